"""GPU: the partition ablation.  Equal co-rank segments and the classic
cross-rank segments both give the oracle's merge, bit for bit; the segment
bounds are checked exactly: floor(w (m + n) / P) for the co-rank split, and
for the cross-rank split the cuts of P / 2 equidistant samples of each array
ranked in the other (numpy searchsorted), in output order."""
import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import workloads
from tests.gpu_util import same_bits, to_dev, to_host

pytestmark = pytest.mark.gpu


def cross_rank_bounds(A, B, P):
    """Segment starts of the classic partition, computed on the host."""
    m, n, h = A.size, B.size, P // 2
    cuts = []  # (i, side, index) with A's cut first on equal i
    for side, X, Y, length in ((0, A, B, m), (1, B, A, n)):
        step = -(-length // h) if length else 0
        for r in range(h):
            pos = r * step
            if r == 0:
                i = 0
            elif pos >= length:
                i = m + n
            elif side == 0:
                i = pos + int(np.searchsorted(Y, X[pos], side="left"))
            else:
                i = pos + int(np.searchsorted(Y, X[pos], side="right"))
            cuts.append((i, side, r))
    cuts.sort()
    return np.array([c[0] for c in cuts] + [m + n], dtype=np.uint64)


CASES = [
    ("zipf", lambda: workloads.zipf(m=3_000_000, n=1_000_001)),
    ("same arrays", lambda: (lambda d: dict(d, B=d["A"].copy()))(workloads.dup16(m=1 << 20, n=1 << 20))),
    ("a_below_b", lambda: workloads.structured("a_below_b", 700_000, 300_001)),
    ("interleaved", lambda: workloads.structured("interleaved", 500_000, 500_000)),
    ("empty B", lambda: workloads.structured("a_below_b", 100_000, 0)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("P", [2, 64, 2048])
def test_partitions_merge_exactly(name, make, P):
    d = make()
    A, B = d["A"], d["B"]
    Av, Bv = workloads.origin_payloads(A.size, B.size)
    print(f"[ablation] {name} m={A.size} n={B.size} P={P}", flush=True)
    Ce, Cve = oracle.stable_merge(A, B, Av, Bv)
    N = A.size + B.size
    for part in (0, 1):
        C, Cv, bounds = cm.merge_partition_ablation(to_dev(A), to_dev(B), to_dev(Av), to_dev(Bv),
                                                    P=P, partition=part)
        assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve), f"partition {part}"
        got = to_host(bounds)
        if part == 0:
            want = (np.arange(P + 1, dtype=np.uint64) * N) // P
        else:
            want = cross_rank_bounds(A, B, P)
        assert np.array_equal(got, want), f"partition {part}: bounds differ"


def test_keys_only():
    rng = np.random.default_rng(4)
    A = np.sort(rng.standard_normal(200_000).astype(np.float32))
    B = np.sort(rng.standard_normal(150_000).astype(np.float32))
    for part in (0, 1):
        C, bounds = cm.merge_partition_ablation(to_dev(A), to_dev(B), P=512, partition=part)
        assert same_bits(to_host(C), oracle.stable_merge(A, B))
