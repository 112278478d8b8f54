"""GPU: cm_copy_tiles, the block merge's data movement without the merge.
Each tile must hold A's share of its 16-byte units, then B's share, where
A's share of the first q units is floor(q * (m/4) / (N/4))."""
import numpy as np
import pytest

import paper_1303_4312_amd as cm
from tests.gpu_util import same_bits, to_dev, to_host

pytestmark = pytest.mark.gpu


def expected(A, B, T):
    mq, nq = A.size // 4, B.size // 4
    Nq, TQ = mq + nq, T // 4
    Au, Bu = A.reshape(-1, 4), B.reshape(-1, 4)
    parts = []
    for q0 in range(0, Nq, TQ):
        q1 = min(q0 + TQ, Nq)
        ja, jb = q0 * mq // Nq, q1 * mq // Nq
        parts.append(Au[ja:jb])
        parts.append(Bu[q0 - ja:q1 - jb])
    return np.concatenate(parts).reshape(-1) if parts else np.zeros(0, A.dtype)


@pytest.mark.parametrize("m,n", [(4000, 1236), (0, 512), (512, 0), (4, 4), (1 << 18, (1 << 16) + 4)])
def test_copy_tiles_matches_the_tile_rule(m, n):
    rng = np.random.default_rng(m * 7 + n)
    A = rng.integers(0, 1 << 32, m, dtype=np.uint32)
    B = rng.integers(0, 1 << 32, n, dtype=np.uint32)
    Av = np.arange(m, dtype=np.uint32)
    Bv = np.arange(n, dtype=np.uint32) | np.uint32(1 << 31)
    dA, dB, dAv, dBv = to_dev(A), to_dev(B), to_dev(Av), to_dev(Bv)
    for cfg in range(cm.config_count()):
        nt, e = cm.config_info(cfg)
        C, Cv = cm.copy_tiles(cfg, dA, dAv, dB, dBv)
        assert same_bits(to_host(C), expected(A, B, nt * e)), f"config {cfg}: keys"
        assert same_bits(to_host(Cv), expected(Av, Bv, nt * e)), f"config {cfg}: payloads"
        # every input element appears exactly once
        assert np.array_equal(np.sort(to_host(Cv)), np.sort(np.concatenate([Av, Bv])))
