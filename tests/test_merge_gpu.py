"""GPU parity: the HIP path against the CPU oracle, bit for bit.

Every case runs the library through its C ABI (via the Python binding) on
seeded inputs from paper_1303_4312_amd.workloads and compares keys and
payloads byte for byte with oracle.stable_merge / oracle.co_rank_brute.
Sizes span several blocks and a ragged last block; every tile
configuration and both co-rank searches are covered.
"""
import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import workloads
from tests.gpu_util import first_difference, same_bits, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("restore_settings")]

DTYPES = [np.uint32, np.uint64, np.float32]


def check_pairs(A, B, Av=None, Bv=None, offset=0):
    if Av is None:
        Av, Bv = workloads.origin_payloads(A.size, B.size)
    C, Cv = cm.stable_merge_pairs(to_dev(A, offset), to_dev(Av, offset), to_dev(B, offset),
                                  to_dev(Bv, offset))
    C, Cv = to_host(C), to_host(Cv)
    Ce, Cve = oracle.stable_merge(A, B, Av, Bv)
    assert same_bits(C, Ce), f"keys differ first at {first_difference(C, Ce)}"
    assert same_bits(Cv, Cve), f"payloads differ first at {first_difference(Cv, Cve)}"


def check_keys(A, B, offset=0):
    C = to_host(cm.stable_merge(to_dev(A, offset), to_dev(B, offset)))
    Ce = oracle.stable_merge(A, B)
    assert same_bits(C, Ce), f"keys differ first at {first_difference(C, Ce)}"


def random_sorted(rng, size, dtype, hi):
    if np.dtype(dtype) == np.float32:
        return np.sort((rng.integers(0, hi, size) - hi // 2).astype(np.float32) / 4)
    return np.sort(rng.integers(0, hi, size).astype(dtype))


def test_figure_example(figure):
    A = np.array(figure["A"]["keys"], dtype=np.uint32)
    B = np.array(figure["B"]["keys"], dtype=np.uint32)
    Av, Bv = workloads.origin_payloads(A.size, B.size)
    C, Cv = cm.stable_merge_pairs(to_dev(A), to_dev(Av), to_dev(B), to_dev(Bv))
    C, Cv = to_host(C), to_host(Cv)
    assert C.tolist() == figure["C"]["keys"]
    assert Cv[figure["alpha"]["C_index"]] == figure["alpha"]["A_index"]
    assert Cv[figure["beta"]["C_index"]] == (1 << 31) + figure["beta"]["B_index"]
    assert cm.co_rank(22, to_dev(A), to_dev(B)) == (12, 10)
    check_pairs(A.astype(np.float32) / 100, B.astype(np.float32) / 100)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("search,partition", [(0, 0), (1, 0), (0, 1), (1, 1), (1, 2), (0, 3),
                                              (1, 3), (0, 4), (1, 4)])
def test_all_configs_pairs_and_keys(dtype, search, partition):
    cm.set_search(search)
    cm.set_partition(partition)
    rng = np.random.default_rng(100 + search)
    kt = np.dtype(dtype).name
    for c in range(cm.config_count()):
        nt, e = cm.config_info(c)
        T = nt * e
        cm.set_config(kt, True, c)
        cm.set_config(kt, False, c)
        for m, n, hi in ((3 * T + 5, 2 * T - 7, 50), (T - 1, 1, 1000), (T, T, 3),
                         (5, 4 * T + 1, 1 << 20)):
            A = random_sorted(rng, m, dtype, hi)
            B = random_sorted(rng, n, dtype, hi)
            check_pairs(A, B)
            check_keys(A, B)


@pytest.mark.parametrize("partition,stride,xcd,lanes", [
    (0, 64, 1, 1), (1, 64, 1, 1), (2, 64, 0, 1), (1, 16, 0, 1), (2, 16, 1, 1), (3, 64, 1, 1),
    (4, 64, 1, 1), (4, 64, 0, 1), (2, 64, 1, 2), (2, 16, 0, 4), (1, 64, 1, 4), (2, 64, 1, 4),
    (2, 64, 32, 1), (2, 64, 2, 1), (1, 16, 3, 1), (4, 64, 8, 1), (0, 64, 5, 1)])
def test_two_level_partition_edges(partition, stride, xcd, lanes):
    """Block counts around multiples of the coarse stride, with the co-rank
    windows of the fine pass both wide and degenerate; every block order
    (workgroup order, one run per XCD, runs of c blocks with full groups
    and a partial last group); 1, 2 or 4 lanes per fine boundary."""
    cm.set_partition(partition)
    cm.set_coarse_stride(stride)
    cm.set_block_order(xcd)
    cm.set_fine_lanes(lanes)
    nt, e = cm.config_info(cm.tuning_get(cm.OP_MERGE, "uint32", True, 1 << 30)[0])
    T = nt * e
    rng = np.random.default_rng(21)
    for N in (64 * T, 64 * T + 1, 64 * T - 1, 65 * T, 128 * T + T // 2, 200 * T + 7,
              16 * T + 3, 8 * T + 5):
        m = int(rng.integers(0, N + 1))
        for hi in (3, 1 << 30):
            A = random_sorted(rng, m, np.uint32, hi)
            B = random_sorted(rng, N - m, np.uint32, hi)
            check_pairs(A, B)
    d = workloads.structured("a_below_b", 70 * T, 3 * T + 5)
    check_pairs(d["A"], d["B"], d["Av"], d["Bv"])
    check_pairs(d["B"], d["A"], d["Bv"], d["Av"])


@pytest.mark.parametrize("dtype", DTYPES)
def test_streaming_blocks(dtype):
    """One block per resident workgroup (partition 3): sizes from a few
    elements to many steps per workgroup, skewed and degenerate inputs."""
    cm.set_partition(3)
    rng = np.random.default_rng(33)
    kt = np.dtype(dtype).name
    for c in (0, 4, 6):
        cm.set_config(kt, True, c)
        cm.set_config(kt, False, c)
        for m, n, hi in ((1, 0, 5), (0, 5, 5), (3, 4, 5), (1000, 1, 50),
                         (1 << 20, 3 << 19, 1000), (5, 3_000_001, 1 << 20),
                         (2_000_003, 1_999_999, 2)):
            A = random_sorted(rng, m, dtype, hi)
            B = random_sorted(rng, n, dtype, hi)
            check_pairs(A, B)
            check_keys(A, B)
    for kind in ("a_below_b", "interleaved", "all_equal"):
        d = workloads.structured(kind, 1_500_000, 1_500_000, dtype)
        check_pairs(d["A"], d["B"], d["Av"], d["Bv"])
        check_pairs(d["B"], d["A"], d["Bv"], d["Av"])


@pytest.mark.parametrize("dtype", DTYPES)
def test_empty_and_tiny(dtype):
    rng = np.random.default_rng(3)
    for m, n in ((0, 0), (0, 1), (1, 0), (1, 1), (0, 1000), (1000, 0), (2, 3), (17, 1)):
        A = random_sorted(rng, m, dtype, 5)
        B = random_sorted(rng, n, dtype, 5)
        check_pairs(A, B)
        check_keys(A, B)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("offset", [1, 2, 3])
def test_misaligned_bases(dtype, offset):
    rng = np.random.default_rng(offset)
    A = random_sorted(rng, 12_345, dtype, 100)
    B = random_sorted(rng, 23_456, dtype, 100)
    check_pairs(A, B, offset=offset)
    check_keys(A, B, offset=offset)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kind", ["a_below_b", "interleaved", "all_equal"])
def test_structured(dtype, kind):
    for m, n in ((100_003, 99_999), (1 << 17, 1 << 17), (7, 50_000)):
        if kind == "interleaved":
            n = m
        d = workloads.structured(kind, m, n, dtype)
        check_pairs(d["A"], d["B"], d["Av"], d["Bv"])
        # and with the roles of A and B swapped (all of B below A, etc.)
        check_pairs(d["B"], d["A"], d["Bv"], d["Av"])


def test_dup16_full_size():
    """m = n = 2**20, uint32 keys uniform in [0, 2**16): the small workload."""
    d = workloads.dup16()
    check_pairs(d["A"], d["B"], d["Av"], d["Bv"])
    check_keys(d["A"], d["B"])


def test_zipf_reduced():
    d = workloads.zipf(m=1 << 22, n=1 << 20)
    check_pairs(d["A"], d["B"], d["Av"], d["Bv"])


def test_f32_signed_zeros_and_normal():
    d = workloads.f32(m=300_000, n=200_000, signed_zeros=5000)
    check_pairs(d["A"], d["B"], d["Av"], d["Bv"])
    check_keys(d["A"], d["B"])
    A = np.array([-0.0, 0.0, 1.0], dtype=np.float32)
    B = np.array([0.0, -0.0, 1.0], dtype=np.float32)
    check_pairs(A, B)


def test_u64_high_bits():
    d = workloads.u64(m=250_000, n=333_333)
    check_pairs(d["A"], d["B"], d["Av"], d["Bv"])
    check_keys(d["A"], d["B"])


@pytest.mark.parametrize("dtype", DTYPES)
def test_device_co_rank(dtype):
    rng = np.random.default_rng(9)
    for search in (0, 1):
        cm.set_search(search)
        for m, n, hi in ((0, 0, 2), (0, 100, 4), (70_000, 30_001, 10), (5000, 5000, 2)):
            A = random_sorted(rng, m, dtype, hi)
            B = random_sorted(rng, n, dtype, hi)
            ranks = np.unique(np.concatenate([rng.integers(0, m + n + 1, 300), [0, m + n]]))
            ranks = ranks.astype(np.uint64)
            j = to_host(cm.co_rank(to_dev(ranks), to_dev(A), to_dev(B)))
            expect = np.array([oracle.co_rank_brute(int(i), A, B)[0] for i in ranks],
                              dtype=np.uint64)
            assert np.array_equal(j, expect)
            bad = to_host(cm.co_rank(to_dev(np.array([m + n + 1], dtype=np.uint64)),
                                     to_dev(A), to_dev(B)))
            assert bad[0] == np.iinfo(np.uint64).max


def test_check_sorted():
    x = np.sort(np.random.default_rng(1).integers(0, 1000, 100_000)).astype(np.uint32)
    assert cm.check_sorted(to_dev(x))
    x[50_000] = 0
    assert not cm.check_sorted(to_dev(x))
    assert cm.check_sorted(to_dev(np.array([-0.0, 0.0, -0.0], dtype=np.float32)))


def test_explicit_workspace_and_stream():
    import torch
    d = workloads.dup16(m=70_000, n=50_000)
    need = cm.merge_workspace_size("uint32", True, 70_000, 50_000)
    ws = torch.full((need,), 0xAB, dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        A, Av, B, Bv = (to_dev(d[k]) for k in ("A", "Av", "B", "Bv"))
        C, Cv = cm.stable_merge_pairs(A, Av, B, Bv, workspace=ws, stream=s)
    s.synchronize()
    Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
    assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)
    with pytest.raises(cm.CMError) as e:
        cm.stable_merge_pairs(A, Av, B, Bv, workspace=ws[: need - 256])
    assert e.value.status == -5
