"""GPU: block kernels launched with fewer workgroups than blocks (cm_set_grid),
so every workgroup strides over several blocks of Algorithm 2 and the
barrier between a workgroup's blocks runs.  Single merges (each boundary
mode that runs the block kernel, keys only and with 4- or 8-byte payloads),
segmented batches, batches of separate merges and sorts, each against the
oracle bit for bit, at grids of one workgroup, a few, a round count that
leaves a partial last round, more than a block-order group, and the
resident count of the device."""
import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import workloads
from tests.gpu_util import first_difference, same_bits, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("restore_settings")]

GRIDS = [1, 3, 64, 300, -1]


def sorted_keys(rng, size, dtype, hi):
    if np.dtype(dtype) == np.float32:
        return np.sort((rng.integers(0, hi, size) - hi // 2).astype(np.float32) / 4)
    return np.sort(rng.integers(0, hi, size).astype(dtype))


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("partition", [0, 2, 4])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64, np.float32])
def test_single_merge(grid, partition, dtype):
    print(f"[grid] merge grid={grid} partition={partition} {np.dtype(dtype).name}", flush=True)
    cm.set_grid(grid)
    cm.set_partition(partition)
    rng = np.random.default_rng(400 + partition)
    # about 700 blocks of the 256 x 7 tile, a ragged last block
    m, n = 700_001, 554_321
    for hi in (5, 1 << 20):
        A, B = sorted_keys(rng, m, dtype, hi), sorted_keys(rng, n, dtype, hi)
        Av, Bv = workloads.origin_payloads(m, n)
        C, Cv = cm.stable_merge_pairs(to_dev(A), to_dev(Av), to_dev(B), to_dev(Bv))
        Ce, Cve = oracle.stable_merge(A, B, Av, Bv)
        C, Cv = to_host(C), to_host(Cv)
        assert same_bits(C, Ce), f"keys differ first at {first_difference(C, Ce)}"
        assert same_bits(Cv, Cve), f"payloads differ first at {first_difference(Cv, Cve)}"
        Ck = to_host(cm.stable_merge(to_dev(A, 1), to_dev(B, 1)))  # unaligned: element-wise staging
        assert same_bits(Ck, Ce), f"keys only: first difference at {first_difference(Ck, Ce)}"


@pytest.mark.parametrize("grid", [1, 64, -1])
def test_pairs64(grid):
    print(f"[grid] pairs64 grid={grid}", flush=True)
    cm.set_grid(grid)
    rng = np.random.default_rng(410)
    m, n = 300_007, 400_009
    A, B = sorted_keys(rng, m, np.uint32, 1000), sorted_keys(rng, n, np.uint32, 1000)
    Arec = rng.integers(0, 1 << 62, m, dtype=np.uint64)
    Brec = rng.integers(0, 1 << 62, n, dtype=np.uint64)
    C, Cv = cm.stable_merge_pairs(to_dev(A), to_dev(Arec), to_dev(B), to_dev(Brec))
    # the oracle merges origin codes; the 8-byte records follow them on the host
    Av, Bv = workloads.origin_payloads(m, n)
    Ce, codes = oracle.stable_merge(A, B, Av, Bv)
    idx = np.where(codes < (1 << 31), codes, m + (codes & 0x7FFFFFFF)).astype(np.int64)
    assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), np.concatenate([Arec, Brec])[idx])


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("partition", [0, 2])
def test_segmented(grid, partition):
    print(f"[grid] segmented grid={grid} partition={partition}", flush=True)
    cm.set_grid(grid)
    cm.set_partition(partition)
    d = workloads.segmented(seed=420 + partition, num_seg=4000, max_side=1 << 10, min_side=0)
    A, B = to_dev(d["A"]), to_dev(d["B"])
    a_off, b_off = to_dev(d["a_off"]), to_dev(d["b_off"])
    C, Cv = cm.stable_merge_segmented(A, a_off, B, b_off, to_dev(d["Av"]), to_dev(d["Bv"]))
    Ce, Cve = oracle.stable_merge_segmented(d["A"], d["a_off"], d["B"], d["b_off"], d["Av"], d["Bv"])
    C, Cv = to_host(C), to_host(Cv)
    assert same_bits(C, Ce), f"keys differ first at {first_difference(C, Ce)}"
    assert same_bits(Cv, Cve), f"payloads differ first at {first_difference(Cv, Cve)}"


@pytest.mark.parametrize("grid", GRIDS)
def test_batch(grid):
    print(f"[grid] batch grid={grid}", flush=True)
    cm.set_grid(grid)
    rng = np.random.default_rng(430)
    host, merges = [], []
    for m, n in ((0, 0), (1, 0), (0, 3), (150_000, 70_001), (1, 1 << 17), (90_001, 3), (2048, 2048),
                 (300_000, 300_001)):
        A, B = sorted_keys(rng, m, np.uint32, 100), sorted_keys(rng, n, np.uint32, 100)
        Av, Bv = workloads.origin_payloads(m, n)
        host.append((A, B, Av, Bv))
        merges.append((to_dev(A), to_dev(Av), to_dev(B), to_dev(Bv)))
    outs = cm.stable_merge_batch(merges)
    for (A, B, Av, Bv), (C, Cv) in zip(host, outs):
        Ce, Cve = oracle.stable_merge(A, B, Av, Bv)
        assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)


@pytest.mark.parametrize("grid", [1, 7, 300, -1])
@pytest.mark.parametrize("payload", [True, False])
def test_sort(grid, payload):
    print(f"[grid] sort grid={grid} payload={payload}", flush=True)
    cm.set_grid(grid)
    rng = np.random.default_rng(440)
    keys = rng.integers(0, 1000, 1_000_003).astype(np.uint32)
    if payload:
        vals = np.arange(keys.size, dtype=np.uint32)
        C, Cv = cm.stable_sort(to_dev(keys), to_dev(vals))
        Ce, Cve = oracle.stable_sort(keys, vals)
        assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)
    else:
        assert same_bits(to_host(cm.stable_sort(to_dev(keys))), oracle.stable_sort(keys))


def test_grid_setting():
    assert cm.get_grid() == 0
    for g in (-1, 0, 1, 1 << 20):
        cm.set_grid(g)
        assert cm.get_grid() == g
    with pytest.raises(cm.CMError):
        cm.set_grid(-2)
