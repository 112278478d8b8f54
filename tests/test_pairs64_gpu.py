"""GPU: the stable merge with 8-byte payloads (cm_stable_merge_pairs64).

Each payload must land beside its key: the result must equal the oracle's
merge with origin payloads followed by a host gather of the 8-byte records
(bit for bit), for every key type and order, every boundary mode, every
tile configuration, ragged sizes around the tile and unaligned bases (the
element-wise staging path)."""
import zlib

import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import workloads
from tests.gpu_util import same_bits, to_dev, to_host

pytestmark = pytest.mark.gpu


def sorted_keys(rng, size, dtype, hi, descending):
    if np.dtype(dtype) == np.float32:
        k = np.sort((rng.integers(0, hi, size) - hi // 2).astype(np.float32) / 4)
    else:
        k = np.sort(rng.integers(0, hi, size).astype(dtype))
    return k[::-1].copy() if descending else k


def expected(A, B, Arec, Brec, descending):
    Av, Bv = workloads.origin_payloads(A.size, B.size)
    C, codes = oracle.stable_merge(A, B, Av, Bv, descending=descending)
    src = np.concatenate([Arec, Brec])
    idx = np.where(codes < (1 << 31), codes, A.size + (codes & 0x7FFFFFFF)).astype(np.int64)
    return C, src[idx]


def check(A, B, descending=False, offset=0, seed=0):
    rng = np.random.default_rng(seed)
    Arec = rng.integers(0, 1 << 63, A.size, dtype=np.uint64)
    Brec = rng.integers(0, 1 << 63, B.size, dtype=np.uint64)
    C, Cv = cm.stable_merge_pairs(to_dev(A, offset), to_dev(Arec, offset), to_dev(B), to_dev(Brec),
                                  descending=descending)
    Ce, Cve = expected(A, B, Arec, Brec, descending)
    assert same_bits(to_host(C), Ce)
    assert same_bits(to_host(Cv), Cve)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64, np.float32])
@pytest.mark.parametrize("descending", [False, True])
@pytest.mark.parametrize("partition", [0, 1, 2, 3, 4])
def test_pairs64_key_types_orders_and_boundary_modes(dtype, descending, partition, restore_settings):
    cm.set_partition(partition)
    rng = np.random.default_rng(zlib.crc32(f"{np.dtype(dtype).name}{descending}{partition}".encode()))
    print(f"[pairs64] {np.dtype(dtype).name} descending={descending} partition={partition}", flush=True)
    for m, n, hi in ((70_001, 33_333, 5000), (1, 0, 9), (0, 5, 9), (3000, 1, 2), (2, 300_000, 1 << 20)):
        check(sorted_keys(rng, m, dtype, hi, descending), sorted_keys(rng, n, dtype, hi, descending),
              descending, seed=m + n)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_pairs64_every_tile_ragged_and_unaligned(dtype, restore_settings):
    rng = np.random.default_rng(7)
    for cfg in range(cm.config_count()):
        cm.set_config(np.dtype(dtype).name, True, cfg)
        nt, e = cm.config_info(cfg)
        T = nt * e
        print(f"[pairs64] {np.dtype(dtype).name} tile {nt}x{e}", flush=True)
        for part in (2, 4):
            cm.set_partition(part)
            for m, n, offset in ((3 * T + 5, 2 * T - 7, 0), (T - 1, 1, 1), (T, T, 0), (5, 4 * T + 1, 3)):
                check(sorted_keys(rng, m, dtype, 50, False), sorted_keys(rng, n, dtype, 50, False),
                      offset=offset, seed=cfg * 100 + part)


def test_pairs64_headline_size():
    """The headline arrays (m = 2^28, n = 2^26, Zipf keys) with 8-byte
    payloads 3 x (origin index) + 1: element by element against the
    oracle's merge with origin payloads, the codes mapped on the host."""
    import torch
    d = workloads.zipf()
    A, B = d["A"], d["B"]
    m, n = A.size, B.size
    print(f"[pairs64] headline m={m} n={n}", flush=True)
    Arec = torch.arange(m, dtype=torch.int64, device="cuda:0") * 3 + 1
    Brec = (torch.arange(n, dtype=torch.int64, device="cuda:0") + m) * 3 + 1
    C, Cv = cm.stable_merge_pairs(to_dev(A), Arec.view(torch.uint64), to_dev(B), Brec.view(torch.uint64))
    C, Cv = to_host(C), to_host(Cv.view(torch.int64))
    del Arec, Brec
    torch.cuda.empty_cache()
    Ce, codes = oracle.stable_merge(A, B, d["Av"], d["Bv"])
    origin = np.where(codes < (1 << 31), codes, m + (codes & 0x7FFFFFFF)).astype(np.int64)
    assert same_bits(C, Ce)
    assert np.array_equal(Cv, origin * 3 + 1)
