"""GPU: seeded random cases across everything a merge call can vary at
once: key type and order, payload or not, sizes (zero, tiny, ragged, up to
3e5 per side), key distribution (few distinct values, wide, all equal, long
runs of one side), base alignment, tile configuration, co-rank search and
boundary mode, single merge and segmented form.  Every result bit for bit
against the oracle."""
import zlib

import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from tests.gpu_util import first_difference, same_bits, to_dev, to_host

pytestmark = pytest.mark.gpu

DTYPES = (np.uint32, np.uint64, np.float32)


def draw_keys(rng, size, dtype, dist, descending):
    if dist == "few":
        k = rng.integers(0, 5, size)
    elif dist == "equal":
        k = np.full(size, 3)
    elif dist == "runs":  # long stretches of one value, blocks of distinct ones
        k = np.repeat(rng.integers(0, 1 << 20, max(1, size // 4096 + 1)), 4096)[:size]
    else:
        k = rng.integers(0, 1 << 30, size)
    if np.dtype(dtype) == np.float32:
        k = (k.astype(np.float64) - (1 << 29)).astype(np.float32) / 8
        k[rng.random(size) < 0.02] = -0.0
        k[rng.random(size) < 0.02] = 0.0
        order = np.argsort(-k if descending else k, kind="stable")
        return k[order]
    k = np.sort(k.astype(dtype))
    return k[::-1].copy() if descending else k


def draw_size(rng):
    r = rng.random()
    if r < 0.1:
        return 0
    if r < 0.25:
        return int(rng.integers(1, 40))
    return int(np.exp(rng.uniform(np.log(40), np.log(300_000))))


@pytest.mark.parametrize("case", range(160))
def test_random_merge_case(case, restore_settings):
    rng = np.random.default_rng(zlib.crc32(b"fuzz") + case)
    dtype = DTYPES[case % 3]
    descending = bool(rng.integers(0, 2))
    payload = bool(rng.integers(0, 2))
    dist = ("few", "wide", "equal", "runs")[int(rng.integers(0, 4))]
    m, n = draw_size(rng), draw_size(rng)
    offset = int(rng.integers(0, 2)) * int(rng.integers(1, 4))
    cfg = int(rng.integers(0, cm.config_count()))
    search = int(rng.integers(0, 2))
    partition = int(rng.choice([-1, 0, 1, 2, 3, 4]))
    print(f"\n[fuzz {case}] {np.dtype(dtype).name} desc={descending} pairs={payload} {dist} "
          f"m={m} n={n} offset={offset} cfg={cfg} search={search} partition={partition}",
          flush=True)
    A = draw_keys(rng, m, dtype, dist, descending)
    B = draw_keys(rng, n, dtype, dist, descending)
    kd = np.dtype(dtype).name
    cm.set_config(kd, payload, cfg)
    cm.set_search(search)
    cm.set_partition(partition)
    if payload:
        Av = rng.integers(0, 1 << 32, m, dtype=np.uint64).astype(np.uint32)
        Bv = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
        C, Cv = cm.stable_merge_pairs(to_dev(A, offset), to_dev(Av, offset), to_dev(B, offset),
                                      to_dev(Bv, offset), descending=descending)
        Ce, Cve = oracle.stable_merge(A, B, Av, Bv, descending=descending)
        C, Cv = to_host(C), to_host(Cv)
        assert same_bits(C, Ce), f"keys differ at {first_difference(C, Ce)}"
        assert same_bits(Cv, Cve), f"payloads differ at {first_difference(Cv, Cve)}"
    else:
        C = to_host(cm.stable_merge(to_dev(A, offset), to_dev(B, offset), descending=descending))
        Ce = oracle.stable_merge(A, B, descending=descending)
        assert same_bits(C, Ce), f"keys differ at {first_difference(C, Ce)}"


@pytest.mark.parametrize("case", range(40))
def test_random_segmented_case(case, restore_settings):
    import torch
    rng = np.random.default_rng(zlib.crc32(b"fuzz-seg") + case)
    dtype = DTYPES[case % 3]
    descending = bool(rng.integers(0, 2))
    S = int(rng.integers(1, 3000))
    la = rng.integers(0, 200, S) * (rng.random(S) < 0.8)
    lb = rng.integers(0, 200, S) * (rng.random(S) < 0.8)
    a_off = np.concatenate([[0], np.cumsum(la)]).astype(np.uint64)
    b_off = np.concatenate([[0], np.cumsum(lb)]).astype(np.uint64)
    dist = ("few", "wide", "equal")[int(rng.integers(0, 3))]
    A = np.concatenate([draw_keys(rng, int(x), dtype, dist, descending) for x in la] or [np.zeros(0, dtype)])
    B = np.concatenate([draw_keys(rng, int(x), dtype, dist, descending) for x in lb] or [np.zeros(0, dtype)])
    A, B = A.astype(dtype), B.astype(dtype)
    Av = np.arange(A.size, dtype=np.uint32)
    Bv = (np.arange(B.size, dtype=np.uint32) | np.uint32(1 << 31)).astype(np.uint32)
    cfg = int(rng.integers(0, cm.config_count()))
    search = int(rng.integers(0, 2))
    print(f"\n[fuzz seg {case}] {np.dtype(dtype).name} desc={descending} S={S} {dist} "
          f"m={A.size} n={B.size} cfg={cfg} search={search}", flush=True)
    cm.set_config(np.dtype(dtype).name, True, cfg)
    cm.set_search(search)
    C, Cv = cm.stable_merge_segmented(to_dev(A), to_dev(a_off), to_dev(B), to_dev(b_off), to_dev(Av),
                                      to_dev(Bv), descending=descending)
    Ce, Cve = oracle.stable_merge_segmented(A, a_off, B, b_off, Av, Bv, descending=descending)
    C, Cv = to_host(C), to_host(Cv)
    assert same_bits(C, Ce), f"keys differ at {first_difference(C, Ce)}"
    assert same_bits(Cv, Cve), f"payloads differ at {first_difference(Cv, Cve)}"
