"""GPU: seeded random cases across everything a merge call can vary at
once: key type and order, payload or not, sizes (zero, tiny, ragged, up to
3e5 per side), key distribution (few distinct values, wide, all equal, long
runs of one side), base alignment, tile configuration, co-rank search and
boundary mode, single merge, segmented form, merge sort and batches of
separate merges.  Every result bit for bit against the oracle."""
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


@pytest.mark.parametrize("case", range(60))
def test_random_merge_case_8byte_payloads(case, restore_settings):
    """As above with uint64 payloads (cm_stable_merge_pairs64); expected:
    the oracle's merge with origin payloads, the records gathered by origin
    on the host."""
    from paper_1303_4312_amd import workloads
    rng = np.random.default_rng(zlib.crc32(b"fuzz-pairs64") + case)
    dtype = DTYPES[case % 3]
    descending = bool(rng.integers(0, 2))
    dist = ("few", "wide", "equal", "runs")[int(rng.integers(0, 4))]
    m, n = draw_size(rng), draw_size(rng)
    offset = int(rng.integers(0, 2)) * int(rng.integers(1, 4))
    cfg = int(rng.integers(0, cm.config_count()))
    search = int(rng.integers(0, 2))
    partition = int(rng.choice([-1, 0, 1, 2, 3, 4]))
    print(f"\n[fuzz pairs64 {case}] {np.dtype(dtype).name} desc={descending} {dist} m={m} n={n} "
          f"offset={offset} cfg={cfg} search={search} partition={partition}", flush=True)
    A = draw_keys(rng, m, dtype, dist, descending)
    B = draw_keys(rng, n, dtype, dist, descending)
    cm.set_config(np.dtype(dtype).name, True, cfg)
    cm.set_search(search)
    cm.set_partition(partition)
    Arec = rng.integers(0, 1 << 63, m, dtype=np.uint64)
    Brec = rng.integers(0, 1 << 63, n, dtype=np.uint64)
    C, Cv = cm.stable_merge_pairs(to_dev(A, offset), to_dev(Arec, offset), to_dev(B, offset),
                                  to_dev(Brec, offset), descending=descending)
    Av, Bv = workloads.origin_payloads(m, n)
    Ce, codes = oracle.stable_merge(A, B, Av, Bv, descending=descending)
    origin = np.where(codes < (1 << 31), codes, m + (codes & 0x7FFFFFFF)).astype(np.int64)
    Cve = np.concatenate([Arec, Brec])[origin]
    C, Cv = to_host(C), to_host(Cv)
    assert same_bits(C, Ce), f"keys differ at {first_difference(C, Ce)}"
    assert same_bits(Cv, Cve), f"payloads differ at {first_difference(Cv, Cve)}"


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


@pytest.mark.parametrize("case", range(24))
def test_random_sort_case(case, restore_settings):
    """Stable merge sort of random keys (ties broken by input position),
    keys only or with payloads, in place or not, any tile configuration."""
    import torch
    rng = np.random.default_rng(zlib.crc32(b"fuzz-sort") + case)
    dtype = DTYPES[case % 3]
    descending = bool(rng.integers(0, 2))
    payload = bool(rng.integers(0, 2))
    in_place = bool(rng.integers(0, 2))
    n = draw_size(rng) * int(rng.integers(1, 4))
    cfg = int(rng.integers(0, cm.config_count()))
    print(f"\n[fuzz sort {case}] {np.dtype(dtype).name} desc={descending} pairs={payload} "
          f"n={n} cfg={cfg} in_place={in_place}", flush=True)
    span = int(rng.choice([3, 1000, 1 << 30]))
    keys = rng.integers(0, span, n)
    keys = (keys.astype(np.float32) / 4 if np.dtype(dtype) == np.float32 else keys.astype(dtype))
    vals = np.arange(n, dtype=np.uint32)
    cm.set_config(np.dtype(dtype).name, payload, cfg)
    dk = to_dev(keys)
    dv = to_dev(vals) if payload else None
    out = (dk, dv) if in_place else (None, None)
    res = cm.stable_sort(dk, dv, out[0], out[1], descending=descending)
    if payload:
        Ke, Ve = oracle.stable_sort(keys, vals, descending=descending)
        assert same_bits(to_host(res[0]), Ke) and same_bits(to_host(res[1]), Ve)
    else:
        assert same_bits(to_host(res), oracle.stable_sort(keys, descending=descending))


@pytest.mark.parametrize("case", range(12))
def test_random_batch_case(case):
    """A batch of separately allocated merges of random sizes (some empty)
    in one launch, each against the oracle."""
    rng = np.random.default_rng(zlib.crc32(b"fuzz-batch") + case)
    dtype = DTYPES[case % 3]
    count = int(rng.integers(1, 40))
    merges, host = [], []
    for _ in range(count):
        m, n = draw_size(rng) // 4, draw_size(rng) // 4
        A = draw_keys(rng, m, dtype, "few", False)
        B = draw_keys(rng, n, dtype, "wide", False)
        Av = np.arange(m, dtype=np.uint32)
        Bv = (np.arange(n, dtype=np.uint32) | np.uint32(1 << 31)).astype(np.uint32)
        merges.append((to_dev(A), to_dev(Av), to_dev(B), to_dev(Bv)))
        host.append((A, Av, B, Bv))
    print(f"\n[fuzz batch {case}] {np.dtype(dtype).name} {count} merges, "
          f"{sum(a.size + b.size for a, _, b, _ in host)} outputs", flush=True)
    outs = cm.stable_merge_batch(merges)
    for (A, Av, B, Bv), (C, Cv) in zip(host, outs):
        Ce, Cve = oracle.stable_merge(A, B, Av, Bv)
        assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)
