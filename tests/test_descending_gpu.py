"""GPU: keys in nonincreasing order (the CM_KEY_*_DESC types), bit-exact
against the oracle under the reversed order: single merges in every
boundary mode and search, tile configurations, the segmented batch, the
merge sort, device and host co-ranks, the sortedness check and the native
server."""
import time

import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import serve, workloads
from tests.gpu_util import first_difference, same_bits, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("restore_settings")]

DTYPES = [np.uint32, np.uint64, np.float32]


def desc_sorted(rng, n, dtype, hi):
    if np.dtype(dtype) == np.float32:
        k = (rng.integers(0, hi, n) - hi // 2).astype(np.float32) / 4
        k[rng.random(n) < 0.05] = -0.0
        return k[np.argsort(-k, kind="stable")]
    return np.sort(rng.integers(0, hi, n).astype(dtype))[::-1].copy()


def check_pairs(A, B, offset=0):
    print(f"[desc] merge m={A.size} n={B.size} {A.dtype} offset={offset}", flush=True)
    Av, Bv = workloads.origin_payloads(A.size, B.size)
    C, Cv = cm.stable_merge_pairs(to_dev(A, offset), to_dev(Av, offset), to_dev(B, offset),
                                  to_dev(Bv, offset), descending=True)
    Ce, Cve = oracle.stable_merge(A, B, Av, Bv, descending=True)
    C, Cv = to_host(C), to_host(Cv)
    assert same_bits(C, Ce), f"keys differ first at {first_difference(C, Ce)}"
    assert same_bits(Cv, Cve), f"payloads differ first at {first_difference(Cv, Cve)}"
    Ck = to_host(cm.stable_merge(to_dev(A), to_dev(B), descending=True))
    assert same_bits(Ck, Ce)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("search,partition", [(0, 0), (1, 2), (1, 4), (0, 3), (1, -1)])
def test_merge_modes(dtype, search, partition):
    cm.set_search(search)
    cm.set_partition(partition)
    rng = np.random.default_rng(31)
    for m, n, hi in ((0, 5, 9), (1, 0, 9), (7, 9, 3), (3000, 1, 50), (20_001, 30_000, 100),
                     (250_000, 70_003, 1 << 20)):
        check_pairs(desc_sorted(rng, m, dtype, hi), desc_sorted(rng, n, dtype, hi))


def test_configurations_and_misaligned():
    rng = np.random.default_rng(32)
    for c in range(cm.config_count()):
        cm.set_config("uint32", True, c)
        cm.set_config("uint32", False, c)
        check_pairs(desc_sorted(rng, 40_000, np.uint32, 30), desc_sorted(rng, 33_333, np.uint32, 30))
    for off in (1, 3):
        check_pairs(desc_sorted(rng, 50_000, np.float32, 64),
                    desc_sorted(rng, 40_001, np.float32, 64), offset=off)


def test_co_rank_and_check_sorted():
    rng = np.random.default_rng(33)
    A = desc_sorted(rng, 5000, np.uint64, 40)
    B = desc_sorted(rng, 3000, np.uint64, 40)
    ranks = np.array([0, 1, 17, 4000, 7999, 8000], dtype=np.uint64)
    j = to_host(cm.co_rank(to_dev(ranks), to_dev(A), to_dev(B), descending=True))
    for r, jj in zip(ranks.tolist(), j.tolist()):
        assert (jj, r - jj) == oracle.co_rank_brute(r, A, B, descending=True)
        assert cm.co_rank_host(r, A, B, descending=True) == (jj, r - jj)
    assert cm.check_sorted(to_dev(A), descending=True)
    assert not cm.check_sorted(to_dev(A))
    assert cm.check_sorted(to_dev(A[::-1].copy()))


def test_segmented():
    rng = np.random.default_rng(34)
    d = workloads.segmented(seed=7, num_seg=3000, max_side=1 << 10)
    A, B = d["A"].astype(np.uint32), d["B"].astype(np.uint32)
    for s in range(3000):  # reverse each segment: nonincreasing per segment
        a0, a1 = int(d["a_off"][s]), int(d["a_off"][s + 1])
        b0, b1 = int(d["b_off"][s]), int(d["b_off"][s + 1])
        A[a0:a1] = A[a0:a1][::-1]
        B[b0:b1] = B[b0:b1][::-1]
    print("[desc] segmented 3000 segments", flush=True)
    C, Cv = cm.stable_merge_segmented(to_dev(A), to_dev(d["a_off"]), to_dev(B), to_dev(d["b_off"]),
                                      to_dev(d["Av"]), to_dev(d["Bv"]), descending=True)
    Ce, Cve = oracle.stable_merge_segmented(A, d["a_off"], B, d["b_off"], d["Av"], d["Bv"],
                                            descending=True)
    assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)
    del rng


@pytest.mark.parametrize("dtype", DTYPES)
def test_sort(dtype):
    rng = np.random.default_rng(35)
    for n in (1, 1791, 1793, 100_003, 1 << 20):
        keys = desc_sorted(rng, n, dtype, 1000)
        rng.shuffle(keys)
        print(f"[desc] sort n={n} {np.dtype(dtype).name}", flush=True)
        vals = np.arange(n, dtype=np.uint32)
        C, Cv = cm.stable_sort(to_dev(keys), to_dev(vals), descending=True)
        Ce, Cve = oracle.stable_sort(keys, vals, descending=True)
        assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)


def test_native_server_descending():
    rng = np.random.default_rng(36)
    with serve.NativeServer("float32", True, arena_bytes=1 << 24, descending=True) as srv:
        host, tickets = {}, []
        for k in range(10):
            A = desc_sorted(rng, int(rng.integers(0, 40_000)), np.float32, 300)
            B = desc_sorted(rng, int(rng.integers(0, 40_000)), np.float32, 300)
            Av, Bv = workloads.origin_payloads(A.size, B.size)
            dev = [to_dev(x) for x in (A, B, Av, Bv)]  # kept alive until reported
            t = srv.submit(*dev)
            tickets.append(t)
            host[t] = (A, B, Av, Bv, dev)
        seen = {}
        t_end = time.time() + 60
        while len(seen) < len(tickets):
            assert time.time() < t_end
            for d in srv.poll(wait_us=2000):
                assert d.status == 0
                A, B, Av, Bv, _ = host[d.ticket]
                C, Cv = srv.outputs(d, A.size + B.size)
                seen[d.ticket] = (to_host(C), to_host(Cv))
                srv.release(d.ticket)
    for t in tickets:
        A, B, Av, Bv, _ = host[t]
        Ce, Cve = oracle.stable_merge(A, B, Av, Bv, descending=True)
        assert same_bits(seen[t][0], Ce) and same_bits(seen[t][1], Cve)
