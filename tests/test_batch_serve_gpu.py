"""GPU: the batch of separate merges and the serving loop.

Each request's result must be the same bits whether it runs alone (a single
merge call) or in a batch mixed with other requests, and equal the oracle."""
import time

import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import serve, workloads
from tests.gpu_util import same_bits, to_dev, to_host

pytestmark = pytest.mark.gpu


def requests(count, seed, lo=1 << 10, hi=1 << 18):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = workloads.request(int(rng.integers(1 << 30)), lo=lo, hi=hi)
        out.append(d)
    return out


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64, np.float32])
def test_batch_call_matches_oracle(dtype):
    rng = np.random.default_rng(1)
    sizes = [(0, 0), (1, 0), (0, 3), (5000, 7000), (1, 1 << 17), (70_001, 3), (2048, 2048)]
    host, merges = [], []
    for m, n in sizes:
        if np.dtype(dtype) == np.float32:
            A = np.sort(rng.standard_normal(m).astype(np.float32))
            B = np.sort(rng.standard_normal(n).astype(np.float32))
        else:
            A = np.sort(rng.integers(0, 100, m)).astype(dtype)
            B = np.sort(rng.integers(0, 100, n)).astype(dtype)
        Av, Bv = workloads.origin_payloads(m, n)
        host.append((A, B, Av, Bv))
        merges.append((to_dev(A), to_dev(Av), to_dev(B), to_dev(Bv)))
    outs = cm.stable_merge_batch(merges)
    for (A, B, Av, Bv), (C, Cv) in zip(host, outs):
        Ce, Cve = oracle.stable_merge(A, B, Av, Bv)
        assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)
    keys_only = cm.stable_merge_batch([(m[0], m[2]) for m in merges])
    for (A, B, _, _), C in zip(host, keys_only):
        assert same_bits(to_host(C), oracle.stable_merge(A, B))


def test_batch_all_configs():
    reqs = requests(12, seed=2, lo=1, hi=1 << 14)
    merges = [(to_dev(d["A"]), to_dev(d["Av"]), to_dev(d["B"]), to_dev(d["Bv"])) for d in reqs]
    total = sum(d["A"].size + d["B"].size for d in reqs)
    try:
        for c in range(cm.config_count()):
            for search in (0, 1):
                cm.tuning_set(cm.OP_BATCH, "uint32", True, int(total).bit_length(), c, search, 0)
                outs = cm.stable_merge_batch(merges)
                for d, (C, Cv) in zip(reqs, outs):
                    Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
                    assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)
    finally:
        cm.tuning_clear()


@pytest.mark.parametrize("order", [0, 1, 2, 3, 32])
def test_batch_every_block_order(order, restore_settings):
    """The batch kernel's block order (runs of c blocks per XCD with full
    groups and a partial last group, one run per XCD, workgroup order) only
    changes which workgroup merges which block."""
    reqs = requests(12, seed=3, lo=1, hi=1 << 15)
    merges = [(to_dev(d["A"]), to_dev(d["Av"]), to_dev(d["B"]), to_dev(d["Bv"])) for d in reqs]
    cm.set_block_order(order)
    outs = cm.stable_merge_batch(merges)
    for d, (C, Cv) in zip(reqs, outs):
        Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)


def test_serving_result_alone_equals_in_the_mix():
    import torch
    reqs = requests(24, seed=3)
    dev_reqs = [(to_dev(d["A"]), to_dev(d["B"]), to_dev(d["Av"]), to_dev(d["Bv"])) for d in reqs]
    alone = []
    for A, B, Av, Bv in dev_reqs:
        C, Cv = cm.stable_merge_pairs(A, Av, B, Bv)
        alone.append((to_host(C), to_host(Cv)))
    ex = serve.GpuExecutor()
    budget = sum(ex.footprint(*r) for r in dev_reqs) // 3  # forces queueing
    srv = serve.Server(ex, budget_bytes=budget, max_batch=16, max_inflight=2)
    torch.cuda.synchronize()
    with srv:
        futs = []
        for r in dev_reqs:
            futs.append(srv.submit(*r))
            time.sleep(0.0005)
        mixed = [f.result(timeout=60) for f in futs]
    torch.cuda.synchronize()
    for k, ((C, Cv), (Ca, Cva)) in enumerate(zip(mixed, alone)):
        assert same_bits(to_host(C), Ca), f"request {k} keys differ alone vs in the mix"
        assert same_bits(to_host(Cv), Cva), f"request {k} payloads differ alone vs in the mix"
    for d, (Ca, Cva) in list(zip(reqs, alone))[:6]:
        Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        assert same_bits(Ca, Ce) and same_bits(Cva, Cve)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert srv.budget.peak <= budget and srv.budget.used == 0
    assert st["batches"] >= 2


def test_serving_refuses_request_over_budget():
    d = workloads.request(5, lo=1 << 12, hi=1 << 12)
    r = (to_dev(d["A"]), to_dev(d["B"]), to_dev(d["Av"]), to_dev(d["Bv"]))
    ex = serve.GpuExecutor()
    srv = serve.Server(ex, budget_bytes=ex.footprint(*r) - 1)
    with srv:
        with pytest.raises(serve.BudgetError):
            srv.submit(*r).result(timeout=30)


@pytest.mark.parametrize("partition", [0, 1, 2, 4])
@pytest.mark.parametrize("count,upload", [(9, False), (9, True), (16, False), (40, True)])
@pytest.mark.parametrize("stride", [16, 64])
def test_batch_boundary_modes(partition, count, upload, stride, restore_settings):
    """Every boundary mode of a batch (one-level pass, two-level pass with
    64- or 16-lane coarse searches, no pass), descriptors in the kernel
    arguments or uploaded, coarse strides that put coarse slots in some
    merges and none in others; empty, one-element and lopsided merges among
    them, keys and payloads against the oracle."""
    print(f"[batch modes] partition={partition} count={count} upload={upload} stride={stride}",
          flush=True)
    cm.set_partition(partition)
    cm.set_coarse_stride(stride)
    rng = np.random.default_rng(600 + count)
    host, merges = [], []
    fixed = [(0, 0), (1, 0), (0, 1), (1 << 16, 3), (5, 200_001)]
    for k in range(count):
        if k < len(fixed):
            m, n = fixed[k]
        else:
            m, n = (int(x) for x in np.exp(rng.uniform(0, np.log(300_000), 2)))
        hi = (3, 1000, 1 << 30)[k % 3]
        A = np.sort(rng.integers(0, hi, m)).astype(np.uint32)
        B = np.sort(rng.integers(0, hi, n)).astype(np.uint32)
        Av, Bv = workloads.origin_payloads(m, n)
        host.append((A, B, Av, Bv))
        merges.append((to_dev(A), to_dev(Av), to_dev(B), to_dev(Bv)))
    outs = cm.stable_merge_batch(merges, upload=upload)
    for k, ((A, B, Av, Bv), (C, Cv)) in enumerate(zip(host, outs)):
        Ce, Cve = oracle.stable_merge(A, B, Av, Bv)
        assert same_bits(to_host(C), Ce), f"merge {k} ({A.size}, {B.size}): keys"
        assert same_bits(to_host(Cv), Cve), f"merge {k} ({A.size}, {B.size}): payloads"
    keys_only = cm.stable_merge_batch([(m[0], m[2]) for m in merges], upload=upload)
    for k, ((A, B, _, _), C) in enumerate(zip(host, keys_only)):
        assert same_bits(to_host(C), oracle.stable_merge(A, B)), f"merge {k}: keys only"


@pytest.mark.parametrize("dtype", [np.uint64, np.float32])
@pytest.mark.parametrize("partition", [2, 4])
def test_batch_modes_other_keys(dtype, partition, restore_settings):
    cm.set_partition(partition)
    rng = np.random.default_rng(650)
    host, merges = [], []
    for m, n in ((70_001, 3), (0, 5), (40_000, 90_000), (1, 1), (123_457, 65_536)):
        if np.dtype(dtype) == np.float32:
            A = np.sort(rng.standard_normal(m).astype(np.float32))
            B = np.sort(rng.standard_normal(n).astype(np.float32))
        else:
            A = np.sort(rng.integers(0, 1 << 63, m, dtype=np.uint64))
            B = np.sort(rng.integers(0, 1 << 63, n, dtype=np.uint64))
        Av, Bv = workloads.origin_payloads(m, n)
        host.append((A, B, Av, Bv))
        merges.append((to_dev(A), to_dev(Av), to_dev(B), to_dev(Bv)))
    for upload in (False, True):
        outs = cm.stable_merge_batch(merges, upload=upload)
        for (A, B, Av, Bv), (C, Cv) in zip(host, outs):
            Ce, Cve = oracle.stable_merge(A, B, Av, Bv)
            assert same_bits(to_host(C), Ce) and same_bits(to_host(Cv), Cve)
