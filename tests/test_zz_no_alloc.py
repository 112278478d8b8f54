"""GPU: the allocation-free merge (cm_stable_merge_pairs_noalloc) against the
merge with a caller's workspace (cm_stable_merge_pairs), bit for bit, and
against the oracle: two calls in a row on one GPU, the second smaller than
the first (the per-GPU scratch array keeps the first call's contents, which
the second must not depend on), keys with payloads and keys only, uint32
and float32 keys, an unaligned case; a merge too large for the scratch
array is refused with CM_ENOSPC before anything runs.  Called through the
C ABI (ctypes) with outputs the test allocates beforehand."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import workloads
from tests.gpu_util import first_difference, same_bits, to_dev, to_host

pytestmark = pytest.mark.gpu

ENOSPC = -5


def call_noalloc(A, Av, B, Bv, C, Cv, key_type=0):
    import torch
    lib = cm.load()
    ptr = lambda t: None if t is None else t.data_ptr()
    return lib.cm_stable_merge_pairs_noalloc(key_type, ptr(A), ptr(Av), A.numel(), ptr(B), ptr(Bv), B.numel(),
                                             ptr(C), ptr(Cv), torch.cuda.current_stream().cuda_stream)


def check_case(d, key_type=0, offset=0, payload=True):
    import torch
    A, B = to_dev(d["A"], offset), to_dev(d["B"], offset)
    Av, Bv = (to_dev(d["Av"], offset), to_dev(d["Bv"], offset)) if payload else (None, None)
    N = A.numel() + B.numel()
    C = torch.full((N,), 0x7F7F7F7F, dtype=A.dtype, device=A.device)
    Cv = torch.full((N,), 0x5A5A5A5A, dtype=torch.uint32, device=A.device) if payload else None
    print(f"[noalloc] m={A.numel()} n={B.numel()} key_type={key_type} offset={offset} payload={payload}",
          flush=True)
    assert call_noalloc(A, Av, B, Bv, C, Cv, key_type) == 0
    if payload:
        Cw, Cvw = cm.stable_merge_pairs(A, Av, B, Bv)  # the same merge with a workspace
        Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        assert same_bits(to_host(Cv), to_host(Cvw)), f"payloads differ first at {first_difference(to_host(Cv), to_host(Cvw))}"
        assert same_bits(to_host(Cv), Cve)
    else:
        Cw = cm.stable_merge(A, B)
        Ce = oracle.stable_merge(d["A"], d["B"])
    assert same_bits(to_host(C), to_host(Cw)), f"keys differ first at {first_difference(to_host(C), to_host(Cw))}"
    assert same_bits(to_host(C), Ce)


def test_two_calls_second_smaller():
    # a large merge (two-level boundary pass, 3.4e7 co-ranked block ends'
    # worth of scratch), then a small one (no pass) and a mid-sized one
    check_case(workloads.zipf(seed=11, m=1 << 25, n=(1 << 23) + 5))
    check_case(workloads.dup16(seed=12, m=300_001, n=200_003))
    check_case(workloads.dup16(seed=13, m=3_000_017, n=2_000_011))


def test_keys_only_float_and_unaligned():
    d = workloads.dup16(seed=14, m=1_000_003, n=777_777)
    check_case(d, payload=False)
    f = dict(d)
    f["A"] = (d["A"].astype(np.float32) - 30000.0) / 8
    f["B"] = (d["B"].astype(np.float32) - 30000.0) / 8
    check_case(f, key_type=2)
    check_case(workloads.dup16(seed=15, m=500_001, n=400_003), offset=1)


def test_refuses_merges_beyond_the_scratch():
    import torch
    lib = cm.load()
    # the largest merge the scratch array serves, by the workspace rule
    lo, hi = 1, 1 << 40
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if lib.cm_merge_workspace_size(0, 1, mid, 0) <= cm.NOALLOC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid - 1
    assert lo > 400_000_000  # the single-merge workloads here all fit
    fake = ctypes.c_void_p(1 << 44)
    assert lib.cm_stable_merge_pairs_noalloc(0, fake, fake, lo + 1, fake, fake, 0, fake, fake, None) == ENOSPC
    # and a call after the refusal still works
    check_case(workloads.dup16(seed=16, m=70_001, n=50_003))
