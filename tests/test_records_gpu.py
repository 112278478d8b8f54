"""GPU: payloads of any width.  Keys are merged with origin codes as their
payloads and records of W bytes follow by code; the result must equal the
oracle's merge with origin payloads followed by a host gather of the
records, for widths that take every word size of the gather (16, 8, 4 and
1 bytes) and for both key orders."""
import zlib

import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import workloads
from tests.gpu_util import same_bits, to_dev, to_host

pytestmark = pytest.mark.gpu


def expected(A, B, Arec, Brec, descending):
    Av, Bv = workloads.origin_payloads(A.size, B.size)
    C, codes = oracle.stable_merge(A, B, Av, Bv, descending=descending)
    src = np.concatenate([Arec, Brec])
    idx = np.where(codes < (1 << 31), codes, A.size + (codes & 0x7FFFFFFF)).astype(np.int64)
    return C, src[idx]


@pytest.mark.parametrize("shape,dtype", [((), np.uint8), ((3,), np.uint8), ((), np.uint32),
                                         ((), np.uint64), ((3,), np.uint32), ((4,), np.uint32),
                                         ((2, 4), np.float32), ((4,), np.uint64)])
@pytest.mark.parametrize("descending", [False, True])
def test_merge_records(shape, dtype, descending):
    import torch
    rng = np.random.default_rng(zlib.crc32(f"{shape}{np.dtype(dtype).name}".encode()))
    m, n = 70_001, 33_333
    A = np.sort(rng.integers(0, 5000, m).astype(np.uint32))
    B = np.sort(rng.integers(0, 5000, n).astype(np.uint32))
    if descending:
        A, B = A[::-1].copy(), B[::-1].copy()
    Arec = rng.integers(0, 255, (m,) + shape).astype(dtype)
    Brec = rng.integers(0, 255, (n,) + shape).astype(dtype)
    print(f"[records] {np.dtype(dtype).name}{shape} descending={descending}", flush=True)
    C, Crec = cm.merge_records(to_dev(A), to_dev(B), torch.from_numpy(Arec).cuda(),
                               torch.from_numpy(Brec).cuda(), descending=descending)
    Ce, Crec_e = expected(A, B, Arec, Brec, descending)
    assert same_bits(to_host(C), Ce)
    assert np.array_equal(to_host(Crec).view(np.uint8), np.ascontiguousarray(Crec_e).view(np.uint8))


def test_origin_codes_and_empty():
    import torch
    a, b = cm.origin_codes(5, 3)
    assert to_host(a).tolist() == [0, 1, 2, 3, 4]
    assert to_host(b).tolist() == [(1 << 31) + y for y in range(3)]
    a, b = cm.origin_codes(0, 0)
    assert a.numel() == 0 and b.numel() == 0
    out = cm.gather_records(torch.empty(0, dtype=torch.uint32, device="cuda:0"),
                            torch.zeros((4, 8), dtype=torch.uint8, device="cuda:0"),
                            torch.zeros((2, 8), dtype=torch.uint8, device="cuda:0"))
    assert out.shape == (0, 8)
