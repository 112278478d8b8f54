"""GPU: a single merge past 2^32 outputs (every rank, co-rank and window
offset above 32 bits), checked against the closed form that the oracle is
pinned to on small sizes (tests/test_oracle.py::test_pair_duplicates_closed_form):
keys A[x] = x >> 1, B[y] = y >> 1 with m = n odd, payloads x and y, so
C[p] = p >> 2 and C_val[p] = 2 (p >> 2) + (p & 1) below N - 2, then A's last
element and B's.  m = n = 2^31 + 3: N = 2^32 + 6 outputs, about 69 GB of
device memory for inputs and outputs."""
import pytest

import paper_1303_4312_amd as cm

pytestmark = pytest.mark.gpu

CHUNK = 1 << 28


def fill(dst, s, e, fn):
    import torch
    x = torch.arange(s, e, dtype=torch.int64, device=dst.device)
    dst[s:e].view(torch.int32).copy_(fn(x).to(torch.int32))  # low 32 bits


def check(C, Cv, m, n):
    import torch
    N = m + n
    bad = 0
    for s in range(0, N, CHUNK):
        e = min(N, s + CHUNK)
        p = torch.arange(s, e, dtype=torch.int64, device=C.device)
        ek, ev = p >> 2, 2 * (p >> 2) + (p & 1)
        for q, key, val in ((N - 2, (m - 1) >> 1, m - 1), (N - 1, (n - 1) >> 1, n - 1)):
            if s <= q < e:
                ek[q - s], ev[q - s] = key, val
        got_k = C[s:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        got_v = Cv[s:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        bad += int((got_k != ek).sum()) + int((got_v != ev).sum())
    return bad


@pytest.mark.parametrize("partition", [-1, 0, 4])
def test_merge_past_2_32_outputs(partition, restore_settings):
    import torch
    free, _ = torch.cuda.mem_get_info()
    if free < (80 << 30):
        pytest.skip("needs about 69 GB of free device memory")
    m = n = (1 << 31) + 3
    print(f"\n[max size] m = n = {m}, partition {partition}", flush=True)
    A = torch.empty(m, dtype=torch.uint32, device="cuda")
    B = torch.empty(n, dtype=torch.uint32, device="cuda")
    Av = torch.empty(m, dtype=torch.uint32, device="cuda")
    Bv = torch.empty(n, dtype=torch.uint32, device="cuda")
    for s in range(0, m, CHUNK):
        e = min(m, s + CHUNK)
        fill(A, s, e, lambda x: x >> 1)
        fill(B, s, e, lambda x: x >> 1)
        fill(Av, s, e, lambda x: x)
        fill(Bv, s, e, lambda x: x)
    cm.set_partition(partition)
    C, Cv = cm.stable_merge_pairs(A, Av, B, Bv)
    torch.cuda.synchronize()
    del A, B, Av, Bv
    assert check(C, Cv, m, n) == 0
    del C, Cv
    torch.cuda.empty_cache()


def test_segmented_past_2_32_outputs():
    """The segmented form over the same arrays: an empty segment, the whole
    merge, an empty segment (offsets past 2^32), same closed form."""
    import torch
    free, _ = torch.cuda.mem_get_info()
    if free < (80 << 30):
        pytest.skip("needs about 69 GB of free device memory")
    m = n = (1 << 31) + 3
    print(f"\n[max size] segmented, m = n = {m}", flush=True)
    A = torch.empty(m, dtype=torch.uint32, device="cuda")
    B = torch.empty(n, dtype=torch.uint32, device="cuda")
    Av = torch.empty(m, dtype=torch.uint32, device="cuda")
    Bv = torch.empty(n, dtype=torch.uint32, device="cuda")
    for s in range(0, m, CHUNK):
        e = min(m, s + CHUNK)
        fill(A, s, e, lambda x: x >> 1)
        fill(B, s, e, lambda x: x >> 1)
        fill(Av, s, e, lambda x: x)
        fill(Bv, s, e, lambda x: x)
    a_off = torch.tensor([0, 0, m, m], dtype=torch.uint64, device="cuda")
    b_off = torch.tensor([0, 0, n, n], dtype=torch.uint64, device="cuda")
    C, Cv = cm.stable_merge_segmented(A, a_off, B, b_off, Av, Bv)
    torch.cuda.synchronize()
    del A, B, Av, Bv
    assert check(C, Cv, m, n) == 0
    del C, Cv
    torch.cuda.empty_cache()
