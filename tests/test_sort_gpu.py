"""GPU: the stable merge sort built from the co-rank merge, bit-exact
against the oracle's stable sort: every key type, keys only and with
payloads, every tile configuration, sizes around one block and around pass
boundaries, duplicate-heavy, sorted, reversed and all-equal inputs, signed
zeros, in place, and a large input."""
import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from tests.gpu_util import first_difference, same_bits, to_dev, to_host

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("restore_settings")]

DTYPES = [np.uint32, np.uint64, np.float32]


def keys_of(rng, n, dtype, hi):
    if np.dtype(dtype) == np.float32:
        k = (rng.integers(0, hi, n) - hi // 2).astype(np.float32) / 4
        k[rng.random(n) < 0.05] = -0.0
        return k
    return rng.integers(0, hi, n).astype(dtype)


def check(keys, payload=True, offset=0):
    n = keys.size
    print(f"[sort] n={n} {keys.dtype} payload={payload} offset={offset}", flush=True)
    vals = np.arange(n, dtype=np.uint32)
    if payload:
        C, Cv = cm.stable_sort(to_dev(keys, offset), to_dev(vals, offset))
        C, Cv = to_host(C), to_host(Cv)
        Ce, Cve = oracle.stable_sort(keys, vals)
        assert same_bits(C, Ce), f"n={n}: keys differ first at {first_difference(C, Ce)}"
        assert same_bits(Cv, Cve), f"n={n}: payloads differ first at {first_difference(Cv, Cve)}"
    else:
        C = to_host(cm.stable_sort(to_dev(keys, offset)))
        Ce = oracle.stable_sort(keys)
        assert same_bits(C, Ce), f"n={n}: keys differ first at {first_difference(C, Ce)}"


@pytest.mark.parametrize("dtype", DTYPES)
def test_sizes_around_blocks_and_passes(dtype):
    rng = np.random.default_rng(11)
    nt, e = cm.config_info(cm.tuning_get(cm.OP_SORT, np.dtype(dtype).name, True, 1 << 20)[0])
    T = nt * e
    # the first sorted runs are 1, 2 or 4 blocks long (as LDS allows)
    for n in (0, 1, 2, 7, T - 1, T, T + 1, 2 * T, 2 * T + 1, 3 * T + 5, 4 * T, 4 * T - 1,
              4 * T + 1, 8 * T + 3, 16 * T - 1, 16 * T + 1, 33 * T + 17, 100_003):
        for hi in (3, 1 << 20):
            check(keys_of(rng, n, dtype, hi))
    check(keys_of(rng, 50_001, dtype, 1000), payload=False)


@pytest.mark.parametrize("dtype", DTYPES)
def test_every_configuration(dtype):
    rng = np.random.default_rng(12)
    kt = np.dtype(dtype).name
    for c in range(cm.config_count()):
        for search in (0, 1):
            nt, e = cm.config_info(c)
            n = 5 * nt * e + 123
            cm.tuning_set(cm.OP_SORT, kt, True, n.bit_length(), c, search, 0)
            cm.tuning_set(cm.OP_SORT, kt, False, n.bit_length(), c, search, 0)
            try:
                k = keys_of(rng, n, dtype, 64)
                check(k)
                check(k, payload=False)
            finally:
                cm.tuning_clear()


@pytest.mark.parametrize("stride", [16, 64])
def test_two_level_pass_boundaries(stride):
    """Passes whose pairs span more than the coarse stride co-rank every
    stride-th block start first and search the others between them (by
    bisection, or by groups of 2 or 4 lanes); sizes
    put pairs just past one and two strides, ragged last pairs included, and
    the one-level pass must give the same bits."""
    rng = np.random.default_rng(16 + stride)
    cm.set_coarse_stride(stride)
    nt, e = cm.config_info(cm.tuning_get(cm.OP_SORT, "uint32", True, 1 << 20)[0])
    T = nt * e
    for n in (2 * stride * T + 1, 2 * stride * T + T - 1, 3 * stride * T + 17, 5 * stride * T - 3):
        for hi in (5, 1 << 30):
            k = keys_of(rng, n, np.uint32, hi)
            for part, lanes in ((2, 1), (2, 4), (2, 2), (0, 1)):
                cm.set_partition(part)
                cm.set_fine_lanes(lanes)
                check(k)
    cm.set_fine_lanes(1)
    cm.set_partition(2)
    check(keys_of(rng, 2 * stride * T + 333, np.uint64, 1 << 40), payload=False)
    check(keys_of(rng, 3 * stride * T + 1, np.float32, 1 << 16))


def test_structured_inputs_and_misaligned_bases():
    n = 300_001
    up = np.arange(n, dtype=np.uint32) * 2
    check(up)
    check(up[::-1].copy())
    check(np.full(n, 9, dtype=np.uint32))
    check(np.full(n, 0xFFFFFFFF, dtype=np.uint32))  # equal to the padding key
    check(np.full(n, np.inf, dtype=np.float32))
    alt = np.where(np.arange(n) % 2 == 0, 5, 3).astype(np.uint64)
    check(alt)
    rng = np.random.default_rng(13)
    for off in (1, 2, 3):
        check(keys_of(rng, 70_000, np.uint32, 100), offset=off)


def test_in_place():
    import torch
    rng = np.random.default_rng(14)
    k = keys_of(rng, 123_457, np.float32, 200)
    v = np.arange(k.size, dtype=np.uint32)
    K, V = to_dev(k), to_dev(v)
    out = cm.stable_sort(K, V, out=K, out_vals=V)
    assert out[0].data_ptr() == K.data_ptr()
    torch.cuda.synchronize()
    Ce, Cve = oracle.stable_sort(k, v)
    assert same_bits(to_host(K), Ce) and same_bits(to_host(V), Cve)


def test_large_duplicate_heavy():
    rng = np.random.default_rng(15)
    n = (1 << 25) + 12345
    k = rng.integers(0, 1 << 12, n).astype(np.uint32)
    check(k)


def test_argument_errors():
    import torch
    lib = cm.load()
    K = torch.zeros(1000, dtype=torch.uint32, device="cuda:0")
    ws = torch.empty(cm.sort_workspace_size("uint32", False, 1000), dtype=torch.uint8,
                     device="cuda:0")
    P = lambda t: t.data_ptr()
    assert lib.cm_stable_sort(0, P(K), 1000, None, P(ws), ws.numel(), None) == -1
    assert lib.cm_stable_sort(0, P(K), 1000, P(K) + 4, P(ws), ws.numel(), None) == -4
    assert lib.cm_stable_sort(0, P(K), 1000, P(K), P(ws), ws.numel() - 1, None) == -5
    assert lib.cm_stable_sort(0, P(K), 1000, P(K), P(K), ws.numel(), None) == -4
    assert lib.cm_stable_sort(7, P(K), 1000, P(K), P(ws), ws.numel(), None) == -3
    assert lib.cm_stable_sort(0, None, 0, None, None, 0, None) == 0
