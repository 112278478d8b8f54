"""Co-rank stable merge on MI355X (gfx950).

Python binding of ``libcorank_merge.so`` (C ABI in ``include/corank_merge.h``).
Each function marshals torch tensors into pointers, sizes and the current HIP
stream and calls the C function of the same name (``cm_`` prefix in C); all
of the merge and co-rank work runs in the library's HIP kernels.  torch is
used only to allocate device memory and to name the stream.

The operations follow Siebert and Traeff, arXiv:1303.4312: ``co_rank``
(Section 2, Lemma 1 and Algorithm 1), ``stable_merge`` /
``stable_merge_pairs`` (Sections 1-3, Algorithm 2), and
``stable_merge_segmented`` (a batch of independent merges).

If the library has not been built, every call raises; nothing falls back to
the CPU.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "CMError", "library_path", "co_rank_host", "co_rank", "stable_merge",
    "stable_merge_pairs", "stable_merge_segmented", "merge_workspace_size",
    "segmented_workspace_size", "check_sorted", "config_count", "config_info",
    "set_config", "get_config", "set_search", "KEY_TYPES",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libcorank_merge.so")

# C enum cm_key_type
KEY_U32, KEY_U64, KEY_F32 = 0, 1, 2
KEY_TYPES = {"uint32": KEY_U32, "uint64": KEY_U64, "float32": KEY_F32}

EXPORTS = [
    "cm_status_string", "cm_version", "cm_co_rank_host", "cm_co_rank",
    "cm_merge_workspace_size", "cm_stable_merge", "cm_stable_merge_pairs",
    "cm_segmented_workspace_size", "cm_stable_merge_segmented", "cm_check_sorted",
    "cm_config_count", "cm_config_info", "cm_set_config", "cm_get_config",
    "cm_set_search",
]

_lib = None


class CMError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


def load():
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise RuntimeError(
            f"{library_path} is missing: build it with "
            "`python -m paper_1303_4312_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(library_path)
    c_int, c_u64, c_size, vp = ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p
    p64 = ctypes.POINTER(ctypes.c_uint64)
    sig = {
        "cm_status_string": (ctypes.c_char_p, [c_int]),
        "cm_version": (c_int, []),
        "cm_co_rank_host": (c_int, [c_int, c_u64, vp, c_u64, vp, c_u64, p64, p64]),
        "cm_co_rank": (c_int, [c_int, vp, c_u64, vp, c_u64, vp, c_u64, vp, vp]),
        "cm_merge_workspace_size": (c_size, [c_int, c_int, c_u64, c_u64]),
        "cm_stable_merge": (c_int, [c_int, vp, c_u64, vp, c_u64, vp, vp, c_size, vp]),
        "cm_stable_merge_pairs": (c_int, [c_int, vp, vp, c_u64, vp, vp, c_u64, vp, vp, vp,
                                          c_size, vp]),
        "cm_segmented_workspace_size": (c_size, [c_int, c_int, c_u64, c_u64, c_u64]),
        "cm_stable_merge_segmented": (c_int, [c_int, vp, vp, vp, c_u64, vp, vp, vp, c_u64,
                                              c_u64, vp, vp, vp, c_size, vp]),
        "cm_check_sorted": (c_int, [c_int, vp, c_u64, vp, vp]),
        "cm_config_count": (c_int, []),
        "cm_config_info": (c_int, [c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
        "cm_set_config": (c_int, [c_int, c_int, c_int]),
        "cm_get_config": (c_int, [c_int, c_int]),
        "cm_set_search": (c_int, [c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().cm_status_string(status).decode()


def _check(status: int, where: str):
    if status != 0:
        raise CMError(status, where)


def _torch():
    import torch
    return torch


def _key_type(t) -> int:
    torch = _torch()
    kt = {torch.uint32: KEY_U32, torch.uint64: KEY_U64, torch.float32: KEY_F32}.get(t.dtype)
    if kt is None:
        raise TypeError(f"unsupported key dtype {t.dtype} (uint32, uint64, float32)")
    return kt


def _dev(t, name, dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    return t


def _ptr(t):
    return None if t is None or t.numel() == 0 else ctypes.c_void_p(t.data_ptr())


def _stream(stream, device):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def merge_workspace_size(key_dtype, with_payload: bool, m: int, n: int) -> int:
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    return load().cm_merge_workspace_size(kt, int(bool(with_payload)), m, n)


def segmented_workspace_size(key_dtype, with_payload: bool, total_a: int, total_b: int,
                             num_seg: int) -> int:
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    return load().cm_segmented_workspace_size(kt, int(bool(with_payload)), total_a, total_b,
                                              num_seg)


def _workspace(nbytes, device, workspace):
    torch = _torch()
    if nbytes == 0:
        return None, 0
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
    return workspace, workspace.numel() * workspace.element_size()


def co_rank_host(i: int, A, B):
    """Co-ranks (j, k) of rank i for host arrays (numpy or CPU tensors)."""
    import numpy as np
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B, dtype=A.dtype)
    kt = {np.dtype(np.uint32): KEY_U32, np.dtype(np.uint64): KEY_U64,
          np.dtype(np.float32): KEY_F32}.get(A.dtype)
    if kt is None:
        raise TypeError(f"unsupported key dtype {A.dtype}")
    j, k = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().cm_co_rank_host(kt, i, A.ctypes.data_as(ctypes.c_void_p), A.size,
                                  B.ctypes.data_as(ctypes.c_void_p), B.size,
                                  ctypes.byref(j), ctypes.byref(k)), "cm_co_rank_host")
    return j.value, k.value


def co_rank(ranks, A, B, j_out=None, stream=None):
    """A co-ranks of device rank tensor `ranks` (uint64) over device arrays A
    and B; returns j (uint64 tensor; k = ranks - j).  A plain int rank
    returns the pair (j, k) and synchronises."""
    torch = _torch()
    A = _dev(A, "A")
    B = _dev(B, "B", A.dtype)
    scalar = isinstance(ranks, int)
    if scalar:
        ranks = torch.tensor([ranks], dtype=torch.uint64, device=A.device)
    ranks = _dev(ranks, "ranks", torch.uint64)
    if j_out is None:
        j_out = torch.empty_like(ranks)
    _check(load().cm_co_rank(_key_type(A), _ptr(ranks), ranks.numel(), _ptr(A), A.numel(),
                             _ptr(B), B.numel(), _ptr(j_out), _stream(stream, A.device)),
           "cm_co_rank")
    if scalar:
        j = int(j_out.cpu()[0])
        if j == 2**64 - 1:
            raise CMError(-2, "cm_co_rank")
        return j, int(ranks.cpu()[0]) - j
    return j_out


def stable_merge(A, B, C=None, workspace=None, stream=None):
    """Stable merge of sorted device key arrays A and B; returns C."""
    torch = _torch()
    A = _dev(A, "A")
    B = _dev(B, "B", A.dtype)
    m, n = A.numel(), B.numel()
    if C is None:
        C = torch.empty(m + n, dtype=A.dtype, device=A.device)
    C = _dev(C, "C", A.dtype)
    if C.numel() != m + n:
        raise ValueError("C must hold m + n keys")
    kt = _key_type(A)
    ws, wsb = _workspace(load().cm_merge_workspace_size(kt, 0, m, n), A.device, workspace)
    _check(load().cm_stable_merge(kt, _ptr(A), m, _ptr(B), n, _ptr(C), _ptr(ws), wsb,
                                  _stream(stream, A.device)), "cm_stable_merge")
    return C


def stable_merge_pairs(A, A_val, B, B_val, C=None, C_val=None, workspace=None, stream=None):
    """Stable merge of (key, uint32 payload) pairs; returns (C, C_val)."""
    torch = _torch()
    A = _dev(A, "A")
    B = _dev(B, "B", A.dtype)
    A_val = _dev(A_val, "A_val", torch.uint32)
    B_val = _dev(B_val, "B_val", torch.uint32)
    m, n = A.numel(), B.numel()
    if A_val.numel() != m or B_val.numel() != n:
        raise ValueError("payload lengths must match key lengths")
    if C is None:
        C = torch.empty(m + n, dtype=A.dtype, device=A.device)
    if C_val is None:
        C_val = torch.empty(m + n, dtype=torch.uint32, device=A.device)
    C = _dev(C, "C", A.dtype)
    C_val = _dev(C_val, "C_val", torch.uint32)
    if C.numel() != m + n or C_val.numel() != m + n:
        raise ValueError("C and C_val must hold m + n elements")
    kt = _key_type(A)
    ws, wsb = _workspace(load().cm_merge_workspace_size(kt, 1, m, n), A.device, workspace)
    _check(load().cm_stable_merge_pairs(kt, _ptr(A), _ptr(A_val), m, _ptr(B), _ptr(B_val), n,
                                        _ptr(C), _ptr(C_val), _ptr(ws), wsb,
                                        _stream(stream, A.device)), "cm_stable_merge_pairs")
    return C, C_val


def stable_merge_segmented(A, a_off, B, b_off, A_val=None, B_val=None, C=None, C_val=None,
                           workspace=None, stream=None):
    """Merge segment s of A (A[a_off[s]:a_off[s+1]]) with segment s of B into
    C at a_off[s] + b_off[s].  a_off, b_off: uint64 device tensors of
    num_seg + 1 entries.  Returns C or (C, C_val)."""
    torch = _torch()
    A = _dev(A, "A")
    B = _dev(B, "B", A.dtype)
    a_off = _dev(a_off, "a_off", torch.uint64)
    b_off = _dev(b_off, "b_off", torch.uint64)
    if a_off.numel() != b_off.numel() or a_off.numel() < 1:
        raise ValueError("a_off and b_off need num_seg + 1 entries each")
    with_val = A_val is not None
    if with_val != (B_val is not None):
        raise ValueError("give payloads for both inputs or neither")
    ta, tb = A.numel(), B.numel()
    if C is None:
        C = torch.empty(ta + tb, dtype=A.dtype, device=A.device)
    C = _dev(C, "C", A.dtype)
    if with_val:
        A_val = _dev(A_val, "A_val", torch.uint32)
        B_val = _dev(B_val, "B_val", torch.uint32)
        if C_val is None:
            C_val = torch.empty(ta + tb, dtype=torch.uint32, device=A.device)
        C_val = _dev(C_val, "C_val", torch.uint32)
    kt = _key_type(A)
    S = a_off.numel() - 1
    ws, wsb = _workspace(load().cm_segmented_workspace_size(kt, int(with_val), ta, tb, S),
                         A.device, workspace)
    _check(load().cm_stable_merge_segmented(
        kt, _ptr(A), _ptr(A_val) if with_val else None, _ptr(a_off), ta,
        _ptr(B), _ptr(B_val) if with_val else None, _ptr(b_off), tb, S,
        _ptr(C), _ptr(C_val) if with_val else None, _ptr(ws), wsb,
        _stream(stream, A.device)), "cm_stable_merge_segmented")
    return (C, C_val) if with_val else C


def check_sorted(X, stream=None) -> bool:
    """True if the device key array X is nondecreasing (synchronises)."""
    torch = _torch()
    X = _dev(X, "X")
    flag = torch.empty(1, dtype=torch.uint32, device=X.device)
    _check(load().cm_check_sorted(_key_type(X), _ptr(X), X.numel(), _ptr(flag),
                                  _stream(stream, X.device)), "cm_check_sorted")
    return int(flag.cpu()[0]) == 0


def config_count() -> int:
    return load().cm_config_count()


def config_info(config_id: int):
    nt, e = ctypes.c_int(), ctypes.c_int()
    _check(load().cm_config_info(config_id, ctypes.byref(nt), ctypes.byref(e)), "cm_config_info")
    return nt.value, e.value


def set_config(key_dtype, with_payload: bool, config_id: int):
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    _check(load().cm_set_config(kt, int(bool(with_payload)), config_id), "cm_set_config")


def get_config(key_dtype, with_payload: bool) -> int:
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    return load().cm_get_config(kt, int(bool(with_payload)))


def set_search(mode: int):
    """0 = Algorithm 1 (default), 1 = bisection."""
    _check(load().cm_set_search(mode), "cm_set_search")
