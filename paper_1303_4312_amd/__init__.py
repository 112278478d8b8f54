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
    "CMError", "library_path", "co_rank_host", "co_rank", "stable_merge", "KEY_DESC_OFFSET",
    "stable_merge_pairs", "stable_merge_segmented", "merge_workspace_size",
    "segmented_workspace_size", "check_sorted", "config_count", "config_info",
    "set_config", "get_config", "set_search", "KEY_TYPES", "stable_merge_segmented_each",
    "copy", "timing_start", "timing_stop", "get_search", "set_partition", "get_partition",
    "autotune_merge", "autotune_segmented", "tuning_set", "tuning_get", "tuning_save",
    "tuning_load", "tuning_clear", "tuning_count", "build_id", "ESTALE", "Plan", "plan_merge", "plan_segmented",
    "OP_MERGE", "OP_SEGMENTED", "OP_BATCH", "OP_SORT", "stable_merge_batch", "batch_descriptors",
    "stable_sort", "sort_workspace_size", "merge_partition_ablation", "origin_codes",
    "gather_records", "merge_records", "stable_merge_pairs_noalloc", "NOALLOC_SCRATCH_BYTES",
    "launch_batch", "set_coarse_stride", "set_block_order", "set_fine_lanes", "get_block_order",
    "get_coarse_stride", "get_fine_lanes", "set_grid", "get_grid",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libcorank_merge.so")

# C enum cm_key_type
KEY_U32, KEY_U64, KEY_F32 = 0, 1, 2
KEY_DESC_OFFSET = 3  # CM_KEY_*_DESC = CM_KEY_* + 3: the same keys, nonincreasing order
ESTALE = -11  # CM_ESTALE: a tuning table made for another device, runtime or build
# operations of the tuning table
OP_MERGE, OP_SEGMENTED, OP_BATCH, OP_SORT = 0, 1, 2, 3
KEY_TYPES = {"uint32": KEY_U32, "uint64": KEY_U64, "float32": KEY_F32}

EXPORTS = [
    "cm_status_string", "cm_version", "cm_co_rank_host", "cm_co_rank",
    "cm_merge_workspace_size", "cm_stable_merge", "cm_stable_merge_pairs", "cm_stable_merge_pairs64",
    "cm_stable_merge_pairs_noalloc",
    "cm_segmented_workspace_size", "cm_stable_merge_segmented", "cm_check_sorted",
    "cm_config_count", "cm_config_info", "cm_set_config", "cm_get_config",
    "cm_set_search", "cm_get_search", "cm_set_partition", "cm_get_partition",
    "cm_stable_merge_segmented_each", "cm_copy", "cm_copy_tiles", "cm_timing_start", "cm_timing_stop",
    "cm_autotune_merge", "cm_autotune_segmented", "cm_tuning_set", "cm_tuning_get",
    "cm_tuning_save", "cm_tuning_load", "cm_tuning_clear", "cm_tuning_count", "cm_build_id",
    "cm_plan_create_merge", "cm_plan_create_segmented", "cm_plan_launch", "cm_plan_destroy",
    "cm_plan_update_merge", "cm_plan_update_segmented", "cm_get_block_order",
    "cm_get_coarse_stride", "cm_get_fine_lanes", "cm_set_grid", "cm_get_grid",
    "cm_batch_prepare", "cm_batch_workspace_size", "cm_stable_merge_batch",
    "cm_set_coarse_stride", "cm_set_block_order", "cm_set_fine_lanes",
    "cm_server_create", "cm_server_submit", "cm_server_submit_host", "cm_server_poll",
    "cm_server_release",
    "cm_server_get_stats", "cm_server_destroy", "cm_sort_workspace_size", "cm_sort_run_length", "cm_stable_sort",
    "cm_stable_sort_pairs", "cm_partition_ablation_workspace_size", "cm_merge_partition_ablation",
    "cm_origin_codes", "cm_gather_records",
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
    # torch first: its HIP runtime (requested under the name libamdhip64.so)
    # must be the one the library binds (libamdhip64.so.7, satisfied by the
    # already-loaded runtime's soname).  Loaded the other way round, the
    # process would hold two HIP runtimes and torch's streams and memory would
    # be foreign to the library's launches.
    import torch  # noqa: F401
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
        "cm_stable_merge_pairs_noalloc": (c_int, [c_int, vp, vp, c_u64, vp, vp, c_u64, vp, vp, vp]),
        "cm_stable_merge_pairs64": (c_int, [c_int, vp, vp, c_u64, vp, vp, c_u64, vp, vp, vp,
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
        "cm_get_search": (c_int, []),
        "cm_set_partition": (c_int, [c_int]),
        "cm_set_coarse_stride": (c_int, [ctypes.c_uint32]),
        "cm_set_block_order": (c_int, [c_int]),
        "cm_get_block_order": (c_int, []),
        "cm_get_coarse_stride": (c_int, []),
        "cm_get_fine_lanes": (c_int, []),
        "cm_set_fine_lanes": (c_int, [c_int]),
        "cm_set_grid": (c_int, [c_int]),
        "cm_get_grid": (c_int, []),
        "cm_get_partition": (c_int, []),
        "cm_stable_merge_segmented_each": (c_int, [c_int, vp, vp, vp, c_u64, vp, vp, vp, c_u64,
                                                   c_u64, vp, vp, vp, c_size, vp]),
        "cm_copy": (c_int, [vp, vp, c_u64, vp]),
        "cm_copy_tiles": (c_int, [c_int, vp, vp, c_u64, vp, vp, c_u64, vp, vp, vp]),
        "cm_autotune_merge": (c_int, [c_int, vp, vp, c_u64, vp, vp, c_u64, vp, vp, vp, c_size,
                                      c_int, vp, ctypes.POINTER(c_int)]),
        "cm_autotune_segmented": (c_int, [c_int, vp, vp, vp, c_u64, vp, vp, vp, c_u64, c_u64, vp,
                                          vp, vp, c_size, c_int, vp, ctypes.POINTER(c_int)]),
        "cm_tuning_set": (c_int, [c_int, c_int, c_int, c_int, c_int, c_int, c_int]),
        "cm_tuning_get": (c_int, [c_int, c_int, c_int, c_u64, ctypes.POINTER(c_int)]),
        "cm_tuning_save": (c_int, [ctypes.c_char_p]),
        "cm_build_id": (ctypes.c_char_p, []),
        "cm_tuning_load": (c_int, [ctypes.c_char_p]),
        "cm_tuning_clear": (c_int, []),
        "cm_tuning_count": (c_int, []),
        "cm_plan_create_merge": (c_int, [c_int, vp, vp, c_u64, vp, vp, c_u64, vp, vp, vp, c_size,
                                         ctypes.POINTER(vp)]),
        "cm_plan_create_segmented": (c_int, [c_int, vp, vp, vp, c_u64, vp, vp, vp, c_u64, c_u64,
                                             vp, vp, vp, c_size, ctypes.POINTER(vp)]),
        "cm_plan_launch": (c_int, [vp, vp]),
        "cm_plan_update_merge": (c_int, [vp, c_int, vp, vp, c_u64, vp, vp, c_u64, vp, vp, vp, c_size]),
        "cm_plan_update_segmented": (c_int, [vp, c_int, vp, vp, vp, c_u64, vp, vp, vp, c_u64, c_u64,
                                             vp, vp, vp, c_size]),
        "cm_batch_prepare": (c_int, [c_int, c_int, vp, ctypes.c_uint32, ctypes.POINTER(c_u64)]),
        "cm_batch_workspace_size": (c_size, [c_u64, ctypes.c_uint32]),
        "cm_stable_merge_batch": (c_int, [c_int, c_int, vp, vp, ctypes.c_uint32, c_u64, vp, c_size,
                                          vp]),
        "cm_plan_destroy": (c_int, [vp]),
        "cm_timing_start": (c_int, [ctypes.c_uint32]),
        "cm_server_create": (c_int, [c_int, c_int, vp, c_u64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.POINTER(vp)]),
        "cm_server_submit": (c_int, [vp, vp, vp, c_u64, vp, vp, c_u64, vp, c_int,
                                     ctypes.POINTER(c_u64)]),
        "cm_server_submit_host": (c_int, [vp, vp, vp, c_u64, vp, vp, c_u64, vp, vp,
                                          ctypes.POINTER(c_u64)]),
        "cm_server_poll": (c_int, [vp, vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.c_int64]),
        "cm_server_release": (c_int, [vp, c_u64]),
        "cm_server_get_stats": (c_int, [vp, vp]),
        "cm_server_destroy": (c_int, [vp]),
        "cm_sort_workspace_size": (c_size, [c_int, c_int, c_u64]),
        "cm_sort_run_length": (c_u64, [c_int, c_int, c_u64]),
        "cm_stable_sort": (c_int, [c_int, vp, c_u64, vp, vp, c_size, vp]),
        "cm_stable_sort_pairs": (c_int, [c_int, vp, vp, c_u64, vp, vp, vp, c_size, vp]),
        "cm_partition_ablation_workspace_size": (c_size, [ctypes.c_uint32]),
        "cm_origin_codes": (c_int, [c_u64, c_u64, vp, vp, vp]),
        "cm_gather_records": (c_int, [vp, c_u64, vp, c_u64, vp, c_u64, c_u64, vp, vp]),
        "cm_merge_partition_ablation": (c_int, [c_int, vp, vp, c_u64, vp, vp, c_u64, vp, vp,
                                                ctypes.c_uint32, c_int, vp, vp, c_size, vp]),
        "cm_timing_stop": (c_int, [ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float),
                                   ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
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


_torch_mod = None
_key_of_dtype = None


def _torch():
    global _torch_mod
    if _torch_mod is None:
        import torch
        _torch_mod = torch
    return _torch_mod


def _key_type(t, descending: bool = False) -> int:
    """C key type of tensor t: the ascending type, or its _DESC twin."""
    global _key_of_dtype
    if _key_of_dtype is None:
        torch = _torch()
        _key_of_dtype = {torch.uint32: KEY_U32, torch.uint64: KEY_U64, torch.float32: KEY_F32}
    kt = _key_of_dtype.get(t.dtype)
    if kt is None:
        raise TypeError(f"unsupported key dtype {t.dtype} (uint32, uint64, float32)")
    return kt + (KEY_DESC_OFFSET if descending else 0)


def _dev(t, name, dtype=None):
    if not isinstance(t, _torch().Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}")
    return t


def _ptr(t):
    """Device address of a tensor (None when empty): a plain int, which the
    declared c_void_p argument types convert."""
    return None if t is None or t.numel() == 0 else t.data_ptr()


def _stream(stream, device):
    """Raw HIP stream handle: the given torch stream, else the device's
    current one (read without building a Stream object when torch offers
    that)."""
    if stream is not None:
        return stream.cuda_stream
    torch = _torch()
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        index = device.index if device.index is not None else torch.cuda.current_device()
        return raw(index)
    return torch.cuda.current_stream(device).cuda_stream


def merge_workspace_size(key_dtype, with_payload: bool, m: int, n: int) -> int:
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    return load().cm_merge_workspace_size(kt, int(bool(with_payload)), m, n)


def segmented_workspace_size(key_dtype, with_payload: bool, total_a: int, total_b: int,
                             num_seg: int) -> int:
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    return load().cm_segmented_workspace_size(kt, int(bool(with_payload)), total_a, total_b,
                                              num_seg)


def _workspace(nbytes, device, workspace):
    """(workspace, its bytes): the caller's, or a new one of `nbytes` bytes
    (nbytes may be a callable, asked only when no workspace is given; the
    library checks a given workspace's size itself)."""
    if workspace is not None:
        torch = _torch()
        if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda \
                or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous tensor on the GPU")
        return workspace, workspace.numel() * workspace.element_size()
    if callable(nbytes):
        nbytes = nbytes()
    if nbytes == 0:
        return None, 0
    torch = _torch()
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def co_rank_host(i: int, A, B, descending=False):
    """Co-ranks (j, k) of rank i for host arrays (numpy or CPU tensors),
    sorted nonincreasingly if descending."""
    import numpy as np
    A = np.ascontiguousarray(A)
    B = np.ascontiguousarray(B, dtype=A.dtype)
    kt = {np.dtype(np.uint32): KEY_U32, np.dtype(np.uint64): KEY_U64,
          np.dtype(np.float32): KEY_F32}.get(A.dtype)
    if kt is None:
        raise TypeError(f"unsupported key dtype {A.dtype}")
    kt += KEY_DESC_OFFSET if descending else 0
    j, k = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().cm_co_rank_host(kt, i, A.ctypes.data_as(ctypes.c_void_p), A.size,
                                  B.ctypes.data_as(ctypes.c_void_p), B.size,
                                  ctypes.byref(j), ctypes.byref(k)), "cm_co_rank_host")
    return j.value, k.value


def co_rank(ranks, A, B, j_out=None, stream=None, descending=False):
    """A co-ranks of device rank tensor `ranks` (uint64) over device arrays A
    and B (sorted nonincreasingly if descending); returns j (uint64 tensor;
    k = ranks - j).  A plain int rank returns the pair (j, k) and
    synchronises."""
    torch = _torch()
    A = _dev(A, "A")
    B = _dev(B, "B", A.dtype)
    scalar = isinstance(ranks, int)
    if scalar:
        ranks = torch.tensor([ranks], dtype=torch.uint64, device=A.device)
    ranks = _dev(ranks, "ranks", torch.uint64)
    if j_out is None:
        j_out = torch.empty_like(ranks)
    _check(load().cm_co_rank(_key_type(A, descending), _ptr(ranks), ranks.numel(), _ptr(A),
                             A.numel(),
                             _ptr(B), B.numel(), _ptr(j_out), _stream(stream, A.device)),
           "cm_co_rank")
    if scalar:
        j = int(j_out.cpu()[0])
        if j == 2**64 - 1:
            raise CMError(-2, "cm_co_rank")
        return j, int(ranks.cpu()[0]) - j
    return j_out


def stable_merge(A, B, C=None, workspace=None, stream=None, descending=False):
    """Stable merge of sorted device key arrays A and B (both nonincreasing
    if descending); returns C."""
    torch = _torch()
    A = _dev(A, "A")
    B = _dev(B, "B", A.dtype)
    m, n = A.numel(), B.numel()
    if C is None:
        C = torch.empty(m + n, dtype=A.dtype, device=A.device)
    C = _dev(C, "C", A.dtype)
    if C.numel() != m + n:
        raise ValueError("C must hold m + n keys")
    kt = _key_type(A, descending)
    ws, wsb = _workspace(lambda: load().cm_merge_workspace_size(kt, 0, m, n), A.device, workspace)
    _check(load().cm_stable_merge(kt, _ptr(A), m, _ptr(B), n, _ptr(C), _ptr(ws), wsb,
                                  _stream(stream, A.device)), "cm_stable_merge")
    return C


def stable_merge_pairs(A, A_val, B, B_val, C=None, C_val=None, workspace=None, stream=None,
                       descending=False):
    """Stable merge of (key, payload) pairs with uint32 payloads
    (cm_stable_merge_pairs) or uint64 payloads (cm_stable_merge_pairs64);
    returns (C, C_val)."""
    torch = _torch()
    A = _dev(A, "A")
    B = _dev(B, "B", A.dtype)
    A_val = _dev(A_val, "A_val")
    if A_val.dtype not in (torch.uint32, torch.uint64):
        raise TypeError("payloads must be uint32 or uint64")
    vt = A_val.dtype
    B_val = _dev(B_val, "B_val", vt)
    m, n = A.numel(), B.numel()
    if A_val.numel() != m or B_val.numel() != n:
        raise ValueError("payload lengths must match key lengths")
    if C is None:
        C = torch.empty(m + n, dtype=A.dtype, device=A.device)
    if C_val is None:
        C_val = torch.empty(m + n, dtype=vt, device=A.device)
    C = _dev(C, "C", A.dtype)
    C_val = _dev(C_val, "C_val", vt)
    if C.numel() != m + n or C_val.numel() != m + n:
        raise ValueError("C and C_val must hold m + n elements")
    kt = _key_type(A, descending)
    ws, wsb = _workspace(lambda: load().cm_merge_workspace_size(kt, 1, m, n), A.device, workspace)
    fn, name = ((load().cm_stable_merge_pairs, "cm_stable_merge_pairs") if vt == torch.uint32 else
                (load().cm_stable_merge_pairs64, "cm_stable_merge_pairs64"))
    _check(fn(kt, _ptr(A), _ptr(A_val), m, _ptr(B), _ptr(B_val), n, _ptr(C), _ptr(C_val), _ptr(ws), wsb,
              _stream(stream, A.device)), name)
    return C, C_val


NOALLOC_SCRATCH_BYTES = 4 << 20  # CM_NOALLOC_SCRATCH_BYTES


def stable_merge_pairs_noalloc(A, A_val, B, B_val, C, C_val, stream=None, descending=False):
    """cm_stable_merge_pairs_noalloc: the merge of stable_merge_pairs into the
    caller's C / C_val with no workspace and no allocation (the library's
    per-GPU scratch array holds the block co-ranks).  Payload arguments all
    None for keys only.  Returns (C, C_val)."""
    A, B, C = _dev(A, "A"), _dev(B, "B"), _dev(C, "C")
    if A_val is not None or B_val is not None or C_val is not None:
        torch = _torch()
        A_val, B_val = _dev(A_val, "A_val", torch.uint32), _dev(B_val, "B_val", torch.uint32)
        C_val = _dev(C_val, "C_val", torch.uint32)
    kt = _key_type(A, descending)
    _check(load().cm_stable_merge_pairs_noalloc(kt, _ptr(A), _ptr(A_val), A.numel(), _ptr(B), _ptr(B_val),
                                                B.numel(), _ptr(C), _ptr(C_val), _stream(stream, A.device)),
           "cm_stable_merge_pairs_noalloc")
    return C, C_val


def stable_merge_segmented(A, a_off, B, b_off, A_val=None, B_val=None, C=None, C_val=None,
                           workspace=None, stream=None, descending=False):
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
    kt = _key_type(A, descending)
    S = a_off.numel() - 1
    ws, wsb = _workspace(load().cm_segmented_workspace_size(kt, int(with_val), ta, tb, S),
                         A.device, workspace)
    _check(load().cm_stable_merge_segmented(
        kt, _ptr(A), _ptr(A_val) if with_val else None, _ptr(a_off), ta,
        _ptr(B), _ptr(B_val) if with_val else None, _ptr(b_off), tb, S,
        _ptr(C), _ptr(C_val) if with_val else None, _ptr(ws), wsb,
        _stream(stream, A.device)), "cm_stable_merge_segmented")
    return (C, C_val) if with_val else C


def stable_merge_segmented_each(A, a_off, B, b_off, A_val=None, B_val=None, C=None, C_val=None,
                                workspace=None, stream=None):
    """The batch of stable_merge_segmented run as one merge call per segment
    (the per-merge-launch baseline).  a_off, b_off: host (numpy uint64)
    offsets.  Returns C or (C, C_val)."""
    import numpy as np
    torch = _torch()
    A = _dev(A, "A")
    B = _dev(B, "B", A.dtype)
    a_off = np.ascontiguousarray(a_off, dtype=np.uint64)
    b_off = np.ascontiguousarray(b_off, dtype=np.uint64)
    if a_off.shape != b_off.shape or a_off.size < 1:
        raise ValueError("a_off and b_off need num_seg + 1 entries each")
    with_val = A_val is not None
    ta, tb = A.numel(), B.numel()
    if C is None:
        C = torch.empty(ta + tb, dtype=A.dtype, device=A.device)
    if with_val:
        A_val = _dev(A_val, "A_val", torch.uint32)
        B_val = _dev(B_val, "B_val", torch.uint32)
        if C_val is None:
            C_val = torch.empty(ta + tb, dtype=torch.uint32, device=A.device)
    kt = _key_type(A)
    la = np.diff(a_off.astype(np.int64))
    lb = np.diff(b_off.astype(np.int64))
    biggest = int((la + lb).max()) if la.size else 0
    ws, wsb = _workspace(load().cm_merge_workspace_size(kt, int(with_val), biggest, 0), A.device,
                         workspace)
    _check(load().cm_stable_merge_segmented_each(
        kt, _ptr(A), _ptr(A_val) if with_val else None, a_off.ctypes.data_as(ctypes.c_void_p), ta,
        _ptr(B), _ptr(B_val) if with_val else None, b_off.ctypes.data_as(ctypes.c_void_p), tb,
        a_off.size - 1, _ptr(C), _ptr(C_val) if with_val else None, _ptr(ws), wsb,
        _stream(stream, A.device)), "cm_stable_merge_segmented_each")
    return (C, C_val) if with_val else C


def copy(src, dst, stream=None):
    """Plain 16-byte-vector device copy of src into dst (measurement helper)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    _check(load().cm_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream, src.device)), "cm_copy")


def copy_tiles(config, A, A_val, B, B_val, C=None, C_val=None, stream=None):
    """The block merge's data movement in tile configuration `config`
    without the merge (measurement helper): uint32 keys and payloads, tile t
    copies A's and B's shares of its outputs, A's first (cm_copy_tiles).
    Returns (C, C_val)."""
    torch = _torch()
    for t, name in ((A, "A"), (A_val, "A_val"), (B, "B"), (B_val, "B_val")):
        _dev(t, name)
        if t.dtype != torch.uint32:
            raise TypeError(f"{name} must be uint32")
    N = A.numel() + B.numel()
    if C is None:
        C = torch.empty(N, dtype=torch.uint32, device=A.device)
    if C_val is None:
        C_val = torch.empty(N, dtype=torch.uint32, device=A.device)
    _check(load().cm_copy_tiles(int(config), _ptr(A), _ptr(A_val), A.numel(), _ptr(B), _ptr(B_val),
                                B.numel(), _ptr(C), _ptr(C_val), _stream(stream, A.device)),
           "cm_copy_tiles")
    return C, C_val


_timing_capacity = [0]


def timing_start(capacity: int):
    """Record kernel events around the next `capacity` merge calls."""
    _check(load().cm_timing_start(capacity), "cm_timing_start")
    _timing_capacity[0] = capacity


def timing_stop(per_call=False):
    """Returns (calls, mean co-rank pass ms, mean block-merge kernel ms); with
    per_call, also the lists of each call's start (ms after call 0's start),
    whole duration and block-merge kernel duration (ms)."""
    calls, tb, tm = ctypes.c_uint32(), ctypes.c_double(), ctypes.c_double()
    cap = max(_timing_capacity[0] if per_call else 0, 1)
    arrays = [(ctypes.c_float * cap)() for _ in range(3)]
    _check(load().cm_timing_stop(ctypes.byref(calls), ctypes.byref(tb), ctypes.byref(tm),
                                 *(a if per_call else None for a in arrays)), "cm_timing_stop")
    if not per_call:
        return calls.value, tb.value, tm.value
    return (calls.value, tb.value, tm.value) + tuple(list(a[:calls.value]) for a in arrays)


def sort_workspace_size(key_dtype, with_payload: bool, n: int) -> int:
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    return load().cm_sort_workspace_size(kt, int(bool(with_payload)), n)


def sort_run_length(key_dtype, with_payload: bool, n: int) -> int:
    """Elements per run of the LDS run sort that a sort of n keys would use
    now (its merge passes then number ceil(log2(n / run)))."""
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    return load().cm_sort_run_length(kt, int(bool(with_payload)), n)


def stable_sort(keys, vals=None, out=None, out_vals=None, workspace=None, stream=None,
                descending=False):
    """Stable merge sort of a device key array (with uint32 payloads if vals
    is given).  out / out_vals may be the inputs themselves (in place).
    Returns the sorted keys, or (keys, payloads)."""
    torch = _torch()
    keys = _dev(keys, "keys")
    kt = _key_type(keys, descending)
    n = keys.numel()
    with_val = vals is not None
    if with_val:
        vals = _dev(vals, "vals", torch.uint32)
        if vals.numel() != n:
            raise ValueError("vals must be as long as keys")
    if out is None:
        out = torch.empty_like(keys)
    if with_val and out_vals is None:
        out_vals = torch.empty_like(vals)
    out = _dev(out, "out", keys.dtype)
    if out.numel() != n or (with_val and _dev(out_vals, "out_vals", torch.uint32).numel() != n):
        raise ValueError("outputs must be as long as keys")
    ws, wsb = _workspace(load().cm_sort_workspace_size(kt, int(with_val), n), keys.device,
                         workspace)
    s = _stream(stream, keys.device)
    if with_val:
        _check(load().cm_stable_sort_pairs(kt, _ptr(keys), _ptr(vals), n, _ptr(out),
                                           _ptr(out_vals), _ptr(ws), wsb, s),
               "cm_stable_sort_pairs")
        return out, out_vals
    _check(load().cm_stable_sort(kt, _ptr(keys), n, _ptr(out), _ptr(ws), wsb, s),
           "cm_stable_sort")
    return out


def merge_partition_ablation(A, B, A_val=None, B_val=None, P=2048, partition=0, C=None,
                             C_val=None, stream=None):
    """The merge with P workgroups each merging one output segment; segments
    cut by co-ranking (partition 0) or by the classic cross-rank partition
    (1).  Returns (C[, C_val], bounds) with bounds the P + 1 segment starts
    (a device uint64 tensor)."""
    torch = _torch()
    kt, with_val, m, n, A, A_val, B, B_val, C, C_val = _pair_args(A, B, A_val, B_val, C, C_val)
    bounds = torch.empty(P + 1, dtype=torch.uint64, device=A.device)
    ws, wsb = _workspace(load().cm_partition_ablation_workspace_size(P), A.device, None)
    _check(load().cm_merge_partition_ablation(kt, _ptr(A), _ptr(A_val), m, _ptr(B), _ptr(B_val), n,
                                              _ptr(C), _ptr(C_val), P, partition, _ptr(bounds),
                                              _ptr(ws), wsb, _stream(stream, A.device)),
           "cm_merge_partition_ablation")
    return ((C, C_val) if with_val else (C,)) + (bounds,)


def origin_codes(m: int, n: int, device="cuda:0", stream=None):
    """(A_codes, B_codes): A_codes[x] = x, B_codes[y] = 2^31 + y (uint32)."""
    torch = _torch()
    a = torch.empty(m, dtype=torch.uint32, device=device)
    b = torch.empty(n, dtype=torch.uint32, device=device)
    _check(load().cm_origin_codes(m, n, _ptr(a), _ptr(b), _stream(stream, a.device)),
           "cm_origin_codes")
    return a, b


def _record_width(t):
    width = t.element_size()
    for d in t.shape[1:]:
        width *= d
    return width


def gather_records(codes, A_rec, B_rec, out=None, stream=None):
    """out[i] = A_rec[codes[i]] or B_rec[codes[i] - 2^31]: records are the
    rows of A_rec / B_rec (same dtype and row shape, contiguous)."""
    torch = _torch()
    codes = _dev(codes, "codes", torch.uint32)
    if A_rec.dtype != B_rec.dtype or A_rec.shape[1:] != B_rec.shape[1:]:
        raise ValueError("A_rec and B_rec need the same dtype and row shape")
    for t, name in ((A_rec, "A_rec"), (B_rec, "B_rec")):
        if t.device.type != "cuda" or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous GPU tensor")
    N = codes.numel()
    if out is None:
        out = torch.empty((N,) + tuple(A_rec.shape[1:]), dtype=A_rec.dtype, device=codes.device)
    width = _record_width(A_rec)
    _check(load().cm_gather_records(_ptr(codes), N, _ptr(A_rec), A_rec.shape[0], _ptr(B_rec),
                                    B_rec.shape[0], width, _ptr(out),
                                    _stream(stream, codes.device)), "cm_gather_records")
    return out


def merge_records(A, B, A_rec, B_rec, descending=False, stream=None):
    """Stable merge of key arrays A and B whose payloads are records of any
    width (rows of A_rec / B_rec): the keys are merged with origin codes as
    payloads, then the records are gathered by code.  Returns (C, C_rec)."""
    if A_rec.shape[0] != A.numel() or B_rec.shape[0] != B.numel():
        raise ValueError("one record per key")
    a_codes, b_codes = origin_codes(A.numel(), B.numel(), A.device, stream)
    C, codes = stable_merge_pairs(A, a_codes, B, b_codes, stream=stream, descending=descending)
    return C, gather_records(codes, A_rec, B_rec, stream=stream)


def check_sorted(X, stream=None, descending=False) -> bool:
    """True if the device key array X is nondecreasing (nonincreasing if
    descending); synchronises."""
    torch = _torch()
    X = _dev(X, "X")
    flag = torch.empty(1, dtype=torch.uint32, device=X.device)
    _check(load().cm_check_sorted(_key_type(X, descending), _ptr(X), X.numel(), _ptr(flag),
                                  _stream(stream, X.device)), "cm_check_sorted")
    return int(flag.cpu()[0]) == 0


def config_count() -> int:
    return load().cm_config_count()


def config_info(config_id: int):
    nt, e = ctypes.c_int(), ctypes.c_int()
    _check(load().cm_config_info(config_id, ctypes.byref(nt), ctypes.byref(e)), "cm_config_info")
    return nt.value, e.value


def set_config(key_dtype, with_payload: bool, config_id: int):
    """Tile configuration of the merge calls for (key type, payload mode);
    -1 returns the pair to the per-operation defaults."""
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    _check(load().cm_set_config(kt, int(bool(with_payload)), config_id), "cm_set_config")


def get_config(key_dtype, with_payload: bool) -> int:
    """The configuration set for (key type, payload mode), or -1 while none
    is set (tuning_get gives the one a call would use)."""
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    return load().cm_get_config(kt, int(bool(with_payload)))


def set_search(mode: int):
    """Per-thread / one-level co-rank search: 0 = Algorithm 1, 1 = bisection."""
    _check(load().cm_set_search(mode), "cm_set_search")


def get_search() -> int:
    return load().cm_get_search()


def set_partition(mode: int):
    """Block-boundary pass: -1 = automatic (the default: 4 below 2^24
    outputs for a single merge, else 2), 0 = one thread per boundary, 1 = two-level with a
    64-lane coarse search, 2 = two-level with a 16-lane coarse search, 3 =
    one block per resident workgroup (streaming), 4 = no pass, each block
    co-ranks its own ends."""
    _check(load().cm_set_partition(mode), "cm_set_partition")


def get_partition() -> int:
    return load().cm_get_partition()


def set_grid(workgroups: int):
    """Workgroups of the block-merge kernels: 0 = one per block (default),
    -1 = a persistent grid of the resident workgroups, g > 0 = at most g;
    the workgroups stride over the blocks."""
    _check(load().cm_set_grid(workgroups), "cm_set_grid")


def get_grid() -> int:
    return load().cm_get_grid()


def set_coarse_stride(blocks: int):
    """Blocks between coarse boundaries of the two-level pass (>= 16)."""
    _check(load().cm_set_coarse_stride(blocks), "cm_set_coarse_stride")


def set_fine_lanes(lanes: int):
    """Lanes per boundary in the fine step of the two-level pass (1, 2, 4)."""
    _check(load().cm_set_fine_lanes(lanes), "cm_set_fine_lanes")


def set_block_order(order: int):
    """Block order of single merges, batches of separate merges, sort passes
    and copy_tiles: c >= 2 (default 32) runs of c blocks per XCD, 1 one
    contiguous run per XCD, 0 workgroup order."""
    _check(load().cm_set_block_order(order), "cm_set_block_order")


def get_block_order() -> int:
    return load().cm_get_block_order()


def get_coarse_stride() -> int:
    return load().cm_get_coarse_stride()


def get_fine_lanes() -> int:
    return load().cm_get_fine_lanes()


# ---------------------------------------------------------------------------
# argument marshalling shared by merge calls, tuner and plans


def _pair_args(A, B, A_val, B_val, C, C_val):
    """Validated (kt, with_val, m, n, A, Av, B, Bv, C, Cv) for one merge;
    allocates C / C_val when not given."""
    torch = _torch()
    A = _dev(A, "A")
    B = _dev(B, "B", A.dtype)
    with_val = A_val is not None
    if with_val != (B_val is not None):
        raise ValueError("give payloads for both inputs or neither")
    m, n = A.numel(), B.numel()
    if C is None:
        C = torch.empty(m + n, dtype=A.dtype, device=A.device)
    C = _dev(C, "C", A.dtype)
    if C.numel() != m + n:
        raise ValueError("C must hold m + n keys")
    if with_val:
        A_val = _dev(A_val, "A_val", torch.uint32)
        B_val = _dev(B_val, "B_val", torch.uint32)
        if A_val.numel() != m or B_val.numel() != n:
            raise ValueError("payload lengths must match key lengths")
        if C_val is None:
            C_val = torch.empty(m + n, dtype=torch.uint32, device=A.device)
        C_val = _dev(C_val, "C_val", torch.uint32)
        if C_val.numel() != m + n:
            raise ValueError("C_val must hold m + n payloads")
    else:
        A_val = B_val = C_val = None
    return _key_type(A), with_val, m, n, A, A_val, B, B_val, C, C_val


def _seg_args(A, a_off, B, b_off, A_val, B_val, C, C_val):
    torch = _torch()
    kt, with_val, ta, tb, A, A_val, B, B_val, C, C_val = _pair_args(A, B, A_val, B_val, C, C_val)
    a_off = _dev(a_off, "a_off", torch.uint64)
    b_off = _dev(b_off, "b_off", torch.uint64)
    if a_off.numel() != b_off.numel() or a_off.numel() < 1:
        raise ValueError("a_off and b_off need num_seg + 1 entries each")
    return kt, with_val, ta, tb, a_off.numel() - 1, A, A_val, a_off, B, B_val, b_off, C, C_val


def autotune_merge(A, B, A_val=None, B_val=None, reps=5, stream=None):
    """Time every (config, search, partition) on these inputs and record the
    fastest for their size class; returns (config, search, partition)."""
    kt, with_val, m, n, A, A_val, B, B_val, C, C_val = _pair_args(A, B, A_val, B_val, None, None)
    ws, wsb = _workspace(load().cm_merge_workspace_size(kt, int(with_val), m, n), A.device, None)
    best = (ctypes.c_int * 3)()
    _check(load().cm_autotune_merge(kt, _ptr(A), _ptr(A_val), m, _ptr(B), _ptr(B_val), n, _ptr(C),
                                    _ptr(C_val), _ptr(ws), wsb, reps, _stream(stream, A.device),
                                    best), "cm_autotune_merge")
    return tuple(best)


def autotune_segmented(A, a_off, B, b_off, A_val=None, B_val=None, reps=5, stream=None):
    """Tuner for the segmented batch; returns (config, search, partition)."""
    kt, with_val, ta, tb, S, A, A_val, a_off, B, B_val, b_off, C, C_val = _seg_args(
        A, a_off, B, b_off, A_val, B_val, None, None)
    ws, wsb = _workspace(load().cm_segmented_workspace_size(kt, int(with_val), ta, tb, S), A.device,
                         None)
    best = (ctypes.c_int * 3)()
    _check(load().cm_autotune_segmented(kt, _ptr(A), _ptr(A_val), _ptr(a_off), ta, _ptr(B),
                                        _ptr(B_val), _ptr(b_off), tb, S, _ptr(C), _ptr(C_val),
                                        _ptr(ws), wsb, reps, _stream(stream, A.device), best),
           "cm_autotune_segmented")
    return tuple(best)


def tuning_set(op, key_dtype, with_payload, size_class, config, search, partition):
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    _check(load().cm_tuning_set(op, kt, int(bool(with_payload)), size_class, config, search,
                                partition), "cm_tuning_set")


def tuning_get(op, key_dtype, with_payload, num_outputs):
    """(config, search, partition) a call of num_outputs outputs would use."""
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    out = (ctypes.c_int * 3)()
    _check(load().cm_tuning_get(op, kt, int(bool(with_payload)), num_outputs, out),
           "cm_tuning_get")
    return tuple(out)


def tuning_save(path=None):
    """Save the tuning table (path None: $CM_TUNING_FILE, else the user's
    cache directory)."""
    _check(load().cm_tuning_save(None if path is None else os.fsencode(path)), "cm_tuning_save")


def tuning_load(path=None):
    """Merge a saved tuning table into the library's (path None: as for
    tuning_save).  Raises CMError with status ESTALE for a table made for
    another device, HIP runtime or library build."""
    _check(load().cm_tuning_load(None if path is None else os.fsencode(path)), "cm_tuning_load")


def build_id() -> str:
    """The library's build id (a hash of its sources)."""
    return load().cm_build_id().decode()


def tuning_clear():
    _check(load().cm_tuning_clear(), "cm_tuning_clear")


def tuning_count() -> int:
    return load().cm_tuning_count()


class Plan:
    """A merge call captured once into a HIP graph; launch() replays it.
    Holds references to every buffer it was built on (they must stay alive
    and in place); outputs are the attributes C and C_val."""

    def __init__(self, handle, device, keep, C, C_val, kind="merge"):
        self._handle = handle
        self._device = device
        self._keep = keep
        self.C = C
        self.C_val = C_val
        self._kind = kind

    def update(self, A, B, A_val=None, B_val=None, C=None, C_val=None, workspace=None):
        """Re-point a single-merge plan at other arrays (cm_plan_update_merge);
        waits for the device first, so no earlier launch is still running."""
        if self._handle is None or self._kind != "merge":
            raise RuntimeError("update() needs an open plan made by plan_merge")
        kt, with_val, m, n, A, A_val, B, B_val, C, C_val = _pair_args(A, B, A_val, B_val, C, C_val)
        ws, wsb = _workspace(load().cm_merge_workspace_size(kt, int(with_val), m, n), A.device,
                             workspace)
        _torch().cuda.synchronize(self._device)
        _check(load().cm_plan_update_merge(self._handle, kt, _ptr(A), _ptr(A_val), m, _ptr(B),
                                           _ptr(B_val), n, _ptr(C), _ptr(C_val), _ptr(ws), wsb),
               "cm_plan_update_merge")
        self._keep = (A, A_val, B, B_val, ws)
        self.C, self.C_val = C, C_val

    def update_segmented(self, A, a_off, B, b_off, A_val=None, B_val=None, C=None, C_val=None,
                         workspace=None):
        """Re-point a segmented plan (cm_plan_update_segmented); waits for the
        device first."""
        if self._handle is None or self._kind != "segmented":
            raise RuntimeError("update_segmented() needs an open plan made by plan_segmented")
        kt, with_val, ta, tb, S, A, A_val, a_off, B, B_val, b_off, C, C_val = _seg_args(
            A, a_off, B, b_off, A_val, B_val, C, C_val)
        ws, wsb = _workspace(load().cm_segmented_workspace_size(kt, int(with_val), ta, tb, S),
                             A.device, workspace)
        _torch().cuda.synchronize(self._device)
        _check(load().cm_plan_update_segmented(self._handle, kt, _ptr(A), _ptr(A_val), _ptr(a_off),
                                               ta, _ptr(B), _ptr(B_val), _ptr(b_off), tb, S,
                                               _ptr(C), _ptr(C_val), _ptr(ws), wsb),
               "cm_plan_update_segmented")
        self._keep = (A, A_val, a_off, B, B_val, b_off, ws)
        self.C, self.C_val = C, C_val

    def launch(self, stream=None):
        if self._handle is None:
            raise RuntimeError("plan already closed")
        _check(load().cm_plan_launch(self._handle, _stream(stream, self._device)),
               "cm_plan_launch")
        return (self.C, self.C_val) if self.C_val is not None else self.C

    def close(self):
        if self._handle is not None:
            _torch().cuda.synchronize(self._device)
            _check(load().cm_plan_destroy(self._handle), "cm_plan_destroy")
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_merge(A, B, A_val=None, B_val=None, C=None, C_val=None, workspace=None) -> Plan:
    kt, with_val, m, n, A, A_val, B, B_val, C, C_val = _pair_args(A, B, A_val, B_val, C, C_val)
    ws, wsb = _workspace(load().cm_merge_workspace_size(kt, int(with_val), m, n), A.device,
                         workspace)
    h = ctypes.c_void_p()
    _check(load().cm_plan_create_merge(kt, _ptr(A), _ptr(A_val), m, _ptr(B), _ptr(B_val), n,
                                       _ptr(C), _ptr(C_val), _ptr(ws), wsb, ctypes.byref(h)),
           "cm_plan_create_merge")
    return Plan(h, A.device, (A, A_val, B, B_val, ws), C, C_val)


def plan_segmented(A, a_off, B, b_off, A_val=None, B_val=None, C=None, C_val=None,
                   workspace=None) -> Plan:
    kt, with_val, ta, tb, S, A, A_val, a_off, B, B_val, b_off, C, C_val = _seg_args(
        A, a_off, B, b_off, A_val, B_val, C, C_val)
    ws, wsb = _workspace(load().cm_segmented_workspace_size(kt, int(with_val), ta, tb, S), A.device,
                         workspace)
    h = ctypes.c_void_p()
    _check(load().cm_plan_create_segmented(kt, _ptr(A), _ptr(A_val), _ptr(a_off), ta, _ptr(B),
                                           _ptr(B_val), _ptr(b_off), tb, S, _ptr(C), _ptr(C_val),
                                           _ptr(ws), wsb, ctypes.byref(h)),
           "cm_plan_create_segmented")
    return Plan(h, A.device, (A, A_val, a_off, B, B_val, b_off, ws), C, C_val, kind="segmented")


# layout of cm_merge_desc (nine 64-bit fields)
_DESC_FIELDS = ("A", "A_val", "m", "B", "B_val", "n", "C", "C_val", "first_block")


def stable_merge_batch(merges, with_payload=None, stream=None, upload=None):
    """Merge several separately allocated pairs of sorted device arrays in one
    launch (cm_stable_merge_batch).  merges: list of (A, B) or
    (A, A_val, B, B_val) tuples, all of one key dtype.  upload: copy the
    descriptors to the device (default: only for more than
    CM_BATCH_INLINE_MAX merges; fewer travel in the kernel arguments).
    Returns a list of C or (C, C_val) in the same order."""
    import numpy as np
    torch = _torch()
    if not merges:
        return []
    if with_payload is None:
        with_payload = len(merges[0]) == 4
    device = merges[0][0].device
    s = stream if stream is not None else torch.cuda.current_stream(device)
    with torch.cuda.stream(s):  # outputs, descriptor upload and workspace all on s
        return _merge_batch_on(merges, with_payload, s, upload)


def batch_descriptors(count):
    """Zeroed host array laid out as cm_merge_desc[count]."""
    import numpy as np
    return np.zeros(count, dtype=np.dtype([(f, np.uint64) for f in _DESC_FIELDS]))


BATCH_INLINE_MAX = 16  # CM_BATCH_INLINE_MAX


def launch_batch(key_dtype, with_payload, descs, device, stream, upload=None):
    """cm_batch_prepare + (upload) + cm_stable_merge_batch for descriptors the
    caller filled (pointers and sizes; first_block is set here).  Without an
    upload (the default for at most BATCH_INLINE_MAX merges) the descriptors
    travel in the kernel arguments.  Returns the device buffers the call
    uses; they must stay alive until the stream has run it (torch's
    allocator keeps them ordered on `stream`)."""
    import numpy as np
    torch = _torch()
    kt = KEY_TYPES[str(key_dtype).replace("torch.", "")]
    total = ctypes.c_uint64()
    _check(load().cm_batch_prepare(kt, int(with_payload), descs.ctypes.data_as(ctypes.c_void_p),
                                   len(descs), ctypes.byref(total)), "cm_batch_prepare")
    if upload is None:
        upload = len(descs) > BATCH_INLINE_MAX
    with torch.cuda.stream(stream):
        # pinned staging so the upload is stream-ordered and does not block the host
        descs_dev = torch.from_numpy(descs.view(np.uint8)).pin_memory().to(
            device, non_blocking=True) if upload else None
        ws, wsb = _workspace(load().cm_batch_workspace_size(total.value, len(descs)), device,
                             None)
    _check(load().cm_stable_merge_batch(kt, int(with_payload),
                                        descs.ctypes.data_as(ctypes.c_void_p), _ptr(descs_dev),
                                        len(descs), total.value, _ptr(ws), wsb,
                                        ctypes.c_void_p(stream.cuda_stream)),
           "cm_stable_merge_batch")
    return descs_dev, ws


def _merge_batch_on(merges, with_payload, stream, upload=None):
    import numpy as np
    torch = _torch()
    prepared = []
    for item in merges:
        if with_payload:
            A, A_val, B, B_val = item
        else:
            (A, B), A_val, B_val = item, None, None
        prepared.append(_pair_args(A, B, A_val, B_val, None, None))
    kt = prepared[0][0]
    device = prepared[0][4].device
    if any(p[0] != kt for p in prepared):
        raise TypeError("all merges of a batch must have the same key dtype")
    descs = batch_descriptors(len(prepared))
    for r, (_, _, m, n, A, Av, B, Bv, C, Cv) in enumerate(prepared):
        descs[r] = (A.data_ptr() if m else 0, Av.data_ptr() if with_payload and m else 0, m,
                    B.data_ptr() if n else 0, Bv.data_ptr() if with_payload and n else 0, n,
                    C.data_ptr() if m + n else 0, Cv.data_ptr() if with_payload and m + n else 0, 0)
    launch_batch(prepared[0][4].dtype, with_payload, descs, device, stream, upload)
    return [(p[8], p[9]) if with_payload else p[8] for p in prepared]
