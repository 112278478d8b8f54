"""CPU oracle for the stable merge and co-ranking (arXiv:1303.4312).

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU library in ``paper_1303_4312_amd`` and the GPU library never
imports it.

The arithmetic lives in ``oracle.c`` (plain single-threaded C); this module
only compiles it, loads it and marshals numpy arrays:

- :func:`stable_merge` -- the sequential stable merge (Section 1), equal keys
  from A before equal keys from B (Section 2).
- :func:`co_rank_brute` -- co-ranks by definition (Section 2, Lemma 1):
  merge i outputs and count those taken from A.
- :func:`co_rank_alg1` -- Algorithm 1 (Section 2) with its state trace.
- :func:`stable_merge_segmented` -- the merge applied to each segment of a
  batch independently.
- :func:`stable_sort` -- the stable sort merge sort computes (Section 1
  names merging as the step of merge sort): the permutation that orders the
  keys, equal keys in input order.  numpy's stable argsort is the step; no
  merge code is involved, so the GPU merge sort is checked against the
  definition rather than against another merge sort.

Every function takes ``descending=True`` for keys ordered nonincreasingly:
the same method under the reversed total order (Section 2 merges under any
total order), equal keys still A first.

Key types: numpy uint32, uint64, float32. Payloads: uint32 or None.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_KT = {np.dtype(np.uint32): 0, np.dtype(np.uint64): 1, np.dtype(np.float32): 2}
_DESC = 3  # key types 3..5: the same keys under the reversed order

_lib = None


def build() -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, -O2, no threads)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", _LIB_PATH, _SRC]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB_PATH)
                or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        _lib = open_library(_LIB_PATH)
    return _lib


def open_library(path):
    """Load a compiled copy of oracle.c and declare its signatures."""
    lib = ctypes.CDLL(path)
    vp, u64, p64, p32 = (ctypes.c_void_p, ctypes.c_uint64,
                         ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p)
    lib.oracle_stable_merge.argtypes = [ctypes.c_int, vp, p32, u64, vp, p32, u64, vp, p32]
    lib.oracle_stable_merge.restype = None
    lib.oracle_co_rank_brute.argtypes = [ctypes.c_int, u64, vp, u64, vp, u64]
    lib.oracle_co_rank_brute.restype = u64
    lib.oracle_co_rank_alg1.argtypes = [ctypes.c_int, u64, vp, u64, vp, u64,
                                        p64, p64, vp, u64, p64, p64]
    lib.oracle_co_rank_alg1.restype = ctypes.c_int
    lib.oracle_stable_merge_segmented.argtypes = [ctypes.c_int, vp, p32, vp, vp, p32, vp,
                                                  u64, vp, p32]
    lib.oracle_stable_merge_segmented.restype = None
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _keys(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype=dtype))
    if a.dtype not in _KT:
        raise TypeError(f"oracle: unsupported key dtype {a.dtype}")
    return a


def _pay(v, length):
    if v is None:
        return None
    v = np.ascontiguousarray(v, dtype=np.uint32)
    if v.shape != (length,):
        raise ValueError("oracle: payload length differs from key length")
    return v


def _kt(dtype, descending):
    return _KT[dtype] + (_DESC if descending else 0)


def stable_merge(A, B, Av=None, Bv=None, descending=False):
    """Stable merge of sorted A and B (both nonincreasing, merged under the
    reversed order, if descending); returns C, or (C, Cv) with payloads."""
    A = _keys(A)
    B = _keys(B, A.dtype)
    if (Av is None) != (Bv is None):
        raise ValueError("oracle: give payloads for both inputs or neither")
    Av, Bv = _pay(Av, A.size), _pay(Bv, B.size)
    C = np.empty(A.size + B.size, dtype=A.dtype)
    Cv = None if Av is None else np.empty(A.size + B.size, dtype=np.uint32)
    _load().oracle_stable_merge(_kt(A.dtype, descending), _ptr(A), _ptr(Av), A.size,
                                _ptr(B), _ptr(Bv), B.size, _ptr(C), _ptr(Cv))
    return C if Cv is None else (C, Cv)


def co_rank_brute(i, A, B, descending=False):
    """(j, k) for output rank i, by merging i outputs and counting A's."""
    A = _keys(A)
    B = _keys(B, A.dtype)
    if not 0 <= i <= A.size + B.size:
        raise ValueError("oracle: rank out of range")
    j = int(_load().oracle_co_rank_brute(_kt(A.dtype, descending), i, _ptr(A), A.size, _ptr(B),
                                         B.size))
    return j, i - j


def co_rank_alg1(i, A, B, trace_cap=0, descending=False):
    """Algorithm 1. Returns (j, k, iters) or, with trace_cap > 0,
    (j, k, iters, states) where states is a list of (j, k, j_low, k_low)
    tuples (k_low is None before it is first assigned)."""
    A = _keys(A)
    B = _keys(B, A.dtype)
    if not 0 <= i <= A.size + B.size:
        raise ValueError("oracle: rank out of range")
    j = ctypes.c_uint64()
    k = ctypes.c_uint64()
    ns = ctypes.c_uint64()
    it = ctypes.c_uint64()
    tr = np.zeros(4 * max(trace_cap, 1), dtype=np.uint64)
    rc = _load().oracle_co_rank_alg1(_kt(A.dtype, descending), i, _ptr(A), A.size, _ptr(B), B.size,
                                     ctypes.byref(j), ctypes.byref(k),
                                     _ptr(tr) if trace_cap else None, trace_cap,
                                     ctypes.byref(ns), ctypes.byref(it))
    if rc != 0:
        raise RuntimeError("oracle: Algorithm 1 did not terminate")
    if not trace_cap:
        return j.value, k.value, it.value
    states = []
    for s in range(min(ns.value, trace_cap)):
        jj, kk, jl, kl = (int(x) for x in tr[4 * s:4 * s + 4])
        states.append((jj, kk, jl, None if kl == 2**64 - 1 else kl))
    return j.value, k.value, it.value, states


def stable_merge_segmented(A, a_off, B, b_off, Av=None, Bv=None, descending=False):
    """Merge segment s of A with segment s of B into C at a_off[s]+b_off[s]."""
    A = _keys(A)
    B = _keys(B, A.dtype)
    a_off = np.ascontiguousarray(a_off, dtype=np.uint64)
    b_off = np.ascontiguousarray(b_off, dtype=np.uint64)
    if a_off.shape != b_off.shape or a_off.size < 1:
        raise ValueError("oracle: offset arrays must both have num_seg+1 entries")
    if int(a_off[-1]) != A.size or int(b_off[-1]) != B.size:
        raise ValueError("oracle: last offset must equal the array length")
    if (Av is None) != (Bv is None):
        raise ValueError("oracle: give payloads for both inputs or neither")
    Av, Bv = _pay(Av, A.size), _pay(Bv, B.size)
    C = np.empty(A.size + B.size, dtype=A.dtype)
    Cv = None if Av is None else np.empty(A.size + B.size, dtype=np.uint32)
    _load().oracle_stable_merge_segmented(_kt(A.dtype, descending), _ptr(A), _ptr(Av),
                                          _ptr(a_off),
                                          _ptr(B), _ptr(Bv), _ptr(b_off), a_off.size - 1,
                                          _ptr(C), _ptr(Cv))
    return C if Cv is None else (C, Cv)


def stable_sort(keys, vals=None, descending=False):
    """Keys sorted nondecreasingly (nonincreasingly if descending), equal
    keys keeping their input order (IEEE comparison for float32: -0.0 and
    +0.0 are equal keys); payloads follow their keys.  Returns keys, or
    (keys, payloads).  The nonincreasing order is the nondecreasing order of
    an order-reversing image of the keys (bitwise complement for unsigned
    keys, negation for floats, which keeps -0.0 and +0.0 equal)."""
    k = _keys(keys)
    if descending:
        image = -k if k.dtype == np.float32 else ~k
        order = np.argsort(image, kind="stable")
    else:
        order = np.argsort(k, kind="stable")
    if vals is None:
        return k[order]
    v = _pay(vals, k.size)
    return k[order], v[order]
