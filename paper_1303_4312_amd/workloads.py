"""Seeded synthetic inputs for the stable merge.

This module only draws random sorted arrays (and the payloads and offsets
that go with them). It holds none of the merge or co-ranking arithmetic, so
the GPU path and the CPU oracle can both take their inputs from it.

Every generator is a pure function of its arguments and seed (numpy PCG64).
Payloads are "origin" indices: A[x] carries x and B[y] carries 2**31 + y, so
that the stability of a merge can be read off its output payloads.

Recipes (sizes are the defaults; tests pass smaller ones):

- ``dup16``       m = n = 2**20, uint32 keys uniform in [0, 2**16), sorted
                  (about 32 copies of every key).
- ``zipf``        m = 2**28, n = 2**26, uint32 keys from an alphabet of 1024
                  distinct seeded values with Zipf(1.1) frequencies, sorted.
- ``u64``         m = n = 2**27, uint64 keys uniform on [0, 2**64), sorted.
- ``f32``         m = n = 2**27, float32 keys ~ N(0, 1) (no NaN), sorted; the
                  test variant also plants -0.0 and +0.0 keys.
- ``a_below_b``   all of A below all of B: A[x] = x, B[y] = m + y.
- ``interleaved`` A[x] = 2x, B[y] = 2y + 1.
- ``all_equal``   every key of A and B equal to 7.
- ``segmented``   num_seg independent merges, each side's length drawn
                  log-uniform in [1, 2**16], uint32 keys uniform in
                  [0, 2**20) sorted within each segment.
- ``request``     one serving request: each side's length log-uniform in
                  [2**10, 2**24], uint32 keys uniform, sorted.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 13034312
PAYLOAD_B_BIT = np.uint32(1 << 31)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def origin_payloads(m: int, n: int):
    """A[x] carries x, B[y] carries 2**31 + y (requires m, n < 2**31)."""
    if m >= 1 << 31 or n >= 1 << 31:
        raise ValueError("origin payloads need m, n < 2**31")
    av = np.arange(m, dtype=np.uint32)
    bv = np.arange(n, dtype=np.uint32) | PAYLOAD_B_BIT
    return av, bv


def _pack(A, B, payload):
    out = {"A": A, "B": B}
    if payload:
        out["Av"], out["Bv"] = origin_payloads(A.size, B.size)
    return out


def dup16(seed: int = SEED_BASE + 1000, m: int = 1 << 20, n: int = 1 << 20,
          high: int = 1 << 16, payload: bool = True):
    """uint32 keys i.i.d. uniform on [0, high), each array sorted."""
    rng = rng_for(seed)
    A = np.sort(rng.integers(0, high, size=m, dtype=np.uint32))
    B = np.sort(rng.integers(0, high, size=n, dtype=np.uint32))
    return _pack(A, B, payload)


def zipf_alphabet(rng: np.random.Generator, size: int = 1024, s: float = 1.1):
    """Sorted alphabet of `size` distinct uint32 values and, for each value in
    sorted order, its probability; the Zipf ranks are assigned to the values
    through a seeded permutation so frequent keys are spread over the range."""
    values = np.sort(rng.choice(np.uint64(1) << np.uint64(32), size=size,
                                replace=False)).astype(np.uint32)
    ranks = np.arange(1, size + 1, dtype=np.float64)
    p_rank = ranks ** (-s)
    p_rank /= p_rank.sum()
    perm = rng.permutation(size)          # value index v gets rank perm[v]+1
    return values, p_rank[perm]


def zipf(seed: int = SEED_BASE + 2000, m: int = 1 << 28, n: int = 1 << 26,
         alphabet: int = 1024, s: float = 1.1, payload: bool = True):
    """uint32 keys drawn from a Zipf(s) distribution over `alphabet` distinct
    values, sorted (generated sorted: multinomial counts per value)."""
    rng = rng_for(seed)
    values, p = zipf_alphabet(rng, alphabet, s)
    A = np.repeat(values, rng.multinomial(m, p))
    B = np.repeat(values, rng.multinomial(n, p))
    return _pack(A, B, payload)


def u64(seed: int = SEED_BASE + 3001, m: int = 1 << 27, n: int = 1 << 27,
        payload: bool = True):
    rng = rng_for(seed)
    A = np.sort(rng.integers(0, np.iinfo(np.uint64).max, size=m, dtype=np.uint64,
                             endpoint=True))
    B = np.sort(rng.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64,
                             endpoint=True))
    return _pack(A, B, payload)


def f32(seed: int = SEED_BASE + 3002, m: int = 1 << 27, n: int = 1 << 27,
        payload: bool = True, signed_zeros: int = 0):
    """float32 keys ~ N(0,1), sorted. `signed_zeros` > 0 overwrites that many
    random positions of each array with -0.0 or +0.0 before sorting."""
    rng = rng_for(seed)
    A = rng.standard_normal(m, dtype=np.float32)
    B = rng.standard_normal(n, dtype=np.float32)
    if signed_zeros:
        for X in (A, B):
            if X.size:
                pos = rng.integers(0, X.size, size=signed_zeros)
                X[pos] = np.where(rng.integers(0, 2, size=signed_zeros) == 1,
                                  np.float32(-0.0), np.float32(0.0))
    # np.sort orders -0.0 and +0.0 as equal and may leave them in any
    # relative order, which is a valid sorted array under IEEE comparison.
    return _pack(np.sort(A), np.sort(B), payload)


def structured(kind: str, m: int = 1 << 27, n: int = 1 << 27,
               dtype=np.uint32, payload: bool = True):
    """The three degenerate cases: 'a_below_b', 'interleaved', 'all_equal'."""
    dt = np.dtype(dtype)
    if kind == "a_below_b":
        A = np.arange(m, dtype=np.float64)
        B = np.arange(n, dtype=np.float64) + m
    elif kind == "interleaved":
        A = 2.0 * np.arange(m, dtype=np.float64)
        B = 2.0 * np.arange(n, dtype=np.float64) + 1.0
    elif kind == "all_equal":
        A = np.full(m, 7.0)
        B = np.full(n, 7.0)
    else:
        raise ValueError(f"unknown structured kind {kind!r}")
    if dt == np.float32 and max(A.max(initial=0), B.max(initial=0)) >= 1 << 24:
        raise ValueError("float32 cannot hold these integers exactly")
    if dt.kind == "u":
        # exact integer construction (float64 is exact below 2**53)
        A = A.astype(np.uint64).astype(dt)
        B = B.astype(np.uint64).astype(dt)
    else:
        A = A.astype(dt)
        B = B.astype(dt)
    return _pack(A, B, payload)


def log_uniform_lengths(rng: np.random.Generator, count: int, lo: int, hi: int):
    """Log-uniform integers in [lo, hi]: floor(exp(ln lo + U (ln(hi+1) - ln lo)))
    with U uniform on [0, 1).  lo = 0 shifts the range [1, hi + 1] down by one
    so that empty sides occur."""
    if lo == 0:
        return log_uniform_lengths(rng, count, 1, hi + 1) - 1
    u = rng.random(count)
    L = np.floor(np.exp(np.log(lo) + u * (np.log(hi + 1) - np.log(lo)))).astype(np.int64)
    return np.clip(L, lo, hi)


def _sorted_within_segments(rng, lengths, high):
    """Uniform keys in [0, high) sorted inside each segment (one global sort
    on (segment, key), which sorts each segment and keeps segments apart)."""
    total = int(lengths.sum())
    seg = np.repeat(np.arange(lengths.size, dtype=np.uint64), lengths)
    keys = rng.integers(0, high, size=total, dtype=np.uint64)
    shift = np.uint64(int(high - 1).bit_length())
    combo = np.sort((seg << shift) | keys)
    del seg, keys
    return (combo & np.uint64((1 << int(shift)) - 1)).astype(np.uint32)


def segmented(seed: int = SEED_BASE + 4000, num_seg: int = 65536,
              max_side: int = 1 << 16, key_high: int = 1 << 20,
              min_side: int = 1, payload: bool = True):
    """num_seg independent merge problems laid out back to back.
    Returns A, B (concatenated keys), a_off, b_off (uint64, num_seg + 1
    entries) and, with payload, Av, Bv = global origin indices."""
    rng = rng_for(seed)
    la = log_uniform_lengths(rng, num_seg, min_side, max_side)
    lb = log_uniform_lengths(rng, num_seg, min_side, max_side)
    a_off = np.zeros(num_seg + 1, dtype=np.uint64)
    b_off = np.zeros(num_seg + 1, dtype=np.uint64)
    np.cumsum(la, out=a_off[1:])
    np.cumsum(lb, out=b_off[1:])
    A = _sorted_within_segments(rng, la, key_high)
    B = _sorted_within_segments(rng, lb, key_high)
    out = _pack(A, B, payload)
    out["a_off"], out["b_off"] = a_off, b_off
    return out


def request(seed: int, lo: int = 1 << 10, hi: int = 1 << 24, payload: bool = True):
    """One serving request: each side log-uniform in [lo, hi], uint32 keys
    uniform on [0, 2**32), sorted."""
    rng = rng_for(seed)
    m, n = (int(x) for x in log_uniform_lengths(rng, 2, lo, hi))
    A = np.sort(rng.integers(0, 1 << 32, size=m, dtype=np.uint64).astype(np.uint32))
    B = np.sort(rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32))
    return _pack(A, B, payload)
