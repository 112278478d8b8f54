"""Pins of oracle.stable_sort (CPU).  The oracle's sort is numpy's stable
argsort; each pin below reaches the same result by a different route:

- brute force: every sequence over a 3-letter alphabet up to length 7,
  sorted by adjacent swaps of strictly out-of-order neighbours (a stable
  insertion sort in plain Python);
- merge sort from the oracle's own stable merge, itself pinned to the
  paper's Figure 1 (bottom-up: runs of 1, 2, 4, ... merged pairwise with
  the left run as A, so equal keys keep input order);
- closed forms: sorted input is unchanged, strictly decreasing input is
  reversed, all-equal input is unchanged;
- IEEE order for float keys: -0.0 and +0.0 are equal and keep input order.
Origin payloads (position x carries x) make stability visible: the sorted
(key, payload) pairs must be strictly increasing.
"""
import itertools

import numpy as np
import pytest

import oracle


def insertion_sort(keys):
    idx = list(range(len(keys)))
    k = list(keys)
    for a in range(1, len(k)):
        j = a
        while j > 0 and k[j] < k[j - 1]:  # strictly out of order only
            k[j], k[j - 1] = k[j - 1], k[j]
            idx[j], idx[j - 1] = idx[j - 1], idx[j]
            j -= 1
    return k, idx


def merge_sort_from_oracle_merge(keys, vals):
    runs = [(keys[x:x + 1], vals[x:x + 1]) for x in range(keys.size)]
    while len(runs) > 1:
        nxt = []
        for r in range(0, len(runs) - 1, 2):
            (a, av), (b, bv) = runs[r], runs[r + 1]
            nxt.append(oracle.stable_merge(a, b, av, bv))
        if len(runs) % 2:
            nxt.append(runs[-1])
        runs = nxt
    return runs[0] if runs else (keys[:0], vals[:0])


def test_brute_force_small_alphabet():
    cases = 0
    for n in range(0, 8):
        for seq in itertools.product(range(3), repeat=n):
            keys = np.array(seq, dtype=np.uint32)
            vals = np.arange(n, dtype=np.uint32)
            k, v = oracle.stable_sort(keys, vals)
            ek, ev = insertion_sort(seq)
            assert k.tolist() == ek and v.tolist() == ev
            cases += 1
    assert cases == sum(3 ** n for n in range(8))


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64, np.float32])
def test_equals_merge_sort_built_from_the_pinned_merge(dtype):
    rng = np.random.default_rng(7)
    for n in (1, 2, 3, 17, 64, 1000, 4097):
        if np.dtype(dtype) == np.float32:
            keys = rng.integers(-20, 20, n).astype(np.float32) / 4
            keys[rng.random(n) < 0.1] = -0.0
        else:
            keys = rng.integers(0, 50, n).astype(dtype)
        vals = np.arange(n, dtype=np.uint32)
        k, v = oracle.stable_sort(keys, vals)
        ek, ev = merge_sort_from_oracle_merge(keys, vals)
        assert np.array_equal(k.view(np.uint8), ek.view(np.uint8)) and np.array_equal(v, ev)
        order = np.lexsort((v, k))
        assert np.array_equal(order, np.arange(n))  # (key, payload) increasing: stable
        assert sorted(v.tolist()) == list(range(n))


def test_closed_forms():
    n = 1000
    up = np.arange(n, dtype=np.uint32) * 3
    k, v = oracle.stable_sort(up, np.arange(n, dtype=np.uint32))
    assert np.array_equal(k, up) and np.array_equal(v, np.arange(n))
    down = up[::-1].copy()
    k, v = oracle.stable_sort(down, np.arange(n, dtype=np.uint32))
    assert np.array_equal(k, up) and np.array_equal(v, np.arange(n)[::-1])
    same = np.full(n, 7, dtype=np.uint64)
    k, v = oracle.stable_sort(same, np.arange(n, dtype=np.uint32))
    assert np.array_equal(v, np.arange(n))
    assert oracle.stable_sort(np.zeros(0, np.uint32)).size == 0


def test_signed_zeros_are_equal_keys():
    keys = np.array([0.0, -0.0, 1.0, -0.0, 0.0, -1.0], dtype=np.float32)
    k, v = oracle.stable_sort(keys, np.arange(6, dtype=np.uint32))
    assert v.tolist() == [5, 0, 1, 3, 4, 2]
    assert np.signbit(k).tolist() == [True, False, True, True, False, False]


def _pins_pass(sort_fn):
    """The brute-force and merge-sort pins, run against any sort function."""
    rng = np.random.default_rng(3)
    try:
        for n in range(0, 7):
            for seq in itertools.product(range(3), repeat=n):
                k, v = sort_fn(np.array(seq, dtype=np.uint32), np.arange(n, dtype=np.uint32))
                ek, ev = insertion_sort(seq)
                if k.tolist() != ek or v.tolist() != ev:
                    return False
        for n in (100, 4097):
            keys = rng.integers(0, 10, n).astype(np.float32) - 5
            keys[rng.random(n) < 0.2] = -0.0
            keys[rng.random(n) < 0.2] = 0.0
            vals = np.arange(n, dtype=np.uint32)
            k, v = sort_fn(keys, vals)
            ek, ev = merge_sort_from_oracle_merge(keys, vals)
            if not (np.array_equal(k.view(np.uint8), ek.view(np.uint8)) and np.array_equal(v, ev)):
                return False
    except Exception:
        return False
    return True


def test_pins_catch_plausible_mistakes():
    assert _pins_pass(oracle.stable_sort)
    mutants = {
        "unstable algorithm": lambda k, v: (np.sort(k, kind="heapsort"),
                                            v[np.argsort(k, kind="heapsort")]),
        "descending": lambda k, v: (k[np.argsort(k, kind="stable")[::-1]],
                                    v[np.argsort(k, kind="stable")[::-1]]),
        "payloads not moved": lambda k, v: (np.sort(k, kind="stable"), v),
        "float keys by bit pattern": lambda k, v: (
            k[np.argsort(k.view(np.int32) if k.dtype == np.float32 else k, kind="stable")],
            v[np.argsort(k.view(np.int32) if k.dtype == np.float32 else k, kind="stable")]),
    }
    for name, fn in mutants.items():
        assert not _pins_pass(fn), f"mutant '{name}' passed the pins"
