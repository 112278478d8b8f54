"""Pins of the oracle under the reversed key order (CPU).

The method merges under any total order (Section 2), so the descending
variants must satisfy, under x <=' y :<=> x >= y:
- the merge equals numpy's stable argsort of A ++ B applied to an
  order-reversing image of the keys (bitwise complement for unsigned keys,
  negation for floats), A's equal keys first;
- Lemma 1 with the reversed comparisons, exhaustively on tiny inputs, with
  its uniqueness; Algorithm 1 finds the same pair;
- closed forms: all keys equal gives A then B; A entirely above B gives
  j = min(i, m).
Planted mistakes in the descending branch of oracle.c must fail a pin."""
import itertools
import os
import subprocess

import numpy as np
import pytest

import oracle


def image(x):
    return -x if x.dtype == np.float32 else ~x


def desc_sorted(rng, n, dtype, hi):
    if np.dtype(dtype) == np.float32:
        k = (rng.integers(0, hi, n) - hi // 2).astype(np.float32) / 4
        k[rng.random(n) < 0.1] = -0.0
        k[rng.random(n) < 0.1] = 0.0
        return k[np.argsort(-k, kind="stable")]
    return np.sort(rng.integers(0, hi, n).astype(dtype))[::-1].copy()


def check_numpy_route(dtype, seed=0):
    rng = np.random.default_rng(seed)
    for m, n in ((0, 0), (1, 0), (0, 3), (5, 7), (100, 1), (333, 444), (2000, 1999)):
        for hi in (3, 1 << 16):
            A, B = desc_sorted(rng, m, dtype, hi), desc_sorted(rng, n, dtype, hi)
            Av = np.arange(m, dtype=np.uint32)
            Bv = (np.arange(n, dtype=np.uint32) + np.uint32(1 << 31)).astype(np.uint32)
            C, Cv = oracle.stable_merge(A, B, Av, Bv, descending=True)
            cat = np.concatenate([A, B])
            order = np.argsort(image(cat), kind="stable")
            assert np.array_equal(C.view(np.uint8), cat[order].view(np.uint8))
            assert np.array_equal(Cv, np.concatenate([Av, Bv])[order])


def check_lemma_exhaustive(letters=3, max_len=5):
    cases = 0
    for m in range(max_len + 1):
        for n in range(max_len + 1):
            for a in itertools.combinations_with_replacement(range(letters), m):
                A = np.array(a[::-1], dtype=np.uint32)  # nonincreasing
                for b in itertools.combinations_with_replacement(range(letters), n):
                    B = np.array(b[::-1], dtype=np.uint32)
                    for i in range(m + n + 1):
                        j, k = oracle.co_rank_brute(i, A, B, descending=True)
                        j1, k1, _ = oracle.co_rank_alg1(i, A, B, descending=True)
                        assert (j, k) == (j1, k1)
                        ok = [jj for jj in range(max(0, i - n), min(i, m) + 1)
                              if (jj == 0 or i - jj == n or A[jj - 1] >= B[i - jj])
                              and (i - jj == 0 or jj == m or B[i - jj - 1] > A[jj])]
                        assert ok == [j], (A, B, i, ok, j)
                        cases += 1
    return cases


def check_closed_forms():
    m, n = 40, 25
    eq = np.full(m, 5, np.uint64), np.full(n, 5, np.uint64)
    for i in range(m + n + 1):
        assert oracle.co_rank_brute(i, *eq, descending=True)[0] == min(i, m)
    A = np.arange(m, dtype=np.uint32)[::-1].copy() + np.uint32(100)  # all above B
    B = np.arange(n, dtype=np.uint32)[::-1].copy()
    for i in range(m + n + 1):
        assert oracle.co_rank_alg1(i, A, B, descending=True)[0] == min(i, m)
    assert np.array_equal(oracle.stable_merge(A, B, descending=True), np.concatenate([A, B]))


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64, np.float32])
def test_merge_equals_numpy_route(dtype):
    check_numpy_route(dtype)


def test_lemma_and_algorithm1_exhaustive():
    assert check_lemma_exhaustive() > 10000


def test_closed_forms():
    check_closed_forms()


def test_sort_descending():
    rng = np.random.default_rng(9)
    for dtype in (np.uint32, np.uint64, np.float32):
        keys = desc_sorted(rng, 500, dtype, 20)
        rng.shuffle(keys)
        k, v = oracle.stable_sort(keys, np.arange(500, dtype=np.uint32), descending=True)
        # nonincreasing; equal keys in input order; a permutation
        assert np.all(k[:-1] >= k[1:])
        for x in range(499):
            if k[x] == k[x + 1]:
                assert v[x] < v[x + 1]
        assert sorted(v.tolist()) == list(range(500))
        # equals merge sort built from the descending oracle merge
        runs = [(keys[x:x + 1], np.array([x], np.uint32)) for x in range(500)]
        while len(runs) > 1:
            nxt = [oracle.stable_merge(runs[r][0], runs[r + 1][0], runs[r][1], runs[r + 1][1],
                                       descending=True) for r in range(0, len(runs) - 1, 2)]
            runs = nxt + ([runs[-1]] if len(runs) % 2 else [])
        assert np.array_equal(runs[0][0].view(np.uint8), k.view(np.uint8))
        assert np.array_equal(runs[0][1], v)


SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
MUTANTS = {
    # the descending order compared ascending in the merge
    "desc_le_ascending": ("return kt >= ORACLE_DESC ? num_le(base_type(kt), B, b, A, a) : num_le(kt, A, a, B, b);",
                          "return kt >= ORACLE_DESC ? num_le(base_type(kt), A, a, B, b) : num_le(kt, A, a, B, b);"),
    # descending tie rule flipped (B's equal keys first)
    "desc_tie_strict": ("return kt >= ORACLE_DESC ? num_le(base_type(kt), B, b, A, a) : num_le(kt, A, a, B, b);",
                        "return kt >= ORACLE_DESC ? num_lt(base_type(kt), B, b, A, a) : num_le(kt, A, a, B, b);"),
    # Algorithm 1's first test with the ascending order under descending keys
    "desc_gt_ascending": ("return kt >= ORACLE_DESC ? num_lt(base_type(kt), A, a, B, b) : num_lt(kt, B, b, A, a);",
                          "return kt >= ORACLE_DESC ? num_lt(base_type(kt), B, b, A, a) : num_lt(kt, B, b, A, a);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_descending_mutant(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found"
    c_path = tmp_path / "oracle_mutant.c"
    so_path = tmp_path / "liboracle_mutant.so"
    c_path.write_text(src.replace(old, new))
    subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", str(so_path),
                    str(c_path)], check=True)
    monkeypatch.setattr(oracle, "_lib", oracle.open_library(str(so_path)))
    caught = 0
    for check in (lambda: check_numpy_route(np.uint32), lambda: check_lemma_exhaustive(3, 3),
                  check_closed_forms):
        try:
            check()
        except (AssertionError, RuntimeError):
            caught += 1
    assert caught >= 1, f"mutant {name} passed every pin"
