"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself:
- the paper's worked example (Figures 1, 2 and 3), stored in
  tests/golden/figure_example.json with citations;
- Lemma 1 written out directly (the two conditions, with the sentinels
  A[-1] = B[-1] = -inf and A[m] = B[n] = +inf), including uniqueness, by
  exhaustive enumeration of all sorted arrays over small alphabets;
- numpy's stable argsort of the concatenation A ++ B (a stable sort keeps
  A's copies of a key before B's, which is the paper's tie rule) and the
  rank formula pos(A[x]) = x + #{B < A[x]}, pos(B[y]) = y + #{A <= B[y]};
- closed forms for the degenerate inputs (all equal, A below B,
  interleaved);
- Proposition 1's iteration bound, in the corrected form.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1303_4312_amd import workloads

# ----------------------------------------------------------------------------
# independent views (not the oracle)


def lemma1_holds(A, B, i, j):
    """Both conditions of Lemma 1 for (j, k = i - j), sentinels included."""
    m, n = len(A), len(B)
    k = i - j
    if not (0 <= j <= m and 0 <= k <= n):
        return False
    cond1 = j == 0 or k == n or A[j - 1] <= B[k]
    cond2 = k == 0 or j == m or B[k - 1] < A[j]
    return cond1 and cond2


def numpy_stable_merge(A, B, Av=None, Bv=None):
    keys = np.concatenate([A, B])
    order = np.argsort(keys, kind="stable")
    if Av is None:
        return keys[order]
    return keys[order], np.concatenate([Av, Bv])[order]


def rank_formula_co_rank(A, B, i):
    """j(i) = #{x : pos(A[x]) < i} with pos(A[x]) = x + #{y : B[y] < A[x]}."""
    posA = np.arange(len(A)) + np.searchsorted(B, A, side="left")
    j = int(np.count_nonzero(posA < i))
    return j, i - j


def corrected_bound(m, n, i):
    """Rounds of Algorithm 1 never exceed ceil(log2(min(m, n, i, m+n-i) + 1))."""
    mn = min(m, n, i, m + n - i)
    return math.ceil(math.log2(mn + 1))


def sorted_arrays(alphabet, max_len):
    for L in range(max_len + 1):
        for combo in itertools.combinations_with_replacement(range(alphabet), L):
            yield np.array(combo, dtype=np.uint32)


# ----------------------------------------------------------------------------
# pin checks, written as plain functions so the mutant test can rerun them


def check_figure1_merge(fig):
    A = np.array(fig["A"]["keys"], dtype=np.uint32)
    B = np.array(fig["B"]["keys"], dtype=np.uint32)
    C = oracle.stable_merge(A, B)
    assert C.tolist() == fig["C"]["keys"]
    # the same with float32 keys (the figure's bar heights)
    Cf = oracle.stable_merge(A.astype(np.float32) / 100, B.astype(np.float32) / 100)
    assert np.array_equal(Cf, np.array(fig["C"]["keys"], dtype=np.float32) / 100)


def check_figure1_stability(fig):
    A = np.array(fig["A"]["keys"], dtype=np.uint32)
    B = np.array(fig["B"]["keys"], dtype=np.uint32)
    Av, Bv = workloads.origin_payloads(A.size, B.size)
    C, Cv = oracle.stable_merge(A, B, Av, Bv)
    assert Cv[fig["alpha"]["C_index"]] == fig["alpha"]["A_index"]
    assert Cv[fig["beta"]["C_index"]] == (1 << 31) + fig["beta"]["B_index"]


def check_figure2_co_rank(fig):
    A = np.array(fig["A"]["keys"], dtype=np.uint32)
    B = np.array(fig["B"]["keys"], dtype=np.uint32)
    i, j, k = fig["co_rank"]["i"], fig["co_rank"]["j"], fig["co_rank"]["k"]
    assert oracle.co_rank_brute(i, A, B) == (j, k)
    assert oracle.co_rank_alg1(i, A, B)[:2] == (j, k)


def check_figure3_trace(fig):
    A = np.array(fig["A"]["keys"], dtype=np.uint32)
    B = np.array(fig["B"]["keys"], dtype=np.uint32)
    tr = fig["alg1_trace"]
    j, k, iters, states = oracle.co_rank_alg1(tr["i"], A, B, trace_cap=64)
    expect = [tuple(s) for s in tr["states_j_k_jlow_klow"]]
    assert states[:len(expect)] == expect
    assert (j, k) == (fig["co_rank"]["j"], fig["co_rank"]["k"])
    assert states[-1][:2] == (j, k)
    assert iters == len(states) - 1


def check_exhaustive(alphabet, max_len):
    """All sorted arrays over `alphabet` letters with m, n <= max_len and all
    ranks: brute force and Algorithm 1 return the unique Lemma 1 pair, Alg. 1
    within the corrected round bound, and the merge equals numpy's stable
    argsort of the concatenation."""
    arrays = list(sorted_arrays(alphabet, max_len))
    cases = 0
    for A in arrays:
        for B in arrays:
            m, n = len(A), len(B)
            assert np.array_equal(oracle.stable_merge(A, B), numpy_stable_merge(A, B))
            for i in range(m + n + 1):
                sat = [j for j in range(max(0, i - n), min(i, m) + 1)
                       if lemma1_holds(A, B, i, j)]
                assert len(sat) == 1, (A, B, i, sat)
                jb, kb = oracle.co_rank_brute(i, A, B)
                assert (jb, kb) == (sat[0], i - sat[0])
                ja, ka, it = oracle.co_rank_alg1(i, A, B)
                assert (ja, ka) == (jb, kb)
                assert it <= corrected_bound(m, n, i)
                cases += 1
    return cases


def check_closed_forms():
    for dtype in (np.uint32, np.uint64, np.float32):
        for m, n in ((37, 53), (64, 64), (1, 0), (0, 5), (33, 1)):
            d = workloads.structured("all_equal", m, n, dtype)
            C, Cv = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
            assert np.array_equal(Cv, np.concatenate([d["Av"], d["Bv"]]))
            d2 = workloads.structured("a_below_b", m, n, dtype)
            C2 = oracle.stable_merge(d2["A"], d2["B"])
            assert np.array_equal(C2, np.arange(m + n).astype(dtype))
            for i in range(m + n + 1):
                assert oracle.co_rank_brute(i, d["A"], d["B"]) == (min(i, m), i - min(i, m))
                assert oracle.co_rank_alg1(i, d["A"], d["B"])[:2] == (min(i, m), i - min(i, m))
                assert oracle.co_rank_alg1(i, d2["A"], d2["B"])[:2] == (min(i, m), i - min(i, m))
        for m in (1, 2, 31, 64):
            d = workloads.structured("interleaved", m, m, dtype)
            C = oracle.stable_merge(d["A"], d["B"])
            assert np.array_equal(C, np.arange(2 * m).astype(dtype))
            for i in range(2 * m + 1):
                j = (i + 1) // 2
                assert oracle.co_rank_brute(i, d["A"], d["B"]) == (j, i - j)
                assert oracle.co_rank_alg1(i, d["A"], d["B"])[:2] == (j, i - j)


def check_random_vs_numpy(seed=7):
    rng = np.random.default_rng(seed)
    for dtype in (np.uint32, np.uint64, np.float32):
        for m, n, hi in ((1000, 3000, 50), (2048, 2048, 2), (777, 5, 1000), (0, 9, 3)):
            if dtype == np.float32:
                A = np.sort(rng.integers(0, hi, m).astype(np.float32) - hi / 2)
                B = np.sort(rng.integers(0, hi, n).astype(np.float32) - hi / 2)
            else:
                A = np.sort(rng.integers(0, hi, m).astype(dtype))
                B = np.sort(rng.integers(0, hi, n).astype(dtype))
            Av, Bv = workloads.origin_payloads(m, n)
            C, Cv = oracle.stable_merge(A, B, Av, Bv)
            Ce, Cve = numpy_stable_merge(A, B, Av, Bv)
            assert np.array_equal(C.view(np.uint8), Ce.view(np.uint8))
            assert np.array_equal(Cv, Cve)
            for i in sorted(set(rng.integers(0, m + n + 1, 25).tolist()) | {0, m + n}):
                ref = rank_formula_co_rank(A, B, i)
                assert oracle.co_rank_brute(i, A, B) == ref
                assert oracle.co_rank_alg1(i, A, B)[:2] == ref


def check_segmented(seed=11):
    d = workloads.segmented(seed=seed, num_seg=300, max_side=40, key_high=8, min_side=0)
    A, B, a_off, b_off = d["A"], d["B"], d["a_off"], d["b_off"]
    C, Cv = oracle.stable_merge_segmented(A, a_off, B, b_off, d["Av"], d["Bv"])
    # per segment against numpy
    for s in range(a_off.size - 1):
        a0, a1, b0, b1 = int(a_off[s]), int(a_off[s + 1]), int(b_off[s]), int(b_off[s + 1])
        ek, ev = numpy_stable_merge(A[a0:a1], B[b0:b1], d["Av"][a0:a1], d["Bv"][b0:b1])
        assert np.array_equal(C[a0 + b0:a1 + b1], ek)
        assert np.array_equal(Cv[a0 + b0:a1 + b1], ev)
    # the whole batch is one stable merge under the (segment, key) order
    segA = np.repeat(np.arange(a_off.size - 1), np.diff(a_off).astype(np.int64))
    segB = np.repeat(np.arange(b_off.size - 1), np.diff(b_off).astype(np.int64))
    seg = np.concatenate([segA, segB])
    keys = np.concatenate([A, B])
    order = np.lexsort((np.arange(keys.size), keys, seg))
    assert np.array_equal(C, keys[order])
    assert np.array_equal(Cv, np.concatenate([d["Av"], d["Bv"]])[order])


PIN_CHECKS = [check_figure1_merge, check_figure1_stability, check_figure2_co_rank,
              check_figure3_trace, check_closed_forms, check_random_vs_numpy,
              check_segmented]


# ----------------------------------------------------------------------------
# tests


def test_figure1_merge(figure):
    check_figure1_merge(figure)


def test_figure1_stability(figure):
    check_figure1_stability(figure)


def test_figure2_co_rank(figure):
    check_figure2_co_rank(figure)


def test_figure3_trace(figure):
    check_figure3_trace(figure)


def test_exhaustive_three_letters():
    assert check_exhaustive(3, 6) > 50_000


def test_exhaustive_four_letters():
    assert check_exhaustive(4, 4) > 20_000


def test_closed_forms():
    check_closed_forms()


def test_random_vs_numpy():
    check_random_vs_numpy()


def test_segmented():
    check_segmented()


def test_float_signed_zero_ties():
    """-0.0 == +0.0 under IEEE comparison: the tie rule keeps A's first and
    the bit patterns travel unchanged."""
    A = np.array([-0.0, 0.0, 1.0], dtype=np.float32)
    B = np.array([0.0, -0.0, 1.0], dtype=np.float32)
    C, Cv = oracle.stable_merge(A, B, *workloads.origin_payloads(3, 3))
    assert Cv.tolist() == [0, 1, 1 << 31, (1 << 31) + 1, 2, (1 << 31) + 2]
    assert np.signbit(C).tolist() == [True, False, False, True, False, False]
    assert oracle.co_rank_alg1(2, A, B)[:2] == (2, 0)
    assert oracle.co_rank_brute(2, B, A) == (2, 0)


def test_paper_iteration_bound_is_off_by_one():
    """Proposition 1 states at most ceil(log2 min(m, n, i, m+n-i)) rounds; with
    m = n = i = 1 that is 0, yet one round is needed (reading recorded in the
    design notes: the bound used in tests is ceil(log2(min + 1)))."""
    A = np.array([1], dtype=np.uint32)
    B = np.array([0], dtype=np.uint32)
    j, k, iters = oracle.co_rank_alg1(1, A, B)
    assert (j, k) == (0, 1)
    assert iters == 1
    assert math.ceil(math.log2(min(1, 1, 1, 1))) == 0
    assert iters <= corrected_bound(1, 1, 1)


def test_origin_payload_encodes_stability():
    """With origin payloads, a merge is stable iff (key, payload) pairs of the
    output are strictly increasing; a deliberately unstable order fails."""
    d = workloads.dup16(m=3000, n=2000, high=40)
    C, Cv = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
    pairs = C.astype(np.uint64) << np.uint64(32) | Cv.astype(np.uint64)
    assert np.all(np.diff(pairs.astype(np.int64)) > 0)
    # B before A on ties is sorted by key but not stable: the check catches it
    keys = np.concatenate([d["B"], d["A"]])
    order = np.argsort(keys, kind="stable")
    bad_v = np.concatenate([d["Bv"], d["Av"]])[order]
    bad = keys[order].astype(np.uint64) << np.uint64(32) | bad_v.astype(np.uint64)
    assert not np.all(np.diff(bad.astype(np.int64)) > 0)


@pytest.mark.parametrize("m", [1, 3, 11, 1001, 65537])
def test_pair_duplicates_closed_form(m):
    """Keys A[x] = x >> 1 and B[y] = y >> 1 (each value twice; m = n odd, so
    the last value once on each side), payloads x and y.  Ties go to A first
    (Section 2's stable merge), so value v's two A copies precede its two B
    copies: C[p] = p >> 2 and C_val[p] = 2 (p >> 2) + (p & 1) for p < N - 2,
    then A's last element, then B's.  The GPU test past 2^32 outputs uses
    this closed form."""
    n = m
    A = (np.arange(m) >> 1).astype(np.uint32)
    B = (np.arange(n) >> 1).astype(np.uint32)
    Av = np.arange(m, dtype=np.uint32)
    Bv = np.arange(n, dtype=np.uint32)
    C, Cv = oracle.stable_merge(A, B, Av, Bv)
    N = m + n
    p = np.arange(N, dtype=np.int64)
    ek, ev = p >> 2, 2 * (p >> 2) + (p & 1)
    ek[N - 2], ev[N - 2] = (m - 1) >> 1, m - 1
    ek[N - 1], ev[N - 1] = (n - 1) >> 1, n - 1
    assert np.array_equal(C, ek.astype(np.uint32))
    assert np.array_equal(Cv, ev.astype(np.uint32))
