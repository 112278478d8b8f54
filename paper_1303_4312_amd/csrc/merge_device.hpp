// Device-side building blocks of the co-rank merge (gfx950, wave64).
//
// co_rank_alg1 is Algorithm 1 of Section 2 (Siebert and Traeff,
// arXiv:1303.4312); co_rank_bisect finds the same pair by plain bisection on
// the first Lemma 1 condition.  Both return the unique A co-rank j of rank i
// (Lemma 1); the B co-rank is i - j.  The block merge follows Algorithm 2 of
// Section 3 at two levels: workgroups take equal output blocks whose ends are
// co-ranked in global memory, and threads take equal runs of E outputs whose
// starts are co-ranked inside the block's windows held in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "order.hpp"

namespace cm {

// Non-temporal store of one key or payload (a Desc key stores its bits).
template <typename X>
__device__ __forceinline__ void store_nt(X v, X* p) {
  if constexpr (is_desc<X>::value)
    __builtin_nontemporal_store(v.v, &p->v);
  else
    __builtin_nontemporal_store(v, p);
}

enum SearchMode : int { kSearchAlg1 = 0, kSearchBisect = 1 };

// Algorithm 1 (Section 2).  State j + k = i with lower bounds j_low, k_low.
// The four keys a round may look at are fetched together, each only when its
// index guard holds (the paper's conditional and), so positions -1, m and n
// are never read.  Reading all four at once costs one memory round trip per
// round: A[j-1], A[j] and B[k-1], B[k] are neighbours.
// k_low is left unset by the paper; it is assigned in the first round before
// any read (only the first condition can fail there), and starts at 0 here.
// On sorted input a violated condition always has a nonzero step (the
// co-rank lies strictly inside the interval being halved).  The zero-step
// exits only matter for unsorted input, outside the paper's precondition:
// there they keep the loop finite (the result is then meaningless but lies
// in [max(0, i - n), min(i, m)]).
template <typename K, typename I, typename RA, typename RB>
__device__ __forceinline__ I co_rank_alg1(I i, RA A, I m, RB B, I n) {
  I j = i < m ? i : m;
  I k = i - j;
  I j_low = i > n ? i - n : I(0);
  I k_low = 0;
  while (true) {
    const bool g1 = j > 0 && k < n;  // guards of the first condition
    const bool g2 = k > 0 && j < m;  // guards of the second condition
    K a_prev{}, b_here{}, b_prev{}, a_here{};
    if (g1) {
      a_prev = A(j - 1);
      b_here = B(k);
    }
    if (g2) {
      b_prev = B(k - 1);
      a_here = A(j);
    }
    if (g1 && a_prev > b_here) {  // first condition violated: j too large
      const I d = (j - j_low + 1) >> 1;
      if (d == 0) return j;
      k_low = k;
      j -= d;
      k += d;
    } else if (g2 && b_prev >= a_here) {  // second violated: k too large
      const I d = (k - k_low + 1) >> 1;
      if (d == 0) return j;
      j_low = j;
      j += d;
      k -= d;
    } else {
      return j;
    }
  }
}

// The same pair by bisection: j is the largest value in
// [max(0, i - n), min(i, m)] that is the lower end or satisfies
// A[j-1] <= B[i-j]; that predicate is true then false along the diagonal.
template <typename K, typename I, typename RA, typename RB>
__device__ __forceinline__ I co_rank_bisect(I i, RA A, I m, RB B, I n) {
  I lo = i > n ? i - n : I(0);
  I hi = i < m ? i : m;
  while (lo < hi) {
    const I mid = lo + ((hi - lo + 1) >> 1);  // lo < mid <= hi
    if (A(mid - 1) <= B(i - mid))
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Bisection restricted to [lo, hi], an interval already known to contain the
// co-rank of i (lo >= max(0, i - n), hi <= min(i, m)).
template <typename K, typename I, typename RA, typename RB>
__device__ __forceinline__ I co_rank_bisect_in(I i, RA A, RB B, I lo, I hi) {
  while (lo < hi) {
    const I mid = lo + ((hi - lo + 1) >> 1);
    if (A(mid - 1) <= B(i - mid))
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Co-rank of i by one whole wave (64 lanes): each round the lanes test 64
// evenly spaced candidates of the current interval at once, a ballot finds
// where the first Lemma condition turns false, and the interval shrinks
// 64-fold, so an interval of L candidates takes ceil(log64(L + 1)) rounds of
// one memory round trip each instead of ceil(log2(L + 1)).  Every lane
// returns the result.  All 64 lanes of the wave must call it together.
template <typename K, typename RA, typename RB>
__device__ __forceinline__ uint64_t co_rank_wave64(uint64_t i, RA A, RB B, uint64_t lo, uint64_t hi) {
  const int lane = (int)(threadIdx.x & 63);
  while (lo < hi) {
    const uint64_t L = hi - lo;
    // lo + floor(L * (lane + 1) / 64), nondecreasing in lane, last = hi
    const uint64_t cand = lo + (L >> 6) * (uint64_t)(lane + 1) + (((L & 63) * (uint64_t)(lane + 1)) >> 6);
    const bool p = cand == lo || A(cand - 1) <= B(i - cand);
    const uint64_t mask = __ballot(p);
    const int t = __popcll(mask);  // the true lanes form a prefix
    const uint64_t c_last_true = __shfl(cand, t > 0 ? t - 1 : 0);
    const uint64_t c_first_false = __shfl(cand, t < 64 ? t : 63);
    if (t == 64) return hi;
    hi = c_first_false - 1;
    lo = t > 0 ? c_last_true : lo;
  }
  return lo;
}

// The same search by a group of G lanes (G a power of two dividing 64,
// aligned inside the wave): each round tests G evenly spaced candidates and
// shrinks the interval G-fold.  Fewer probes per round than the whole-wave
// form (less memory traffic), at the price of more rounds.  Every lane of
// the group returns the result; all lanes of the wave must call it together.
template <typename K, int G, typename RA, typename RB>
__device__ __forceinline__ uint64_t co_rank_group(uint64_t i, RA A, RB B, uint64_t lo, uint64_t hi) {
  static_assert(G >= 2 && G <= 64 && (G & (G - 1)) == 0, "group size");
  constexpr int kShift = G == 2 ? 1 : G == 4 ? 2 : G == 8 ? 3 : G == 16 ? 4 : G == 32 ? 5 : 6;
  const int lane = (int)(threadIdx.x & 63);
  const int g = lane & (G - 1);       // position in the group
  const int base = lane - g;          // first lane of the group
  bool live = lo < hi;
  while (__any(live)) {
    uint64_t cand = lo;
    bool p = true;
    if (live) {
      const uint64_t L = hi - lo;
      cand = lo + (L >> kShift) * (uint64_t)(g + 1) + (((L & (G - 1)) * (uint64_t)(g + 1)) >> kShift);
      p = cand == lo || A(cand - 1) <= B(i - cand);
    }
    const uint64_t mask = (__ballot(p) >> base) & (G == 64 ? ~0ull : ((1ull << (G & 63)) - 1));
    const int t = __popcll(mask);  // true lanes form a prefix of the group
    const uint64_t c_last_true = __shfl(cand, base + (t > 0 ? t - 1 : 0));
    const uint64_t c_first_false = __shfl(cand, base + (t < G ? t : G - 1));
    if (live) {
      if (t == G) {
        lo = hi;
      } else {
        hi = c_first_false - 1;
        lo = t > 0 ? c_last_true : lo;
      }
      live = lo < hi;
    }
  }
  return lo;
}

template <typename K, typename I, typename RA, typename RB>
__device__ __forceinline__ I co_rank(int mode, I i, RA A, I m, RB B, I n) {
  return mode == kSearchBisect ? co_rank_bisect<K>(i, A, m, B, n)
                               : co_rank_alg1<K>(i, A, m, B, n);
}

// Length of a block's A window from the co-ranks of its two ends.  With
// sorted input j0 <= j1 <= j0 + len always holds; the clamp (with the
// callers starting the windows at min(j0, j1)) only keeps every access in
// bounds when the precondition is broken.
__device__ __forceinline__ int window_a_len(uint64_t j0, uint64_t j1, int len) {
  return j1 < j0 ? 0 : (int)(j1 - j0 < (uint64_t)len ? j1 - j0 : (uint64_t)len);
}

// Streams the two windows of a block into LDS: s_key[0, a_len) holds
// A[ja, ja + a_len) and s_key[a_len, len) holds B[kb, kb + len - a_len);
// payloads likewise.  Split in a load phase (registers) and an LDS-write
// phase so that a caller can put other loads in flight beside these; every
// thread issues all of its E (2E with payloads) loads before its first LDS
// write.  The loads are unconditional (a slot past the block re-reads its
// first element, len >= 1), so no copy between branches waits on a load in
// flight.  Consecutive lanes read consecutive addresses (one break at a_len).
template <typename K, bool VAL, int NT, int E, typename V = uint32_t>
struct WindowRegs {
  K k[E];
  V v[VAL ? E : 1];
};

template <typename K, bool VAL, int NT, int E, typename V = uint32_t>
__device__ __forceinline__ void load_window_regs(const K* __restrict__ A, const V* __restrict__ Av,
                                                 uint64_t ja, const K* __restrict__ B,
                                                 const V* __restrict__ Bv, uint64_t kb, int a_len,
                                                 int len, WindowRegs<K, VAL, NT, E, V>& w) {
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int x0 = (int)threadIdx.x + r * NT;
    const int x = x0 < len ? x0 : 0;
    const bool from_a = x < a_len;
    const uint64_t g = from_a ? ja + (uint64_t)x : kb + (uint64_t)(x - a_len);
    const K* pk = from_a ? A : B;
    w.k[r] = pk[g];
    if constexpr (VAL) {
      const V* pv = from_a ? Av : Bv;
      w.v[r] = pv[g];
    }
  }
}

template <typename K, bool VAL, int NT, int E, typename V = uint32_t>
__device__ __forceinline__ void write_window_regs(int len, const WindowRegs<K, VAL, NT, E, V>& w, K* s_key,
                                                  V* s_val) {
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int x = (int)threadIdx.x + r * NT;
    if (x < len) {
      s_key[x] = w.k[r];
      if constexpr (VAL) s_val[x] = w.v[r];
    }
  }
}

template <typename K, bool VAL, int NT, int E, typename V = uint32_t>
__device__ __forceinline__ void load_windows(const K* __restrict__ A, const V* __restrict__ Av,
                                             uint64_t ja, const K* __restrict__ B,
                                             const V* __restrict__ Bv, uint64_t kb, int a_len,
                                             int len, K* s_key, V* s_val) {
  WindowRegs<K, VAL, NT, E, V> w;
  load_window_regs<K, VAL, NT, E, V>(A, Av, ja, B, Bv, kb, a_len, len, w);
  write_window_regs<K, VAL, NT, E, V>(len, w, s_key, s_val);
}

// Writes the block's LDS contents (already in output order) to C[i0, i0 + len)
// with lane-contiguous stores.
template <typename K, bool VAL, int NT, int E, typename V = uint32_t>
__device__ __forceinline__ void store_block(K* __restrict__ C, V* __restrict__ Cv, uint64_t i0,
                                            int len, const K* s_key, const V* s_val) {
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int x = (int)threadIdx.x + r * NT;
    if (x < len) {
      store_nt(s_key[x], C + i0 + x);
      if constexpr (VAL) store_nt(s_val[x], Cv + i0 + x);
    }
  }
}

// ---- 16-byte vector paths ---------------------------------------------------

typedef uint32_t vec16 __attribute__((ext_vector_type(4)));  // one 16-byte access

template <typename X>
constexpr int kPerVec = 16 / (int)sizeof(X);

__device__ __forceinline__ bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Vectors that cover the span X[g0, g0 + cnt) (none when cnt == 0).
template <typename X>
__device__ __forceinline__ int span_vectors(uint64_t g0, int cnt) {
  constexpr int V = kPerVec<X>;
  return cnt ? (int)((g0 + (uint64_t)cnt + V - 1) / V - g0 / V) : 0;
}

// Loads vector q of the span starting at g0 of array X (length total, 16-byte
// aligned base) as a whole 16-byte access; the last vector of the array may
// be partial, and its elements past the end are not read (zero).  Elements of
// the vector outside the span are real array elements and land in padding.
template <typename X>
__device__ __forceinline__ vec16 load_span_vec(const X* __restrict__ Xp, uint64_t total, uint64_t g0, int q) {
  constexpr int V = kPerVec<X>;
  const uint64_t first = (g0 / V + (uint64_t)q) * V;
  if (first + V <= total) return __builtin_nontemporal_load((const vec16*)(Xp + first));
  union {
    vec16 v;
    X e[V];
  } u;
  u.v = vec16{0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < V; ++k)
    if (first + k < total) u.e[k] = Xp[first + k];
  return u.v;
}

// The windows X_A[ga, ga + na) and X_B[gb, gb + nb) of one array pair, as
// staged in LDS by 16-byte vectors: element ga + x of the A window lands at
// dst[pa + x] with pa = ga % V, element gb + y of the B window at dst[pb + y]
// with pb = rb + gb % V and rb = roundup(pa + na, V), so every aligned global
// vector maps onto an aligned LDS vector.  dst must hold na + nb + 3 V
// elements.
struct PairSpan {
  int pa, pb, rb, nva, nvb;
};

template <typename X>
__device__ __forceinline__ PairSpan pair_span(uint64_t ga, int na, uint64_t gb, int nb) {
  constexpr int V = kPerVec<X>;
  PairSpan p;
  p.pa = (int)(ga % V);
  p.rb = (p.pa + na + V - 1) / V * V;
  p.pb = p.rb + (int)(gb % V);
  p.nva = span_vectors<X>(ga, na);
  p.nvb = span_vectors<X>(gb, nb);
  return p;
}

// True when a vector of the pair's span runs past the end of its array (the
// array's length is not a multiple of V and the window reaches its end): only
// then must a vector be read element by element.  Uniform over the block.
template <typename X>
__device__ __forceinline__ bool pair_has_partial(uint64_t totA, uint64_t ga, uint64_t totB, uint64_t gb,
                                                 const PairSpan& p) {
  constexpr int V = kPerVec<X>;
  return (p.nva && (ga / V + (uint64_t)p.nva) * V > totA) || (p.nvb && (gb / V + (uint64_t)p.nvb) * V > totB);
}

// Issues this thread's loads of the pair's vectors (R per thread at most)
// into registers; write_pair_vec puts them in LDS.  Split in two so that a
// caller staging keys and payloads issues every load before the first wait.
// FULL (no vector of the span is partial): one 16-byte load per slot with no
// branch; a slot past the span re-reads the span's first vector, so every
// lane issues the same loads and the waits before the LDS writes count them
// exactly.  Otherwise each vector is read through load_span_vec.
template <typename X, int NT, int R, bool FULL>
__device__ __forceinline__ void load_pair_vec(const X* __restrict__ XA, uint64_t totA, uint64_t ga,
                                              const X* __restrict__ XB, uint64_t totB, uint64_t gb,
                                              const PairSpan& p, vec16 (&reg)[R]) {
  constexpr int V = kPerVec<X>;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = (int)threadIdx.x + r * NT;
    if constexpr (FULL) {
      const bool in_a = q < p.nva || (q >= p.nva + p.nvb && p.nva > 0);
      const int v = q < p.nva ? q : (q < p.nva + p.nvb ? q - p.nva : 0);
      const X* src = in_a ? XA + (ga / V + (uint64_t)v) * V : XB + (gb / V + (uint64_t)v) * V;
      reg[r] = __builtin_nontemporal_load((const vec16*)src);
    } else {
      if (q < p.nva)
        reg[r] = load_span_vec(XA, totA, ga, q);
      else if (q < p.nva + p.nvb)
        reg[r] = load_span_vec(XB, totB, gb, q - p.nva);
    }
  }
}

template <typename X, int NT, int R>
__device__ __forceinline__ void write_pair_vec(X* dst, const PairSpan& p, const vec16 (&reg)[R]) {
  constexpr int V = kPerVec<X>;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = (int)threadIdx.x + r * NT;
    if (q < p.nva + p.nvb) *(vec16*)(dst + (q < p.nva ? q * V : p.rb + (q - p.nva) * V)) = reg[r];
  }
}

// Stores dst[0, len) (LDS, output order) to G[i0, i0 + len) with 16-byte
// stores (G + i0 16-byte aligned, dst 16-byte aligned); the tail of fewer
// than V elements element by element.
template <typename X, int NT>
__device__ __forceinline__ void store_span_vec(X* __restrict__ G, uint64_t i0, int len, const X* src) {
  constexpr int V = kPerVec<X>;
  const int nv = len / V;
  for (int q = (int)threadIdx.x; q < nv; q += NT)
    __builtin_nontemporal_store(*(const vec16*)(src + q * V), (vec16*)(G + i0 + (uint64_t)q * V));
  const int x = nv * V + (int)threadIdx.x;
  if (x < len) store_nt(src[x], G + i0 + x);
}

}  // namespace cm
