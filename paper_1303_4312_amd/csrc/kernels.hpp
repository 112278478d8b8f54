// Kernels of the co-rank stable merge for MI355X (gfx950).
//
// Single merge (Sections 2 and 3 of Siebert and Traeff, arXiv:1303.4312):
//   1. block-boundary co-ranks: j_t = co_rank(i_t) for i_t = t * T, either
//      one thread per boundary (k_block_co_rank) or in two levels
//      (k_coarse_co_rank: a whole wave per 64th boundary with a 64-ary
//      search; k_fine_co_rank: bisection between coarse neighbours).  Running
//      the boundary searches as their own pass is the synchronised variant of
//      Algorithm 2 described after Proposition 2: every boundary is searched
//      once and read by the two blocks that share it (the kernel boundary is
//      the synchronisation).
//   2. k_merge_blocks: workgroup t stages A[j_t, j_t+1) and B[k_t, k_t+1)
//      (exactly T elements together, Proposition 2) in LDS; thread q
//      co-ranks its own start q * E inside those windows (the window-local
//      co-rank plus the window offsets is the global co-rank, because the
//      windows are cut at exact co-ranks), merges E outputs sequentially in
//      registers, and the block leaves through an LDS transpose as
//      lane-contiguous non-temporal stores.
// Segmented batch: the same two steps over the concatenation of many
// problems, partitioned as one merge under the order (segment, key).
#pragma once

#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "merge_device.hpp"

namespace cm {

// ---------------------------------------------------------------------------
// kernels

// j_out[t] = A co-rank of rank min(t * tile, m + n), t in [0, num_bounds).
template <typename K>
__global__ __launch_bounds__(256) void k_block_co_rank(const K* __restrict__ A, uint64_t m,
                                                       const K* __restrict__ B, uint64_t n,
                                                       uint64_t tile, uint64_t num_bounds,
                                                       uint64_t* __restrict__ j_out, int search) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= num_bounds) return;
  const uint64_t N = m + n;
  const uint64_t i = std::min(t * tile, N);
  auto ra = [=](uint64_t x) { return A[x]; };
  auto rb = [=](uint64_t x) { return B[x]; };
  j_out[t] = co_rank<K, uint64_t>(search, i, ra, m, rb, n);
}

// Two-level boundary co-ranks.  Coarse pass: a group of G lanes per coarse
// boundary c * stride, G-ary search over the whole diagonal (G = 64: one
// wave per boundary).
template <typename K, int G>
__global__ __launch_bounds__(256) void k_coarse_co_rank(const K* __restrict__ A, uint64_t m,
                                                        const K* __restrict__ B, uint64_t n, uint64_t stride,
                                                        uint64_t num_coarse, uint64_t* __restrict__ jc) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((gid & ~63ull) / G >= num_coarse) return;  // whole waves with no boundary leave
  const uint64_t c = gid / G;
  const bool mine = c < num_coarse;  // groups past the end run along with an empty interval
  const uint64_t N = m + n;
  const uint64_t i = mine ? std::min(c * stride, N) : 0;
  auto ra = [=](uint64_t x) { return A[x]; };
  auto rb = [=](uint64_t x) { return B[x]; };
  const uint64_t lo = i > n ? i - n : 0;
  const uint64_t hi = mine ? std::min(i, m) : lo;
  const uint64_t j = G == 64 ? co_rank_wave64<K>(i, ra, rb, lo, hi) : co_rank_group<K, G>(i, ra, rb, lo, hi);
  if (mine && (gid & (G - 1)) == 0) jc[c] = j;
}

// Fine pass: block boundary t lies between coarse boundaries c = t / G and
// c + 1, so its co-ranks lie between theirs (co-ranks are monotone in the
// rank); bisection runs only over that window.
template <typename K>
__global__ __launch_bounds__(256) void k_fine_co_rank(const K* __restrict__ A, uint64_t m,
                                                      const K* __restrict__ B, uint64_t n, uint64_t tile,
                                                      uint64_t num_bounds, uint32_t G,
                                                      const uint64_t* __restrict__ jc,
                                                      uint64_t* __restrict__ j_out) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= num_bounds) return;
  const uint64_t N = m + n;
  const uint64_t c = t / G;
  if (t % G == 0) {
    j_out[t] = jc[c];
    return;
  }
  const uint64_t i = std::min(t * tile, N);
  const uint64_t i0 = std::min(c * G * tile, N), i1 = std::min((c + 1) * G * tile, N);
  const uint64_t j0 = jc[c], j1 = jc[c + 1];
  const uint64_t k0 = i0 - j0, k1 = i1 - j1;
  uint64_t lo = std::max(i > n ? i - n : 0, j0);
  if (i > k1) lo = std::max(lo, i - k1);
  uint64_t hi = std::min(std::min(i, m), j1);
  hi = std::min(hi, i - std::min(k0, i));
  if (hi < lo) hi = lo;  // only for unsorted input (monotonicity broken)
  auto ra = [=](uint64_t x) { return A[x]; };
  auto rb = [=](uint64_t x) { return B[x]; };
  j_out[t] = co_rank_bisect_in<K>(i, ra, rb, lo, hi);
}

// Arbitrary ranks: j_out[r] = A co-rank of ranks[r], UINT64_MAX if out of range.
// The fine pass with L lanes per boundary (L = 2 or 4): each group searches
// its window L-ary (co_rank_group), ceil(log_{L+1} w) rounds instead of
// ceil(log2 w).  Whole waves run together: groups past the end and coarse
// boundaries take an empty interval.
template <typename K, int L>
__global__ __launch_bounds__(256) void k_fine_co_rank_group(const K* __restrict__ A, uint64_t m,
                                                            const K* __restrict__ B, uint64_t n, uint64_t tile,
                                                            uint64_t num_bounds, uint32_t G,
                                                            const uint64_t* __restrict__ jc,
                                                            uint64_t* __restrict__ j_out) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((gid & ~63ull) / L >= num_bounds) return;  // whole waves with no boundary leave
  const uint64_t t = gid / L;
  const bool mine = t < num_bounds;
  const uint64_t N = m + n;
  const uint64_t c = mine ? t / G : 0;
  const bool coarse = mine && t % G == 0;
  uint64_t lo = 0, hi = 0, i = 0;
  if (mine && !coarse) {
    i = std::min(t * tile, N);
    const uint64_t i0 = std::min(c * G * tile, N), i1 = std::min((c + 1) * G * tile, N);
    const uint64_t j0 = jc[c], j1 = jc[c + 1];
    const uint64_t k0 = i0 - j0, k1 = i1 - j1;
    lo = std::max(i > n ? i - n : 0, j0);
    if (i > k1) lo = std::max(lo, i - k1);
    hi = std::min(std::min(i, m), j1);
    hi = std::min(hi, i - std::min(k0, i));
    if (hi < lo) hi = lo;  // only for unsorted input (monotonicity broken)
  }
  auto ra = [=](uint64_t x) { return A[x]; };
  auto rb = [=](uint64_t x) { return B[x]; };
  const uint64_t j = co_rank_group<K, L>(i, ra, rb, lo, hi);
  if (mine && (gid & (L - 1)) == 0) j_out[t] = coarse ? jc[c] : j;
}

template <typename K>
__global__ __launch_bounds__(256) void k_co_rank_many(const uint64_t* __restrict__ ranks, uint64_t q,
                                                      const K* __restrict__ A, uint64_t m,
                                                      const K* __restrict__ B, uint64_t n,
                                                      uint64_t* __restrict__ j_out, int search) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= q) return;
  const uint64_t i = ranks[r];
  if (i > m + n) {
    j_out[r] = UINT64_MAX;
    return;
  }
  auto ra = [=](uint64_t x) { return A[x]; };
  auto rb = [=](uint64_t x) { return B[x]; };
  j_out[r] = co_rank<K, uint64_t>(search, i, ra, m, rb, n);
}

// Per-thread sequential stable merge of E outputs starting at window
// position (a, b), in registers.  sA / sB are the block's A and B windows in
// LDS (a_len and b_len elements).  Takes A while A has elements left and B
// is exhausted or A's key <= B's key (the tie rule: A first).  ka / kb hold
// the next key of each side; one LDS read refills the side just consumed.
// out_src[e] is the window position the output came from: a for A, ~b for
// B (used to move payloads).  Outputs at or beyond `avail` are not produced.
template <typename K, int E>
__device__ __forceinline__ void merge_run(const K* sA, int a_len, const K* sB, int b_len, int a, int b, int avail,
                                          K (&out_key)[E], int (&out_src)[E]) {
  K ka = a < a_len ? sA[a] : K{};
  K kb = b < b_len ? sB[b] : K{};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e < avail) {
      const bool take_a = (a < a_len) && (b >= b_len || ka <= kb);
      out_key[e] = take_a ? ka : kb;
      out_src[e] = take_a ? a : ~b;
      a += take_a ? 1 : 0;
      b += take_a ? 0 : 1;
      const bool more = take_a ? (a < a_len) : (b < b_len);
      const K next = more ? (take_a ? sA[a] : sB[b]) : K{};
      if (take_a)
        ka = next;
      else
        kb = next;
    }
  }
}

// One block of Algorithm 2: outputs C[i0, i0 + len) from the windows
// A[j0, j1) and B[i0 - j0, ...) (j0, j1 = co-ranks of the block's ends).
// VEC (every base address 16-byte aligned, and i0 a multiple of 4): the
// windows are staged with 16-byte loads (in a layout shifted so global and
// LDS alignment agree) and the block leaves with 16-byte stores; otherwise
// element by element.  s_key / s_val hold T + 16 elements.  Called by every
// thread of the workgroup; ends with the block stored (LDS reusable after a
// barrier).
template <typename K, bool VAL, int NT, int E, bool VEC, typename V = uint32_t>
__device__ __forceinline__ void merge_block(const K* __restrict__ A, const V* __restrict__ Av, uint64_t m,
                                            const K* __restrict__ B, const V* __restrict__ Bv, uint64_t n,
                                            K* __restrict__ C, V* __restrict__ Cv, uint64_t i0, int len,
                                            uint64_t j0, uint64_t j1, int search, K* s_key, V* s_val) {
  // with sorted input j0 <= j1; for unsorted input (co-ranks out of order)
  // starting at the smaller one keeps both windows inside A and B: the B
  // window then ends at i0 + len - j1, which the end's search bounds by n
  j0 = std::min(j0, j1);
  const int a_len = window_a_len(j0, j1, len);
  const int b_len = len - a_len;
  const uint64_t k0 = i0 - j0;
  int pak = 0, pbk = a_len, pav = 0, pbv = a_len;  // window offsets in LDS
  if constexpr (VEC) {
    // the two windows span at most T / V + 4 vectors; keys and payloads are
    // all requested before the first LDS write waits for them
    constexpr int T = NT * E;
    constexpr int RK = (T / kPerVec<K> + 4 + NT - 1) / NT;
    constexpr int RV = VAL ? (T / kPerVec<V> + 4 + NT - 1) / NT : 1;
    const PairSpan sk = pair_span<K>(j0, a_len, k0, b_len);
    const PairSpan sv = pair_span<V>(j0, a_len, k0, b_len);
    auto stage = [&](auto full) {
      constexpr bool FULL = decltype(full)::value;
      vec16 rk[RK], rv[RV];
      load_pair_vec<K, NT, RK, FULL>(A, m, j0, B, n, k0, sk, rk);
      if constexpr (VAL) load_pair_vec<V, NT, RV, FULL>(Av, m, j0, Bv, n, k0, sv, rv);
      write_pair_vec<K, NT, RK>(s_key, sk, rk);
      if constexpr (VAL) write_pair_vec<V, NT, RV>(s_val, sv, rv);
    };
    if (pair_has_partial<K>(m, j0, n, k0, sk) || (VAL && pair_has_partial<V>(m, j0, n, k0, sv)))
      stage(std::false_type{});
    else
      stage(std::true_type{});
    pak = sk.pa;
    pbk = sk.pb;
    pav = sv.pa;
    pbv = sv.pb;
  } else {
    load_windows<K, VAL, NT, E, V>(A, Av, j0, B, Bv, k0, a_len, len, s_key, s_val);
  }
  __syncthreads();

  const int d = std::min((int)threadIdx.x * E, len);
  const K* sA = s_key + pak;
  const K* sB = s_key + pbk;
  auto ra = [=](int x) { return sA[x]; };
  auto rb = [=](int x) { return sB[x]; };
  const int a = co_rank<K, int>(search, d, ra, a_len, rb, b_len);
  K ok[E];
  int os[E];
  const int avail = len - d;
  merge_run<K, E>(sA, a_len, sB, b_len, a, d - a, avail, ok, os);
  V ov[E];
  if constexpr (VAL) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (e < avail) ov[e] = os[e] >= 0 ? s_val[pav + os[e]] : s_val[pbv + ~os[e]];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e < avail) {
      s_key[d + e] = ok[e];
      if constexpr (VAL) s_val[d + e] = ov[e];
    }
  }
  __syncthreads();
  if constexpr (VEC) {
    store_span_vec<K, NT>(C, i0, len, s_key);
    if constexpr (VAL) store_span_vec<V, NT>(Cv, i0, len, s_val);
  } else {
    store_block<K, VAL, NT, E, V>(C, Cv, i0, len, s_key, s_val);
  }
}

// Workgroups are handed to the 8 XCDs of the chip round-robin by index.
// block_order is a bijection of [0, P) that hands each XCD runs of
// neighbouring blocks, which share the cache lines at their window edges,
// so that they run under the same L2.  xcd = 1: workgroup b takes block
// x * q + min(x, r) + b / 8 (x = b % 8, q = P / 8, r = P % 8), one contiguous
// run per XCD, so eight distant address ranges stream at once.  xcd = c >= 2:
// runs of c blocks, the XCDs side by side, so the blocks in flight at any
// time cover one narrow address range (measured faster: see Shape).
__device__ __forceinline__ uint64_t block_order(uint64_t b, uint64_t P, int xcd) {
  if (!xcd) return b;
  if (xcd == 1) {
    const uint64_t x = b & 7, q = P >> 3, r = P & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
  }
  // runs of c = xcd tiles: in each group of 8c tiles, XCD x takes tiles
  // [x c, (x + 1) c); a last partial group keeps workgroup order
  const uint64_t c = (uint64_t)xcd, group = 8 * c, g = b / group;
  if ((g + 1) * group > P) return b;
  const uint64_t w = b - g * group;
  return g * group + (w & 7) * c + (w >> 3);
}

// Block taken by this workgroup at grid-stride step b (b = blockIdx.x + r G
// for a grid of G workgroups).  With one workgroup per block (G = P) that is
// block_order(b); a smaller, persistent grid takes the blocks in rounds of
// G, each full round in block_order over its G blocks (so the XCDs again
// take runs of neighbouring blocks), the last partial round in workgroup
// order.  Either way a bijection of [0, P).
__device__ __forceinline__ uint64_t grid_block(uint64_t b, uint64_t P, int xcd) {
  const uint64_t G = gridDim.x, base = b - blockIdx.x;
  return base + G <= P ? base + block_order(blockIdx.x, G, xcd) : b;
}

template <typename K, bool VAL, int NT, int E, bool VEC, typename V = uint32_t>
__global__ __launch_bounds__(NT) void k_merge_blocks(const K* __restrict__ A, const V* __restrict__ Av,
                                                     uint64_t m, const K* __restrict__ B,
                                                     const V* __restrict__ Bv, uint64_t n,
                                                     K* __restrict__ C, V* __restrict__ Cv,
                                                     const uint64_t* __restrict__ bj, uint64_t num_tiles,
                                                     int search, int xcd) {
  constexpr int T = NT * E;
  __shared__ __attribute__((aligned(16))) K s_key[T + 16];
  __shared__ __attribute__((aligned(16))) V s_val[VAL ? T + 16 : 1];
  const uint64_t N = m + n;
  for (uint64_t b = blockIdx.x; b < num_tiles; b += gridDim.x) {
    const uint64_t t = grid_block(b, num_tiles, xcd);
    const uint64_t i0 = t * (uint64_t)T;
    const int len = (int)std::min((uint64_t)T, N - i0);
    merge_block<K, VAL, NT, E, VEC, V>(A, Av, m, B, Bv, n, C, Cv, i0, len, bj[t], bj[t + 1], search, s_key, s_val);
    if (b + gridDim.x < num_tiles) __syncthreads();
  }
}

// Algorithm 2 as the paper states it, with no separate boundary pass: every
// workgroup co-ranks the two ends of its own block (wave 0 the start, wave 1
// the end, each with the 64-ary wave search over the whole diagonal), then
// merges the block as k_merge_blocks does.  Each inner boundary is searched
// twice, once by each block that shares it; no workspace is read or written.
// Worth it where the launch and the pass cost more than a few extra memory
// round trips per block (small merges).
template <typename K, bool VAL, int NT, int E, bool VEC, typename V = uint32_t>
__global__ __launch_bounds__(NT) void k_merge_blocks_self(const K* __restrict__ A, const V* __restrict__ Av,
                                                          uint64_t m, const K* __restrict__ B,
                                                          const V* __restrict__ Bv, uint64_t n,
                                                          K* __restrict__ C, V* __restrict__ Cv,
                                                          uint64_t num_tiles, int search, int xcd) {
  static_assert(NT >= 128, "two waves search the block ends");
  constexpr int T = NT * E;
  __shared__ __attribute__((aligned(16))) K s_key[T + 16];
  __shared__ __attribute__((aligned(16))) V s_val[VAL ? T + 16 : 1];
  __shared__ uint64_t s_j[2];
  const uint64_t N = m + n;
  const int wave = (int)(threadIdx.x >> 6);
  for (uint64_t b = blockIdx.x; b < num_tiles; b += gridDim.x) {
    const uint64_t t = grid_block(b, num_tiles, xcd);
    const uint64_t i0 = t * (uint64_t)T;
    const int len = (int)std::min((uint64_t)T, N - i0);
    if (wave < 2) {  // wave-uniform
      const uint64_t i = i0 + (wave ? (uint64_t)len : 0);
      auto ra = [=](uint64_t x) { return A[x]; };
      auto rb = [=](uint64_t x) { return B[x]; };
      const uint64_t j = co_rank_wave64<K>(i, ra, rb, i > n ? i - n : 0, std::min(i, m));
      if ((threadIdx.x & 63) == 0) s_j[wave] = j;
    }
    __syncthreads();
    merge_block<K, VAL, NT, E, VEC, V>(A, Av, m, B, Bv, n, C, Cv, i0, len, s_j[0], s_j[1], search, s_key, s_val);
    if (b + gridDim.x < num_tiles) __syncthreads();
  }
}

// ---- Algorithm 2 with one processing element per resident workgroup --------

// First output of block w of P: floor(w * N / P), exactly (no 128-bit product).
__device__ __forceinline__ uint64_t stream_block_start(uint64_t w, uint64_t N, uint64_t P) {
  return (N / P) * w + ((N % P) * w) / P;
}

// J[w] = A co-rank of stream_block_start(w), w in [0, P]; one wave per
// boundary with the 64-ary search.
template <typename K>
__global__ __launch_bounds__(256) void k_stream_co_rank(const K* __restrict__ A, uint64_t m,
                                                        const K* __restrict__ B, uint64_t n, uint32_t P,
                                                        uint64_t* __restrict__ J) {
  const uint64_t w = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w > P) return;  // whole waves leave
  const uint64_t i = stream_block_start(w, m + n, P);
  auto ra = [=](uint64_t x) { return A[x]; };
  auto rb = [=](uint64_t x) { return B[x]; };
  const uint64_t j = co_rank_wave64<K>(i, ra, rb, i > n ? i - n : 0, std::min(i, m));
  if ((threadIdx.x & 63) == 0) J[w] = j;
}

// ---- the classic cross-rank partition (the prior art of Section 1) -----------
//
// h equidistant samples of A and h of B; each sample is ranked in the other
// array by binary search: A[j] has k = #{B < A[j]} elements of B before it
// (equal keys: A first), B[k] has j = #{A <= B[k]} elements of A before it.
// Each sample gives an exact cut (j, k) of the output at i = j + k; sample 0
// of each side is the cut (0, 0), and samples past the end give (m, n).
// Segments between consecutive cuts hold at most ceil(m / h) elements of A
// and ceil(n / h) of B, so their lengths can differ by a factor of two.
template <typename K>
__global__ __launch_bounds__(256) void k_cross_rank_cuts(const K* __restrict__ A, uint64_t m,
                                                         const K* __restrict__ B, uint64_t n, uint32_t h,
                                                         uint64_t* __restrict__ ia, uint64_t* __restrict__ ja,
                                                         uint64_t* __restrict__ ib, uint64_t* __restrict__ jb) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= 2ull * h) return;
  const bool from_a = x < h;
  const uint64_t r = from_a ? x : x - h;
  const uint64_t len = from_a ? m : n;
  const uint64_t step = (len + h - 1) / h;
  const uint64_t pos = r * step;
  uint64_t j, k;
  if (r == 0) {
    j = 0;
    k = 0;
  } else if (pos >= len) {
    j = m;
    k = n;
  } else if (from_a) {
    const K key = A[pos];
    uint64_t lo = 0, hi = n;  // first B index with B[y] >= key
    while (lo < hi) {
      const uint64_t mid = lo + (hi - lo) / 2;
      if (B[mid] < key) lo = mid + 1; else hi = mid;
    }
    j = pos;
    k = lo;
  } else {
    const K key = B[pos];
    uint64_t lo = 0, hi = m;  // first A index with A[y] > key
    while (lo < hi) {
      const uint64_t mid = lo + (hi - lo) / 2;
      if (A[mid] <= key) lo = mid + 1; else hi = mid;
    }
    j = lo;
    k = pos;
  }
  if (from_a) {
    ia[r] = j + k;
    ja[r] = j;
  } else {
    ib[r] = j + k;
    jb[r] = j;
  }
}

// Ring of T slots: slot of position x (x < T) after head h (h < T).
template <int T>
__device__ __forceinline__ int ring_slot(int h, int x) {
  const int s = h + x;
  return s < T ? s : s - T;
}

// Workgroup w merges its whole output block [o_w, o_{w+1}) of Algorithm 2
// (P blocks, sizes differing by at most one) from the windows A[J_w, J_{w+1})
// and B[o_w - J_w, o_{w+1} - J_{w+1}), in steps of T = NT * E outputs.
// Two LDS rings of T slots hold the next min(T, remaining) elements of each
// window.  A step co-ranks every thread's start q * E inside the rings (the
// co-rank of d <= T needs no element past position T of either window),
// merges E outputs per thread, and finds how many A elements the step used
// (a_take: the final A cursor of the thread that produces the step's last
// output).  The step's outputs are then staged in exactly the ring slots it
// consumed (a_take slots of ring A, len - a_take of ring B), stored to C in
// order, and those slots are refilled from global memory with the next
// elements of each window; the refill loads are issued before the stores so
// that both are in flight together.
template <typename K, bool VAL, int NT, int E>
__global__ __launch_bounds__(NT) void k_merge_stream(const K* __restrict__ A, const uint32_t* __restrict__ Av,
                                                     uint64_t m, const K* __restrict__ B,
                                                     const uint32_t* __restrict__ Bv, uint64_t n,
                                                     K* __restrict__ C, uint32_t* __restrict__ Cv,
                                                     const uint64_t* __restrict__ I, const uint64_t* __restrict__ J,
                                                     uint32_t P, int search) {
  constexpr int T = NT * E;
  __shared__ K ra_key[T];
  __shared__ K rb_key[T];
  __shared__ uint32_t ra_val[VAL ? T : 1];
  __shared__ uint32_t rb_val[VAL ? T : 1];
  __shared__ int s_take;
  const uint64_t N = m + n;
  const uint64_t w = blockIdx.x;
  if (w >= P) return;
  // segment w: equal shares, or the starts I gives (any monotone cuts with J)
  uint64_t o = I ? I[w] : stream_block_start(w, N, P);
  const uint64_t o_end = std::max(I ? I[w + 1] : stream_block_start(w + 1, N, P), o);
  uint64_t ja = J[w];
  const uint64_t ja_end = std::max(J[w + 1], ja);  // the max only matters for unsorted input
  uint64_t kb = o - ja;
  const uint64_t kb_end = std::max(o_end - std::min(J[w + 1], o_end), kb);
  int ha = 0, hb = 0;  // ring heads
  int fa = (int)std::min<uint64_t>(T, ja_end - ja);
  int fb = (int)std::min<uint64_t>(T, kb_end - kb);
  // initial fill
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int x = (int)threadIdx.x + r * NT;
    if (x < fa) {
      ra_key[x] = A[ja + x];
      if constexpr (VAL) ra_val[x] = Av[ja + x];
    }
    if (x < fb) {
      rb_key[x] = B[kb + x];
      if constexpr (VAL) rb_val[x] = Bv[kb + x];
    }
  }
  __syncthreads();

  while (o < o_end) {
    // fa + fb >= the step with sorted input; the clamp and the exit only
    // keep unsorted input in bounds and finite
    const int len = (int)std::min<uint64_t>(std::min<uint64_t>(T, o_end - o), (uint64_t)(fa + fb));
    if (len == 0) break;
    const int d = std::min((int)threadIdx.x * E, len);
    const int avail = len - d;
    auto rka = [&](int x) { return ra_key[ring_slot<T>(ha, x)]; };
    auto rkb = [&](int x) { return rb_key[ring_slot<T>(hb, x)]; };
    int a = co_rank<K, int>(search, d, rka, fa, rkb, fb);
    int b = d - a;
    K ok[E];
    int os[E];  // ring slot of each output: slot in A, or T + slot in B
    K ka = a < fa ? rka(a) : K{};
    K kbv = b < fb ? rkb(b) : K{};
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (e < avail) {
        const bool take_a = (a < fa) && (b >= fb || ka <= kbv);
        ok[e] = take_a ? ka : kbv;
        os[e] = take_a ? ring_slot<T>(ha, a) : T + ring_slot<T>(hb, b);
        a += take_a ? 1 : 0;
        b += take_a ? 0 : 1;
        const bool more = take_a ? (a < fa) : (b < fb);
        const K next = more ? (take_a ? rka(a) : rkb(b)) : K{};
        if (take_a)
          ka = next;
        else
          kbv = next;
      }
    }
    if (avail > 0 && avail <= E) s_take = a;  // this thread produced the step's last output
    uint32_t ov[E];
    if constexpr (VAL) {
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (e < avail) ov[e] = os[e] < T ? ra_val[os[e]] : rb_val[os[e] - T];
    }
    __syncthreads();  // every ring read of this step is done; s_take is visible
    const int a_take = s_take;
    const int b_take = len - a_take;
    // stage output x in the x-th consumed slot: A's for x < a_take, then B's
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (e < avail) {
        const int x = d + e;
        if (x < a_take) {
          const int sl = ring_slot<T>(ha, x);
          ra_key[sl] = ok[e];
          if constexpr (VAL) ra_val[sl] = ov[e];
        } else {
          const int sl = ring_slot<T>(hb, x - a_take);
          rb_key[sl] = ok[e];
          if constexpr (VAL) rb_val[sl] = ov[e];
        }
      }
    }
    // refill: after the step ring A must hold min(T, remaining) elements
    // again; the new ones are window positions [fa, a_take + fa_next) of the
    // old head, i.e. [fa - a_take, fa_next) of the new one
    const uint64_t ja_next = ja + (uint64_t)a_take, kb_next = kb + (uint64_t)b_take;
    const int fa_next = (int)std::min<uint64_t>(T, ja_end - ja_next);
    const int fb_next = (int)std::min<uint64_t>(T, kb_end - kb_next);
    const int new_a = a_take + fa_next - fa;  // >= 0
    const int new_b = b_take + fb_next - fb;
    const int ha_next = ring_slot<T>(ha, a_take);
    const int hb_next = ring_slot<T>(hb, b_take);
    K nk[E];
    uint32_t nv[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int x = (int)threadIdx.x + r * NT;
      if (x < new_a) {
        const uint64_t g = ja + fa + x;
        nk[r] = A[g];
        if constexpr (VAL) nv[r] = Av[g];
      } else if (x < new_a + new_b) {
        const uint64_t g = kb + fb + (x - new_a);
        nk[r] = B[g];
        if constexpr (VAL) nv[r] = Bv[g];
      }
    }
    __syncthreads();  // staging complete
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int x = (int)threadIdx.x + r * NT;
      if (x < len) {
        const int sl = x < a_take ? ring_slot<T>(ha, x) : ring_slot<T>(hb, x - a_take);
        const K key = x < a_take ? ra_key[sl] : rb_key[sl];
        store_nt(key, C + o + x);
        if constexpr (VAL) {
          const uint32_t v = x < a_take ? ra_val[sl] : rb_val[sl];
          store_nt(v, Cv + o + x);
        }
      }
    }
    __syncthreads();  // staging read; the consumed slots may be overwritten
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int x = (int)threadIdx.x + r * NT;
      if (x < new_a) {
        const int sl = ring_slot<T>(ha_next, fa - a_take + x);
        ra_key[sl] = nk[r];
        if constexpr (VAL) ra_val[sl] = nv[r];
      } else if (x < new_a + new_b) {
        const int sl = ring_slot<T>(hb_next, fb - b_take + (x - new_a));
        rb_key[sl] = nk[r];
        if constexpr (VAL) rb_val[sl] = nv[r];
      }
    }
    ja = ja_next;
    kb = kb_next;
    ha = ha_next;
    hb = hb_next;
    fa = fa_next;
    fb = fb_next;
    o += (uint64_t)len;
    __syncthreads();  // refill visible to the next step
  }
}

// ---- batch of separately allocated merges ----------------------------------

// One merge of a batch.  Same layout as the C ABI's cm_merge_desc.
struct MergeDesc {
  const void* A;
  const uint32_t* A_val;
  uint64_t m;
  const void* B;
  const uint32_t* B_val;
  uint64_t n;
  void* C;
  uint32_t* C_val;
  uint64_t first_block;  // blocks of merges before this one
};

// Up to kInlineDescs descriptors of a batch travel in the kernel arguments,
// so that a small batch needs no upload before its kernels run.
constexpr uint32_t kInlineDescs = 16;
struct DescPack {
  MergeDesc d[kInlineDescs];
};

// Boundary slots of a batch: merge r (nb_r blocks) owns the nb_r + 1 slots
// [first_block[r] + r, first_block[r] + r + nb_r], one per block end; slot
// s0 + t holds the A co-rank of rank min(t * tile, m + n) of merge r.
// Block g of the batch is block g - first_block[r] of merge r.

// Largest r in [0, count) with fb(r) + r * extra <= x (merges with no
// blocks share first_block with their successor and are skipped).
template <typename FB>
__device__ __forceinline__ uint32_t merge_of(FB fb, uint32_t count, uint64_t x, uint64_t extra) {
  uint32_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo + 1) >> 1);
    if (fb(mid) + mid * extra <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

struct BatchSlot {
  MergeDesc q;
  uint32_t r;   // the merge
  uint64_t s0;  // its first slot
  uint64_t i;   // rank of the slot inside the merge
};

// Slot b: its merge from the prep kernel's table, the descriptor from the
// workspace copy.
__device__ __forceinline__ BatchSlot batch_slot(const MergeDesc* __restrict__ d, const uint32_t* __restrict__ sm,
                                                uint64_t tile, uint64_t b) {
  BatchSlot x;
  x.r = sm[b];
  x.q = d[x.r];
  x.s0 = x.q.first_block + x.r;
  x.i = std::min((b - x.s0) * tile, x.q.m + x.q.n);
  return x;
}

// One-level boundary pass of a batch: one thread per slot, searching the
// whole diagonal of its merge.
template <typename K>
__global__ __launch_bounds__(256) void k_batch_co_rank(const MergeDesc* __restrict__ d,
                                                       const uint32_t* __restrict__ sm, uint64_t tile,
                                                       uint64_t num_bounds, uint64_t* __restrict__ bj, int search) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= num_bounds) return;
  const BatchSlot x = batch_slot(d, sm, tile, b);
  const K* A = (const K*)x.q.A;
  const K* B = (const K*)x.q.B;
  auto ra = [=](uint64_t y) { return A[y]; };
  auto rb = [=](uint64_t y) { return B[y]; };
  bj[b] = co_rank<K, uint64_t>(search, x.i, ra, x.q.m, rb, x.q.n);
}

// Two-level boundary pass of a batch.  Coarse step: every G-th slot of the
// whole batch (slot c * G), whatever merge it falls in, co-ranked over its
// merge's diagonal by a group of L lanes (L-ary search).
template <typename K, int L>
__global__ __launch_bounds__(256) void k_batch_coarse_co_rank(const MergeDesc* __restrict__ d,
                                                              const uint32_t* __restrict__ sm, uint64_t tile,
                                                              uint32_t G, uint64_t num_coarse,
                                                              uint64_t* __restrict__ jc) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((gid & ~63ull) / L >= num_coarse) return;  // whole waves with no coarse slot leave
  const uint64_t c = gid / L;
  const bool mine = c < num_coarse;  // groups past the end run along with an empty interval
  uint64_t i = 0, lo = 0, hi = 0;
  const K* A = nullptr;
  const K* B = nullptr;
  if (mine) {
    const BatchSlot x = batch_slot(d, sm, tile, c * G);
    A = (const K*)x.q.A;
    B = (const K*)x.q.B;
    i = x.i;
    lo = i > x.q.n ? i - x.q.n : 0;
    hi = std::min(i, x.q.m);
  }
  auto ra = [=](uint64_t y) { return A[y]; };
  auto rb = [=](uint64_t y) { return B[y]; };
  const uint64_t j = co_rank_group<K, L>(i, ra, rb, lo, hi);
  if (mine && (gid & (L - 1)) == 0) jc[c] = j;
}

// Fine step: slot b of merge r lies between the coarse slots c * G and
// (c + 1) * G (c = b / G).  Each of them bounds b's co-rank when it belongs
// to the same merge (co-ranks grow with the rank); otherwise the merge's own
// start (rank 0, co-rank 0) or end (rank m + n, co-rank m) does.  Bisection
// then runs only over that window.
template <typename K>
__global__ __launch_bounds__(256) void k_batch_fine_co_rank(const MergeDesc* __restrict__ d,
                                                            const uint32_t* __restrict__ sm, uint64_t tile,
                                                            uint64_t num_bounds, uint32_t G,
                                                            const uint64_t* __restrict__ jc,
                                                            uint64_t* __restrict__ bj) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= num_bounds) return;
  const uint64_t c = b / G;
  if (b == c * G) {
    bj[b] = jc[c];
    return;
  }
  const BatchSlot x = batch_slot(d, sm, tile, b);
  const uint64_t m = x.q.m, n = x.q.n, N = m + n, i = x.i;
  const uint64_t nb = (N + tile - 1) / tile;  // the merge's slots are s0 .. s0 + nb
  uint64_t i0 = 0, j0 = 0, i1 = N, j1 = m;
  if (c * G >= x.s0) {
    i0 = std::min((c * G - x.s0) * tile, N);
    j0 = jc[c];
  }
  if ((c + 1) * G <= x.s0 + nb) {
    i1 = std::min(((c + 1) * G - x.s0) * tile, N);
    j1 = jc[c + 1];
  }
  const uint64_t k0 = i0 - j0, k1 = i1 - j1;
  uint64_t lo = std::max(i > n ? i - n : 0, j0);
  if (i > k1) lo = std::max(lo, i - k1);
  uint64_t hi = std::min(std::min(i, m), j1);
  hi = std::min(hi, i - std::min(k0, i));
  if (hi < lo) hi = lo;  // only for unsorted input (monotonicity broken)
  const K* A = (const K*)x.q.A;
  const K* B = (const K*)x.q.B;
  auto ra = [=](uint64_t y) { return A[y]; };
  auto rb = [=](uint64_t y) { return B[y]; };
  bj[b] = co_rank_bisect_in<K>(i, ra, rb, lo, hi);
}

// Waves 0 and 1 of the workgroup co-rank the start i0 and the end i0 + len
// of a block of merge q over its whole diagonal (64-ary wave search) into
// s_j[0], s_j[1]; the workgroup then waits for both.
template <typename K>
__device__ __forceinline__ void block_ends(const MergeDesc& q, uint64_t i0, int len, uint64_t* s_j) {
  const int wave = (int)(threadIdx.x >> 6);
  if (wave < 2) {  // wave-uniform
    const uint64_t i = i0 + (wave ? (uint64_t)len : 0);
    const K* A = (const K*)q.A;
    const K* B = (const K*)q.B;
    auto ra = [=](uint64_t y) { return A[y]; };
    auto rb = [=](uint64_t y) { return B[y]; };
    const uint64_t j = co_rank_wave64<K>(i, ra, rb, i > q.n ? i - q.n : 0, std::min(i, q.m));
    if ((threadIdx.x & 63) == 0) s_j[wave] = j;
  }
  __syncthreads();
}

// Block merge of a batch after the prep kernel: block g's merge comes from
// bm, its descriptor from d (device memory).  Its end co-ranks come from
// the boundary pass (bj), or, with SELF (no pass: Algorithm 2 as the paper
// states it), the block finds them itself (block_ends).
template <typename K, bool VAL, int NT, int E, bool VEC, bool SELF>
__global__ __launch_bounds__(NT) void k_batch_merge_blocks(const MergeDesc* __restrict__ d,
                                                           const uint32_t* __restrict__ bm,
                                                           const uint64_t* __restrict__ bj, uint64_t num_tiles,
                                                           int search, int xcd) {
  static_assert(NT >= 128, "two waves search the block ends");
  constexpr int T = NT * E;
  __shared__ __attribute__((aligned(16))) K s_key[T + 16];
  __shared__ __attribute__((aligned(16))) uint32_t s_val[VAL ? T + 16 : 1];
  __shared__ uint64_t s_j[2];
  for (uint64_t b = blockIdx.x; b < num_tiles; b += gridDim.x) {
    const uint64_t g = grid_block(b, num_tiles, xcd);
    const uint32_t r = bm[g];
    const MergeDesc q = d[r];
    const uint64_t t = g - q.first_block;
    const uint64_t i0 = t * (uint64_t)T;
    const int len = (int)std::min((uint64_t)T, q.m + q.n - i0);
    uint64_t j0, j1;
    if constexpr (SELF) {
      block_ends<K>(q, i0, len, s_j);
      j0 = s_j[0];
      j1 = s_j[1];
    } else {
      j0 = bj[g + r];  // block g starts at slot g + r
      j1 = bj[g + r + 1];
    }
    merge_block<K, VAL, NT, E, VEC>((const K*)q.A, q.A_val, q.m, (const K*)q.B, q.B_val, q.n, (K*)q.C, q.C_val, i0,
                                    len, j0, j1, search, s_key, s_val);
    if (b + gridDim.x < num_tiles) __syncthreads();
  }
}

// The single-launch form for a small batch: the descriptors come in the
// kernel arguments, the block finds its merge by searching them and
// co-ranks its own ends (no prep, no pass).
template <typename K, bool VAL, int NT, int E, bool VEC>
__global__ __launch_bounds__(NT) void k_batch_merge_blocks_args(DescPack pk, uint32_t count, uint64_t num_tiles,
                                                                int search, int xcd) {
  static_assert(NT >= 128, "two waves search the block ends");
  constexpr int T = NT * E;
  __shared__ __attribute__((aligned(16))) K s_key[T + 16];
  __shared__ __attribute__((aligned(16))) uint32_t s_val[VAL ? T + 16 : 1];
  __shared__ uint64_t s_j[2];
  auto fb = [&](uint32_t r) { return pk.d[r < kInlineDescs ? r : 0].first_block; };
  for (uint64_t b = blockIdx.x; b < num_tiles; b += gridDim.x) {
    const uint64_t g = grid_block(b, num_tiles, xcd);
    const uint32_t r = merge_of(fb, count, g, 0);
    const MergeDesc q = pk.d[r < kInlineDescs ? r : 0];
    const uint64_t t = g - q.first_block;
    const uint64_t i0 = t * (uint64_t)T;
    const int len = (int)std::min((uint64_t)T, q.m + q.n - i0);
    block_ends<K>(q, i0, len, s_j);
    merge_block<K, VAL, NT, E, VEC>((const K*)q.A, q.A_val, q.m, (const K*)q.B, q.B_val, q.n, (K*)q.C, q.C_val, i0,
                                    len, s_j[0], s_j[1], search, s_key, s_val);
    if (b + gridDim.x < num_tiles) __syncthreads();
  }
}

// ---- segmented batch -------------------------------------------------------

// Largest s in [lo, hi] with a_off[s] + b_off[s] <= g (the segment holding
// output position g; empty segments before it are skipped).
__device__ __forceinline__ uint32_t seg_of(const uint64_t* __restrict__ a_off,
                                           const uint64_t* __restrict__ b_off, uint32_t lo, uint32_t hi,
                                           uint64_t g) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo + 1) >> 1);
    if (a_off[mid] + b_off[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// The same search over offset accessors (LDS table or global arrays).
template <typename AO, typename BO>
__device__ __forceinline__ uint32_t seg_of_at(AO ao, BO bo, uint32_t lo, uint32_t hi, uint64_t g) {
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo + 1) >> 1);
    if (ao(mid) + bo(mid) <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Block boundaries of the batch seen as one merge under (segment, key):
// boundary i lies in segment s; its co-rank is a_off[s] plus the co-rank of
// i - c_off[s] inside segment s (Algorithm 1 on that segment's arrays).
template <typename K>
__global__ __launch_bounds__(256) void k_seg_block_co_rank(const K* __restrict__ A,
                                                           const uint64_t* __restrict__ a_off,
                                                           const K* __restrict__ B,
                                                           const uint64_t* __restrict__ b_off, uint32_t S,
                                                           uint64_t N, uint64_t tile, uint64_t num_bounds,
                                                           uint64_t* __restrict__ j_out,
                                                           uint32_t* __restrict__ s_out,
                                                           const uint32_t* __restrict__ flag, int search) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= num_bounds || *flag) return;
  const uint64_t i = std::min(t * tile, N);
  const uint32_t s = seg_of(a_off, b_off, 0, S - 1, i);
  const uint64_t a0 = a_off[s], b0 = b_off[s];
  const uint64_t ms = a_off[s + 1] - a0, ns = b_off[s + 1] - b0;
  const uint64_t d = i - a0 - b0;
  const K* As = A + a0;
  const K* Bs = B + b0;
  auto ra = [=](uint64_t x) { return As[x]; };
  auto rb = [=](uint64_t x) { return Bs[x]; };
  j_out[t] = a0 + co_rank<K, uint64_t>(search, d, ra, ms, rb, ns);
  s_out[t] = s;
}

// Two-level form for the batch: block boundary t lies between coarse
// boundaries c = t / G and c + 1 (computed by k_seg_block_co_rank with a
// G-times longer stride into jc, sc).  Its segment lies in [sc[c], sc[c+1]]
// and, inside that segment, its co-ranks lie between the coarse ones (the
// batch is one merge under (segment, key), so co-ranks are monotone), so
// both searches run over short ranges.
template <typename K>
__global__ __launch_bounds__(256) void k_seg_fine_co_rank(const K* __restrict__ A, const uint64_t* __restrict__ a_off,
                                                          const K* __restrict__ B, const uint64_t* __restrict__ b_off,
                                                          uint64_t N, uint64_t tile, uint64_t num_bounds, uint32_t G,
                                                          const uint64_t* __restrict__ jc,
                                                          const uint32_t* __restrict__ sc,
                                                          uint64_t* __restrict__ j_out, uint32_t* __restrict__ s_out,
                                                          const uint32_t* __restrict__ flag) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= num_bounds || *flag) return;
  const uint64_t c = t / G;
  if (t % G == 0) {
    j_out[t] = jc[c];
    s_out[t] = sc[c];
    return;
  }
  const uint64_t i = std::min(t * tile, N);
  const uint64_t i0 = std::min(c * G * tile, N), i1 = std::min((c + 1) * G * tile, N);
  const uint64_t J0 = jc[c], J1 = jc[c + 1];
  const uint64_t K0 = i0 - J0, K1 = i1 - J1;
  const uint32_t s = seg_of(a_off, b_off, sc[c], std::max(sc[c], sc[c + 1]), i);
  const uint64_t a0 = a_off[s], b0 = b_off[s];
  const uint64_t ms = a_off[s + 1] - a0, ns = b_off[s + 1] - b0;
  const uint64_t d = i - a0 - b0;
  // local j in [max(0, d - ns), min(d, ms)], also J0 <= a0 + j <= J1 and
  // K0 <= b0 + d - j <= K1
  uint64_t lo = d > ns ? d - ns : 0;
  if (J0 > a0) lo = std::max(lo, J0 - a0);
  if (b0 + d > K1) lo = std::max(lo, b0 + d - K1);
  uint64_t hi = std::min(d, ms);
  hi = std::min(hi, J1 > a0 ? J1 - a0 : 0);
  hi = std::min(hi, b0 + d > K0 ? b0 + d - K0 : 0);
  if (hi < lo) hi = lo;  // only for unsorted input
  const K* As = A + a0;
  const K* Bs = B + b0;
  auto ra = [=](uint64_t x) { return As[x]; };
  auto rb = [=](uint64_t x) { return Bs[x]; };
  j_out[t] = a0 + co_rank_bisect_in<K>(d, ra, rb, lo, hi);
  s_out[t] = s;
}

// Segmented merge run: like merge_run, but the run may cross segment ends.
// s is the segment of the run's first output; a_end / b_end are the window
// positions where segment s ends on each side (they may lie beyond the
// window).  When both sides of the current segment are used up the run moves
// on to the next non-empty segment.
template <typename K, int E, typename AO, typename BO>
__device__ __forceinline__ void merge_run_seg(const K* s_key, int a_len, int len, int a, int b, int avail, AO ao,
                                              BO bo, uint32_t S, uint32_t s, uint64_t j0, uint64_t k0,
                                              K (&out_key)[E], int (&out_src)[E]) {
  const int b_len = len - a_len;
  auto clamp_end = [](uint64_t end, uint64_t base) -> int {
    return (int)std::min(end - base, (uint64_t)INT_MAX);
  };
  int a_end = clamp_end(ao(s + 1), j0);
  int b_end = clamp_end(bo(s + 1), k0);
  K ka = a < a_len ? s_key[a] : K{};
  K kb = b < b_len ? s_key[a_len + b] : K{};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e < avail) {
      while (a == a_end && b == b_end && s + 1 < S) {
        ++s;
        a_end = clamp_end(ao(s + 1), j0);
        b_end = clamp_end(bo(s + 1), k0);
      }
      const bool has_a = a < std::min(a_end, a_len);
      const bool has_b = b < std::min(b_end, b_len);
      const bool take_a = has_a && (!has_b || ka <= kb);
      out_key[e] = take_a ? ka : kb;
      out_src[e] = take_a ? a : a_len + b;
      a += take_a ? 1 : 0;
      b += take_a ? 0 : 1;
      const bool more = take_a ? (a < a_len) : (b < b_len);
      const int pos = take_a ? a : a_len + b;
      const K next = more ? s_key[pos] : K{};
      if (take_a)
        ka = next;
      else
        kb = next;
    }
  }
}

// Offsets of the segments a block's outputs can lie in (s_first..s_last, so
// entries s_first..s_last + 1) are staged in LDS when there are at most this
// many segments; blocks over more (tiny) segments read them from HBM.
constexpr uint32_t kSegTable = 256;

// VST: C (and C_val) 16-byte aligned: the block leaves with 16-byte stores.
template <typename K, bool VAL, int NT, int E, bool VST>
__global__ __launch_bounds__(NT) void k_seg_merge_blocks(
    const K* __restrict__ A, const uint32_t* __restrict__ Av, const uint64_t* __restrict__ a_off,
    const K* __restrict__ B, const uint32_t* __restrict__ Bv, const uint64_t* __restrict__ b_off, uint32_t S,
    uint64_t N, K* __restrict__ C, uint32_t* __restrict__ Cv, const uint64_t* __restrict__ bj,
    const uint32_t* __restrict__ bs, uint64_t num_tiles, const uint32_t* __restrict__ flag, int search) {
  constexpr int T = NT * E;
  __shared__ __attribute__((aligned(16))) K s_key[T];
  __shared__ __attribute__((aligned(16))) uint32_t s_val[VAL ? T : 1];
  __shared__ uint64_t s_aoff[kSegTable + 1], s_boff[kSegTable + 1];
  if (*flag) return;
  for (uint64_t t = blockIdx.x; t < num_tiles; t += gridDim.x) {
    const uint64_t i0 = t * (uint64_t)T;
    const int len = (int)std::min((uint64_t)T, N - i0);
    // the smaller of the two co-ranks starts the windows: equal to bj[t] for
    // sorted segments, inside A and B for unsorted ones (as in merge_block)
    const uint64_t j0 = std::min(bj[t], bj[t + 1]);
    const uint64_t k0 = i0 - j0;
    const int a_len = window_a_len(j0, bj[t + 1], len);
    const int b_len = len - a_len;
    const uint64_t j1 = j0 + (uint64_t)a_len;
    const uint32_t s_first = bs[t];
    const uint32_t s_last = bs[t + 1];
    const uint32_t entries = s_last - s_first + 2;  // s_last + 1 <= S: inside a_off / b_off
    const bool table = entries <= kSegTable + 1;     // block-uniform
    // the table's loads and the windows' loads are all issued before the
    // first LDS write waits for any of them (entries s_first .. s_last + 1
    // exist; a slot past them re-reads entry s_first)
    constexpr int RT = (kSegTable + 1 + NT - 1) / NT;
    uint64_t ta[RT], tb[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const uint32_t x0 = threadIdx.x + (uint32_t)(r * NT);
      const uint32_t x = x0 < entries ? x0 : 0;
      ta[r] = a_off[s_first + x];
      tb[r] = b_off[s_first + x];
    }
    WindowRegs<K, VAL, NT, E> w;
    load_window_regs<K, VAL, NT, E>(A, Av, j0, B, Bv, k0, a_len, len, w);
    if (table) {
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const uint32_t x = threadIdx.x + (uint32_t)(r * NT);
        if (x < entries) {
          s_aoff[x] = ta[r];
          s_boff[x] = tb[r];
        }
      }
    }
    write_window_regs<K, VAL, NT, E>(len, w, s_key, s_val);
    __syncthreads();

    // offsets of segment s (s >= s_first): from the table when it holds s
    auto ao = [&](uint32_t q) -> uint64_t {
      const uint32_t x = q - s_first;
      return table && x < entries ? s_aoff[x] : a_off[q];
    };
    auto bo = [&](uint32_t q) -> uint64_t {
      const uint32_t x = q - s_first;
      return table && x < entries ? s_boff[x] : b_off[q];
    };
    const int d = std::min((int)threadIdx.x * E, len);
    const int avail = len - d;
    K ok[E];
    int os[E];
    if (avail > 0) {
      const uint64_t g = i0 + (uint64_t)d;
      const uint32_t s = seg_of_at(ao, bo, s_first, s_last, g);
      const uint64_t sa0 = ao(s), sa1 = ao(s + 1);
      const uint64_t sb0 = bo(s), sb1 = bo(s + 1);
      // the part of segment s inside this block, in window coordinates; its
      // ends are exact co-rank cuts (block ends or segment ends)
      // (clamped into the windows so that unsorted input cannot lead outside)
      const int wa0 = (int)std::min(std::max(sa0, j0) - j0, (uint64_t)a_len);
      const int wa1 = std::max(wa0, (int)std::min(std::max(std::min(sa1, j1), j0) - j0, (uint64_t)a_len));
      const int wb0 = (int)std::min(std::max(sb0, k0) - k0, (uint64_t)b_len);
      const int wb1 = std::max(wb0, (int)std::min(std::max(std::min(sb1, k0 + (uint64_t)b_len), k0) - k0,
                                                  (uint64_t)b_len));
      const int64_t dd64 = (int64_t)(g - j0 - k0) - wa0 - wb0;
      const int dd = (int)std::min<int64_t>(std::max<int64_t>(dd64, 0), (wa1 - wa0) + (wb1 - wb0));
      const K* sA = s_key + wa0;
      const K* sB = s_key + a_len + wb0;
      auto ra = [=](int x) { return sA[x]; };
      auto rb = [=](int x) { return sB[x]; };
      const int ja = co_rank<K, int>(search, dd, ra, wa1 - wa0, rb, wb1 - wb0);
      merge_run_seg<K, E>(s_key, a_len, len, wa0 + ja, wb0 + (dd - ja), avail, ao, bo, S, s, j0, k0, ok, os);
    }
    uint32_t ov[E];
    if constexpr (VAL) {
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (e < avail) ov[e] = s_val[os[e]];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (e < avail) {
        s_key[d + e] = ok[e];
        if constexpr (VAL) s_val[d + e] = ov[e];
      }
    }
    __syncthreads();
    if constexpr (VST) {
      store_span_vec<K, NT>(C, i0, len, s_key);
      if constexpr (VAL) store_span_vec<uint32_t, NT>(Cv, i0, len, s_val);
    } else {
      store_block<K, VAL, NT, E>(C, Cv, i0, len, s_key, s_val);
    }
    if (t + gridDim.x < num_tiles) __syncthreads();
  }
}

// flag |= 1 if some X[x-1] > X[x].
template <typename K>
__global__ __launch_bounds__(256) void k_check_sorted(const K* __restrict__ X, uint64_t len,
                                                      uint32_t* __restrict__ flag) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; x < len; x += stride)
    if (X[x - 1] > X[x]) bad = 1;
  if (__any(bad) && (threadIdx.x % warpSize) == 0) atomicOr(flag, 1u);
}

}  // namespace cm
