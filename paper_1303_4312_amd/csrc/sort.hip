// Stable merge sort built from the co-rank merge (Siebert and Traeff,
// arXiv:1303.4312: the merge of Sections 2-3 applied pass after pass, the way
// merge sort uses merging, Section 1).
//
//   1. k_sort_runs: every workgroup sorts one run of M pass blocks (M * T
//      elements, T = NT * E the pass tile, M = 4, 2 or 1 as LDS allows) in
//      LDS: each thread sorts its E keys with an odd-even transposition
//      network (compare-exchange only on strictly greater keys, so equal keys
//      never cross: stable), then rounds merge pairs of runs inside LDS, each
//      thread co-ranking its own E outputs (Lemma 1) and merging them
//      sequentially, payloads alongside.
//   2. Passes: runs of length L = MT, 2MT, 4MT, ... are merged pairwise, the
//      pair p being X[2pL, 2pL + L) and X[2pL + L, 2pL + 2L) (clipped to N).
//      Each pass is Algorithm 2 on every pair at once: boundary kernels
//      co-rank the start of every output block inside its pair (one level,
//      or every G-th start first and the others between those), and the
//      block merge of the single merge (merge_block) merges the block.  L is
//      a multiple of T, so no block straddles two pairs.
#include <hip/hip_runtime.h>

#include <stddef.h>

#include <algorithm>
#include <type_traits>

#include "corank_merge.h"
#include "dispatch.hpp"
#include "internal.hpp"
#include "kernels.hpp"

namespace cm {

// Orders this wave's LDS writes before its later LDS reads (lanes of one
// wave exchanging data through LDS; no other wave takes part).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Blocks of the pass tile per initial run: the largest of 4, 2, 1 that keeps
// a workgroup within 1024 threads and its LDS (one run of keys and payloads)
// within 80 KB, so that two workgroups share a CU.  Longer runs leave fewer
// passes over HBM.
template <typename K, bool VAL, int NT, int E>
constexpr int run_blocks() {
  constexpr long bytes = (long)NT * E * (long)(sizeof(K) + (VAL ? sizeof(uint32_t) : 0));
  if (NT * 4 <= 1024 && bytes * 4 <= 80 * 1024) return 4;
  if (NT * 2 <= 1024 && bytes * 2 <= 80 * 1024) return 2;
  return 1;
}

// Waves per SIMD of the run sort with payloads: as many as its LDS (TR keys
// and payloads) allows per CU over 4 SIMDs, in whole workgroups, at most 8;
// asked of the compiler as for the pass kernel.  Keys alone ask for nothing
// (1): at 8 some of those instantiations would spill a register or two.
template <typename K, bool VAL, int NTR, int E>
constexpr int run_waves_per_simd() {
  constexpr long bytes = (long)NTR * E * (long)(sizeof(K) + (VAL ? sizeof(uint32_t) : 0));
  constexpr long per_group = NTR >= 256 ? NTR / 256 : 1;  // waves per SIMD of one workgroup
  long groups = 160l * 1024 / bytes;
  while (groups > 1 && groups * per_group > 8) --groups;
  const long w = groups * per_group;
  return !VAL || w < 1 ? 1 : w > 8 ? 8 : (int)w;
}

// Orders the LDS accesses of the threads of one merged pair: the wave alone
// while a pair's threads fit in one wave (pairs are aligned to waves),
// otherwise the whole workgroup.
__device__ __forceinline__ void pair_sync(int threads_per_pair) {
  if (threads_per_pair <= 64)
    wave_sync();
  else
    __syncthreads();
}

// A 4-byte key and its payload side by side in LDS: one 8-byte access moves
// both (the run sort's merge steps then read each element once).
template <typename K>
struct alignas(8) KeyVal {
  K k;
  uint32_t v;
};

// One run's elements in LDS.  4-byte keys with payloads: KeyVal pairs;
// otherwise keys, then (with payloads) the payloads.
template <typename K, bool VAL, int T>
struct RunStore {
  static constexpr bool kPack = VAL && sizeof(K) == 4;
  static constexpr size_t kBytes = (size_t)T * (sizeof(K) + (VAL ? sizeof(uint32_t) : 0));
  unsigned char* raw;
  __device__ KeyVal<K>* kv() const { return (KeyVal<K>*)raw; }
  __device__ K* keys() const { return (K*)raw; }
  __device__ uint32_t* vals() const { return (uint32_t*)(raw + (size_t)T * sizeof(K)); }
  __device__ K key(int x) const {
    if constexpr (kPack)
      return kv()[x].k;
    else
      return keys()[x];
  }
  __device__ void put(int x, K k, uint32_t v) const {
    if constexpr (kPack) {
      kv()[x] = KeyVal<K>{k, v};
    } else {
      keys()[x] = k;
      if constexpr (VAL) vals()[x] = v;
    }
  }
  __device__ uint32_t val(int x) const {
    if constexpr (kPack)
      return kv()[x].v;
    else
      return vals()[x];
  }
};

// E outputs of the merge of the pair's runs sA = [base, base + R) and
// sB = [base + R, base + 2R), from co-ranks a, b (a + b = the first output's
// rank), keys to ok and payloads to ov: A wins ties (stability).  Packed
// stores read each element once (key and payload together); otherwise the
// payloads are gathered after the keys from their source positions.
template <typename K, bool VAL, int T, int E>
__device__ __forceinline__ void merge_run_store(const RunStore<K, VAL, T>& st, int base, int R, int a, int b,
                                                K (&ok)[E], uint32_t (&ov)[VAL ? E : 1]) {
  if constexpr (RunStore<K, VAL, T>::kPack) {
    const KeyVal<K>* sA = st.kv() + base;
    const KeyVal<K>* sB = sA + R;
    KeyVal<K> ha = a < R ? sA[a] : KeyVal<K>{};
    KeyVal<K> hb = b < R ? sB[b] : KeyVal<K>{};
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool take_a = (a < R) && (b >= R || ha.k <= hb.k);
      ok[e] = take_a ? ha.k : hb.k;
      ov[e] = take_a ? ha.v : hb.v;
      a += take_a ? 1 : 0;
      b += take_a ? 0 : 1;
      const bool more = take_a ? (a < R) : (b < R);
      const KeyVal<K> next = more ? (take_a ? sA[a] : sB[b]) : KeyVal<K>{};
      if (take_a)
        ha = next;
      else
        hb = next;
    }
  } else {
    const K* sA = st.keys() + base;
    const K* sB = sA + R;
    int os[E];
    merge_run<K, E>(sA, R, sB, R, a, b, E, ok, os);
    if constexpr (VAL) {
      const uint32_t* va = st.vals() + base;
#pragma unroll
      for (int e = 0; e < E; ++e) ov[e] = os[e] >= 0 ? va[os[e]] : va[R + ~os[e]];
    }
  }
}

// Every workgroup sorts one run of TR = NTR * E elements in LDS: each thread
// sorts its E keys with an odd-even transposition network (compare-exchange
// only on strictly greater keys, so equal keys never cross: stable), then
// log2(NTR) rounds merge pairs of runs, each thread co-ranking its own E
// outputs (Lemma 1) and merging them sequentially, payloads alongside.  One
// LDS buffer: a thread's E outputs of a round are exactly the E slots it
// writes at the start of the next (its own), so it holds them in registers
// until every thread of its pair has read the round's inputs.
template <typename K, bool VAL, int NTR, int E>
__global__ __launch_bounds__(NTR) __attribute__((amdgpu_waves_per_eu(run_waves_per_simd<K, VAL, NTR, E>())))
void k_sort_runs(const K* __restrict__ X, const uint32_t* __restrict__ Xv, uint64_t N, K* __restrict__ Y,
                 uint32_t* __restrict__ Yv, uint64_t num_runs) {
  static_assert((NTR & (NTR - 1)) == 0 && NTR >= 64, "pairs of runs are whole waves or within one");
  constexpr int T = NTR * E;
  __shared__ __attribute__((aligned(16))) unsigned char s_raw[RunStore<K, VAL, T>::kBytes];
  const RunStore<K, VAL, T> st{s_raw};
  const int q0 = (int)threadIdx.x * E;
  for (uint64_t t = blockIdx.x; t < num_runs; t += gridDim.x) {
    const uint64_t i0 = t * (uint64_t)T;
    const int len = (int)std::min((uint64_t)T, N - i0);
    // every load in flight before the first LDS write waits for one (a slot
    // past the run re-reads its first element: len >= 1)
    K k[E];
    uint32_t v[VAL ? E : 1];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int x = (int)threadIdx.x + r * NTR;
      const uint64_t g = i0 + (uint64_t)(x < len ? x : 0);
      k[r] = X[g];
      if constexpr (VAL) v[r] = Xv[g];
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int x = (int)threadIdx.x + r * NTR;  // < T
      // pads: the last key of the order, after every real key (and after
      // equal real keys, being later), so the run's first len slots end up
      // holding exactly the real elements
      st.put(x, x < len ? k[r] : key_last<K>(), VAL ? v[r] : 0u);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      k[e] = st.key(q0 + e);
      if constexpr (VAL) v[e] = st.val(q0 + e);
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
#pragma unroll
      for (int e = r & 1; e + 1 < E; e += 2) {
        if (k[e + 1] < k[e]) {  // strictly out of order only
          const K tk = k[e];
          k[e] = k[e + 1];
          k[e + 1] = tk;
          if constexpr (VAL) {
            const uint32_t tv = v[e];
            v[e] = v[e + 1];
            v[e + 1] = tv;
          }
        }
      }
    }

    for (int R = E; R < T; R <<= 1) {
      const int per = (2 * R) / E;  // threads per merged pair (a power of two)
      pair_sync(per);               // the pair's reads of the last round are done
#pragma unroll
      for (int e = 0; e < E; ++e) st.put(q0 + e, k[e], VAL ? v[e] : 0u);
      pair_sync(per);
      const int base = ((int)threadIdx.x / per) * 2 * R;
      const int d = q0 - base;
      auto ra = [=](int x) { return st.key(base + x); };
      auto rb = [=](int x) { return st.key(base + R + x); };
      const int a = co_rank<K, int>(kSearchBisect, d, ra, R, rb, R);
      merge_run_store<K, VAL, T, E>(st, base, R, a, d - a, k, v);
    }

    __syncthreads();  // every thread has read the last round's inputs
#pragma unroll
    for (int e = 0; e < E; ++e) st.put(q0 + e, k[e], VAL ? v[e] : 0u);
    __syncthreads();
    for (int x = (int)threadIdx.x; x < len; x += NTR) {
      store_nt(st.key(x), Y + i0 + x);
      if constexpr (VAL) store_nt(st.val(x), Yv + i0 + x);
    }
    if (t + gridDim.x < num_runs) __syncthreads();
  }
}

// The pair holding output block t of a pass whose runs are 2^(sh-1) blocks
// long (a pair is 2^sh blocks of T outputs; shifts, not divisions).
struct PassPair {
  uint64_t base;  // first element of the pair (of X and of Y)
  uint64_t m, n;  // lengths of its two runs
  uint64_t il;    // the block's first output inside the pair
};

__device__ __forceinline__ PassPair pass_pair(uint64_t t, uint64_t T, int sh, uint64_t N) {
  PassPair p;
  const uint64_t first = t >> sh << sh;  // first block of the pair
  const uint64_t L = T << (sh - 1);
  p.base = first * T;
  p.m = std::min(L, N - p.base);
  p.n = std::min(L, N - p.base - p.m);
  p.il = (t - first) * T;
  return p;
}

// bj[t] = A co-rank of block t's first output inside its pair.
template <typename K>
__global__ __launch_bounds__(256) void k_sort_pass_co_rank(const K* __restrict__ X, uint64_t N, int sh,
                                                           uint64_t T, uint64_t num_tiles,
                                                           uint64_t* __restrict__ bj, int search) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= num_tiles) return;
  const PassPair p = pass_pair(t, T, sh, N);
  const K* A = X + p.base;
  const K* B = A + p.m;
  auto ra = [=](uint64_t x) { return A[x]; };
  auto rb = [=](uint64_t x) { return B[x]; };
  bj[t] = co_rank<K, uint64_t>(search, p.il, ra, p.m, rb, p.n);
}

// Two-level form for passes whose pairs span more than G blocks (the
// one-level search above then walks up to log2 of the whole pair).  Coarse
// step: every G-th block start of the pass (block c * G), co-ranked inside
// its pair by a group of 16 lanes (16-ary search).
template <typename K>
__global__ __launch_bounds__(256) void k_sort_pass_coarse(const K* __restrict__ X, uint64_t N, int sh, uint64_t T,
                                                          uint32_t G, uint64_t num_coarse,
                                                          uint64_t* __restrict__ jc) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((gid & ~63ull) / 16 >= num_coarse) return;  // whole waves with no coarse block leave
  const uint64_t c = gid / 16;
  const bool mine = c < num_coarse;  // groups past the end run along with an empty interval
  uint64_t i = 0, lo = 0, hi = 0;
  const K* A = X;
  const K* B = X;
  if (mine) {
    const PassPair p = pass_pair(c * G, T, sh, N);
    A = X + p.base;
    B = A + p.m;
    i = p.il;
    lo = i > p.n ? i - p.n : 0;
    hi = std::min(i, p.m);
  }
  auto ra = [=](uint64_t x) { return A[x]; };
  auto rb = [=](uint64_t x) { return B[x]; };
  const uint64_t j = co_rank_group<K, 16>(i, ra, rb, lo, hi);
  if (mine && (gid & 15) == 0) jc[c] = j;
}

// Fine step: block t's start lies between the coarse blocks c * G and
// (c + 1) * G (c = t / G); each bounds its co-rank when it lies in the same
// pair (co-ranks grow with the rank), else the pair's start (co-rank 0) or
// end (co-rank m) does; the search runs only over that window, by bisection
// (L = 1) or by a group of L lanes (L-ary, co_rank_group; whole waves run
// together, groups past the end and coarse blocks taking an empty window).
template <typename K, int L>
__global__ __launch_bounds__(256) void k_sort_pass_fine(const K* __restrict__ X, uint64_t N, int sh, uint64_t T,
                                                        uint64_t num_tiles, uint32_t G,
                                                        const uint64_t* __restrict__ jc, uint64_t* __restrict__ bj) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (L == 1 ? gid >= num_tiles : (gid & ~63ull) / L >= num_tiles) return;
  const uint64_t t = gid / L;
  const bool mine = t < num_tiles;
  const uint64_t c = mine ? t / G : 0;
  const bool coarse = mine && t == c * G;
  uint64_t i = 0, lo = 0, hi = 0;
  const K* A = X;
  const K* B = X;
  if (mine && !coarse) {
    const PassPair p = pass_pair(t, T, sh, N);
    const uint64_t f = t >> sh << sh;              // the pair's first block
    const uint64_t nbp = (p.m + p.n + T - 1) / T;  // its blocks
    const uint64_t m = p.m, n = p.n;
    i = p.il;
    uint64_t i0 = 0, j0 = 0, i1 = m + n, j1 = m;
    if (c * G >= f) {
      i0 = (c * G - f) * T;
      j0 = jc[c];
    }
    if ((c + 1) * G < f + nbp) {
      i1 = ((c + 1) * G - f) * T;
      j1 = jc[c + 1];
    }
    const uint64_t k0 = i0 - j0, k1 = i1 - j1;
    lo = std::max(i > n ? i - n : 0, j0);
    if (i > k1) lo = std::max(lo, i - k1);
    hi = std::min(std::min(i, m), j1);
    hi = std::min(hi, i - std::min(k0, i));
    if (hi < lo) hi = lo;  // only for unsorted input (monotonicity broken)
    A = X + p.base;
    B = A + m;
  }
  auto ra = [=](uint64_t x) { return A[x]; };
  auto rb = [=](uint64_t x) { return B[x]; };
  uint64_t j;
  if constexpr (L == 1)
    j = co_rank_bisect_in<K>(i, ra, rb, lo, hi);
  else
    j = co_rank_group<K, L>(i, ra, rb, lo, hi);
  if (mine && gid % L == 0) bj[t] = coarse ? jc[c] : j;
}

// The same value in every lane, said so to the compiler: the block index
// from grid_block is, but the pair arithmetic on it otherwise lands in vector
// registers (98 of them for 256 x 9 with payloads, which halves the waves a
// CU holds against the 64 of the single merge's kernel).
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return (uint64_t)hi << 32 | lo;
}

// Waves per SIMD that the LDS of one pass workgroup (T + 16 keys and, with
// payloads, T + 16 uint32 values) leaves room for: 160 KB per CU shared by
// 4 SIMDs.  The pass kernel asks the compiler for that many
// (amdgpu_waves_per_eu), so registers are not the tighter limit; at most 8
// (64 VGPRs) for uint32 keys, at most 7 for the other key types, whose
// comparisons or wider keys would spill a register or two at 8.
template <typename K, bool VAL, int NT, int E>
constexpr int pass_waves_per_simd() {
  constexpr long bytes = (long)(NT * E + 16) * (long)(sizeof(K) + (VAL ? sizeof(uint32_t) : 0));
  constexpr long w = (160l * 1024 / bytes) * (NT / 64) / 4;
  constexpr long cap = std::is_same<K, uint32_t>::value || std::is_same<K, Desc<uint32_t>>::value ? 8 : 7;
  return w < 1 ? 1 : w > cap ? (int)cap : (int)w;
}

template <typename K, bool VAL, int NT, int E, bool VEC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(pass_waves_per_simd<K, VAL, NT, E>())))
void k_sort_pass_merge(const K* __restrict__ X, const uint32_t* __restrict__ Xv,
                                                        uint64_t N, int sh, K* __restrict__ Y,
                                                        uint32_t* __restrict__ Yv, const uint64_t* __restrict__ bj,
                                                        uint64_t num_tiles, int search, int xcd) {
  constexpr int T = NT * E;
  __shared__ __attribute__((aligned(16))) K s_key[T + 16];
  __shared__ __attribute__((aligned(16))) uint32_t s_val[VAL ? T + 16 : 1];
  for (uint64_t b = blockIdx.x; b < num_tiles; b += gridDim.x) {
    const uint64_t t = uniform_u64(grid_block(b, num_tiles, xcd));
    const PassPair p = pass_pair(t, (uint64_t)T, sh, N);
    const int len = (int)std::min((uint64_t)T, N - t * (uint64_t)T);
    const uint64_t j0 = bj[t];
    // the block's end co-rank: the next block's start in the same pair, or the pair's end
    const uint64_t j1 = p.il + (uint64_t)len == p.m + p.n ? p.m : bj[t + 1];
    const K* A = X + p.base;
    const uint32_t* Av = VAL ? Xv + p.base : nullptr;
    merge_block<K, VAL, NT, E, VEC>(A, Av, p.m, A + p.m, VAL ? Av + p.m : nullptr, p.n, Y + p.base,
                                    VAL ? Yv + p.base : nullptr, p.il, len, j0, j1, search, s_key, s_val);
    if (b + gridDim.x < num_tiles) __syncthreads();
  }
}

uint32_t sort_run_blocks(int kt, bool val, int cfg) {
  return (uint32_t)by_key(kt, [&](auto key) -> int {
    using K = decltype(key);
    return by_cfg(cfg, [&](auto nt, auto e) -> int {
      constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
      return val ? run_blocks<K, true, NT, E>() : run_blocks<K, false, NT, E>();
    });
  });
}

int launch_sort_blocks(int kt, bool val, const Choice& ch, const void* X, const uint32_t* Xv, uint64_t N, void* Y,
                       uint32_t* Yv, uint64_t runs, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int {
    using K = decltype(key);
    return by_cfg(ch.cfg, [&](auto nt, auto e) -> int {
      constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
      auto go = [&](auto val_c) {
        constexpr bool V = decltype(val_c)::value;
        constexpr int NTR = NT * run_blocks<K, V, NT, E>();
        hipLaunchKernelGGL((k_sort_runs<K, V, NTR, E>),
                           dim3(launch_grid((const void*)k_sort_runs<K, V, NTR, E>, NTR, runs, ch.grid)), dim3(NTR),
                           0, st, (const K*)X, Xv, N, (K*)Y, Yv, runs);
      };
      if (val)
        go(std::true_type{});
      else
        go(std::false_type{});
      return launch_status();
    });
  });
}

int launch_sort_pass(int kt, bool val, const Choice& ch, const Shape& shape, const void* X, const uint32_t* Xv,
                     uint64_t N, int sh, void* Y, uint32_t* Yv, uint64_t* bj, uint64_t* coarse, uint64_t tiles,
                     hipStream_t st) {
  return by_key(kt, [&](auto key) -> int {
    using K = decltype(key);
    return by_cfg(ch.cfg, [&](auto nt, auto e) -> int {
      constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
      constexpr uint64_t T = (uint64_t)NT * E;
      const uint32_t G = shape.coarse_stride;
      if (ch.partition != 0 && coarse && (1ull << sh) > G) {  // pairs longer than G blocks: two levels
        const uint64_t nc = (tiles + G - 1) / G;
        hipLaunchKernelGGL((k_sort_pass_coarse<K>), dim3((unsigned)((nc + 15) / 16)), dim3(256), 0, st, (const K*)X,
                           N, sh, T, G, nc, coarse);
        if (launch_status() != CM_OK) return CM_EHIP;
        const int L = shape.fine_lanes == 2 || shape.fine_lanes == 4 ? shape.fine_lanes : 1;
        const unsigned fine_grid = (unsigned)((tiles * (uint64_t)L + 255) / 256);
        if (L == 4)
          hipLaunchKernelGGL((k_sort_pass_fine<K, 4>), dim3(fine_grid), dim3(256), 0, st, (const K*)X, N, sh, T, tiles,
                             G, (const uint64_t*)coarse, bj);
        else if (L == 2)
          hipLaunchKernelGGL((k_sort_pass_fine<K, 2>), dim3(fine_grid), dim3(256), 0, st, (const K*)X, N, sh, T, tiles,
                             G, (const uint64_t*)coarse, bj);
        else
          hipLaunchKernelGGL((k_sort_pass_fine<K, 1>), dim3(fine_grid), dim3(256), 0, st, (const K*)X, N, sh, T, tiles,
                             G, (const uint64_t*)coarse, bj);
      } else {
        hipLaunchKernelGGL((k_sort_pass_co_rank<K>), dim3((unsigned)((tiles + 255) / 256)), dim3(256), 0, st,
                           (const K*)X, N, sh, T, tiles, bj, ch.search);
      }
      if (launch_status() != CM_OK) return CM_EHIP;
      // every pair starts at a multiple of T elements of X and Y
      const bool vec = val ? all_aligned16({X, Y, Xv, Yv}) : all_aligned16({X, Y});
      auto go = [&](auto val_c, auto vec_c) {
        constexpr bool V = decltype(val_c)::value, W = decltype(vec_c)::value;
        hipLaunchKernelGGL((k_sort_pass_merge<K, V, NT, E, W>),
                           dim3(launch_grid((const void*)k_sort_pass_merge<K, V, NT, E, W>, NT, tiles, ch.grid)),
                           dim3(NT), 0, st, (const K*)X, Xv, N, sh, (K*)Y, Yv, (const uint64_t*)bj, tiles,
                           ch.search, shape.xcd_order);
      };
      using T_ = std::true_type;
      using F_ = std::false_type;
      if (val && vec)
        go(T_{}, T_{});
      else if (val)
        go(T_{}, F_{});
      else if (vec)
        go(F_{}, T_{});
      else
        go(F_{}, F_{});
      return launch_status();
    });
  });
}

}  // namespace cm
