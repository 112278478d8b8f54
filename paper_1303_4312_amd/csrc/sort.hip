// Stable merge sort built from the co-rank merge (Siebert and Traeff,
// arXiv:1303.4312: the merge of Sections 2-3 applied pass after pass, the way
// merge sort uses merging, Section 1).
//
//   1. k_sort_blocks: every workgroup sorts one run of T = NT * E elements in
//      LDS: each thread sorts its E keys with an odd-even transposition
//      network (compare-exchange only on strictly greater keys, so equal keys
//      never cross: stable), then log2(NT) rounds merge pairs of runs inside
//      LDS, each thread co-ranking its own E outputs (Lemma 1) and merging
//      them sequentially; payloads follow through the run position.
//   2. Passes: runs of length L = T, 2T, 4T, ... are merged pairwise, the
//      pair p being X[2pL, 2pL + L) and X[2pL + L, 2pL + 2L) (clipped to N).
//      Each pass is Algorithm 2 on every pair at once: a boundary kernel
//      co-ranks the start of every output block inside its pair, and the
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

template <typename K, bool VAL, int NT, int E>
__global__ __launch_bounds__(NT) void k_sort_blocks(const K* __restrict__ X, const uint32_t* __restrict__ Xv,
                                                    uint64_t N, K* __restrict__ Y, uint32_t* __restrict__ Yv,
                                                    uint64_t num_tiles) {
  static_assert((NT & (NT - 1)) == 0, "runs pair up only for a power-of-two thread count");
  constexpr int T = NT * E;
  static_assert(T <= 65536, "run positions are 16-bit");
  __shared__ K s_k[2][T];
  // position in the run each key came from (payloads follow it; keys alone
  // need none: the merges move the keys themselves, ties in order)
  __shared__ uint16_t s_i[VAL ? 2 : 1][VAL ? T : 1];
  __shared__ uint32_t s_v[VAL ? T : 1];
  for (uint64_t t = blockIdx.x; t < num_tiles; t += gridDim.x) {
    const uint64_t i0 = t * (uint64_t)T;
    const int len = (int)std::min((uint64_t)T, N - i0);
    // every load in flight before the first LDS write waits for one (a slot
    // past the run re-reads its first element: len >= 1)
    K lk[E];
    uint32_t lv[VAL ? E : 1];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int x = (int)threadIdx.x + r * NT;
      const uint64_t g = i0 + (uint64_t)(x < len ? x : 0);
      lk[r] = X[g];
      if constexpr (VAL) lv[r] = Xv[g];
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int x = (int)threadIdx.x + r * NT;  // < T = NT * E
      // pads: the last key of the order, after every real key (and after
      // equal real keys, being later)
      s_k[0][x] = x < len ? lk[r] : key_last<K>();
      if constexpr (VAL)
        if (x < len) s_v[x] = lv[r];
    }
    __syncthreads();

    // this thread's E keys, sorted in registers
    const int q0 = (int)threadIdx.x * E;
    K k[E];
    uint16_t id[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      k[e] = s_k[0][q0 + e];
      if constexpr (VAL) id[e] = (uint16_t)(q0 + e);
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
            const uint16_t ti = id[e];
            id[e] = id[e + 1];
            id[e + 1] = ti;
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      s_k[0][q0 + e] = k[e];
      if constexpr (VAL) s_i[0][q0 + e] = id[e];
    }
    wave_sync();  // the first round pairs neighbouring threads of one wave

    // merge runs of R = E, 2E, 4E, ... pairwise in LDS.  A round reads only
    // what the threads of its own pair wrote in the round before; while a
    // pair's threads (2R / E of them, a power of two) fit in one wave, the
    // rounds need no workgroup barrier.
    int src = 0;
    for (int R = E; R < T; R <<= 1) {
      const int per = (2 * R) / E;  // threads per merged pair
      const int pair = (int)threadIdx.x / per;
      const int d = ((int)threadIdx.x % per) * E;
      const K* sa = s_k[src] + pair * 2 * R;
      const K* sb = sa + R;
      auto ra = [=](int x) { return sa[x]; };
      auto rb = [=](int x) { return sb[x]; };
      const int a = co_rank<K, int>(kSearchBisect, d, ra, R, rb, R);
      K ok[E];
      int os[E];
      merge_run<K, E>(sa, R, sb, R, a, d - a, E, ok, os);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        s_k[src ^ 1][pair * 2 * R + d + e] = ok[e];
        if constexpr (VAL) {
          const uint16_t* si = s_i[src] + pair * 2 * R;
          s_i[src ^ 1][pair * 2 * R + d + e] = os[e] >= 0 ? si[os[e]] : si[R + ~os[e]];
        }
      }
      // the next round's pairs (4R / E threads) inside one wave: wave order
      // suffices; otherwise (and before the stores) the whole workgroup
      if (4 * R < T && 2 * per <= 64)
        wave_sync();
      else
        __syncthreads();
      src ^= 1;
    }

    for (int x = (int)threadIdx.x; x < len; x += NT) {
      store_nt(s_k[src][x], Y + i0 + x);
      if constexpr (VAL) store_nt(s_v[s_i[src][x]], Yv + i0 + x);
    }
    if (t + gridDim.x < num_tiles) __syncthreads();
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

template <typename K, bool VAL, int NT, int E, bool VEC>
__global__ __launch_bounds__(NT) void k_sort_pass_merge(const K* __restrict__ X, const uint32_t* __restrict__ Xv,
                                                        uint64_t N, int sh, K* __restrict__ Y,
                                                        uint32_t* __restrict__ Yv, const uint64_t* __restrict__ bj,
                                                        uint64_t num_tiles, int search, int xcd) {
  constexpr int T = NT * E;
  __shared__ __attribute__((aligned(16))) K s_key[T + 16];
  __shared__ __attribute__((aligned(16))) uint32_t s_val[VAL ? T + 16 : 1];
  for (uint64_t b = blockIdx.x; b < num_tiles; b += gridDim.x) {
    const uint64_t t = grid_block(b, num_tiles, xcd);
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

int launch_sort_blocks(int kt, bool val, const Choice& ch, const void* X, const uint32_t* Xv, uint64_t N, void* Y,
                       uint32_t* Yv, uint64_t tiles, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int {
    using K = decltype(key);
    return by_cfg(ch.cfg, [&](auto nt, auto e) -> int {
      constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
      if (val)
        hipLaunchKernelGGL((k_sort_blocks<K, true, NT, E>),
                           dim3(launch_grid((const void*)k_sort_blocks<K, true, NT, E>, NT, tiles, ch.grid)), dim3(NT),
                           0, st, (const K*)X, Xv, N, (K*)Y, Yv, tiles);
      else
        hipLaunchKernelGGL((k_sort_blocks<K, false, NT, E>),
                           dim3(launch_grid((const void*)k_sort_blocks<K, false, NT, E>, NT, tiles, ch.grid)),
                           dim3(NT), 0, st, (const K*)X, Xv, N, (K*)Y, Yv, tiles);
      return launch_status();
    });
  });
}

int launch_sort_pass(int kt, bool val, const Choice& ch, const Shape& shape, const void* X, const uint32_t* Xv,
                     uint64_t N, int sh, void* Y, uint32_t* Yv, uint64_t* bj, uint64_t tiles, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int {
    using K = decltype(key);
    return by_cfg(ch.cfg, [&](auto nt, auto e) -> int {
      constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
      constexpr uint64_t T = (uint64_t)NT * E;
      hipLaunchKernelGGL((k_sort_pass_co_rank<K>), dim3((unsigned)((tiles + 255) / 256)), dim3(256), 0, st,
                         (const K*)X, N, sh, T, tiles, bj, ch.search);
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
