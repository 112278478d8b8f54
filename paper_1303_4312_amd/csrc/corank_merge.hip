// Kernels and C ABI of the co-rank stable merge for MI355X (gfx950).
//
// Single merge (Sections 2 and 3 of Siebert and Traeff, arXiv:1303.4312):
//   1. k_block_co_rank: one thread per block boundary i_t = t * T computes
//      j_t = co_rank(i_t) over global memory (Algorithm 1).  Running the
//      boundary searches as their own pass is the synchronised variant of
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
// Segmented batch: the same two kernels over the concatenation of many
// problems, partitioned as one merge under the order (segment, key).
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "corank_merge.h"
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

// Arbitrary ranks: j_out[r] = A co-rank of ranks[r], UINT64_MAX if out of range.
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
// position (a, b), in registers.  Takes A while A has elements left and B is
// exhausted or A's key <= B's key (the tie rule: A first).  ka / kb hold the
// next key of each side; one LDS read refills the side just consumed.
// out_src[e] is the window position (0..len) the output came from, used to
// move payloads.  Outputs at or beyond `avail` are not produced.
template <typename K, int E>
__device__ __forceinline__ void merge_run(const K* s_key, int a_len, int len, int a, int b, int avail,
                                          K (&out_key)[E], int (&out_src)[E]) {
  const int b_len = len - a_len;
  K ka = a < a_len ? s_key[a] : K{};
  K kb = b < b_len ? s_key[a_len + b] : K{};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e < avail) {
      const bool take_a = (a < a_len) && (b >= b_len || ka <= kb);
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

template <typename K, bool VAL, int NT, int E>
__global__ __launch_bounds__(NT) void k_merge_blocks(const K* __restrict__ A, const uint32_t* __restrict__ Av,
                                                     uint64_t m, const K* __restrict__ B,
                                                     const uint32_t* __restrict__ Bv, uint64_t n,
                                                     K* __restrict__ C, uint32_t* __restrict__ Cv,
                                                     const uint64_t* __restrict__ bj, uint64_t num_tiles,
                                                     int search) {
  constexpr int T = NT * E;
  __shared__ K s_key[T];
  __shared__ uint32_t s_val[VAL ? T : 1];
  const uint64_t N = m + n;
  for (uint64_t t = blockIdx.x; t < num_tiles; t += gridDim.x) {
    const uint64_t i0 = t * (uint64_t)T;
    const int len = (int)std::min((uint64_t)T, N - i0);
    const uint64_t j0 = bj[t];
    const uint64_t j1 = bj[t + 1];
    const int a_len = window_a_len(j0, j1, len);
    const int b_len = len - a_len;
    load_windows<K, VAL, NT, E>(A, Av, j0, B, Bv, i0 - j0, a_len, len, s_key, s_val);
    __syncthreads();

    const int d = std::min((int)threadIdx.x * E, len);
    const K* sA = s_key;
    const K* sB = s_key + a_len;
    auto ra = [=](int x) { return sA[x]; };
    auto rb = [=](int x) { return sB[x]; };
    const int a = co_rank<K, int>(search, d, ra, a_len, rb, b_len);
    K ok[E];
    int os[E];
    const int avail = len - d;
    merge_run<K, E>(s_key, a_len, len, a, d - a, avail, ok, os);
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
    store_block<K, VAL, NT, E>(C, Cv, i0, len, s_key, s_val);
    if (t + gridDim.x < num_tiles) __syncthreads();
  }
}

// ---- segmented batch -------------------------------------------------------

// One workgroup: flag = 0 if the offsets are consistent (start at 0,
// nondecreasing, end at the host totals), else 1.  Every later kernel of the
// call reads the flag and does nothing when it is set.
__global__ __launch_bounds__(1024) void k_seg_validate(const uint64_t* __restrict__ a_off,
                                                       const uint64_t* __restrict__ b_off, uint64_t S,
                                                       uint64_t total_a, uint64_t total_b,
                                                       uint32_t* __restrict__ flag) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int my_bad = 0;
  for (uint64_t s = threadIdx.x; s < S; s += blockDim.x) {
    if (a_off[s] > a_off[s + 1] || b_off[s] > b_off[s + 1]) my_bad = 1;
  }
  if (threadIdx.x == 0) {
    if (a_off[0] != 0 || b_off[0] != 0 || a_off[S] != total_a || b_off[S] != total_b) my_bad = 1;
  }
  if (my_bad) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) *flag = bad ? 1u : 0u;
}

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

// Segmented merge run: like merge_run, but the run may cross segment ends.
// s is the segment of the run's first output; a_end / b_end are the window
// positions where segment s ends on each side (they may lie beyond the
// window).  When both sides of the current segment are used up the run moves
// on to the next non-empty segment.
template <typename K, int E>
__device__ __forceinline__ void merge_run_seg(const K* s_key, int a_len, int len, int a, int b, int avail,
                                              const uint64_t* __restrict__ a_off,
                                              const uint64_t* __restrict__ b_off, uint32_t S, uint32_t s,
                                              uint64_t j0, uint64_t k0, K (&out_key)[E],
                                              int (&out_src)[E]) {
  const int b_len = len - a_len;
  auto clamp_end = [](uint64_t end, uint64_t base) -> int {
    return (int)std::min(end - base, (uint64_t)INT_MAX);
  };
  int a_end = clamp_end(a_off[s + 1], j0);
  int b_end = clamp_end(b_off[s + 1], k0);
  K ka = a < a_len ? s_key[a] : K{};
  K kb = b < b_len ? s_key[a_len + b] : K{};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e < avail) {
      while (a == a_end && b == b_end && s + 1 < S) {
        ++s;
        a_end = clamp_end(a_off[s + 1], j0);
        b_end = clamp_end(b_off[s + 1], k0);
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

template <typename K, bool VAL, int NT, int E>
__global__ __launch_bounds__(NT) void k_seg_merge_blocks(
    const K* __restrict__ A, const uint32_t* __restrict__ Av, const uint64_t* __restrict__ a_off,
    const K* __restrict__ B, const uint32_t* __restrict__ Bv, const uint64_t* __restrict__ b_off, uint32_t S,
    uint64_t N, K* __restrict__ C, uint32_t* __restrict__ Cv, const uint64_t* __restrict__ bj,
    const uint32_t* __restrict__ bs, uint64_t num_tiles, const uint32_t* __restrict__ flag, int search) {
  constexpr int T = NT * E;
  __shared__ K s_key[T];
  __shared__ uint32_t s_val[VAL ? T : 1];
  if (*flag) return;
  for (uint64_t t = blockIdx.x; t < num_tiles; t += gridDim.x) {
    const uint64_t i0 = t * (uint64_t)T;
    const int len = (int)std::min((uint64_t)T, N - i0);
    const uint64_t j0 = bj[t];
    const uint64_t k0 = i0 - j0;
    const int a_len = window_a_len(j0, bj[t + 1], len);
    const int b_len = len - a_len;
    const uint64_t j1 = j0 + (uint64_t)a_len;
    const uint32_t s_first = bs[t];
    const uint32_t s_last = bs[t + 1];
    load_windows<K, VAL, NT, E>(A, Av, j0, B, Bv, k0, a_len, len, s_key, s_val);
    __syncthreads();

    const int d = std::min((int)threadIdx.x * E, len);
    const int avail = len - d;
    K ok[E];
    int os[E];
    if (avail > 0) {
      const uint64_t g = i0 + (uint64_t)d;
      const uint32_t s = seg_of(a_off, b_off, s_first, s_last, g);
      const uint64_t sa0 = a_off[s], sa1 = a_off[s + 1];
      const uint64_t sb0 = b_off[s], sb1 = b_off[s + 1];
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
      merge_run_seg<K, E>(s_key, a_len, len, wa0 + ja, wb0 + (dd - ja), avail, a_off, b_off, S, s, j0, k0,
                          ok, os);
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
    store_block<K, VAL, NT, E>(C, Cv, i0, len, s_key, s_val);
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

__global__ void k_fill_u32(uint32_t* p, uint32_t v) { *p = v; }

// ---------------------------------------------------------------------------
// host side

struct TileCfg {
  int nt;
  int e;
};

// Every configuration is instantiated for every key type and payload mode.
// E is odd so that the strided LDS accesses of the transposes (stride E
// words) touch distinct banks.
static const TileCfg kCfgs[] = {{256, 7}, {256, 11}, {256, 15}, {128, 15},
                                {512, 7}, {256, 19}, {128, 23}, {512, 11}};
static const int kNumCfgs = (int)(sizeof(kCfgs) / sizeof(kCfgs[0]));

static int g_cfg[3][2] = {{2, 2}, {2, 2}, {2, 2}};
static int g_search = kSearchAlg1;

static bool key_type_ok(int kt) { return kt == CM_KEY_U32 || kt == CM_KEY_U64 || kt == CM_KEY_F32; }
static size_t key_bytes(int kt) { return kt == CM_KEY_U64 ? 8 : 4; }

static bool overlap(const void* p, uint64_t pbytes, const void* q, uint64_t qbytes) {
  if (!p || !q || pbytes == 0 || qbytes == 0) return false;
  const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
  return a < b + qbytes && b < a + pbytes;
}

static uint64_t tile_of(int kt, int with_val) {
  const TileCfg c = kCfgs[g_cfg[kt][with_val ? 1 : 0]];
  return (uint64_t)c.nt * (uint64_t)c.e;
}

static size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

static int launch_status() { return hipGetLastError() == hipSuccess ? CM_OK : CM_EHIP; }

template <typename K, bool VAL, int NT, int E>
static int launch_merge_t(const void* A, const uint32_t* Av, uint64_t m, const void* B, const uint32_t* Bv,
                          uint64_t n, void* C, uint32_t* Cv, const uint64_t* bj, uint64_t tiles,
                          hipStream_t st) {
  hipLaunchKernelGGL((k_merge_blocks<K, VAL, NT, E>), dim3((unsigned)tiles), dim3(NT), 0, st, (const K*)A, Av, m,
                     (const K*)B, Bv, n, (K*)C, Cv, bj, tiles, g_search);
  return launch_status();
}

template <typename K, bool VAL, int NT, int E>
static int launch_seg_t(const void* A, const uint32_t* Av, const uint64_t* a_off, const void* B,
                        const uint32_t* Bv, const uint64_t* b_off, uint32_t S, uint64_t N, void* C, uint32_t* Cv,
                        const uint64_t* bj, const uint32_t* bs, uint64_t tiles, const uint32_t* flag,
                        hipStream_t st) {
  hipLaunchKernelGGL((k_seg_merge_blocks<K, VAL, NT, E>), dim3((unsigned)tiles), dim3(NT), 0, st, (const K*)A,
                     Av, a_off, (const K*)B, Bv, b_off, S, N, (K*)C, Cv, bj, bs, tiles, flag, g_search);
  return launch_status();
}

#define CM_CFG_CASES(FN, K, VAL, ...)        \
  switch (cfg) {                             \
    case 0: return FN<K, VAL, 256, 7>(__VA_ARGS__);   \
    case 1: return FN<K, VAL, 256, 11>(__VA_ARGS__);  \
    case 2: return FN<K, VAL, 256, 15>(__VA_ARGS__);  \
    case 3: return FN<K, VAL, 128, 15>(__VA_ARGS__);  \
    case 4: return FN<K, VAL, 512, 7>(__VA_ARGS__);   \
    case 5: return FN<K, VAL, 256, 19>(__VA_ARGS__);  \
    case 6: return FN<K, VAL, 128, 23>(__VA_ARGS__);  \
    case 7: return FN<K, VAL, 512, 11>(__VA_ARGS__);  \
    default: return CM_ECONFIG;              \
  }

template <typename K, bool VAL>
static int launch_merge_cfg(int cfg, const void* A, const uint32_t* Av, uint64_t m, const void* B,
                            const uint32_t* Bv, uint64_t n, void* C, uint32_t* Cv, const uint64_t* bj,
                            uint64_t tiles, hipStream_t st) {
  CM_CFG_CASES(launch_merge_t, K, VAL, A, Av, m, B, Bv, n, C, Cv, bj, tiles, st)
}

template <typename K, bool VAL>
static int launch_seg_cfg(int cfg, const void* A, const uint32_t* Av, const uint64_t* a_off, const void* B,
                          const uint32_t* Bv, const uint64_t* b_off, uint32_t S, uint64_t N, void* C,
                          uint32_t* Cv, const uint64_t* bj, const uint32_t* bs, uint64_t tiles,
                          const uint32_t* flag, hipStream_t st) {
  CM_CFG_CASES(launch_seg_t, K, VAL, A, Av, a_off, B, Bv, b_off, S, N, C, Cv, bj, bs, tiles, flag, st)
}

template <typename K>
static int launch_bounds_t(const void* A, uint64_t m, const void* B, uint64_t n, uint64_t tile, uint64_t nb,
                           uint64_t* bj, hipStream_t st) {
  const uint64_t blocks = (nb + 255) / 256;
  hipLaunchKernelGGL((k_block_co_rank<K>), dim3((unsigned)blocks), dim3(256), 0, st, (const K*)A, m,
                     (const K*)B, n, tile, nb, bj, g_search);
  return launch_status();
}

static int merge_impl(int kt, bool with_val, const void* A, const uint32_t* Av, uint64_t m, const void* B,
                      const uint32_t* Bv, uint64_t n, void* C, uint32_t* Cv, void* ws, size_t ws_bytes,
                      hipStream_t st) {
  if (!key_type_ok(kt)) return CM_EDTYPE;
  if (m + n < m) return CM_EINVAL;
  const uint64_t N = m + n;
  const size_t ks = key_bytes(kt);
  if ((m && !A) || (n && !B) || (N && !C)) return CM_EINVAL;
  if (with_val && ((m && !Av) || (n && !Bv) || (N && !Cv))) return CM_EINVAL;
  if (overlap(C, N * ks, A, m * ks) || overlap(C, N * ks, B, n * ks)) return CM_EALIAS;
  if (with_val) {
    if (overlap(Cv, N * 4, Av, m * 4) || overlap(Cv, N * 4, Bv, n * 4) || overlap(Cv, N * 4, A, m * ks) ||
        overlap(Cv, N * 4, B, n * ks) || overlap(Cv, N * 4, C, N * ks) || overlap(C, N * ks, Av, m * 4) ||
        overlap(C, N * ks, Bv, n * 4))
      return CM_EALIAS;
  }
  if (N == 0) return CM_OK;
  const uint64_t T = tile_of(kt, with_val);
  const uint64_t tiles = (N + T - 1) / T;
  if (tiles >= (1ull << 31)) return CM_EINVAL;
  const size_t need = round256((tiles + 1) * sizeof(uint64_t));
  if (!ws || ws_bytes < need) return CM_ENOSPC;
  if (overlap(ws, need, A, m * ks) || overlap(ws, need, B, n * ks) || overlap(ws, need, C, N * ks))
    return CM_EALIAS;
  uint64_t* bj = (uint64_t*)ws;
  int rc;
  switch (kt) {
    case CM_KEY_U32: rc = launch_bounds_t<uint32_t>(A, m, B, n, T, tiles + 1, bj, st); break;
    case CM_KEY_U64: rc = launch_bounds_t<uint64_t>(A, m, B, n, T, tiles + 1, bj, st); break;
    default: rc = launch_bounds_t<float>(A, m, B, n, T, tiles + 1, bj, st); break;
  }
  if (rc != CM_OK) return rc;
  const int cfg = g_cfg[kt][with_val ? 1 : 0];
  if (with_val) {
    switch (kt) {
      case CM_KEY_U32: return launch_merge_cfg<uint32_t, true>(cfg, A, Av, m, B, Bv, n, C, Cv, bj, tiles, st);
      case CM_KEY_U64: return launch_merge_cfg<uint64_t, true>(cfg, A, Av, m, B, Bv, n, C, Cv, bj, tiles, st);
      default: return launch_merge_cfg<float, true>(cfg, A, Av, m, B, Bv, n, C, Cv, bj, tiles, st);
    }
  }
  switch (kt) {
    case CM_KEY_U32: return launch_merge_cfg<uint32_t, false>(cfg, A, Av, m, B, Bv, n, C, Cv, bj, tiles, st);
    case CM_KEY_U64: return launch_merge_cfg<uint64_t, false>(cfg, A, Av, m, B, Bv, n, C, Cv, bj, tiles, st);
    default: return launch_merge_cfg<float, false>(cfg, A, Av, m, B, Bv, n, C, Cv, bj, tiles, st);
  }
}

struct SegWorkspace {
  uint32_t* flag;
  uint64_t* bj;
  uint32_t* bs;
  size_t bytes;
};

static SegWorkspace seg_layout(void* ws, uint64_t tiles) {
  SegWorkspace w;
  char* p = (char*)ws;
  w.flag = (uint32_t*)p;
  size_t off = 256;
  w.bj = (uint64_t*)(p + off);
  off += round256((tiles + 1) * sizeof(uint64_t));
  w.bs = (uint32_t*)(p + off);
  off += round256((tiles + 1) * sizeof(uint32_t));
  w.bytes = off;
  return w;
}

template <typename K>
static int launch_seg_bounds_t(const void* A, const uint64_t* a_off, const void* B, const uint64_t* b_off,
                               uint32_t S, uint64_t N, uint64_t T, uint64_t nb, uint64_t* bj, uint32_t* bs,
                               const uint32_t* flag, hipStream_t st) {
  const uint64_t blocks = (nb + 255) / 256;
  hipLaunchKernelGGL((k_seg_block_co_rank<K>), dim3((unsigned)blocks), dim3(256), 0, st, (const K*)A, a_off,
                     (const K*)B, b_off, S, N, T, nb, bj, bs, flag, g_search);
  return launch_status();
}

static int seg_impl(int kt, const void* A, const uint32_t* Av, const uint64_t* a_off, uint64_t total_a,
                    const void* B, const uint32_t* Bv, const uint64_t* b_off, uint64_t total_b, uint64_t S,
                    void* C, uint32_t* Cv, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!key_type_ok(kt)) return CM_EDTYPE;
  const bool with_val = Av || Bv || Cv;
  if (with_val && (!Av && total_a)) return CM_EINVAL;
  if (with_val && ((!Bv && total_b) || !Cv)) return CM_EINVAL;
  if (total_a + total_b < total_a) return CM_EINVAL;
  const uint64_t N = total_a + total_b;
  if (S >= (1ull << 32)) return CM_EINVAL;
  if (S == 0) return N == 0 ? CM_OK : CM_EINVAL;
  if (!a_off || !b_off) return CM_EINVAL;
  const size_t ks = key_bytes(kt);
  if ((total_a && !A) || (total_b && !B) || (N && !C)) return CM_EINVAL;
  if (overlap(C, N * ks, A, total_a * ks) || overlap(C, N * ks, B, total_b * ks) ||
      overlap(C, N * ks, a_off, (S + 1) * 8) || overlap(C, N * ks, b_off, (S + 1) * 8))
    return CM_EALIAS;
  if (with_val && (overlap(Cv, N * 4, Av, total_a * 4) || overlap(Cv, N * 4, Bv, total_b * 4) ||
                   overlap(Cv, N * 4, A, total_a * ks) || overlap(Cv, N * 4, B, total_b * ks) ||
                   overlap(Cv, N * 4, C, N * ks) || overlap(Cv, N * 4, a_off, (S + 1) * 8) ||
                   overlap(Cv, N * 4, b_off, (S + 1) * 8)))
    return CM_EALIAS;
  const uint64_t T = tile_of(kt, with_val);
  const uint64_t tiles = (N + T - 1) / T;
  if (tiles >= (1ull << 31)) return CM_EINVAL;
  SegWorkspace w = seg_layout(ws, tiles);
  if (!ws || ws_bytes < w.bytes) return CM_ENOSPC;
  if (overlap(ws, w.bytes, C, N * ks) || overlap(ws, w.bytes, a_off, (S + 1) * 8) ||
      overlap(ws, w.bytes, b_off, (S + 1) * 8))
    return CM_EALIAS;
  hipLaunchKernelGGL(k_seg_validate, dim3(1), dim3(1024), 0, st, a_off, b_off, S, total_a, total_b, w.flag);
  if (launch_status() != CM_OK) return CM_EHIP;
  if (N == 0) return CM_OK;
  int rc;
  switch (kt) {
    case CM_KEY_U32:
      rc = launch_seg_bounds_t<uint32_t>(A, a_off, B, b_off, (uint32_t)S, N, T, tiles + 1, w.bj, w.bs, w.flag, st);
      break;
    case CM_KEY_U64:
      rc = launch_seg_bounds_t<uint64_t>(A, a_off, B, b_off, (uint32_t)S, N, T, tiles + 1, w.bj, w.bs, w.flag, st);
      break;
    default:
      rc = launch_seg_bounds_t<float>(A, a_off, B, b_off, (uint32_t)S, N, T, tiles + 1, w.bj, w.bs, w.flag, st);
      break;
  }
  if (rc != CM_OK) return rc;
  const int cfg = g_cfg[kt][with_val ? 1 : 0];
  const uint32_t S32 = (uint32_t)S;
  if (with_val) {
    switch (kt) {
      case CM_KEY_U32:
        return launch_seg_cfg<uint32_t, true>(cfg, A, Av, a_off, B, Bv, b_off, S32, N, C, Cv, w.bj, w.bs, tiles,
                                              w.flag, st);
      case CM_KEY_U64:
        return launch_seg_cfg<uint64_t, true>(cfg, A, Av, a_off, B, Bv, b_off, S32, N, C, Cv, w.bj, w.bs, tiles,
                                              w.flag, st);
      default:
        return launch_seg_cfg<float, true>(cfg, A, Av, a_off, B, Bv, b_off, S32, N, C, Cv, w.bj, w.bs, tiles,
                                           w.flag, st);
    }
  }
  switch (kt) {
    case CM_KEY_U32:
      return launch_seg_cfg<uint32_t, false>(cfg, A, Av, a_off, B, Bv, b_off, S32, N, C, Cv, w.bj, w.bs, tiles,
                                             w.flag, st);
    case CM_KEY_U64:
      return launch_seg_cfg<uint64_t, false>(cfg, A, Av, a_off, B, Bv, b_off, S32, N, C, Cv, w.bj, w.bs, tiles,
                                             w.flag, st);
    default:
      return launch_seg_cfg<float, false>(cfg, A, Av, a_off, B, Bv, b_off, S32, N, C, Cv, w.bj, w.bs, tiles,
                                          w.flag, st);
  }
}

}  // namespace cm

// ---------------------------------------------------------------------------
// C ABI

using namespace cm;

extern "C" {

const char* cm_status_string(int status) {
  switch (status) {
    case CM_OK: return "ok";
    case CM_EINVAL: return "invalid argument";
    case CM_ERANGE: return "rank out of range";
    case CM_EDTYPE: return "unknown key type";
    case CM_EALIAS: return "output overlaps an input";
    case CM_ENOSPC: return "workspace too small";
    case CM_EHIP: return "HIP runtime error";
    case CM_EUNSORTED: return "array not sorted";
    case CM_ECONFIG: return "unknown tile configuration";
    default: return "unknown status";
  }
}

int cm_version(void) { return 1; }

int cm_co_rank(int key_type, const uint64_t* ranks, uint64_t q, const void* A, uint64_t m, const void* B,
               uint64_t n, uint64_t* j_out, hipStream_t stream) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (m + n < m) return CM_EINVAL;
  if ((m && !A) || (n && !B) || (q && (!ranks || !j_out))) return CM_EINVAL;
  const size_t ks = key_bytes(key_type);
  if (overlap(j_out, q * 8, ranks, q * 8) || overlap(j_out, q * 8, A, m * ks) || overlap(j_out, q * 8, B, n * ks))
    return CM_EALIAS;
  if (q == 0) return CM_OK;
  const uint64_t blocks = (q + 255) / 256;
  if (blocks >= (1ull << 31)) return CM_EINVAL;
  switch (key_type) {
    case CM_KEY_U32:
      hipLaunchKernelGGL(k_co_rank_many<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, stream, ranks, q,
                         (const uint32_t*)A, m, (const uint32_t*)B, n, j_out, g_search);
      break;
    case CM_KEY_U64:
      hipLaunchKernelGGL(k_co_rank_many<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, stream, ranks, q,
                         (const uint64_t*)A, m, (const uint64_t*)B, n, j_out, g_search);
      break;
    default:
      hipLaunchKernelGGL(k_co_rank_many<float>, dim3((unsigned)blocks), dim3(256), 0, stream, ranks, q,
                         (const float*)A, m, (const float*)B, n, j_out, g_search);
      break;
  }
  return launch_status();
}

size_t cm_merge_workspace_size(int key_type, int with_payload, uint64_t m, uint64_t n) {
  if (!key_type_ok(key_type) || m + n == 0) return 0;
  const uint64_t T = tile_of(key_type, with_payload != 0);
  const uint64_t tiles = (m + n + T - 1) / T;
  return round256((tiles + 1) * sizeof(uint64_t));
}

int cm_stable_merge(int key_type, const void* A, uint64_t m, const void* B, uint64_t n, void* C, void* workspace,
                    size_t workspace_bytes, hipStream_t stream) {
  return merge_impl(key_type, false, A, nullptr, m, B, nullptr, n, C, nullptr, workspace, workspace_bytes, stream);
}

int cm_stable_merge_pairs(int key_type, const void* A, const uint32_t* A_val, uint64_t m, const void* B,
                          const uint32_t* B_val, uint64_t n, void* C, uint32_t* C_val, void* workspace,
                          size_t workspace_bytes, hipStream_t stream) {
  return merge_impl(key_type, true, A, A_val, m, B, B_val, n, C, C_val, workspace, workspace_bytes, stream);
}

size_t cm_segmented_workspace_size(int key_type, int with_payload, uint64_t total_a, uint64_t total_b,
                                   uint64_t num_seg) {
  (void)num_seg;
  if (!key_type_ok(key_type)) return 0;
  const uint64_t T = tile_of(key_type, with_payload != 0);
  const uint64_t tiles = (total_a + total_b + T - 1) / T;
  return seg_layout(nullptr, tiles).bytes;
}

int cm_stable_merge_segmented(int key_type, const void* A, const uint32_t* A_val, const uint64_t* a_off,
                              uint64_t total_a, const void* B, const uint32_t* B_val, const uint64_t* b_off,
                              uint64_t total_b, uint64_t num_seg, void* C, uint32_t* C_val, void* workspace,
                              size_t workspace_bytes, hipStream_t stream) {
  return seg_impl(key_type, A, A_val, a_off, total_a, B, B_val, b_off, total_b, num_seg, C, C_val, workspace,
                  workspace_bytes, stream);
}

int cm_check_sorted(int key_type, const void* X, uint64_t len, uint32_t* flag, hipStream_t stream) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (!flag || (len && !X)) return CM_EINVAL;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, stream, flag, 0u);
  if (launch_status() != CM_OK) return CM_EHIP;
  if (len < 2) return CM_OK;
  const uint64_t blocks = std::min<uint64_t>((len + 255) / 256, 4096);
  switch (key_type) {
    case CM_KEY_U32:
      hipLaunchKernelGGL(k_check_sorted<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, stream,
                         (const uint32_t*)X, len, flag);
      break;
    case CM_KEY_U64:
      hipLaunchKernelGGL(k_check_sorted<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, stream,
                         (const uint64_t*)X, len, flag);
      break;
    default:
      hipLaunchKernelGGL(k_check_sorted<float>, dim3((unsigned)blocks), dim3(256), 0, stream, (const float*)X,
                         len, flag);
      break;
  }
  return launch_status();
}

int cm_config_count(void) { return kNumCfgs; }

int cm_config_info(int config_id, int* threads, int* items_per_thread) {
  if (config_id < 0 || config_id >= kNumCfgs) return CM_ECONFIG;
  if (threads) *threads = kCfgs[config_id].nt;
  if (items_per_thread) *items_per_thread = kCfgs[config_id].e;
  return CM_OK;
}

int cm_set_config(int key_type, int with_payload, int config_id) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (config_id < 0 || config_id >= kNumCfgs) return CM_ECONFIG;
  g_cfg[key_type][with_payload ? 1 : 0] = config_id;
  return CM_OK;
}

int cm_get_config(int key_type, int with_payload) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  return g_cfg[key_type][with_payload ? 1 : 0];
}

int cm_set_search(int search_mode) {
  if (search_mode != kSearchAlg1 && search_mode != kSearchBisect) return CM_EINVAL;
  g_search = search_mode;
  return CM_OK;
}

}  // extern "C"
