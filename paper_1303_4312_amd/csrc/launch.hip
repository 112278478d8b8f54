// Kernel launchers: template dispatch over key type, payload mode and tile
// configuration.  No argument checking happens here (see internal.hpp).
#include <hip/hip_runtime.h>

#include <stddef.h>
#include <string.h>

#include <map>
#include <mutex>
#include <type_traits>

#include "corank_merge.h"
#include "dispatch.hpp"
#include "internal.hpp"
#include "kernels.hpp"
#include "launch_decl.hpp"

namespace cm {

// The key-dependent launchers are instantiated in launch_keys_*.hip (one file
// per key width, compiled side by side); only the dispatch lives here.
extern template struct Launch<uint32_t>;
extern template struct Launch<Desc<uint32_t>>;
extern template struct Launch<uint64_t>;
extern template struct Launch<Desc<uint64_t>>;
extern template struct Launch<float>;
extern template struct Launch<Desc<float>>;

// ---- scratch of the allocation-free entry point

// The block co-ranks of cm_stable_merge_pairs_noalloc.  Each GPU holds its
// own copy of the array for the life of the process.  In host code the
// name stands for the array but is not a device address: the address is
// looked up per device and kept (noalloc_scratch), and only that is ever
// handed to a kernel.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

int noalloc_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return CM_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return CM_EINVAL;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {  // once per device, with that device current
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return CM_EHIP;
    }
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return CM_OK;
}

// ---- non-template kernels (launched from this file only)

// flag |= 1 if the offsets are inconsistent (not starting at 0, decreasing
// somewhere, or not ending at the host totals).  Grid-stride over the
// segments; the flag is cleared by k_fill_u32 before.  Every later kernel of
// the call reads the flag and does nothing when it is set.
__global__ __launch_bounds__(256) void k_seg_validate(const uint64_t* __restrict__ a_off,
                                                      const uint64_t* __restrict__ b_off, uint64_t S,
                                                      uint64_t total_a, uint64_t total_b,
                                                      uint32_t* __restrict__ flag) {
  int bad = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += stride)
    if (a_off[s] > a_off[s + 1] || b_off[s] > b_off[s + 1]) bad = 1;
  if (blockIdx.x == 0 && threadIdx.x == 0 &&
      (a_off[0] != 0 || b_off[0] != 0 || a_off[S] != total_a || b_off[S] != total_b))
    bad = 1;
  if (__any(bad) && (threadIdx.x % warpSize) == 0) atomicOr(flag, 1u);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v) { *p = v; }

// Merges whose first_block values a prep workgroup holds in LDS.
constexpr uint32_t kPrepTable = 2048;

// First kernel of every batch call but the single-launch form: copies the
// descriptors into the workspace (wd) from the kernel arguments (src null)
// or from src, which may be device memory or host memory the device reads
// (pinned), so that the later kernels read device memory only; and notes
// for every boundary slot and every block the merge it belongs to (sm, bm),
// so that no later kernel searches the descriptors.  The search runs over
// an LDS copy of first_block when the batch has at most kPrepTable merges.
__global__ __launch_bounds__(256) void k_batch_prep(DescPack pk, const MergeDesc* __restrict__ src, uint32_t count,
                                                    uint64_t num_slots, uint64_t num_blocks,
                                                    MergeDesc* __restrict__ wd, uint32_t* __restrict__ sm,
                                                    uint32_t* __restrict__ bm) {
  __shared__ uint64_t s_fb[kPrepTable];
  const bool table = count <= kPrepTable;  // grid-uniform
  auto fb_src = [&](uint32_t r) -> uint64_t {
    return src ? src[r].first_block : pk.d[r < kInlineDescs ? r : 0].first_block;
  };
  if (table)
    for (uint32_t x = threadIdx.x; x < count; x += blockDim.x) s_fb[x] = fb_src(x);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (uint64_t x = gid; x < count; x += stride) wd[x] = src ? src[x] : pk.d[x < kInlineDescs ? x : 0];
  __syncthreads();
  for (uint64_t b = gid; b < num_slots; b += stride) {
    if (table) {
      auto fb = [&](uint32_t r) { return s_fb[r]; };
      sm[b] = merge_of(fb, count, b, 1);
      if (b < num_blocks) bm[b] = merge_of(fb, count, b, 0);
    } else {
      sm[b] = merge_of(fb_src, count, b, 1);
      if (b < num_blocks) bm[b] = merge_of(fb_src, count, b, 0);
    }
  }
}

int launch_batch_prep(const void* h, const void* d, uint32_t count, uint64_t slots, uint64_t blocks, void* wd,
                      uint32_t* sm, uint32_t* bm, hipStream_t st) {
  DescPack pk;
  memset(&pk, 0, sizeof pk);
  if (!d && h) memcpy(pk.d, h, (size_t)std::min(count, kInlineDescs) * sizeof(MergeDesc));
  const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>((slots + 255) / 256, 1024));
  hipLaunchKernelGGL(k_batch_prep, dim3((unsigned)grid), dim3(256), 0, st, pk, (const MergeDesc*)d, count, slots,
                     blocks, (MergeDesc*)wd, sm, bm);
  return launch_status();
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Plain streaming copy, 16 bytes per lane per step, grid-stride.
__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                uint64_t count) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < count; x += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + x), dst + x);
}

// The data movement of a block merge (uint32 keys + uint32 payloads) in its
// tile structure, without the merge: workgroup b takes tile t (XCD order as
// the merge), stages the windows A[ja, jb) and B[q0 - ja, q1 - jb) (units of
// 16 bytes; ja = floor(q0 * mq / Nq), the A share of the tile's first
// output, exact) in LDS with 16-byte loads issued before the first LDS
// write, waits at a barrier, and stores the tile with 16-byte stores, A's
// window first.
template <int NT, int E>
__global__ __launch_bounds__(NT) void k_copy_tiles(const u32x4* __restrict__ A, const u32x4* __restrict__ Av,
                                                   uint64_t mq, const u32x4* __restrict__ B,
                                                   const u32x4* __restrict__ Bv, uint64_t nq, u32x4* __restrict__ C,
                                                   u32x4* __restrict__ Cv, uint64_t tiles, int xcd) {
  constexpr int TQ = NT * E / 4;  // 16-byte units per tile
  constexpr int R = (TQ + NT - 1) / NT;
  __shared__ u32x4 sk[TQ];
  __shared__ u32x4 sv[TQ];
  const uint64_t Nq = mq + nq;
  const uint64_t t = block_order(blockIdx.x, tiles, xcd);
  const uint64_t q0 = t * (uint64_t)TQ;
  const uint64_t q1 = std::min(q0 + (uint64_t)TQ, Nq);
  const uint64_t ja = q0 * mq / Nq, jb = q1 * mq / Nq;  // Nq < 2^32: no overflow
  const int len = (int)(q1 - q0), na = (int)(jb - ja);
  const uint64_t kb = q0 - ja;
  u32x4 rk[R], rv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int x0 = (int)threadIdx.x + r * NT;
    const int x = x0 < len ? x0 : 0;  // a slot past the tile re-reads its first unit
    const bool from_a = x < na;
    const uint64_t g = from_a ? ja + (uint64_t)x : kb + (uint64_t)(x - na);
    rk[r] = __builtin_nontemporal_load((from_a ? A : B) + g);
    rv[r] = __builtin_nontemporal_load((from_a ? Av : Bv) + g);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int x = (int)threadIdx.x + r * NT;
    if (x < len) {
      sk[x] = rk[r];
      sv[x] = rv[r];
    }
  }
  __syncthreads();
  for (int x = (int)threadIdx.x; x < len; x += NT) {
    __builtin_nontemporal_store(sk[x], C + q0 + x);
    __builtin_nontemporal_store(sv[x], Cv + q0 + x);
  }
}

// Puts the 2h cuts in output order (A's cut first on equal ranks, which are
// the same cut) and closes with (m + n, m): I / J get 2h + 1 entries.
__global__ __launch_bounds__(256) void k_cross_rank_place(const uint64_t* __restrict__ ia,
                                                          const uint64_t* __restrict__ ja,
                                                          const uint64_t* __restrict__ ib,
                                                          const uint64_t* __restrict__ jb, uint32_t h,
                                                          uint64_t N, uint64_t m, uint64_t* __restrict__ I,
                                                          uint64_t* __restrict__ J) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x == 0) {
    I[2ull * h] = N;
    J[2ull * h] = m;
  }
  if (x >= 2ull * h) return;
  const bool from_a = x < h;
  const uint64_t r = from_a ? x : x - h;
  const uint64_t key = from_a ? ia[r] : ib[r];
  const uint64_t* other = from_a ? ib : ia;
  uint64_t lo = 0, hi = h;  // cuts of the other side before this one
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (from_a ? other[mid] < key : other[mid] <= key) lo = mid + 1; else hi = mid;
  }
  I[r + lo] = key;
  J[r + lo] = from_a ? ja[r] : jb[r];
}

// Segment starts of the equal split (co-rank partition with P segments).
__global__ __launch_bounds__(256) void k_equal_starts(uint64_t N, uint32_t P, uint64_t* __restrict__ I) {
  const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w <= P) I[w] = stream_block_start(w, N, P);
}

// ---- payloads of any width (records moved by origin code) -----------------

// A_codes[x] = x, B_codes[y] = 2^31 + y (the origin of each element).
__global__ __launch_bounds__(256) void k_origin_codes(uint64_t m, uint64_t n, uint32_t* __restrict__ A_codes,
                                                      uint32_t* __restrict__ B_codes) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m + n; x += stride) {
    if (x < m)
      A_codes[x] = (uint32_t)x;
    else
      B_codes[x - m] = 0x80000000u | (uint32_t)(x - m);
  }
}

// out[i] = record codes[i] of A (code < 2^31) or of B (code - 2^31), each
// record W bytes, moved in words of U bytes (U divides W and every base is
// U-aligned).  Codes outside A and B leave the record untouched.
template <typename U>
__global__ __launch_bounds__(256) void k_gather_records(const uint32_t* __restrict__ codes, uint64_t N,
                                                        const U* __restrict__ A_rec, uint64_t m,
                                                        const U* __restrict__ B_rec, uint64_t n, uint64_t words,
                                                        U* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N * words; t += stride) {
    const uint64_t i = t / words, w = t - i * words;
    const uint32_t c = codes[i];
    const U* src = nullptr;
    if (c < 0x80000000u) {
      if (c < m) src = A_rec + (uint64_t)c * words;
    } else if ((uint64_t)(c & 0x7fffffffu) < n) {
      src = B_rec + (uint64_t)(c & 0x7fffffffu) * words;
    }
    if (src) out[i * words + w] = src[w];
  }
}

int launch_origin_codes(uint64_t m, uint64_t n, uint32_t* A_codes, uint32_t* B_codes, hipStream_t st) {
  const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>((m + n + 255) / 256, 8192));
  hipLaunchKernelGGL(k_origin_codes, dim3((unsigned)blocks), dim3(256), 0, st, m, n, A_codes, B_codes);
  return launch_status();
}

int launch_gather_records(const uint32_t* codes, uint64_t N, const void* A_rec, uint64_t m, const void* B_rec,
                          uint64_t n, uint64_t width, void* out, hipStream_t st) {
  auto aligned = [&](uintptr_t u) {
    return width % u == 0 && ((uintptr_t)A_rec % u) == 0 && ((uintptr_t)B_rec % u) == 0 &&
           ((uintptr_t)out % u) == 0;
  };
  auto go = [&](auto word) {
    using U = decltype(word);
    const uint64_t words = width / sizeof(U);
    const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>((N * words + 255) / 256, 16384));
    hipLaunchKernelGGL((k_gather_records<U>), dim3((unsigned)blocks), dim3(256), 0, st, codes, N, (const U*)A_rec,
                       m, (const U*)B_rec, n, words, (U*)out);
  };
  if (aligned(16))
    go(u32x4{});
  else if (aligned(8))
    go(uint64_t{});
  else if (aligned(4))
    go(uint32_t{});
  else
    go(uint8_t{});
  return launch_status();
}

int launch_block_co_ranks(int kt, const Choice& ch, const Shape& sh, const void* A, uint64_t m, const void* B,
                          uint64_t n, uint64_t tile, uint64_t nb, uint64_t* bj, uint64_t* coarse, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int { return Launch<decltype(key)>::block_co_ranks(ch, sh, A, m, B, n, tile, nb, bj, coarse, st); });
}

int launch_merge_blocks(int kt, bool val, int vbytes, const Choice& ch, const Shape& sh, const void* A,
                        const void* Av, uint64_t m, const void* B, const void* Bv, uint64_t n, void* C, void* Cv,
                        const uint64_t* bj, uint64_t tiles, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int {
    return Launch<decltype(key)>::merge_blocks(val, vbytes, ch, sh, A, Av, m, B, Bv, n, C, Cv, bj, tiles, st);
  });
}

// Resident workgroups per CU of `kernel` at nt threads, times the CU count;
// cached per kernel (the library drives one device type).
uint32_t resident_workgroups(const void* kernel, int nt) {
  static std::mutex mu;
  static std::map<const void*, uint32_t> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(kernel);
    if (it != cache.end()) return it->second;
  }
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) != hipSuccess || cus <= 0 ||
      per_cu <= 0) {
    (void)hipGetLastError();
    return 256;  // a safe count for any device: correctness never depends on it
  }
  const uint32_t r = (uint32_t)cus * (uint32_t)per_cu;
  std::lock_guard<std::mutex> lk(mu);
  cache[kernel] = r;
  return r;
}

uint32_t stream_blocks(int kt, bool val, const Choice& ch, uint64_t N) {
  const uint64_t T = tile_size(ch.cfg);
  const uint64_t tiles = (N + T - 1) / T;
  const int res = by_key(kt, [&](auto key) -> int { return Launch<decltype(key)>::stream_resident(val, ch.cfg); });
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(res > 0 ? (uint64_t)res : 256, tiles));
}

int launch_stream_co_ranks(int kt, const void* A, uint64_t m, const void* B, uint64_t n, uint32_t P, uint64_t* J,
                           hipStream_t st) {
  return by_key(kt, [&](auto key) -> int { return Launch<decltype(key)>::stream_co_ranks(A, m, B, n, P, J, st); });
}

int launch_merge_stream(int kt, bool val, const Choice& ch, const void* A, const uint32_t* Av, uint64_t m,
                        const void* B, const uint32_t* Bv, uint64_t n, void* C, uint32_t* Cv, const uint64_t* I,
                        const uint64_t* J, uint32_t P, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int { return Launch<decltype(key)>::merge_stream(val, ch, A, Av, m, B, Bv, n, C, Cv, I, J, P, st); });
}

int launch_cross_rank_cuts(int kt, const void* A, uint64_t m, const void* B, uint64_t n, uint32_t h, uint64_t* cuts,
                           uint64_t* I, uint64_t* J, hipStream_t st) {
  uint64_t* ia = cuts;
  uint64_t* ja = cuts + h;
  uint64_t* ib = cuts + 2ull * h;
  uint64_t* jb = cuts + 3ull * h;
  const unsigned blocks = (unsigned)((2ull * h + 255) / 256);
  const int rc = by_key(kt, [&](auto key) -> int {
    return Launch<decltype(key)>::cross_rank_cuts(A, m, B, n, h, ia, ja, ib, jb, blocks, st);
  });
  if (rc != CM_OK) return rc;
  hipLaunchKernelGGL(k_cross_rank_place, dim3(blocks), dim3(256), 0, st, (const uint64_t*)ia, (const uint64_t*)ja,
                     (const uint64_t*)ib, (const uint64_t*)jb, h, m + n, m, I, J);
  return launch_status();
}

int launch_equal_starts(uint64_t N, uint32_t P, uint64_t* I, hipStream_t st) {
  hipLaunchKernelGGL(k_equal_starts, dim3((unsigned)(((uint64_t)P + 1 + 255) / 256)), dim3(256), 0, st, N, P, I);
  return launch_status();
}

int launch_seg_validate(const uint64_t* a_off, const uint64_t* b_off, uint64_t S, uint64_t total_a,
                        uint64_t total_b, uint32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, st, flag, 0u);
  if (launch_status() != CM_OK) return CM_EHIP;
  const uint64_t blocks = std::max<uint64_t>(1, std::min<uint64_t>((S + 255) / 256, 2048));
  hipLaunchKernelGGL(k_seg_validate, dim3((unsigned)blocks), dim3(256), 0, st, a_off, b_off, S, total_a, total_b,
                     flag);
  return launch_status();
}

int launch_seg_block_co_ranks(int kt, const Choice& ch, const Shape& sh, const void* A, const uint64_t* a_off,
                              const void* B, const uint64_t* b_off, uint32_t S, uint64_t N, uint64_t tile,
                              uint64_t nb, uint64_t* bj, uint32_t* bs, uint64_t* jc, uint32_t* sc,
                              const uint32_t* flag, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int { return Launch<decltype(key)>::seg_block_co_ranks(ch, sh, A, a_off, B, b_off, S, N, tile, nb, bj, bs, jc, sc, flag, st); });
}

int launch_seg_merge_blocks(int kt, bool val, const Choice& ch, const void* A, const uint32_t* Av,
                            const uint64_t* a_off, const void* B, const uint32_t* Bv, const uint64_t* b_off,
                            uint32_t S, uint64_t N, void* C, uint32_t* Cv, const uint64_t* bj, const uint32_t* bs,
                            uint64_t tiles, const uint32_t* flag, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int { return Launch<decltype(key)>::seg_merge_blocks(val, ch, A, Av, a_off, B, Bv, b_off, S, N, C, Cv, bj, bs, tiles, flag, st); });
}

static_assert(sizeof(MergeDesc) == sizeof(cm_merge_desc), "descriptor layouts differ");
static_assert(offsetof(MergeDesc, first_block) == offsetof(cm_merge_desc, first_block), "descriptor layouts differ");

int launch_batch_co_ranks(int kt, const Choice& ch, const Shape& sh, const void* d, const uint32_t* sm,
                          uint64_t tile, uint64_t nb, uint64_t* bj, uint64_t* coarse, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int {
    return Launch<decltype(key)>::batch_co_ranks(ch, sh, d, sm, tile, nb, bj, coarse, st);
  });
}

int launch_batch_merge_blocks(int kt, bool val, const Choice& ch, int form, const void* h, const void* d,
                              uint32_t count, const uint32_t* bm, const uint64_t* bj, uint64_t tiles, bool vec,
                              int xcd, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int {
    return Launch<decltype(key)>::batch_merge_blocks(val, ch, form, h, d, count, bm, bj, tiles, vec, xcd, st);
  });
}

int launch_co_rank_many(int kt, int search, const uint64_t* ranks, uint64_t q, const void* A, uint64_t m,
                        const void* B, uint64_t n, uint64_t* j_out, hipStream_t st) {
  return by_key(kt, [&](auto key) -> int { return Launch<decltype(key)>::co_rank_many(search, ranks, q, A, m, B, n, j_out, st); });
}

int launch_check_sorted(int kt, const void* X, uint64_t len, uint32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, st, flag, 0u);
  const int rc = launch_status();
  if (rc != CM_OK || len < 2) return rc;
  const uint64_t blocks = std::min<uint64_t>((len + 255) / 256, 4096);
  return by_key(kt, [&](auto key) -> int { return Launch<decltype(key)>::check_sorted(X, len, flag, blocks, st); });
}

int launch_copy_tiles(int cfg, int xcd, const void* A, const uint32_t* Av, uint64_t m, const void* B,
                      const uint32_t* Bv, uint64_t n, void* C, uint32_t* Cv, hipStream_t st) {
  return by_cfg(cfg, [&](auto nt, auto e) -> int {
    constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
    static_assert((NT * E) % 4 == 0, "tiles must hold whole 16-byte units");
    const uint64_t TQ = NT * E / 4, Nq = (m + n) / 4, tiles = (Nq + TQ - 1) / TQ;
    hipLaunchKernelGGL((k_copy_tiles<NT, E>), dim3((unsigned)tiles), dim3(NT), 0, st, (const u32x4*)A,
                       (const u32x4*)Av, m / 4, (const u32x4*)B, (const u32x4*)Bv, n / 4, (u32x4*)C, (u32x4*)Cv,
                       tiles, xcd);
    return launch_status();
  });
}

int launch_copy16(const void* src, void* dst, uint64_t count16, hipStream_t st) {
  // one 16-byte vector per thread where the grid allows, grid-stride beyond
  const uint64_t blocks = std::min<uint64_t>((count16 + 255) / 256, 1ull << 30);
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, st, (const u32x4*)src, (u32x4*)dst, count16);
  return launch_status();
}

}  // namespace cm
