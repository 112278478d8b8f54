// Internal interface between the C ABI (api.cpp) and the kernel launchers
// (launch.hip).  Launchers do no argument checking: the C ABI validates every
// pointer, size and overlap before calling them.  Each returns CM_OK or
// CM_EHIP (launch failure).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include <initializer_list>

namespace cm {

struct TileCfg {
  int nt;  // threads per workgroup
  int e;   // outputs per thread; a block of Algorithm 2 is nt * e outputs
};

extern const TileCfg kCfgs[];
extern const int kNumCfgs;
// Smallest block over all configurations (sizes workspaces so that any
// configuration fits).
extern const uint64_t kMinTile;

// The coarse pass of the two-level boundary scheme searches every
// coarse_stride-th block boundary (at least kMinCoarse, which sizes the
// workspace).
constexpr uint32_t kMinCoarse = 16;

enum Op : int { kOpMerge = 0, kOpSegmented = 1, kOpBatch = 2, kOpSort = 3 };

// How one call runs.
struct Choice {
  int cfg;        // index into kCfgs
  int search;     // per-thread and one-level boundary search: 0 Alg. 1, 1 bisection
  int partition;  // block-boundary pass: 0 one thread per boundary; 1 two-level with a
                  // 64-lane coarse search; 2 two-level with a 16-lane coarse search;
                  // 3 one block per resident workgroup (streaming kernel); 4 no pass,
                  // each block co-ranks its own ends
  int grid = 0;   // workgroups of the block kernels: 0 one per block; -1 as many as
                  // are resident on the device at once; g > 0 at most g (the
                  // workgroups then stride over the blocks)
};

// Workgroups of `kernel` (nt threads each) resident on the whole device at
// once (CUs x occupancy), cached per kernel; 256 if the runtime cannot say.
uint32_t resident_workgroups(const void* kernel, int nt);

// Grid of a block-kernel launch over `tiles` blocks for the choice's grid
// setting (never more workgroups than blocks, at least one).
inline unsigned launch_grid(const void* kernel, int nt, uint64_t tiles, int grid) {
  if (grid == 0 || tiles == 0) return (unsigned)tiles;
  const uint64_t g = grid > 0 ? (uint64_t)grid : (uint64_t)resident_workgroups(kernel, nt);
  return (unsigned)(g < tiles ? (g ? g : 1) : tiles);
}
constexpr int kMaxPartition = 4;
// Every device array of a call holds fewer elements than this, so that no
// byte count or index sum of the host-side checks can wrap (2^48 elements of
// 8 bytes is far beyond one GPU's memory).
constexpr uint64_t kMaxLen = 1ull << 48;
inline bool lengths_ok(uint64_t a, uint64_t b) { return a < kMaxLen && b < kMaxLen; }
// Automatic boundary pass: single merges of fewer outputs than this skip the
// pass (mode 4); larger ones, and batches, use the two-level pass (mode 2).
// Measured on MI355X (uint32 pairs, back-to-back calls): with the 512 x 11
// tile (fewest blocks, so fewest in-block searches) mode 4 takes 14.5 us at
// 2^22 outputs against 20.9-24.8 us with the pass, 35.0 against 35.5-38.6 us
// at 2^23, and draws level at 2^24; the 256 x 7 tile loses from 2^22.  Keys
// only: 10.9 us at 2^22 against 17.7-20.0 us, 23.4 against 25.5 us at 2^23,
// and the pass ahead at 2^24.
constexpr uint64_t kInBlockBelow = 1ull << 24;
constexpr uint64_t kInBlockWideFrom = 1ull << 21;      // from here mode 4 takes the widest tile
constexpr uint64_t kInBlockWideKeysFrom = 1ull << 22;  // the same, keys only
constexpr int kInBlockWideCfg = 7;                     // 512 x 11

// Launch-shape settings that never change results.
struct Shape {
  uint32_t coarse_stride = 64;  // blocks between coarse boundaries
  // Block order of the single-merge and batch kernels (block_order): runs of
  // 32 blocks per XCD.  Measured on MI355X against one contiguous run per XCD
  // (same process, the eight tiles): 3-6 % less time per call for the uint32
  // Zipf merge, 3-9 % for uint64 keys, 3-5 % for float32; runs of 64 within
  // 1 % of 32; workgroup order 0-4 % slower than one run per XCD.  A batch of
  // 64 serving-sized merges: 1-2.5 % faster than workgroup order (8,192
  // small merges: equal).  The segmented kernel keeps workgroup order (runs
  // measured 1-4 % slower there).
  int xcd_order = 32;
  int fine_lanes = 1;           // lanes per boundary in the fine pass (1: bisection; 2, 4)
};

inline uint64_t tile_size(int cfg) { return (uint64_t)kCfgs[cfg].nt * (uint64_t)kCfgs[cfg].e; }
inline uint64_t num_coarse(uint64_t nb, uint32_t stride) { return (nb - 1 + stride - 1) / stride + 1; }

// Block-boundary co-ranks of one merge: bj[t] = A co-rank of min(t * tile, m + n)
// for t < nb.  `coarse` holds num_coarse(nb, sh.coarse_stride) entries
// (two-level pass only).
int launch_block_co_ranks(int kt, const Choice& ch, const Shape& sh, const void* A, uint64_t m, const void* B,
                          uint64_t n, uint64_t tile, uint64_t nb, uint64_t* bj, uint64_t* coarse, hipStream_t st);

// Every pointer 16-byte aligned (the block merge then moves data with
// 16-byte accesses; blocks start at multiples of 4 outputs).
inline bool all_aligned16(std::initializer_list<const void*> ps) {
  for (const void* p : ps)
    if (((uintptr_t)p & 15) != 0) return false;
  return true;
}

// Merge sort (sort.hip): sort every run of sort_run_blocks(kt, val, cfg)
// blocks of T = tile_size(cfg) elements of X into Y (`runs` of them); then
// one pass merging runs of 2^(sh-1) blocks (T << (sh - 1) elements) of X
// pairwise into Y (block co-ranks in bj, `tiles` entries).
uint32_t sort_run_blocks(int kt, bool val, int cfg);
int launch_sort_blocks(int kt, bool val, const Choice& ch, const void* X, const uint32_t* Xv, uint64_t N, void* Y,
                       uint32_t* Yv, uint64_t runs, hipStream_t st);
// ch.partition 0: one thread per block start, bisection over its pair;
// otherwise, for pairs longer than shape.coarse_stride blocks, two levels
// (coarse holds ceil(tiles / coarse_stride) entries), the fine step with
// shape.fine_lanes lanes per block start.
int launch_sort_pass(int kt, bool val, const Choice& ch, const Shape& shape, const void* X, const uint32_t* Xv,
                     uint64_t N, int sh, void* Y, uint32_t* Yv, uint64_t* bj, uint64_t* coarse, uint64_t tiles,
                     hipStream_t st);

// Block merge of one merge over `tiles` blocks whose boundary co-ranks are bj
// (bj == nullptr: each block searches its own two boundary co-ranks).
// Payloads (with val) are vbytes = 4 or 8 bytes wide.
int launch_merge_blocks(int kt, bool val, int vbytes, const Choice& ch, const Shape& sh, const void* A,
                        const void* Av, uint64_t m, const void* B, const void* Bv, uint64_t n, void* C, void* Cv,
                        const uint64_t* bj, uint64_t tiles, hipStream_t st);

// Algorithm 2 with one block per resident workgroup: the number of blocks P
// the streaming kernel uses for an N-output merge (resident workgroups of the
// chip, at most one per T outputs), its P + 1 boundary co-ranks, and the
// kernel.  J holds P + 1 entries.
uint32_t stream_blocks(int kt, bool val, const Choice& ch, uint64_t N);
int launch_stream_co_ranks(int kt, const void* A, uint64_t m, const void* B, uint64_t n, uint32_t P, uint64_t* J,
                           hipStream_t st);
int launch_merge_stream(int kt, bool val, const Choice& ch, const void* A, const uint32_t* Av, uint64_t m,
                        const void* B, const uint32_t* Bv, uint64_t n, void* C, uint32_t* Cv, const uint64_t* I,
                        const uint64_t* J, uint32_t P, hipStream_t st);
// The classic cross-rank partition into P = 2h segments: the 2h sample cuts
// (cuts: 4h uint64 of scratch) in output order into I, J (2h + 1 entries);
// and the starts of the equal split into P segments (I, P + 1 entries).
int launch_cross_rank_cuts(int kt, const void* A, uint64_t m, const void* B, uint64_t n, uint32_t h, uint64_t* cuts,
                           uint64_t* I, uint64_t* J, hipStream_t st);
int launch_equal_starts(uint64_t N, uint32_t P, uint64_t* I, hipStream_t st);
// Payloads of any width: origin codes of A and B, and the gather of W-byte
// records by code.
int launch_origin_codes(uint64_t m, uint64_t n, uint32_t* A_codes, uint32_t* B_codes, hipStream_t st);
int launch_gather_records(const uint32_t* codes, uint64_t N, const void* A_rec, uint64_t m, const void* B_rec,
                          uint64_t n, uint64_t width, void* out, hipStream_t st);

// Segmented batch: offset check, boundary co-ranks (and segments), block merge.
int launch_seg_validate(const uint64_t* a_off, const uint64_t* b_off, uint64_t S, uint64_t total_a,
                        uint64_t total_b, uint32_t* flag, hipStream_t st);
// With ch.partition != 0 and coarse scratch (jc, sc: num_coarse(nb, stride)
// entries each), the boundaries are found in two levels.
int launch_seg_block_co_ranks(int kt, const Choice& ch, const Shape& sh, const void* A, const uint64_t* a_off,
                              const void* B, const uint64_t* b_off, uint32_t S, uint64_t N, uint64_t tile,
                              uint64_t nb, uint64_t* bj, uint32_t* bs, uint64_t* jc, uint32_t* sc,
                              const uint32_t* flag, hipStream_t st);
int launch_seg_merge_blocks(int kt, bool val, const Choice& ch, const void* A, const uint32_t* Av,
                            const uint64_t* a_off, const void* B, const uint32_t* Bv, const uint64_t* b_off,
                            uint32_t S, uint64_t N, void* C, uint32_t* Cv, const uint64_t* bj, const uint32_t* bs,
                            uint64_t tiles, const uint32_t* flag, hipStream_t st);

// Batch of separately allocated merges.
// launch_batch_prep: copies the descriptors into the workspace (wd, count
// entries) from d (device memory, or pinned host memory the device reads)
// or, with d null, from the host array h (at most kBatchInline, passed in
// the kernel arguments); and fills sm (per boundary slot) and bm (per
// block) with the merge each belongs to.  slots = blocks + count.
// launch_batch_co_ranks: the boundary pass over the prep's tables and
// copy (d): ch.partition 0 one-level, 1 or 2 two-level (coarse slots
// searched by 64 or 16 lanes; `coarse` holds ceil(nb / sh.coarse_stride)
// entries).
// launch_batch_merge_blocks, `form`: kBatchPassFed (bj from the pass),
// kBatchSelf (after prep, every block co-ranks its own ends), kBatchArgs
// (no prep: descriptors from h in the kernel arguments, count <=
// kBatchInline, every block finds its merge and co-ranks its ends).
constexpr uint32_t kBatchInline = 16;
enum BatchForm : int { kBatchPassFed = 0, kBatchSelf = 1, kBatchArgs = 2 };

// The allocation-free single merge keeps its block co-ranks in a scratch
// array of this many bytes in the library's device code (one per GPU);
// noalloc_scratch gives its device address on the current device (looked
// up once per device with hipGetSymbolAddress), or CM_EHIP.
constexpr size_t kNoAllocScratchBytes = 4u << 20;
int noalloc_scratch(void** out);
int launch_batch_prep(const void* h, const void* d, uint32_t count, uint64_t slots, uint64_t blocks, void* wd,
                      uint32_t* sm, uint32_t* bm, hipStream_t st);
int launch_batch_co_ranks(int kt, const Choice& ch, const Shape& sh, const void* d, const uint32_t* sm,
                          uint64_t tile, uint64_t nb, uint64_t* bj, uint64_t* coarse, hipStream_t st);
int launch_batch_merge_blocks(int kt, bool val, const Choice& ch, int form, const void* h, const void* d,
                              uint32_t count, const uint32_t* bm, const uint64_t* bj, uint64_t tiles, bool vec,
                              int xcd, hipStream_t st);

// Co-ranks of q arbitrary ranks.
int launch_co_rank_many(int kt, int search, const uint64_t* ranks, uint64_t q, const void* A, uint64_t m,
                        const void* B, uint64_t n, uint64_t* j_out, hipStream_t st);

// flag := 0, then flag |= (some X[x-1] > X[x]).
int launch_check_sorted(int kt, const void* X, uint64_t len, uint32_t* flag, hipStream_t st);

// Streaming copy of count16 16-byte vectors.
int launch_copy16(const void* src, void* dst, uint64_t count16, hipStream_t st);
int launch_copy_tiles(int cfg, int xcd, const void* A, const uint32_t* Av, uint64_t m, const void* B,
                      const uint32_t* Bv, uint64_t n, void* C, uint32_t* Cv, hipStream_t st);

}  // namespace cm
