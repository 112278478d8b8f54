// C ABI of the co-rank stable merge (see include/corank_merge.h): argument
// checks, the per-call choice of tile configuration and co-rank strategy,
// the tuning table and autotuner, graph plans, kernel timing, and the
// per-merge-launch baseline.  Kernel launches live in launch.hip.
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "corank_merge.h"
#include "internal.hpp"

#ifndef CM_BUILD_ID
#define CM_BUILD_ID "unversioned"
#endif

static_assert(cm::kBatchInline == CM_BATCH_INLINE_MAX, "inline descriptor counts differ");
static_assert(cm::kNoAllocScratchBytes == CM_NOALLOC_SCRATCH_BYTES, "scratch sizes differ");

namespace cm {

// Tile configurations (the cases of by_cfg in dispatch.hpp, which
// instantiates every one for every key type and payload mode, must match).
// E is odd so that the strided LDS accesses of the transposes (stride E
// words) fall on distinct banks.
const TileCfg kCfgs[] = {{256, 7}, {256, 11}, {256, 15}, {128, 7}, {512, 7}, {256, 5}, {256, 9}, {512, 11}};
const int kNumCfgs = (int)(sizeof(kCfgs) / sizeof(kCfgs[0]));
const uint64_t kMinTile = 128 * 7;  // smallest nt * e in kCfgs

namespace {

// ---------------------------------------------------------------------------
// process-wide settings

struct Settings {
  int cfg[CM_KEY_F32_DESC + 1][2] = {};       // [key type][payload] default configuration (0)
  bool cfg_set[CM_KEY_F32_DESC + 1][2] = {};  // set by the caller (else the defaults of resolve)
  int search = 1;                             // bisection
  int partition = -1;                         // automatic (see resolve)
  int grid = 0;                               // block-kernel grid (Choice::grid)
  Shape shape;                                // coarse stride, block order
};
Settings g_set;

// Tuning table: (op, key type, payload, size class) -> choice.  The size
// class of a merge of N outputs is the bit length of N.
using TuneKey = std::tuple<int, int, int, int>;
struct TuneEntry {
  Choice ch;
  double ms;
};
std::map<TuneKey, TuneEntry> g_tuning;
std::mutex g_tuning_mu;

int size_class(uint64_t N) { return N ? 64 - __builtin_clzll(N) : 0; }

// Default tiles where the process-wide configuration has not been set for
// the key type (measured on MI355X): a merge sort with payloads, 256 x 9
// (fastest of the eight at 2^26 and 2^28 uint32 keys, within 1 % of the best
// for 2^26 and 2^27 uint64 keys); without payloads 256 x 11 for 4-byte keys
// (8.3 ms for 2^28 uint32 keys against 9.9 ms at 256 x 7) and 256 x 9 for
// uint64 keys (6.9 ms for 2^27 against 7.7 ms); a single merge of keys without payloads, 256 x 9 (within 4 % of
// the best tile for uint32, uint64 and float32 keys at 2^27-2^28 per side,
// where 256 x 7 is up to 39 % slower); a segmented batch and a batch of
// separate merges, 256 x 15 (the 65,536-segment batch: 1.17 ms keys only
// against 1.65 ms at 256 x 7, 2.04 ms against 2.10 ms with payloads; the
// serving runtime's batches: 131k against 123k requests/s at saturation).
constexpr int kSortCfg = 6;
constexpr int kSortKeysCfg = 1;
constexpr int kKeysMergeCfg = 6;
constexpr int kSegCfg = 2;

Choice resolve(int op, int kt, bool val, uint64_t N) {
  {
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    auto it = g_tuning.find(TuneKey{op, kt, val ? 1 : 0, size_class(N)});
    if (it != g_tuning.end()) {
      Choice c = it->second.ch;
      c.grid = g_set.grid;
      return c;
    }
  }
  int part = g_set.partition;
  const bool auto_part = part < 0;
  if (auto_part)  // automatic: small single merges skip the boundary pass
    part = (op == kOpMerge && N < kInBlockBelow) ? 4 : 2;
  int cfg = g_set.cfg[kt][val ? 1 : 0];
  if (!g_set.cfg_set[kt][val ? 1 : 0]) {
    if (op == kOpMerge) {
      if (auto_part && part == 4 && N >= (val ? kInBlockWideFrom : kInBlockWideKeysFrom))
        cfg = kInBlockWideCfg;  // the widest tile: fewest blocks, so fewest in-block searches
      else
        cfg = val ? 0 : kKeysMergeCfg;
    }
    if (op == kOpSort) cfg = (val || kt == CM_KEY_U64 || kt == CM_KEY_U64_DESC) ? kSortCfg : kSortKeysCfg;
    if (op == kOpSegmented || op == kOpBatch) cfg = kSegCfg;
  }
  return Choice{cfg, g_set.search, part, g_set.grid};
}

// ---------------------------------------------------------------------------
// kernel timing (three events per timed call)

struct Timing {
  bool on = false;
  uint32_t capacity = 0;
  uint32_t used = 0;
  hipEvent_t* ev = nullptr;
};
Timing g_timing;
bool g_capturing = false;  // graph capture in progress: record no timing events

void timing_mark(int slot, hipStream_t st) {
  if (!g_timing.on || g_capturing || g_timing.used >= g_timing.capacity) return;
  (void)hipEventRecord(g_timing.ev[3ull * g_timing.used + slot], st);
  if (slot == 2) ++g_timing.used;
}

// ---------------------------------------------------------------------------
// checks

bool key_type_ok(int kt) { return kt >= CM_KEY_U32 && kt <= CM_KEY_F32_DESC; }
size_t key_bytes(int kt) { return kt == CM_KEY_U64 || kt == CM_KEY_U64_DESC ? 8 : 4; }
size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

bool overlap(const void* p, uint64_t pbytes, const void* q, uint64_t qbytes) {
  if (!p || !q || pbytes == 0 || qbytes == 0) return false;
  const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
  return a < b + qbytes && b < a + pbytes;
}

// A region and its size, for overlap checks.
struct Span {
  const void* p;
  uint64_t bytes;
};

bool any_overlap(std::initializer_list<Span> outs, std::initializer_list<Span> ins) {
  for (const Span& o : outs) {
    for (const Span& i : ins)
      if (overlap(o.p, o.bytes, i.p, i.bytes)) return true;
  }
  // outputs must not overlap each other either
  for (auto a = outs.begin(); a != outs.end(); ++a)
    for (auto b = a + 1; b != outs.end(); ++b)
      if (overlap(a->p, a->bytes, b->p, b->bytes)) return true;
  return false;
}

// Workspace of a single merge: block co-ranks + coarse co-ranks, sized for
// the smallest block of any configuration.
size_t merge_ws_bytes(uint64_t N) {
  const uint64_t nb = (N + kMinTile - 1) / kMinTile + 1;
  return round256(nb * sizeof(uint64_t)) + round256(num_coarse(nb, kMinCoarse) * sizeof(uint64_t));
}

struct SegWs {
  uint32_t* flag;
  uint64_t* bj;  // block boundary co-ranks
  uint32_t* bs;  // block boundary segments
  uint64_t* jc;  // coarse boundary co-ranks (two-level pass)
  uint32_t* sc;  // coarse boundary segments
  size_t bytes;
};

// The parts of a segmented merge's workspace at ws (all null when ws is
// null: then only the byte count is wanted).
SegWs seg_ws(void* ws, uint64_t N) {
  const uint64_t nb = (N + kMinTile - 1) / kMinTile + 1;
  const uint64_t nc = num_coarse(nb, kMinCoarse);
  const size_t o_bj = 256;
  const size_t o_bs = o_bj + round256(nb * sizeof(uint64_t));
  const size_t o_jc = o_bs + round256(nb * sizeof(uint32_t));
  const size_t o_sc = o_jc + round256(nc * sizeof(uint64_t));
  char* p = (char*)ws;
  SegWs w;
  w.flag = (uint32_t*)p;
  w.bj = p ? (uint64_t*)(p + o_bj) : nullptr;
  w.bs = p ? (uint32_t*)(p + o_bs) : nullptr;
  w.jc = p ? (uint64_t*)(p + o_jc) : nullptr;
  w.sc = p ? (uint32_t*)(p + o_sc) : nullptr;
  w.bytes = o_sc + round256(nc * sizeof(uint32_t));
  return w;
}

// ---------------------------------------------------------------------------
// implementations

// With dry_run set, only the argument checks run (nothing is launched).
// Payloads (with val) are vb = 4 or 8 bytes wide.
int merge_impl(int kt, bool val, int vb, const void* A, const void* Av, uint64_t m, const void* B, const void* Bv,
               uint64_t n, void* C, void* Cv, void* ws, size_t ws_bytes, hipStream_t st,
               const Choice* forced = nullptr, bool dry_run = false) {
  if (!key_type_ok(kt)) return CM_EDTYPE;
  if (!lengths_ok(m, n)) return CM_EINVAL;
  const uint64_t N = m + n;
  const size_t ks = key_bytes(kt);
  if ((m && !A) || (n && !B) || (N && !C)) return CM_EINVAL;
  if (val && ((m && !Av) || (n && !Bv) || (N && !Cv))) return CM_EINVAL;
  if (N == 0) return CM_OK;
  const size_t need = merge_ws_bytes(N);
  if (!ws || ws_bytes < need) return CM_ENOSPC;
  const uint64_t vs = val ? (uint64_t)vb : 0;
  const Span ins[] = {{A, m * ks}, {B, n * ks}, {Av, m * vs}, {Bv, n * vs}};
  if (any_overlap({{C, N * ks}, {Cv, N * vs}, {ws, need}}, {ins[0], ins[1], ins[2], ins[3]})) return CM_EALIAS;
  Choice ch = forced ? *forced : resolve(kOpMerge, kt, val, N);
  if (vb == 8 && ch.partition == 3) ch.partition = 2;  // the streaming kernel moves 4-byte payloads only
  const uint64_t T = tile_size(ch.cfg);
  const uint64_t tiles = (N + T - 1) / T;
  if (tiles >= (1ull << 31)) return CM_EINVAL;
  if (dry_run) return CM_OK;
  uint64_t* bj = (uint64_t*)ws;
  uint64_t* coarse = (uint64_t*)((char*)ws + round256(((N + kMinTile - 1) / kMinTile + 1) * sizeof(uint64_t)));
  if (ch.partition == 3) {  // one block per resident workgroup; P + 1 <= tiles + 1 co-ranks fit bj
    const uint32_t P = stream_blocks(kt, val, ch, N);
    timing_mark(0, st);
    int rc = launch_stream_co_ranks(kt, A, m, B, n, P, bj, st);
    if (rc != CM_OK) return rc;
    timing_mark(1, st);
    rc = launch_merge_stream(kt, val, ch, A, (const uint32_t*)Av, m, B, (const uint32_t*)Bv, n, C, (uint32_t*)Cv,
                             nullptr, bj, P, st);
    timing_mark(2, st);
    return rc;
  }
  if (ch.partition == 4) {  // every block co-ranks its own ends: no boundary pass
    timing_mark(0, st);
    timing_mark(1, st);
    const int rc = launch_merge_blocks(kt, val, vb, ch, g_set.shape, A, Av, m, B, Bv, n, C, Cv, nullptr, tiles, st);
    timing_mark(2, st);
    return rc;
  }
  timing_mark(0, st);
  int rc = launch_block_co_ranks(kt, ch, g_set.shape, A, m, B, n, T, tiles + 1, bj, coarse, st);
  if (rc != CM_OK) return rc;
  timing_mark(1, st);
  rc = launch_merge_blocks(kt, val, vb, ch, g_set.shape, A, Av, m, B, Bv, n, C, Cv, bj, tiles, st);
  timing_mark(2, st);
  return rc;
}

int seg_impl(int kt, const void* A, const uint32_t* Av, const uint64_t* a_off, uint64_t total_a, const void* B,
             const uint32_t* Bv, const uint64_t* b_off, uint64_t total_b, uint64_t S, void* C, uint32_t* Cv,
             void* ws, size_t ws_bytes, hipStream_t st, const Choice* forced = nullptr, bool dry_run = false) {
  if (!key_type_ok(kt)) return CM_EDTYPE;
  const bool val = Av || Bv || Cv;
  if (!lengths_ok(total_a, total_b)) return CM_EINVAL;
  const uint64_t N = total_a + total_b;
  if (val && ((total_a && !Av) || (total_b && !Bv) || (N && !Cv))) return CM_EINVAL;
  if (S >= (1ull << 32)) return CM_EINVAL;
  if (S == 0) return N == 0 ? CM_OK : CM_EINVAL;
  if (!a_off || !b_off) return CM_EINVAL;
  const size_t ks = key_bytes(kt);
  if ((total_a && !A) || (total_b && !B) || (N && !C)) return CM_EINVAL;
  const SegWs w = seg_ws(ws, N);
  if (!ws || ws_bytes < w.bytes) return CM_ENOSPC;
  if (any_overlap({{C, N * ks}, {Cv, val ? N * 4 : 0}, {ws, w.bytes}},
                  {{A, total_a * ks}, {B, total_b * ks}, {Av, val ? total_a * 4 : 0}, {Bv, val ? total_b * 4 : 0},
                   {a_off, (S + 1) * 8}, {b_off, (S + 1) * 8}}))
    return CM_EALIAS;
  const Choice ch = forced ? *forced : resolve(kOpSegmented, kt, val, N);
  const uint64_t T = tile_size(ch.cfg);
  const uint64_t tiles = (N + T - 1) / T;
  if (tiles >= (1ull << 31)) return CM_EINVAL;
  if (dry_run) return CM_OK;
  if (N == 0) return launch_seg_validate(a_off, b_off, S, total_a, total_b, w.flag, st);
  timing_mark(0, st);
  int rc = launch_seg_validate(a_off, b_off, S, total_a, total_b, w.flag, st);
  if (rc == CM_OK)
    rc = launch_seg_block_co_ranks(kt, ch, g_set.shape, A, a_off, B, b_off, (uint32_t)S, N, T, tiles + 1, w.bj,
                                   w.bs, w.jc, w.sc, w.flag, st);
  if (rc != CM_OK) return rc;
  timing_mark(1, st);
  rc = launch_seg_merge_blocks(kt, val, ch, A, Av, a_off, B, Bv, b_off, (uint32_t)S, N, C, Cv, w.bj, w.bs, tiles,
                               w.flag, st);
  timing_mark(2, st);
  return rc;
}

// Is there a tuning-table entry for this call?
bool tuned(int op, int kt, bool val, uint64_t N) {
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  return g_tuning.count(TuneKey{op, kt, val ? 1 : 0, size_class(N)}) != 0;
}

// Block size and boundary mode of a batch of separate merges (from its
// total output count).  Automatically: no pass (mode 4) for a batch of at
// most kBatchInline merges, each below kInBlockBelow outputs (one launch,
// descriptors in the kernel arguments; measured on the serving runtime's
// low-load batches: p50 0.067-0.073 ms and 2.8-3.0 TB/s while busy,
// against 0.079-0.085 ms and 2.1-2.3 TB/s with a pass), else the two-level
// pass.
Choice batch_choice(int kt, bool val, const cm_merge_desc* d, uint32_t count) {
  uint64_t N = 0, largest = 0;
  for (uint32_t r = 0; r < count; ++r) {  // saturating: only the size class matters here
    const uint64_t x = d[r].m + d[r].n;
    N = (x < d[r].m || N + x < N) ? UINT64_MAX : N + x;
    largest = std::max(largest, x < d[r].m ? UINT64_MAX : x);
  }
  Choice ch = resolve(kOpBatch, kt, val, N);
  if (ch.partition == 3) ch.partition = 2;  // no streaming form for batches: the two-level pass
  if (g_set.partition < 0 && !tuned(kOpBatch, kt, val, N) && count <= kBatchInline && largest < kInBlockBelow)
    ch.partition = 4;
  return ch;
}

// Workspace of a batch: one co-rank per boundary slot (a slot per block end
// of every merge), the coarse slots of the two-level pass (every
// kMinCoarse-th slot at most), and one merge index per block.
uint64_t batch_slots(uint64_t total_blocks, uint32_t count) { return total_blocks + count; }
size_t batch_coarse_offset(uint64_t total_blocks, uint32_t count) {
  return round256(batch_slots(total_blocks, count) * sizeof(uint64_t));
}
size_t batch_index_offset(uint64_t total_blocks, uint32_t count) {  // per block: its merge
  const uint64_t nb = batch_slots(total_blocks, count);
  return batch_coarse_offset(total_blocks, count) + round256((nb + kMinCoarse - 1) / kMinCoarse * sizeof(uint64_t));
}
size_t batch_slot_index_offset(uint64_t total_blocks, uint32_t count) {  // per slot: its merge
  return batch_index_offset(total_blocks, count) + round256(total_blocks * sizeof(uint32_t));
}
size_t batch_descs_offset(uint64_t total_blocks, uint32_t count) {  // the descriptors' device copy
  return batch_slot_index_offset(total_blocks, count) + round256(batch_slots(total_blocks, count) * sizeof(uint32_t));
}

// ---- stable merge sort

// Workspace of a sort: a second key (and payload) buffer for the passes,
// one block co-rank per block and one coarse co-rank per coarse_stride-th
// block (both sized for the smallest block and stride).
size_t sort_ws_bytes(int kt, bool val, uint64_t N) {
  if (N == 0) return 0;
  const uint64_t nb = (N + kMinTile - 1) / kMinTile;
  return round256(N * key_bytes(kt)) + (val ? round256(N * 4) : 0) + round256((nb + 1) * sizeof(uint64_t)) +
         round256(num_coarse(nb, kMinCoarse) * sizeof(uint64_t));
}

int sort_impl(int kt, bool val, const void* X, const uint32_t* Xv, uint64_t N, void* Y, uint32_t* Yv, void* ws,
              size_t ws_bytes, hipStream_t st) {
  if (!key_type_ok(kt)) return CM_EDTYPE;
  if (!lengths_ok(N, 0) || (N && (!X || !Y))) return CM_EINVAL;
  if (val && N && (!Xv || !Yv)) return CM_EINVAL;
  if (N == 0) return CM_OK;
  const size_t ks = key_bytes(kt);
  const size_t need = sort_ws_bytes(kt, val, N);
  if (!ws || ws_bytes < need) return CM_ENOSPC;
  // outputs may be the inputs themselves (in place) but must not overlap them otherwise
  const Span yk{Y == X ? nullptr : Y, N * ks};
  const Span yv{val && Yv != Xv ? Yv : nullptr, val ? N * 4 : 0};
  if (any_overlap({yk, yv, {ws, need}}, {{X, N * ks}, {Xv, val ? N * 4 : 0}}) ||
      any_overlap({{Y, N * ks}, {Yv, val ? N * 4 : 0}, {ws, need}}, {}))
    return CM_EALIAS;
  const Choice ch = resolve(kOpSort, kt, val, N);
  const uint64_t T = tile_size(ch.cfg);
  const uint64_t tiles = (N + T - 1) / T;
  if (tiles >= (1ull << 31)) return CM_EINVAL;
  // the first sorted runs are M blocks long (M a power of two), so the
  // first pass merges pairs of 2M blocks: shift log2(M) + 1
  const uint32_t M = sort_run_blocks(kt, val, ch.cfg);
  int sh0 = 1;
  while ((1u << (sh0 - 1)) < M) ++sh0;
  int passes = 0;
  for (uint64_t L = T * M; L < N; L *= 2) ++passes;
  char* w = (char*)ws;
  void* bk[2] = {Y, w};
  uint32_t* bv[2] = {Yv, val ? (uint32_t*)(w + round256(N * ks)) : nullptr};
  uint64_t* bj = (uint64_t*)(w + round256(N * ks) + (val ? round256(N * 4) : 0));
  uint64_t* coarse = (uint64_t*)((char*)bj + round256(((N + kMinTile - 1) / kMinTile + 1) * sizeof(uint64_t)));
  // ping-pong between Y and the workspace so that the last pass writes Y
  int cur = passes % 2;
  int rc = launch_sort_blocks(kt, val, ch, X, val ? Xv : nullptr, N, bk[cur], bv[cur], (N + T * M - 1) / (T * M), st);
  for (int sh = sh0; rc == CM_OK && sh < sh0 + passes; ++sh) {  // runs of T << (sh - 1)
    rc = launch_sort_pass(kt, val, ch, g_set.shape, bk[cur], bv[cur], N, sh, bk[cur ^ 1], bv[cur ^ 1], bj, coarse,
                          tiles, st);
    cur ^= 1;
  }
  return rc;
}

// Do any of the byte ranges in `outs` overlap each other or any range in
// `ins`?  Sorting keeps this O((outs + ins) log outs) for large batches.
bool spans_overlap(std::vector<Span>& outs, const std::vector<Span>& ins) {
  outs.erase(std::remove_if(outs.begin(), outs.end(), [](const Span& s) { return !s.p || !s.bytes; }),
             outs.end());
  std::sort(outs.begin(), outs.end(), [](const Span& a, const Span& b) { return a.p < b.p; });
  for (size_t x = 1; x < outs.size(); ++x)
    if (overlap(outs[x - 1].p, outs[x - 1].bytes, outs[x].p, outs[x].bytes)) return true;
  for (const Span& in : ins) {
    if (!in.p || !in.bytes) continue;
    // first output starting at or after the input's end cannot overlap; check the one before
    auto it = std::lower_bound(outs.begin(), outs.end(), in,
                               [](const Span& o, const Span& v) { return (uintptr_t)o.p < (uintptr_t)v.p; });
    if (it != outs.end() && overlap(it->p, it->bytes, in.p, in.bytes)) return true;
    if (it != outs.begin() && overlap((it - 1)->p, (it - 1)->bytes, in.p, in.bytes)) return true;
  }
  return false;
}

// Mean milliseconds of `reps` calls of f() on stream st (after one warm call).
template <typename F>
int time_calls(F&& f, int reps, hipStream_t st, double* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return CM_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return CM_EHIP;
  }
  int rc = f();
  if (rc == CM_OK && hipEventRecord(e0, st) != hipSuccess) rc = CM_EHIP;
  for (int r = 0; r < reps && rc == CM_OK; ++r) rc = f();
  if (rc == CM_OK && hipEventRecord(e1, st) != hipSuccess) rc = CM_EHIP;
  float t = 0;
  if (rc == CM_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    rc = CM_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return rc;
}

// The autotuner's choice among `cands`: every candidate is timed once
// (time(ch, &ms): mean of reps calls), then the kTuneFinalists fastest are
// timed again kTuneRounds times, round-robin, so that drift over the sweep
// affects them alike; the winner has the lowest of its timings.  (Single
// sweeps picked tiles within noise of each other, up to 3 % off the best.)
constexpr size_t kTuneFinalists = 4;
constexpr int kTuneRounds = 3;
template <typename F>
int tune_pick(const std::vector<Choice>& cands, F&& time, Choice* win, double* win_ms) {
  std::vector<std::pair<double, size_t>> first;
  first.reserve(cands.size());
  for (size_t c = 0; c < cands.size(); ++c) {
    double ms = 0;
    const int rc = time(cands[c], &ms);
    if (rc != CM_OK) return rc;
    first.emplace_back(ms, c);
  }
  std::sort(first.begin(), first.end());
  const size_t k = std::min(kTuneFinalists, first.size());
  std::vector<double> best(k);
  for (size_t f = 0; f < k; ++f) best[f] = first[f].first;
  for (int round = 0; round < kTuneRounds; ++round)
    for (size_t f = 0; f < k; ++f) {
      double ms = 0;
      const int rc = time(cands[first[f].second], &ms);
      if (rc != CM_OK) return rc;
      best[f] = std::min(best[f], ms);
    }
  size_t w = 0;
  for (size_t f = 1; f < k; ++f)
    if (best[f] < best[w]) w = f;
  *win = cands[first[w].second];
  *win_ms = best[w];
  return CM_OK;
}

// Identity of a saved tuning table: the device architecture (gcnArchName
// of the current device; "none" without one), the HIP runtime version and
// the library's build id (a hash of its sources).
struct Identity {
  std::string arch = "none";
  int runtime = 0;
  std::string build = CM_BUILD_ID;
};

Identity current_identity() {
  Identity id;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.gcnArchName[0])
    id.arch = prop.gcnArchName;
  int v = 0;
  if (hipRuntimeGetVersion(&v) == hipSuccess) id.runtime = v;
  (void)hipGetLastError();  // no device is not an error of later calls
  return id;
}

// The tuning file: `path`, or with path null $CM_TUNING_FILE, else
// $XDG_CACHE_HOME/corank_merge/tuning.txt, else
// $HOME/.cache/corank_merge/tuning.txt.  For a save of the default file its
// directories are created.
bool tuning_path(const char* path, bool for_save, std::string* out) {
  if (path) {
    *out = path;
    return true;
  }
  const char* env = getenv("CM_TUNING_FILE");
  if (env && *env) {
    *out = env;
    return true;
  }
  std::string dir;
  const char* xdg = getenv("XDG_CACHE_HOME");
  const char* home = getenv("HOME");
  if (xdg && *xdg)
    dir = xdg;
  else if (home && *home)
    dir = std::string(home) + "/.cache";
  else
    return false;
  if (for_save) {
    (void)mkdir(dir.c_str(), 0755);
    (void)mkdir((dir + "/corank_merge").c_str(), 0755);
  }
  *out = dir + "/corank_merge/tuning.txt";
  return true;
}

}  // namespace
}  // namespace cm

// ---------------------------------------------------------------------------
// C ABI

using namespace cm;

struct cm_plan {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int kind = 0;  // 0: single merge, 1: segmented batch
};

extern "C" {

const char* cm_status_string(int status) {
  switch (status) {
    case CM_OK: return "ok";
    case CM_EINVAL: return "invalid argument";
    case CM_ERANGE: return "rank out of range";
    case CM_EDTYPE: return "unknown key type";
    case CM_EALIAS: return "output overlaps an input";
    case CM_ENOSPC: return "workspace or arena too small";
    case CM_EHIP: return "HIP runtime error";
    case CM_EUNSORTED: return "array not sorted";
    case CM_ECONFIG: return "unknown tile configuration";
    case CM_EBUSY: return "every request slot is taken";
    case CM_ECANCELED: return "canceled at shutdown";
    case CM_ESTALE: return "tuning table made for another device, runtime or library build";
    default: return "unknown status";
  }
}

int cm_version(void) { return 2; }

int cm_co_rank(int key_type, const uint64_t* ranks, uint64_t q, const void* A, uint64_t m, const void* B,
               uint64_t n, uint64_t* j_out, hipStream_t stream) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (!lengths_ok(m, n) || !lengths_ok(q, 0)) return CM_EINVAL;
  if ((m && !A) || (n && !B) || (q && (!ranks || !j_out))) return CM_EINVAL;
  const size_t ks = key_bytes(key_type);
  if (any_overlap({{j_out, q * 8}}, {{ranks, q * 8}, {A, m * ks}, {B, n * ks}})) return CM_EALIAS;
  if (q == 0) return CM_OK;
  if ((q + 255) / 256 >= (1ull << 31)) return CM_EINVAL;
  return launch_co_rank_many(key_type, g_set.search, ranks, q, A, m, B, n, j_out, stream);
}

size_t cm_merge_workspace_size(int key_type, int with_payload, uint64_t m, uint64_t n) {
  (void)with_payload;
  if (!key_type_ok(key_type) || m + n == 0) return 0;
  return merge_ws_bytes(m + n);
}

int cm_stable_merge(int key_type, const void* A, uint64_t m, const void* B, uint64_t n, void* C, void* workspace,
                    size_t workspace_bytes, hipStream_t stream) {
  return merge_impl(key_type, false, 4, A, nullptr, m, B, nullptr, n, C, nullptr, workspace, workspace_bytes, stream);
}

int cm_stable_merge_pairs(int key_type, const void* A, const uint32_t* A_val, uint64_t m, const void* B,
                          const uint32_t* B_val, uint64_t n, void* C, uint32_t* C_val, void* workspace,
                          size_t workspace_bytes, hipStream_t stream) {
  return merge_impl(key_type, true, 4, A, A_val, m, B, B_val, n, C, C_val, workspace, workspace_bytes, stream);
}

int cm_stable_merge_pairs_noalloc(int key_type, const void* A, const uint32_t* A_val, uint64_t m, const void* B,
                                  const uint32_t* B_val, uint64_t n, void* C, uint32_t* C_val, hipStream_t stream) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (!lengths_ok(m, n)) return CM_EINVAL;
  const bool val = A_val || B_val || C_val;
  // the block co-ranks must fit the scratch array (checked before anything
  // touches the device)
  if (merge_ws_bytes(m + n) > kNoAllocScratchBytes) return CM_ENOSPC;
  void* ws = nullptr;
  if (m + n) {
    const int rc = noalloc_scratch(&ws);
    if (rc != CM_OK) return rc;
  }
  return merge_impl(key_type, val, 4, A, A_val, m, B, B_val, n, C, C_val, ws, kNoAllocScratchBytes, stream);
}

int cm_stable_merge_pairs64(int key_type, const void* A, const uint64_t* A_val, uint64_t m, const void* B,
                            const uint64_t* B_val, uint64_t n, void* C, uint64_t* C_val, void* workspace,
                            size_t workspace_bytes, hipStream_t stream) {
  return merge_impl(key_type, true, 8, A, A_val, m, B, B_val, n, C, C_val, workspace, workspace_bytes, stream);
}

size_t cm_segmented_workspace_size(int key_type, int with_payload, uint64_t total_a, uint64_t total_b,
                                   uint64_t num_seg) {
  (void)with_payload;
  (void)num_seg;
  if (!key_type_ok(key_type)) return 0;
  return seg_ws(nullptr, total_a + total_b).bytes;
}

int cm_stable_merge_segmented(int key_type, const void* A, const uint32_t* A_val, const uint64_t* a_off,
                              uint64_t total_a, const void* B, const uint32_t* B_val, const uint64_t* b_off,
                              uint64_t total_b, uint64_t num_seg, void* C, uint32_t* C_val, void* workspace,
                              size_t workspace_bytes, hipStream_t stream) {
  return seg_impl(key_type, A, A_val, a_off, total_a, B, B_val, b_off, total_b, num_seg, C, C_val, workspace,
                  workspace_bytes, stream);
}

int cm_stable_merge_segmented_each(int key_type, const void* A, const uint32_t* A_val, const uint64_t* a_off_host,
                                   uint64_t total_a, const void* B, const uint32_t* B_val,
                                   const uint64_t* b_off_host, uint64_t total_b, uint64_t num_seg, void* C,
                                   uint32_t* C_val, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  const bool val = A_val || B_val || C_val;
  if (num_seg == 0) return total_a + total_b == 0 ? CM_OK : CM_EINVAL;
  if (!a_off_host || !b_off_host) return CM_EINVAL;
  if (a_off_host[0] != 0 || b_off_host[0] != 0 || a_off_host[num_seg] != total_a ||
      b_off_host[num_seg] != total_b)
    return CM_EINVAL;
  for (uint64_t s = 0; s < num_seg; ++s)
    if (a_off_host[s] > a_off_host[s + 1] || b_off_host[s] > b_off_host[s + 1]) return CM_EINVAL;
  const size_t ks = key_bytes(key_type);
  const bool timing_was_on = g_timing.on;  // this form is not timed per kernel
  g_timing.on = false;
  int rc = CM_OK;
  for (uint64_t s = 0; s < num_seg && rc == CM_OK; ++s) {
    const uint64_t a0 = a_off_host[s], b0 = b_off_host[s];
    const uint64_t ms = a_off_host[s + 1] - a0, ns = b_off_host[s + 1] - b0;
    rc = merge_impl(key_type, val, 4, A ? (const char*)A + a0 * ks : nullptr, val && A_val ? A_val + a0 : nullptr, ms,
                    B ? (const char*)B + b0 * ks : nullptr, val && B_val ? B_val + b0 : nullptr, ns,
                    C ? (char*)C + (a0 + b0) * ks : nullptr, val && C_val ? C_val + a0 + b0 : nullptr, workspace,
                    workspace_bytes, stream);
  }
  g_timing.on = timing_was_on;
  return rc;
}

int cm_batch_prepare(int key_type, int with_payload, cm_merge_desc* descs, uint32_t count,
                     uint64_t* total_blocks) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if ((count && !descs) || !total_blocks) return CM_EINVAL;
  const Choice ch = batch_choice(key_type, with_payload != 0, descs, count);
  const uint64_t T = tile_size(ch.cfg);
  uint64_t blocks = 0;
  for (uint32_t r = 0; r < count; ++r) {
    if (!lengths_ok(descs[r].m, descs[r].n)) return CM_EINVAL;
    descs[r].first_block = blocks;
    blocks += (descs[r].m + descs[r].n + T - 1) / T;
    if (blocks >= (1ull << 31)) return CM_EINVAL;  // checked per merge: the sum cannot wrap
  }
  *total_blocks = blocks;
  return CM_OK;
}

size_t cm_batch_workspace_size(uint64_t total_blocks, uint32_t count) {
  return batch_descs_offset(total_blocks, count) + round256((uint64_t)count * sizeof(cm_merge_desc));
}

int cm_stable_merge_batch(int key_type, int with_payload, const cm_merge_desc* descs_host,
                          const cm_merge_desc* descs_dev, uint32_t count, uint64_t total_blocks, void* workspace,
                          size_t workspace_bytes, hipStream_t stream) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (count == 0) return total_blocks == 0 ? CM_OK : CM_EINVAL;
  // small batches may leave the descriptors on the host: they travel in the kernel arguments
  if (!descs_host || (!descs_dev && count > kBatchInline)) return CM_EINVAL;
  const bool val = with_payload != 0;
  const size_t ks = key_bytes(key_type);
  Choice ch = batch_choice(key_type, val, descs_host, count);
  const uint64_t T = tile_size(ch.cfg);
  std::vector<Span> outs, ins;
  outs.reserve(2 * (size_t)count + 1);
  ins.reserve(4 * (size_t)count + 1);
  uint64_t blocks = 0;
  bool vec = true;  // every array of every merge 16-byte aligned
  for (uint32_t r = 0; r < count; ++r) {
    const cm_merge_desc& q = descs_host[r];
    if (!lengths_ok(q.m, q.n)) return CM_EINVAL;
    const uint64_t N = q.m + q.n;
    if ((q.m && !q.A) || (q.n && !q.B) || (N && !q.C)) return CM_EINVAL;
    if (val && ((q.m && !q.A_val) || (q.n && !q.B_val) || (N && !q.C_val))) return CM_EINVAL;
    if (!val && (q.A_val || q.B_val || q.C_val)) return CM_EINVAL;
    if (q.first_block != blocks) return CM_EINVAL;
    blocks += (N + T - 1) / T;
    if (blocks >= (1ull << 31)) return CM_EINVAL;
    vec = vec && (val ? all_aligned16({q.A, q.B, q.C, q.A_val, q.B_val, q.C_val}) : all_aligned16({q.A, q.B, q.C}));
    outs.push_back({q.C, N * ks});
    if (val) outs.push_back({q.C_val, N * 4});
    ins.push_back({q.A, q.m * ks});
    ins.push_back({q.B, q.n * ks});
    if (val) {
      ins.push_back({q.A_val, q.m * 4});
      ins.push_back({q.B_val, q.n * 4});
    }
  }
  if (blocks != total_blocks || blocks >= (1ull << 31)) return CM_EINVAL;
  const size_t need = cm_batch_workspace_size(total_blocks, count);
  if (!workspace || workspace_bytes < need) return CM_ENOSPC;
  outs.push_back({workspace, need});
  if (descs_dev) ins.push_back({descs_dev, (uint64_t)count * sizeof(cm_merge_desc)});
  if (spans_overlap(outs, ins)) return CM_EALIAS;
  if (total_blocks == 0) return CM_OK;
  uint64_t* bj = (uint64_t*)workspace;
  uint64_t* coarse = (uint64_t*)((char*)workspace + batch_coarse_offset(total_blocks, count));
  uint32_t* bm = (uint32_t*)((char*)workspace + batch_index_offset(total_blocks, count));
  uint32_t* sm = (uint32_t*)((char*)workspace + batch_slot_index_offset(total_blocks, count));
  void* wd = (char*)workspace + batch_descs_offset(total_blocks, count);
  const uint64_t slots = batch_slots(total_blocks, count);
  // no pass: a small batch in one launch with its descriptors in the kernel
  // arguments; otherwise after the prep kernel.  With a pass: prep, pass, merge.
  const int form = ch.partition != 4 ? kBatchPassFed : count <= kBatchInline ? kBatchArgs : kBatchSelf;
  timing_mark(0, stream);
  if (form != kBatchArgs) {
    int rc = launch_batch_prep(descs_host, descs_dev, count, slots, total_blocks, wd, sm, bm, stream);
    if (rc == CM_OK && form == kBatchPassFed)
      rc = launch_batch_co_ranks(key_type, ch, g_set.shape, wd, sm, T, slots, bj, coarse, stream);
    if (rc != CM_OK) return rc;
  }
  timing_mark(1, stream);
  const int rc = launch_batch_merge_blocks(key_type, val, ch, form, descs_host, wd, count, bm, bj, total_blocks, vec,
                                           g_set.shape.xcd_order, stream);
  timing_mark(2, stream);
  return rc;
}

int cm_check_sorted(int key_type, const void* X, uint64_t len, uint32_t* flag, hipStream_t stream) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (!flag || (len && !X)) return CM_EINVAL;
  return launch_check_sorted(key_type, X, len, flag, stream);
}

// ---- configuration and settings

int cm_config_count(void) { return kNumCfgs; }

int cm_config_info(int config_id, int* threads, int* items_per_thread) {
  if (config_id < 0 || config_id >= kNumCfgs) return CM_ECONFIG;
  if (threads) *threads = kCfgs[config_id].nt;
  if (items_per_thread) *items_per_thread = kCfgs[config_id].e;
  return CM_OK;
}

int cm_set_config(int key_type, int with_payload, int config_id) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (config_id < -1 || config_id >= kNumCfgs) return CM_ECONFIG;
  // -1: back to the per-operation defaults of resolve()
  g_set.cfg[key_type][with_payload ? 1 : 0] = config_id < 0 ? 0 : config_id;
  g_set.cfg_set[key_type][with_payload ? 1 : 0] = config_id >= 0;
  return CM_OK;
}

int cm_get_config(int key_type, int with_payload) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  return g_set.cfg_set[key_type][with_payload ? 1 : 0] ? g_set.cfg[key_type][with_payload ? 1 : 0] : -1;
}

int cm_set_search(int search_mode) {
  if (search_mode != 0 && search_mode != 1) return CM_EINVAL;
  g_set.search = search_mode;
  return CM_OK;
}

int cm_get_search(void) { return g_set.search; }

int cm_set_partition(int partition_mode) {
  if (partition_mode < -1 || partition_mode > kMaxPartition) return CM_EINVAL;
  g_set.partition = partition_mode;
  return CM_OK;
}

int cm_get_partition(void) { return g_set.partition; }

int cm_set_coarse_stride(uint32_t blocks) {
  if (blocks < kMinCoarse || blocks > (1u << 20)) return CM_EINVAL;
  g_set.shape.coarse_stride = blocks;
  return CM_OK;
}

int cm_set_fine_lanes(int lanes) {
  if (lanes != 1 && lanes != 2 && lanes != 4) return CM_EINVAL;
  g_set.shape.fine_lanes = lanes;
  return CM_OK;
}

int cm_set_block_order(int order) {
  if (order < 0 || order > (1 << 20)) return CM_EINVAL;
  g_set.shape.xcd_order = order;
  return CM_OK;
}

int cm_get_block_order(void) { return g_set.shape.xcd_order; }

int cm_set_grid(int workgroups) {
  if (workgroups < -1) return CM_EINVAL;
  g_set.grid = workgroups;
  return CM_OK;
}

int cm_get_grid(void) { return g_set.grid; }
int cm_get_coarse_stride(void) { return (int)g_set.shape.coarse_stride; }
int cm_get_fine_lanes(void) { return g_set.shape.fine_lanes; }

// ---- autotuner

int cm_autotune_merge(int key_type, const void* A, const uint32_t* A_val, uint64_t m, const void* B,
                      const uint32_t* B_val, uint64_t n, void* C, uint32_t* C_val, void* workspace,
                      size_t workspace_bytes, int reps, hipStream_t stream, int* best) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (reps < 1 || reps > 10000 || m + n == 0) return CM_EINVAL;
  const bool val = A_val || B_val || C_val;
  const int check = merge_impl(key_type, val, 4, A, A_val, m, B, B_val, n, C, C_val, workspace, workspace_bytes,
                               stream, nullptr, true);
  if (check != CM_OK) return check;
  std::vector<Choice> cands;
  for (int cfg = 0; cfg < kNumCfgs; ++cfg)
    for (int search = 0; search < 2; ++search)
      for (int part = 0; part <= kMaxPartition; ++part) cands.push_back(Choice{cfg, search, part, g_set.grid});
  Choice win{0, 1, 1};
  double win_ms = 0;
  const int picked = tune_pick(
      cands,
      [&](const Choice& ch, double* ms) {
        return time_calls(
            [&] {
              return merge_impl(key_type, val, 4, A, A_val, m, B, B_val, n, C, C_val, workspace, workspace_bytes,
                                stream, &ch);
            },
            reps, stream, ms);
      },
      &win, &win_ms);
  if (picked != CM_OK) return picked;
  {
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    g_tuning[TuneKey{kOpMerge, key_type, val ? 1 : 0, size_class(m + n)}] = TuneEntry{win, win_ms};
  }
  if (best) {
    best[0] = win.cfg;
    best[1] = win.search;
    best[2] = win.partition;
  }
  return CM_OK;
}

int cm_autotune_segmented(int key_type, const void* A, const uint32_t* A_val, const uint64_t* a_off,
                          uint64_t total_a, const void* B, const uint32_t* B_val, const uint64_t* b_off,
                          uint64_t total_b, uint64_t num_seg, void* C, uint32_t* C_val, void* workspace,
                          size_t workspace_bytes, int reps, hipStream_t stream, int* best) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (reps < 1 || reps > 10000 || total_a + total_b == 0) return CM_EINVAL;
  const bool val = A_val || B_val || C_val;
  const int check = seg_impl(key_type, A, A_val, a_off, total_a, B, B_val, b_off, total_b, num_seg, C, C_val,
                             workspace, workspace_bytes, stream, nullptr, true);
  if (check != CM_OK) return check;
  std::vector<Choice> cands;
  for (int cfg = 0; cfg < kNumCfgs; ++cfg)
    for (int search = 0; search < 2; ++search)
      for (int part = 0; part < 3; part += 2) cands.push_back(Choice{cfg, search, part, g_set.grid});
  Choice win{0, 1, 1};
  double win_ms = 0;
  const int picked = tune_pick(
      cands,
      [&](const Choice& ch, double* ms) {
        return time_calls(
            [&] {
              return seg_impl(key_type, A, A_val, a_off, total_a, B, B_val, b_off, total_b, num_seg, C, C_val,
                              workspace, workspace_bytes, stream, &ch);
            },
            reps, stream, ms);
      },
      &win, &win_ms);
  if (picked != CM_OK) return picked;
  {
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    g_tuning[TuneKey{kOpSegmented, key_type, val ? 1 : 0, size_class(total_a + total_b)}] = TuneEntry{win, win_ms};
  }
  if (best) {
    best[0] = win.cfg;
    best[1] = win.search;
    best[2] = win.partition;
  }
  return CM_OK;
}

int cm_tuning_count(void) {
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  return (int)g_tuning.size();
}

int cm_tuning_clear(void) {
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  g_tuning.clear();
  return CM_OK;
}

int cm_tuning_set(int op, int key_type, int with_payload, int size_cls, int config_id, int search_mode,
                  int partition_mode) {
  if (op < kOpMerge || op > kOpSort) return CM_EINVAL;
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (config_id < 0 || config_id >= kNumCfgs) return CM_ECONFIG;
  if (size_cls < 0 || size_cls > 64 || (search_mode != 0 && search_mode != 1) || partition_mode < 0 ||
      partition_mode > kMaxPartition)
    return CM_EINVAL;
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  g_tuning[TuneKey{op, key_type, with_payload ? 1 : 0, size_cls}] =
      TuneEntry{Choice{config_id, search_mode, partition_mode}, 0.0};
  return CM_OK;
}

int cm_tuning_get(int op, int key_type, int with_payload, uint64_t num_outputs, int* choice) {
  if (op < kOpMerge || op > kOpSort) return CM_EINVAL;
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  if (!choice) return CM_EINVAL;
  const Choice ch = resolve(op, key_type, with_payload != 0, num_outputs);
  choice[0] = ch.cfg;
  choice[1] = ch.search;
  choice[2] = op == kOpBatch && ch.partition == 3 ? 2 : ch.partition;  // as batch_choice
  return CM_OK;
}

int cm_tuning_save(const char* path) {
  std::string p;
  if (!tuning_path(path, true, &p)) return CM_EINVAL;
  FILE* f = fopen(p.c_str(), "w");
  if (!f) return CM_EINVAL;
  const Identity id = current_identity();
  fprintf(f, "# corank_merge tuning v2\n# arch %s\n# hip_runtime %d\n# library %s\n", id.arch.c_str(), id.runtime,
          id.build.c_str());
  fprintf(f, "# op key_type with_payload size_class config search partition ms\n");
  {
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    for (const auto& kv : g_tuning) {
      const auto& k = kv.first;
      const auto& e = kv.second;
      fprintf(f, "%d %d %d %d %d %d %d %.6f\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
              e.ch.cfg, e.ch.search, e.ch.partition, e.ms);
    }
  }
  return fclose(f) == 0 ? CM_OK : CM_EINVAL;
}

int cm_tuning_load(const char* path) {
  std::string p;
  if (!tuning_path(path, false, &p)) return CM_EINVAL;
  FILE* f = fopen(p.c_str(), "r");
  if (!f) return CM_EINVAL;
  char line[512];
  int rc = CM_OK;
  std::map<TuneKey, TuneEntry> loaded;
  Identity file_id;
  bool v2 = false, have_arch = false, have_runtime = false, have_build = false;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '\n') continue;
    if (line[0] == '#') {
      char word[256] = {0};
      int num = 0;
      if (strncmp(line, "# corank_merge tuning v2", 24) == 0) {
        v2 = true;
      } else if (sscanf(line, "# arch %255s", word) == 1) {
        file_id.arch = word;
        have_arch = true;
      } else if (sscanf(line, "# hip_runtime %d", &num) == 1) {
        file_id.runtime = num;
        have_runtime = true;
      } else if (sscanf(line, "# library %255s", word) == 1) {
        file_id.build = word;
        have_build = true;
      }
      continue;
    }
    int op, kt, val, sc, cfg, search, part;
    double ms;
    if (sscanf(line, "%d %d %d %d %d %d %d %lf", &op, &kt, &val, &sc, &cfg, &search, &part, &ms) != 8 ||
        op < kOpMerge || op > kOpSort || !key_type_ok(kt) || (val != 0 && val != 1) || sc < 0 ||
        sc > 64 || cfg < 0 || cfg >= kNumCfgs || (search != 0 && search != 1) || part < 0 || part > kMaxPartition) {
      rc = CM_EINVAL;
      break;
    }
    loaded[TuneKey{op, kt, val, sc}] = TuneEntry{Choice{cfg, search, part}, ms};
  }
  fclose(f);
  if (rc != CM_OK) return rc;
  // a table is timed on one device type, runtime and library build: one
  // made elsewhere (or with no identity) is refused
  const Identity id = current_identity();
  if (!v2 || !have_arch || !have_runtime || !have_build || file_id.arch != id.arch ||
      file_id.runtime != id.runtime || file_id.build != id.build)
    return CM_ESTALE;
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  for (const auto& kv : loaded) g_tuning[kv.first] = kv.second;
  return CM_OK;
}

const char* cm_build_id(void) { return CM_BUILD_ID; }

// ---- graph plans

// Captures body(ctx, s) on a private stream into a new graph (*out; left
// null on failure).
static int capture_graph(int (*body)(void*, hipStream_t), void* ctx, hipGraph_t* out) {
  *out = nullptr;
  hipStream_t s;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return CM_EHIP;
  int rc = CM_OK;
  hipGraph_t g = nullptr;
  g_capturing = true;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = CM_EHIP;
  const int body_rc = rc == CM_OK ? body(ctx, s) : rc;
  if (rc == CM_OK && hipStreamEndCapture(s, &g) != hipSuccess) rc = CM_EHIP;
  g_capturing = false;
  if (rc == CM_OK) rc = body_rc;
  (void)hipStreamDestroy(s);
  if (rc != CM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  *out = g;
  return CM_OK;
}

static int plan_capture(cm_plan** out, int kind, int (*body)(void*, hipStream_t), void* ctx) {
  if (!out) return CM_EINVAL;
  *out = nullptr;
  cm_plan* p = new cm_plan;
  p->kind = kind;
  int rc = capture_graph(body, ctx, &p->graph);
  if (rc == CM_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) rc = CM_EHIP;
  if (rc != CM_OK) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
    return rc;
  }
  *out = p;
  return CM_OK;
}

// Do graphs a and b hold the same sequence of nodes, kernel nodes running
// the same kernel functions?  (A tile, payload-width or alignment change
// keeps the node count and types but swaps the kernel instantiation.)
static bool same_kernels(hipGraph_t a, hipGraph_t b) {
  size_t na = 0, nb = 0;
  if (hipGraphGetNodes(a, nullptr, &na) != hipSuccess || hipGraphGetNodes(b, nullptr, &nb) != hipSuccess ||
      na != nb)
    return false;
  std::vector<hipGraphNode_t> xa(na), xb(nb);
  if (na && (hipGraphGetNodes(a, xa.data(), &na) != hipSuccess || hipGraphGetNodes(b, xb.data(), &nb) != hipSuccess))
    return false;
  for (size_t x = 0; x < na; ++x) {
    hipGraphNodeType ta, tb;
    if (hipGraphNodeGetType(xa[x], &ta) != hipSuccess || hipGraphNodeGetType(xb[x], &tb) != hipSuccess || ta != tb)
      return false;
    if (ta != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams pa{}, pb{};
    if (hipGraphKernelNodeGetParams(xa[x], &pa) != hipSuccess || hipGraphKernelNodeGetParams(xb[x], &pb) != hipSuccess ||
        pa.func != pb.func)
      return false;
  }
  return true;
}

// Re-points plan p at the call body(ctx) describes: a new capture, applied
// to the executable graph in place when its topology is unchanged (same
// kernel functions, new arguments and grid sizes), else a new executable
// graph.  On failure the plan is left as it was.
static int plan_recapture(cm_plan* p, int (*body)(void*, hipStream_t), void* ctx) {
  hipGraph_t g = nullptr;
  int rc = capture_graph(body, ctx, &g);
  if (rc != CM_OK) return rc;
  hipGraphNode_t err_node = nullptr;
  hipGraphExecUpdateResult res;
  if (same_kernels(p->graph, g) && hipGraphExecUpdate(p->exec, g, &err_node, &res) == hipSuccess &&
      res == hipGraphExecUpdateSuccess) {
    (void)hipGraphDestroy(p->graph);
    p->graph = g;
    return CM_OK;
  }
  (void)hipGetLastError();  // a refused update is not an error of later calls
  hipGraphExec_t e = nullptr;
  if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return CM_EHIP;
  }
  (void)hipGraphExecDestroy(p->exec);
  (void)hipGraphDestroy(p->graph);
  p->exec = e;
  p->graph = g;
  return CM_OK;
}

struct MergeArgs {
  int kt;
  const void* A;
  const uint32_t* Av;
  uint64_t m;
  const void* B;
  const uint32_t* Bv;
  uint64_t n;
  void* C;
  uint32_t* Cv;
  void* ws;
  size_t ws_bytes;
};

struct SegArgs {
  int kt;
  const void* A;
  const uint32_t* Av;
  const uint64_t* a_off;
  uint64_t ta;
  const void* B;
  const uint32_t* Bv;
  const uint64_t* b_off;
  uint64_t tb;
  uint64_t S;
  void* C;
  uint32_t* Cv;
  void* ws;
  size_t ws_bytes;
};

static int merge_body(void* ctx, hipStream_t s) {
  const MergeArgs& x = *(const MergeArgs*)ctx;
  const bool val = x.Av || x.Bv || x.Cv;
  return merge_impl(x.kt, val, 4, x.A, x.Av, x.m, x.B, x.Bv, x.n, x.C, x.Cv, x.ws, x.ws_bytes, s);
}

static int seg_body(void* ctx, hipStream_t s) {
  const SegArgs& x = *(const SegArgs*)ctx;
  return seg_impl(x.kt, x.A, x.Av, x.a_off, x.ta, x.B, x.Bv, x.b_off, x.tb, x.S, x.C, x.Cv, x.ws, x.ws_bytes, s);
}

int cm_plan_create_merge(int key_type, const void* A, const uint32_t* A_val, uint64_t m, const void* B,
                         const uint32_t* B_val, uint64_t n, void* C, uint32_t* C_val, void* workspace,
                         size_t workspace_bytes, cm_plan** plan) {
  if (!plan) return CM_EINVAL;
  *plan = nullptr;
  const int rc = merge_impl(key_type, A_val || B_val || C_val, 4, A, A_val, m, B, B_val, n, C, C_val, workspace,
                            workspace_bytes, nullptr, nullptr, true);
  if (rc != CM_OK) return rc;
  MergeArgs a{key_type, A, A_val, m, B, B_val, n, C, C_val, workspace, workspace_bytes};
  return plan_capture(plan, 0, merge_body, &a);
}

int cm_plan_update_merge(cm_plan* plan, int key_type, const void* A, const uint32_t* A_val, uint64_t m,
                         const void* B, const uint32_t* B_val, uint64_t n, void* C, uint32_t* C_val,
                         void* workspace, size_t workspace_bytes) {
  if (!plan || !plan->exec || plan->kind != 0) return CM_EINVAL;
  const int rc = merge_impl(key_type, A_val || B_val || C_val, 4, A, A_val, m, B, B_val, n, C, C_val, workspace,
                            workspace_bytes, nullptr, nullptr, true);
  if (rc != CM_OK) return rc;
  MergeArgs a{key_type, A, A_val, m, B, B_val, n, C, C_val, workspace, workspace_bytes};
  return plan_recapture(plan, merge_body, &a);
}

int cm_plan_create_segmented(int key_type, const void* A, const uint32_t* A_val, const uint64_t* a_off,
                             uint64_t total_a, const void* B, const uint32_t* B_val, const uint64_t* b_off,
                             uint64_t total_b, uint64_t num_seg, void* C, uint32_t* C_val, void* workspace,
                             size_t workspace_bytes, cm_plan** plan) {
  if (!plan) return CM_EINVAL;
  *plan = nullptr;
  const int rc = seg_impl(key_type, A, A_val, a_off, total_a, B, B_val, b_off, total_b, num_seg, C, C_val,
                          workspace, workspace_bytes, nullptr, nullptr, true);
  if (rc != CM_OK) return rc;
  SegArgs a{key_type, A, A_val, a_off, total_a, B, B_val, b_off, total_b, num_seg, C, C_val, workspace,
            workspace_bytes};
  return plan_capture(plan, 1, seg_body, &a);
}

int cm_plan_update_segmented(cm_plan* plan, int key_type, const void* A, const uint32_t* A_val,
                             const uint64_t* a_off, uint64_t total_a, const void* B, const uint32_t* B_val,
                             const uint64_t* b_off, uint64_t total_b, uint64_t num_seg, void* C, uint32_t* C_val,
                             void* workspace, size_t workspace_bytes) {
  if (!plan || !plan->exec || plan->kind != 1) return CM_EINVAL;
  const int rc = seg_impl(key_type, A, A_val, a_off, total_a, B, B_val, b_off, total_b, num_seg, C, C_val,
                          workspace, workspace_bytes, nullptr, nullptr, true);
  if (rc != CM_OK) return rc;
  SegArgs a{key_type, A, A_val, a_off, total_a, B, B_val, b_off, total_b, num_seg, C, C_val, workspace,
            workspace_bytes};
  return plan_recapture(plan, seg_body, &a);
}

int cm_plan_launch(cm_plan* plan, hipStream_t stream) {
  if (!plan || !plan->exec) return CM_EINVAL;
  return hipGraphLaunch(plan->exec, stream) == hipSuccess ? CM_OK : CM_EHIP;
}

int cm_plan_destroy(cm_plan* plan) {
  if (!plan) return CM_EINVAL;
  int rc = CM_OK;
  if (plan->exec && hipGraphExecDestroy(plan->exec) != hipSuccess) rc = CM_EHIP;
  if (plan->graph && hipGraphDestroy(plan->graph) != hipSuccess) rc = CM_EHIP;
  delete plan;
  return rc;
}

// ---- measurement helpers

int cm_copy(const void* src, void* dst, uint64_t bytes, hipStream_t stream) {
  if (bytes == 0) return CM_OK;
  if (!src || !dst || (bytes % 16) || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16)) return CM_EINVAL;
  if (overlap(src, bytes, dst, bytes)) return CM_EALIAS;
  return launch_copy16(src, dst, bytes / 16, stream);
}

int cm_copy_tiles(int config, const void* A, const uint32_t* A_val, uint64_t m, const void* B, const uint32_t* B_val,
                  uint64_t n, void* C, uint32_t* C_val, hipStream_t stream) {
  if (config < 0 || config >= kNumCfgs) return CM_EINVAL;
  if ((m % 4) || (n % 4) || m + n >= (1ull << 34)) return CM_EINVAL;
  const uint64_t N = m + n;
  if ((m && (!A || !A_val)) || (n && (!B || !B_val)) || (N && (!C || !C_val))) return CM_EINVAL;
  for (const void* p : {A, (const void*)A_val, B, (const void*)B_val, (const void*)C, (const void*)C_val})
    if ((uintptr_t)p % 16) return CM_EINVAL;
  if (any_overlap({{C, N * 4}, {C_val, N * 4}}, {{A, m * 4}, {A_val, m * 4}, {B, n * 4}, {B_val, n * 4}}))
    return CM_EALIAS;
  if (N == 0) return CM_OK;
  return launch_copy_tiles(config, g_set.shape.xcd_order, A, A_val, m, B, B_val, n, C, C_val, stream);
}

int cm_origin_codes(uint64_t m, uint64_t n, uint32_t* A_codes, uint32_t* B_codes, hipStream_t stream) {
  if ((m && !A_codes) || (n && !B_codes) || m >= (1ull << 31) || n >= (1ull << 31)) return CM_EINVAL;
  if (any_overlap({{A_codes, m * 4}, {B_codes, n * 4}}, {})) return CM_EALIAS;
  if (m + n == 0) return CM_OK;
  return launch_origin_codes(m, n, A_codes, B_codes, stream);
}

int cm_gather_records(const uint32_t* codes, uint64_t N, const void* A_rec, uint64_t m, const void* B_rec,
                      uint64_t n, uint64_t width, void* out, hipStream_t stream) {
  if (width == 0 || (N && (!codes || !out)) || (m && !A_rec) || (n && !B_rec) || m >= (1ull << 31) ||
      n >= (1ull << 31) || (N && width > UINT64_MAX / N) || (m + n && width > UINT64_MAX / (m + n)))
    return CM_EINVAL;
  if (any_overlap({{out, N * width}}, {{codes, N * 4}, {A_rec, m * width}, {B_rec, n * width}})) return CM_EALIAS;
  if (N == 0) return CM_OK;
  return launch_gather_records(codes, N, A_rec, m, B_rec, n, width, out, stream);
}

size_t cm_partition_ablation_workspace_size(uint32_t P) {
  if (P < 2) return 0;
  return round256(((size_t)P + 1) * sizeof(uint64_t)) + round256(2 * (size_t)P * sizeof(uint64_t));
}

int cm_merge_partition_ablation(int key_type, const void* A, const uint32_t* A_val, uint64_t m, const void* B,
                                const uint32_t* B_val, uint64_t n, void* C, uint32_t* C_val, uint32_t P,
                                int partition, uint64_t* bounds, void* workspace, size_t workspace_bytes,
                                hipStream_t stream) {
  if (!key_type_ok(key_type)) return CM_EDTYPE;
  const bool val = A_val || B_val || C_val;
  if (!lengths_ok(m, n) || P < 2 || (P & 1) || P > (1u << 20) || (partition != 0 && partition != 1) || !bounds)
    return CM_EINVAL;
  const uint64_t N = m + n;
  const size_t ks = key_bytes(key_type);
  if ((m && !A) || (n && !B) || (N && !C)) return CM_EINVAL;
  if (val && ((m && !A_val) || (n && !B_val) || (N && !C_val))) return CM_EINVAL;
  const size_t need = cm_partition_ablation_workspace_size(P);
  if (!workspace || workspace_bytes < need) return CM_ENOSPC;
  if (any_overlap({{C, N * ks}, {C_val, val ? N * 4 : 0}, {bounds, ((uint64_t)P + 1) * 8}, {workspace, need}},
                  {{A, m * ks}, {B, n * ks}, {A_val, val ? m * 4 : 0}, {B_val, val ? n * 4 : 0}}))
    return CM_EALIAS;
  const Choice ch = resolve(kOpMerge, key_type, val, N);
  uint64_t* J = (uint64_t*)workspace;
  uint64_t* cuts = (uint64_t*)((char*)workspace + round256(((size_t)P + 1) * sizeof(uint64_t)));
  timing_mark(0, stream);
  int rc = partition == 0 ? launch_stream_co_ranks(key_type, A, m, B, n, P, J, stream)
                          : launch_cross_rank_cuts(key_type, A, m, B, n, P / 2, cuts, bounds, J, stream);
  if (rc == CM_OK && partition == 0) rc = launch_equal_starts(N, P, bounds, stream);
  if (rc != CM_OK) return rc;
  timing_mark(1, stream);
  rc = launch_merge_stream(key_type, val, ch, A, val ? A_val : nullptr, m, B, val ? B_val : nullptr, n, C,
                           val ? C_val : nullptr, bounds, J, P, stream);
  timing_mark(2, stream);
  return rc;
}

size_t cm_sort_workspace_size(int key_type, int with_payload, uint64_t n) {
  if (!key_type_ok(key_type)) return 0;
  return sort_ws_bytes(key_type, with_payload != 0, n);
}

uint64_t cm_sort_run_length(int key_type, int with_payload, uint64_t n) {
  if (!key_type_ok(key_type)) return 0;
  const bool val = with_payload != 0;
  const Choice ch = resolve(kOpSort, key_type, val, n);
  return tile_size(ch.cfg) * sort_run_blocks(key_type, val, ch.cfg);
}

int cm_stable_sort(int key_type, const void* keys, uint64_t n, void* keys_out, void* workspace,
                   size_t workspace_bytes, hipStream_t stream) {
  return sort_impl(key_type, false, keys, nullptr, n, keys_out, nullptr, workspace, workspace_bytes, stream);
}

int cm_stable_sort_pairs(int key_type, const void* keys, const uint32_t* vals, uint64_t n, void* keys_out,
                         uint32_t* vals_out, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  return sort_impl(key_type, true, keys, vals, n, keys_out, vals_out, workspace, workspace_bytes, stream);
}

int cm_timing_start(uint32_t capacity) {
  if (capacity == 0 || capacity > (1u << 20) || g_timing.on) return CM_EINVAL;
  g_timing.ev = new hipEvent_t[3ull * capacity];
  for (uint64_t x = 0; x < 3ull * capacity; ++x) {
    if (hipEventCreate(&g_timing.ev[x]) != hipSuccess) {
      for (uint64_t y = 0; y < x; ++y) (void)hipEventDestroy(g_timing.ev[y]);
      delete[] g_timing.ev;
      g_timing.ev = nullptr;
      return CM_EHIP;
    }
  }
  g_timing.capacity = capacity;
  g_timing.used = 0;
  g_timing.on = true;
  return CM_OK;
}

int cm_timing_stop(uint32_t* calls, double* co_rank_ms_mean, double* merge_ms_mean, float* call_start_ms,
                   float* call_ms, float* merge_ms) {
  if (!g_timing.on && !g_timing.ev) return CM_EINVAL;
  double sum_b = 0, sum_m = 0;
  int rc = CM_OK;
  for (uint32_t c = 0; c < g_timing.used; ++c) {
    float tb = 0, tm = 0;
    hipEvent_t* e = g_timing.ev + 3ull * c;
    if (hipEventSynchronize(e[2]) != hipSuccess || hipEventElapsedTime(&tb, e[0], e[1]) != hipSuccess ||
        hipEventElapsedTime(&tm, e[1], e[2]) != hipSuccess)
      rc = CM_EHIP;
    sum_b += tb;
    sum_m += tm;
    if (call_start_ms) {
      float t0 = 0;
      if (c > 0 && hipEventElapsedTime(&t0, g_timing.ev[0], e[0]) != hipSuccess) rc = CM_EHIP;
      call_start_ms[c] = t0;
    }
    if (call_ms) call_ms[c] = tb + tm;
    if (merge_ms) merge_ms[c] = tm;
  }
  if (calls) *calls = g_timing.used;
  if (co_rank_ms_mean) *co_rank_ms_mean = g_timing.used ? sum_b / g_timing.used : 0.0;
  if (merge_ms_mean) *merge_ms_mean = g_timing.used ? sum_m / g_timing.used : 0.0;
  for (uint64_t x = 0; x < 3ull * g_timing.capacity; ++x) (void)hipEventDestroy(g_timing.ev[x]);
  delete[] g_timing.ev;
  g_timing = Timing{};
  return rc;
}

}  // extern "C"
