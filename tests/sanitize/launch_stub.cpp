// The library's internal kernel-launch interface (internal.hpp) with every
// launcher a no-op that reports success, for the CPU-only sanitizer builds
// of the host code: the C ABI's checks, choices and bookkeeping run end to
// end, and nothing is computed (the sanitizer tests check no merge
// results; parity is the GPU tests' job).  Test infrastructure only.
#include "internal.hpp"

#include "corank_merge.h"

namespace cm {

uint32_t resident_workgroups(const void*, int) { return 256; }

int noalloc_scratch(void** out) {
  static uint64_t scratch[kNoAllocScratchBytes / 8];
  *out = scratch;
  return CM_OK;
}

int launch_block_co_ranks(int, const Choice&, const Shape&, const void*, uint64_t, const void*, uint64_t, uint64_t,
                          uint64_t, uint64_t*, uint64_t*, hipStream_t) {
  return CM_OK;
}
uint32_t sort_run_blocks(int, bool, int) { return 4; }
int launch_sort_blocks(int, bool, const Choice&, const void*, const uint32_t*, uint64_t, void*, uint32_t*, uint64_t,
                       hipStream_t) {
  return CM_OK;
}
int launch_sort_pass(int, bool, const Choice&, const Shape&, const void*, const uint32_t*, uint64_t, int, void*,
                     uint32_t*, uint64_t*, uint64_t*, uint64_t, hipStream_t) {
  return CM_OK;
}
int launch_merge_blocks(int, bool, int, const Choice&, const Shape&, const void*, const void*, uint64_t, const void*,
                        const void*, uint64_t, void*, void*, const uint64_t*, uint64_t, hipStream_t) {
  return CM_OK;
}
uint32_t stream_blocks(int, bool, const Choice& ch, uint64_t N) {
  const uint64_t T = tile_size(ch.cfg), tiles = (N + T - 1) / T;
  return (uint32_t)(tiles < 256 ? (tiles ? tiles : 1) : 256);
}
int launch_stream_co_ranks(int, const void*, uint64_t, const void*, uint64_t, uint32_t, uint64_t*, hipStream_t) {
  return CM_OK;
}
int launch_merge_stream(int, bool, const Choice&, const void*, const uint32_t*, uint64_t, const void*,
                        const uint32_t*, uint64_t, void*, uint32_t*, const uint64_t*, const uint64_t*, uint32_t,
                        hipStream_t) {
  return CM_OK;
}
int launch_cross_rank_cuts(int, const void*, uint64_t, const void*, uint64_t, uint32_t, uint64_t*, uint64_t*,
                           uint64_t*, hipStream_t) {
  return CM_OK;
}
int launch_equal_starts(uint64_t, uint32_t, uint64_t*, hipStream_t) { return CM_OK; }
int launch_origin_codes(uint64_t, uint64_t, uint32_t*, uint32_t*, hipStream_t) { return CM_OK; }
int launch_gather_records(const uint32_t*, uint64_t, const void*, uint64_t, const void*, uint64_t, uint64_t, void*,
                          hipStream_t) {
  return CM_OK;
}
int launch_seg_validate(const uint64_t*, const uint64_t*, uint64_t, uint64_t, uint64_t, uint32_t*, hipStream_t) {
  return CM_OK;
}
int launch_seg_block_co_ranks(int, const Choice&, const Shape&, const void*, const uint64_t*, const void*,
                              const uint64_t*, uint32_t, uint64_t, uint64_t, uint64_t, uint64_t*, uint32_t*,
                              uint64_t*, uint32_t*, const uint32_t*, hipStream_t) {
  return CM_OK;
}
int launch_seg_merge_blocks(int, bool, const Choice&, const void*, const uint32_t*, const uint64_t*, const void*,
                            const uint32_t*, const uint64_t*, uint32_t, uint64_t, void*, uint32_t*, const uint64_t*,
                            const uint32_t*, uint64_t, const uint32_t*, hipStream_t) {
  return CM_OK;
}
int launch_batch_prep(const void*, const void*, uint32_t, uint64_t, uint64_t, void*, uint32_t*, uint32_t*,
                      hipStream_t) {
  return CM_OK;
}
int launch_batch_co_ranks(int, const Choice&, const Shape&, const void*, const uint32_t*, uint64_t, uint64_t,
                          uint64_t*, uint64_t*, hipStream_t) {
  return CM_OK;
}
int launch_batch_merge_blocks(int, bool, const Choice&, int, const void*, const void*, uint32_t, const uint32_t*,
                              const uint64_t*, uint64_t, bool, int, hipStream_t) {
  return CM_OK;
}
int launch_co_rank_many(int, int, const uint64_t*, uint64_t, const void*, uint64_t, const void*, uint64_t, uint64_t*,
                        hipStream_t) {
  return CM_OK;
}
int launch_check_sorted(int, const void*, uint64_t, uint32_t*, hipStream_t) { return CM_OK; }
int launch_copy16(const void*, void*, uint64_t, hipStream_t) { return CM_OK; }
int launch_copy_tiles(int, int, const void*, const uint32_t*, uint64_t, const void*, const uint32_t*, uint64_t, void*,
                      uint32_t*, hipStream_t) {
  return CM_OK;
}

}  // namespace cm
