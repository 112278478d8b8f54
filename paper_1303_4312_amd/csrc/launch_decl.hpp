// Launch<K>: the key-dependent kernel launchers for one key type, declared
// here and defined in launch_impl.hpp.  launch.hip dispatches on the key type
// through these declarations only; each launch_keys_*.hip file includes the
// definitions and instantiates Launch for one key width (ascending and
// descending), so the kernels of the six key types compile side by side.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"
#include "order.hpp"

namespace cm {

template <typename K>
struct Launch {
  static int block_co_ranks(const Choice& ch, const Shape& sh, const void* A, uint64_t m, const void* B, uint64_t n,
                            uint64_t tile, uint64_t nb, uint64_t* bj, uint64_t* coarse, hipStream_t st);
  static int merge_blocks(bool val, int vbytes, const Choice& ch, const Shape& sh, const void* A, const void* Av,
                          uint64_t m, const void* B, const void* Bv, uint64_t n, void* C, void* Cv,
                          const uint64_t* bj, uint64_t tiles, hipStream_t st);
  static int stream_co_ranks(const void* A, uint64_t m, const void* B, uint64_t n, uint32_t P, uint64_t* J,
                             hipStream_t st);
  static int merge_stream(bool val, const Choice& ch, const void* A, const uint32_t* Av, uint64_t m, const void* B,
                          const uint32_t* Bv, uint64_t n, void* C, uint32_t* Cv, const uint64_t* I, const uint64_t* J,
                          uint32_t P, hipStream_t st);
  static int seg_block_co_ranks(const Choice& ch, const Shape& sh, const void* A, const uint64_t* a_off, const void* B,
                                const uint64_t* b_off, uint32_t S, uint64_t N, uint64_t tile, uint64_t nb,
                                uint64_t* bj, uint32_t* bs, uint64_t* jc, uint32_t* sc, const uint32_t* flag,
                                hipStream_t st);
  static int seg_merge_blocks(bool val, const Choice& ch, const void* A, const uint32_t* Av, const uint64_t* a_off,
                              const void* B, const uint32_t* Bv, const uint64_t* b_off, uint32_t S, uint64_t N,
                              void* C, uint32_t* Cv, const uint64_t* bj, const uint32_t* bs, uint64_t tiles,
                              const uint32_t* flag, hipStream_t st);
  static int batch_co_ranks(const Choice& ch, const Shape& sh, const void* d, const uint32_t* sm, uint64_t tile,
                            uint64_t nb, uint64_t* bj, uint64_t* coarse, hipStream_t st);
  static int batch_merge_blocks(bool val, const Choice& ch, int form, const void* h, const void* d, uint32_t count,
                                const uint32_t* bm, const uint64_t* bj, uint64_t tiles, bool vec, int xcd,
                                hipStream_t st);
  static int co_rank_many(int search, const uint64_t* ranks, uint64_t q, const void* A, uint64_t m, const void* B,
                          uint64_t n, uint64_t* j_out, hipStream_t st);
  static int stream_resident(bool val, int cfg);
  static int check_sorted(const void* X, uint64_t len, uint32_t* flag, uint64_t blocks, hipStream_t st);
  static int cross_rank_cuts(const void* A, uint64_t m, const void* B, uint64_t n, uint32_t h, uint64_t* ia,
                             uint64_t* ja, uint64_t* ib, uint64_t* jb, unsigned blocks, hipStream_t st);
};

}  // namespace cm
