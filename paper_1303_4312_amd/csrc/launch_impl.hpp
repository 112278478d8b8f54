// Definitions of the Launch<K> members declared in launch_decl.hpp (included
// only by the launch_keys_*.hip files, which instantiate them).
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "corank_merge.h"
#include "dispatch.hpp"
#include "internal.hpp"
#include "kernels.hpp"
#include "launch_decl.hpp"

namespace cm {

template <typename K>
int Launch<K>::block_co_ranks(const Choice& ch, const Shape& sh, const void* A, uint64_t m, const void* B, uint64_t n,
                              uint64_t tile, uint64_t nb, uint64_t* bj, uint64_t* coarse, hipStream_t st) {
  const uint64_t blocks = (nb + 255) / 256;
  if (ch.partition == 0) {
    hipLaunchKernelGGL((k_block_co_rank<K>), dim3((unsigned)blocks), dim3(256), 0, st, (const K*)A, m,
                       (const K*)B, n, tile, nb, bj, ch.search);
    return launch_status();
  }
  const uint32_t G = sh.coarse_stride;
  const uint64_t nc = num_coarse(nb, G);
  if (ch.partition == 1)
    hipLaunchKernelGGL((k_coarse_co_rank<K, 64>), dim3((unsigned)((nc + 3) / 4)), dim3(256), 0, st,
                       (const K*)A, m, (const K*)B, n, tile * G, nc, coarse);
  else
    hipLaunchKernelGGL((k_coarse_co_rank<K, 16>), dim3((unsigned)((nc + 15) / 16)), dim3(256), 0, st,
                       (const K*)A, m, (const K*)B, n, tile * G, nc, coarse);
  if (launch_status() != CM_OK) return CM_EHIP;
  if (sh.fine_lanes == 2 || sh.fine_lanes == 4) {
    const uint64_t lanes = nb * (uint64_t)sh.fine_lanes;
    if (sh.fine_lanes == 2)
      hipLaunchKernelGGL((k_fine_co_rank_group<K, 2>), dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st,
                         (const K*)A, m, (const K*)B, n, tile, nb, G, (const uint64_t*)coarse, bj);
    else
      hipLaunchKernelGGL((k_fine_co_rank_group<K, 4>), dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st,
                         (const K*)A, m, (const K*)B, n, tile, nb, G, (const uint64_t*)coarse, bj);
  } else {
    hipLaunchKernelGGL((k_fine_co_rank<K>), dim3((unsigned)blocks), dim3(256), 0, st, (const K*)A, m,
                       (const K*)B, n, tile, nb, G, (const uint64_t*)coarse, bj);
  }
  return launch_status();
}

template <typename K>
int Launch<K>::merge_blocks(bool val, int vbytes, const Choice& ch, const Shape& sh, const void* A, const void* Av,
                            uint64_t m, const void* B, const void* Bv, uint64_t n, void* C, void* Cv,
                            const uint64_t* bj, uint64_t tiles, hipStream_t st) {
  return by_cfg(ch.cfg, [&](auto nt, auto e) -> int {
    constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
    static_assert((NT * E) % 4 == 0, "blocks must start at multiples of 4 outputs");
    const bool vec = val ? all_aligned16({A, B, C, Av, Bv, Cv}) : all_aligned16({A, B, C});
    const dim3 b(NT);
    // bj == nullptr: every block co-ranks its own ends (no boundary pass)
    auto go = [&](auto val_c, auto vec_c, auto pay) {
      constexpr bool V = decltype(val_c)::value, W = decltype(vec_c)::value;
      using P = decltype(pay);  // payload type
      if (bj)
        hipLaunchKernelGGL((k_merge_blocks<K, V, NT, E, W, P>),
                           dim3(launch_grid((const void*)k_merge_blocks<K, V, NT, E, W, P>, NT, tiles, ch.grid)), b,
                           0, st, (const K*)A, (const P*)Av, m, (const K*)B, (const P*)Bv, n, (K*)C, (P*)Cv, bj,
                           tiles, ch.search, sh.xcd_order);
      else
        hipLaunchKernelGGL((k_merge_blocks_self<K, V, NT, E, W, P>),
                           dim3(launch_grid((const void*)k_merge_blocks_self<K, V, NT, E, W, P>, NT, tiles, ch.grid)),
                           b, 0, st, (const K*)A, (const P*)Av, m, (const K*)B, (const P*)Bv, n, (K*)C, (P*)Cv,
                           tiles, ch.search, sh.xcd_order);
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    if (val && vbytes == 8) {
      if (vec)
        go(T_{}, T_{}, uint64_t{});
      else
        go(T_{}, F_{}, uint64_t{});
    } else if (val && vec) {
      go(T_{}, T_{}, uint32_t{});
    } else if (val) {
      go(T_{}, F_{}, uint32_t{});
    } else if (vec) {
      go(F_{}, T_{}, uint32_t{});
    } else {
      go(F_{}, F_{}, uint32_t{});
    }
    return launch_status();
  });
}

template <typename K>
int Launch<K>::stream_co_ranks(const void* A, uint64_t m, const void* B, uint64_t n, uint32_t P, uint64_t* J,
                               hipStream_t st) {
  const uint64_t waves = (uint64_t)P + 1;
  hipLaunchKernelGGL((k_stream_co_rank<K>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, (const K*)A, m,
                     (const K*)B, n, P, J);
  return launch_status();
}

template <typename K>
int Launch<K>::merge_stream(bool val, const Choice& ch, const void* A, const uint32_t* Av, uint64_t m, const void* B,
                            const uint32_t* Bv, uint64_t n, void* C, uint32_t* Cv, const uint64_t* I,
                            const uint64_t* J, uint32_t P, hipStream_t st) {
  return by_cfg(ch.cfg, [&](auto nt, auto e) -> int {
    constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
    if (val)
      hipLaunchKernelGGL((k_merge_stream<K, true, NT, E>), dim3(P), dim3(NT), 0, st, (const K*)A, Av, m,
                         (const K*)B, Bv, n, (K*)C, Cv, I, J, P, ch.search);
    else
      hipLaunchKernelGGL((k_merge_stream<K, false, NT, E>), dim3(P), dim3(NT), 0, st, (const K*)A, Av, m,
                         (const K*)B, Bv, n, (K*)C, Cv, I, J, P, ch.search);
    return launch_status();
  });
}

template <typename K>
int Launch<K>::seg_block_co_ranks(const Choice& ch, const Shape& sh, const void* A, const uint64_t* a_off,
                                  const void* B, const uint64_t* b_off, uint32_t S, uint64_t N, uint64_t tile,
                                  uint64_t nb, uint64_t* bj, uint32_t* bs, uint64_t* jc, uint32_t* sc,
                                  const uint32_t* flag, hipStream_t st) {
  if (ch.partition == 0 || !jc || !sc) {
    hipLaunchKernelGGL((k_seg_block_co_rank<K>), dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st,
                       (const K*)A, a_off, (const K*)B, b_off, S, N, tile, nb, bj, bs, flag, ch.search);
    return launch_status();
  }
  const uint32_t G = sh.coarse_stride;
  const uint64_t nc = num_coarse(nb, G);
  hipLaunchKernelGGL((k_seg_block_co_rank<K>), dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, (const K*)A,
                     a_off, (const K*)B, b_off, S, N, tile * G, nc, jc, sc, flag, ch.search);
  if (launch_status() != CM_OK) return CM_EHIP;
  hipLaunchKernelGGL((k_seg_fine_co_rank<K>), dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, (const K*)A,
                     a_off, (const K*)B, b_off, N, tile, nb, G, (const uint64_t*)jc, (const uint32_t*)sc, bj, bs,
                     flag);
  return launch_status();
}

template <typename K>
int Launch<K>::seg_merge_blocks(bool val, const Choice& ch, const void* A, const uint32_t* Av, const uint64_t* a_off,
                                const void* B, const uint32_t* Bv, const uint64_t* b_off, uint32_t S, uint64_t N,
                                void* C, uint32_t* Cv, const uint64_t* bj, const uint32_t* bs, uint64_t tiles,
                                const uint32_t* flag, hipStream_t st) {
  return by_cfg(ch.cfg, [&](auto nt, auto e) -> int {
    constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
    static_assert((NT * E) % 4 == 0, "blocks must start at multiples of 4 outputs");
    // outputs 16-byte aligned: 16-byte stores (the inputs are staged element-wise)
    const bool vst = val ? all_aligned16({C, Cv}) : all_aligned16({C});
    auto go = [&](auto val_c, auto vst_c) {
      constexpr bool V = decltype(val_c)::value, W = decltype(vst_c)::value;
      hipLaunchKernelGGL((k_seg_merge_blocks<K, V, NT, E, W>),
                         dim3(launch_grid((const void*)k_seg_merge_blocks<K, V, NT, E, W>, NT, tiles, ch.grid)),
                         dim3(NT), 0, st, (const K*)A, Av, a_off, (const K*)B, Bv, b_off, S, N, (K*)C, Cv, bj, bs,
                         tiles, flag, ch.search);
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    if (val && vst)
      go(T_{}, T_{});
    else if (val)
      go(T_{}, F_{});
    else if (vst)
      go(F_{}, T_{});
    else
      go(F_{}, F_{});
    return launch_status();
  });
}

template <typename K>
int Launch<K>::batch_co_ranks(const Choice& ch, const Shape& sh, const void* d, const uint32_t* sm, uint64_t tile,
                              uint64_t nb, uint64_t* bj, uint64_t* coarse, hipStream_t st) {
  const MergeDesc* q = (const MergeDesc*)d;
  if (ch.partition == 0) {
    hipLaunchKernelGGL((k_batch_co_rank<K>), dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, q, sm, tile, nb,
                       bj, ch.search);
    return launch_status();
  }
  const uint32_t G = sh.coarse_stride;
  const uint64_t nc = (nb + G - 1) / G;  // coarse slots 0, G, 2G, ... below nb
  if (ch.partition == 1)
    hipLaunchKernelGGL((k_batch_coarse_co_rank<K, 64>), dim3((unsigned)((nc + 3) / 4)), dim3(256), 0, st, q, sm,
                       tile, G, nc, coarse);
  else
    hipLaunchKernelGGL((k_batch_coarse_co_rank<K, 16>), dim3((unsigned)((nc + 15) / 16)), dim3(256), 0, st, q, sm,
                       tile, G, nc, coarse);
  if (launch_status() != CM_OK) return CM_EHIP;
  hipLaunchKernelGGL((k_batch_fine_co_rank<K>), dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, q, sm, tile,
                     nb, G, (const uint64_t*)coarse, bj);
  return launch_status();
}

template <typename K>
int Launch<K>::batch_merge_blocks(bool val, const Choice& ch, int form, const void* h, const void* d, uint32_t count,
                                  const uint32_t* bm, const uint64_t* bj, uint64_t tiles, bool vec, int xcd,
                                  hipStream_t st) {
  static_assert(kInlineDescs == kBatchInline, "inline descriptor counts differ");
  DescPack pk;
  memset(&pk, 0, sizeof pk);
  if (form == kBatchArgs) memcpy(pk.d, h, (size_t)std::min(count, kInlineDescs) * sizeof(MergeDesc));
  return by_cfg(ch.cfg, [&](auto nt, auto e) -> int {
    constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
    const dim3 b(NT);
    const MergeDesc* q = (const MergeDesc*)d;
    auto go = [&](auto val_c, auto vec_c) {
      constexpr bool V = decltype(val_c)::value, W = decltype(vec_c)::value;
      if (form == kBatchArgs) {
        const dim3 g(launch_grid((const void*)k_batch_merge_blocks_args<K, V, NT, E, W>, NT, tiles, ch.grid));
        hipLaunchKernelGGL((k_batch_merge_blocks_args<K, V, NT, E, W>), g, b, 0, st, pk, count, tiles, ch.search,
                           xcd);
      } else if (form == kBatchSelf) {
        const dim3 g(launch_grid((const void*)k_batch_merge_blocks<K, V, NT, E, W, true>, NT, tiles, ch.grid));
        hipLaunchKernelGGL((k_batch_merge_blocks<K, V, NT, E, W, true>), g, b, 0, st, q, bm, bj, tiles, ch.search,
                           xcd);
      } else {
        const dim3 g(launch_grid((const void*)k_batch_merge_blocks<K, V, NT, E, W, false>, NT, tiles, ch.grid));
        hipLaunchKernelGGL((k_batch_merge_blocks<K, V, NT, E, W, false>), g, b, 0, st, q, bm, bj, tiles, ch.search,
                           xcd);
      }
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
}

template <typename K>
int Launch<K>::co_rank_many(int search, const uint64_t* ranks, uint64_t q, const void* A, uint64_t m, const void* B,
                            uint64_t n, uint64_t* j_out, hipStream_t st) {
  hipLaunchKernelGGL((k_co_rank_many<K>), dim3((unsigned)((q + 255) / 256)), dim3(256), 0, st, ranks, q,
                     (const K*)A, m, (const K*)B, n, j_out, search);
  return launch_status();
}

template <typename K>
int Launch<K>::stream_resident(bool val, int cfg) {
  return by_cfg(cfg, [&](auto nt, auto e) -> int {
    constexpr int NT = decltype(nt)::value, E = decltype(e)::value;
    return val ? (int)resident_workgroups((const void*)k_merge_stream<K, true, NT, E>, NT)
               : (int)resident_workgroups((const void*)k_merge_stream<K, false, NT, E>, NT);
  });
}

template <typename K>
int Launch<K>::check_sorted(const void* X, uint64_t len, uint32_t* flag, uint64_t blocks, hipStream_t st) {
  hipLaunchKernelGGL((k_check_sorted<K>), dim3((unsigned)blocks), dim3(256), 0, st, (const K*)X, len, flag);
  return launch_status();
}

template <typename K>
int Launch<K>::cross_rank_cuts(const void* A, uint64_t m, const void* B, uint64_t n, uint32_t h, uint64_t* ia,
                               uint64_t* ja, uint64_t* ib, uint64_t* jb, unsigned blocks, hipStream_t st) {
  hipLaunchKernelGGL((k_cross_rank_cuts<K>), dim3(blocks), dim3(256), 0, st, (const K*)A, m, (const K*)B, n, h, ia,
                     ja, ib, jb);
  return launch_status();
}

}  // namespace cm
