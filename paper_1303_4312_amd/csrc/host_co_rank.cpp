// Co-rank on host arrays: Algorithm 1 of Section 2 (Siebert and Traeff,
// arXiv:1303.4312), run on the CPU for callers whose arrays live in host
// memory.  Same search as the device code: both Lemma 1 conditions are
// tested with their index guards first, so no sentinel position is read.
#include <stdint.h>

#include "corank_merge.h"
#include "order.hpp"

namespace {

template <typename K>
uint64_t co_rank_alg1(uint64_t i, const K* A, uint64_t m, const K* B, uint64_t n) {
  uint64_t j = i < m ? i : m;
  uint64_t k = i - j;
  uint64_t j_low = i > n ? i - n : 0;
  uint64_t k_low = 0;  // assigned in the first round before it is read
  for (;;) {
    if (j > 0 && k < n && A[j - 1] > B[k]) {
      const uint64_t d = (j - j_low + 1) / 2;
      k_low = k;
      j -= d;
      k += d;
    } else if (k > 0 && j < m && B[k - 1] >= A[j]) {
      const uint64_t d = (k - k_low + 1) / 2;
      j_low = j;
      j += d;
      k -= d;
    } else {
      return j;
    }
  }
}

}  // namespace

extern "C" int cm_co_rank_host(int key_type, uint64_t i, const void* A, uint64_t m, const void* B, uint64_t n,
                               uint64_t* j, uint64_t* k) {
  if (key_type < CM_KEY_U32 || key_type > CM_KEY_F32_DESC) return CM_EDTYPE;
  if (!j || !k || (m && !A) || (n && !B) || m + n < m) return CM_EINVAL;
  if (i > m + n) return CM_ERANGE;
  uint64_t jj;
  switch (key_type) {
    case CM_KEY_U32:
      jj = co_rank_alg1(i, static_cast<const uint32_t*>(A), m, static_cast<const uint32_t*>(B), n);
      break;
    case CM_KEY_U64:
      jj = co_rank_alg1(i, static_cast<const uint64_t*>(A), m, static_cast<const uint64_t*>(B), n);
      break;
    case CM_KEY_F32:
      jj = co_rank_alg1(i, static_cast<const float*>(A), m, static_cast<const float*>(B), n);
      break;
    case CM_KEY_U32_DESC:
      jj = co_rank_alg1(i, static_cast<const cm::Desc<uint32_t>*>(A), m, static_cast<const cm::Desc<uint32_t>*>(B),
                        n);
      break;
    case CM_KEY_U64_DESC:
      jj = co_rank_alg1(i, static_cast<const cm::Desc<uint64_t>*>(A), m, static_cast<const cm::Desc<uint64_t>*>(B),
                        n);
      break;
    default:
      jj = co_rank_alg1(i, static_cast<const cm::Desc<float>*>(A), m, static_cast<const cm::Desc<float>*>(B), n);
      break;
  }
  *j = jj;
  *k = i - jj;
  return CM_OK;
}
