// Key orders.  The method merges under any total order on keys (Section 2
// only asks for an ordering <= with ties broken A first).  Desc<K> holds the
// same bits as K and reverses every comparison, so each template that orders
// keys with <=, <, >=, > merges and sorts in nonincreasing order; ties still
// go A first (merge) or keep input order (sort).
#pragma once

#include <stdint.h>

#include <limits>
#include <type_traits>

#if defined(__HIPCC__)
#define CM_HD __host__ __device__
#else
#define CM_HD
#endif

namespace cm {

template <typename K>
struct Desc {
  K v;
  CM_HD friend bool operator<=(Desc a, Desc b) { return b.v <= a.v; }
  CM_HD friend bool operator<(Desc a, Desc b) { return b.v < a.v; }
  CM_HD friend bool operator>=(Desc a, Desc b) { return b.v >= a.v; }
  CM_HD friend bool operator>(Desc a, Desc b) { return b.v > a.v; }
  CM_HD friend bool operator==(Desc a, Desc b) { return a.v == b.v; }
};
static_assert(sizeof(Desc<uint32_t>) == 4 && sizeof(Desc<uint64_t>) == 8 && sizeof(Desc<float>) == 4,
              "Desc keeps the key's layout");

template <typename K>
struct is_desc : std::false_type {};
template <typename K>
struct is_desc<Desc<K>> : std::true_type {};

// The last key of the order (sort pads short runs with it): the largest
// value ascending, the smallest descending; +-infinity for floats.
template <typename K>
CM_HD K key_last() {
  if constexpr (is_desc<K>::value) {
    using R = decltype(K{}.v);
    if constexpr (std::is_same<R, float>::value)
      return K{-std::numeric_limits<float>::infinity()};
    else
      return K{R(0)};
  } else if constexpr (std::is_same<K, float>::value) {
    return std::numeric_limits<float>::infinity();
  } else {
    return ~K(0);
  }
}

}  // namespace cm
