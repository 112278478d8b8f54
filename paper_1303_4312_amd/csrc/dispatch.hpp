// Host-side template dispatch shared by the launcher files: key type and
// tile configuration (the cases of by_cfg must match kCfgs in api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "corank_merge.h"
#include "order.hpp"

namespace cm {

inline int launch_status() { return hipGetLastError() == hipSuccess ? CM_OK : CM_EHIP; }

template <typename F>
int by_key(int kt, F&& f) {
  switch (kt) {
    case CM_KEY_U32: return f(uint32_t{});
    case CM_KEY_U64: return f(uint64_t{});
    case CM_KEY_F32: return f(float{});
    case CM_KEY_U32_DESC: return f(Desc<uint32_t>{});
    case CM_KEY_U64_DESC: return f(Desc<uint64_t>{});
    case CM_KEY_F32_DESC: return f(Desc<float>{});
    default: return CM_EDTYPE;
  }
}

// Calls f(std::integral_constant<int, NT>, std::integral_constant<int, E>)
// for configuration cfg.
template <typename F>
int by_cfg(int cfg, F&& f) {
  switch (cfg) {
    case 0: return f(std::integral_constant<int, 256>{}, std::integral_constant<int, 7>{});
    case 1: return f(std::integral_constant<int, 256>{}, std::integral_constant<int, 11>{});
    case 2: return f(std::integral_constant<int, 256>{}, std::integral_constant<int, 15>{});
    case 3: return f(std::integral_constant<int, 128>{}, std::integral_constant<int, 7>{});
    case 4: return f(std::integral_constant<int, 512>{}, std::integral_constant<int, 7>{});
    case 5: return f(std::integral_constant<int, 256>{}, std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 256>{}, std::integral_constant<int, 9>{});
    case 7: return f(std::integral_constant<int, 512>{}, std::integral_constant<int, 11>{});
    default: return CM_ECONFIG;
  }
}

}  // namespace cm
