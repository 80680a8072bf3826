// Host helpers shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <type_traits>

#include "plan.h"

namespace dpia {

// Number of compute units of the current device (cached per device id).
inline int device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v > 0) return v;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  cache[dev].store(cus, std::memory_order_relaxed);
  return cus;
}

// Work-groups to launch: one per group of `teams_per_wg` items, capped at
// what the device keeps resident (or at the strategy's max_grid).  The
// kernels distribute items by a grid-stride loop, so this never changes a
// result.
inline int64_t grid_size(const Plan& p) {
  int64_t need = (p.items + p.teams_per_wg - 1) / p.teams_per_wg;
  int64_t cap = p.max_grid ? static_cast<int64_t>(p.max_grid)
                           : static_cast<int64_t>(device_cus()) *
                                 (2048 / p.wg_threads > 0 ? 2048 / p.wg_threads : 1);
  return need < cap ? need : cap;
}

inline bool aligned16(const void* ptr) {
  return (reinterpret_cast<uintptr_t>(ptr) & 15u) == 0;
}

inline dpia_status hip_fail(hipError_t e, const std::string& what) {
  set_detail(what + ": " + hipGetErrorString(e));
  return DPIA_ERR_HIP;
}

inline dpia_status bad(dpia_status st, const std::string& msg) {
  set_detail(msg);
  return st;
}

template <int N>
using ic = std::integral_constant<int, N>;

// Calls f(ic<nv>{}) for a runtime vector width nv in {1, 2, 4, ..., MAX}.
template <int MAX, class F>
hipError_t with_nv(int nv, F&& f) {
  switch (nv) {
    case 1: return f(ic<1>{});
    case 2: if constexpr (MAX >= 2) return f(ic<2>{}); break;
    case 4: if constexpr (MAX >= 4) return f(ic<4>{}); break;
    case 8: if constexpr (MAX >= 8) return f(ic<8>{}); break;
    case 16: if constexpr (MAX >= 16) return f(ic<16>{}); break;
  }
  return hipErrorInvalidValue;
}

template <class F>
hipError_t with_order_combine(uint32_t order, uint32_t combine, F&& f) {
  if (order == DPIA_ORDER_STRIDED) {
    if (combine == DPIA_COMBINE_TREE) return f(ic<1>{}, ic<0>{});
    return f(ic<1>{}, ic<1>{});
  }
  if (combine == DPIA_COMBINE_TREE) return f(ic<0>{}, ic<0>{});
  return f(ic<0>{}, ic<1>{});
}

}  // namespace dpia
