// The outer reduceSeq of a strategy: the fold of G chunk values, shared by
// the reduction kernels and the batched engine.
#pragma once

#include "device.h"
#include "plan.h"

namespace dpia {

// Kahan pairs have value s - c, Sum2 pairs s + c; "64": the chunk values are
// folded in binary64.
enum : int {
  kFinalPlain = 0,
  kFinalKahan32 = 1,
  kFinalKahan64 = 2,
  kFinalSum2_32 = 3,
  kFinalSum2_64 = 4
};

// The outer reduceSeq over the G chunk values, from the literal 0, in chunk
// order, by one thread.  The work-group stages blocks of chunk values in LDS
// (coalesced), then thread 0 reads them back 32 at a time into registers
// and folds them in order.
// COHERENT: the chunk values are read with device-coherent loads (values
// written by other work-groups of the same launch with store_coherent).
// R: values thread 0 reads from LDS into registers at a time (fewer
// registers where the fold shares a kernel with other work).
template <class A, int FINAL, bool COHERENT = false, int R = 32>
__device__ void final_fold(const typename A::T* partials, int64_t G, void* out, int out_f64,
                           typename A::T* buf) {
  using T = typename A::T;
  T acc = A::zero();
  double acc64 = 0.0;
  auto fold1 = [&](const T& e) {
    if constexpr (FINAL == kFinalKahan64)
      acc64 = (static_cast<double>(e.s) - static_cast<double>(e.c)) + acc64;
    else if constexpr (FINAL == kFinalSum2_64)
      acc64 = (static_cast<double>(e.s) + static_cast<double>(e.c)) + acc64;
    else
      acc = A::add(e, acc);
  };
  for (int64_t b = 0; b < G; b += kFoldBlock) {
    const int cnt = static_cast<int>(G - b < kFoldBlock ? G - b : kFoldBlock);
    for (int i = threadIdx.x; i < cnt; i += blockDim.x)
      buf[i] = COHERENT ? load_coherent(partials + b + i) : partials[b + i];
    __syncthreads();
    if (threadIdx.x == 0) {
      int i = 0;
      for (; i + R <= cnt; i += R) {
        T r[R];
#pragma unroll
        for (int j = 0; j < R; ++j) r[j] = buf[i + j];
#pragma unroll
        for (int j = 0; j < R; ++j) fold1(r[j]);
      }
      for (; i < cnt; ++i) fold1(buf[i]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if constexpr (FINAL == kFinalKahan64 || FINAL == kFinalSum2_64) {
      if (out_f64)
        *static_cast<double*>(out) = acc64;
      else
        *static_cast<float*>(out) = static_cast<float>(acc64);
    } else if constexpr (FINAL == kFinalKahan32) {
      *static_cast<float*>(out) = acc.s - acc.c;
    } else if constexpr (FINAL == kFinalSum2_32) {
      *static_cast<float*>(out) = acc.s + acc.c;
    } else {
      *static_cast<T*>(out) = acc;
    }
  }
}

}  // namespace dpia
