// The outer reduceSeq of a strategy: the fold of G chunk values, shared by
// the reduction kernels and the batched engine.
#pragma once

#include <type_traits>

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
// order, by one thread.  `buf` (kFoldBlock values of LDS) holds two halves.
// The work-group copies the chunk values into them a step at a time; while
// thread 0 folds one half, every thread already has its loads of the next
// step's values in flight (issued together, into registers), and writes them
// to the other half when the fold of this one has been issued.  Thread 0
// reads its half back R values at a time, the next R requested before the
// current R are added, so the chain of additions waits on memory once per
// step and on LDS once per block of 16 groups.
// COHERENT: the chunk values are read with device-coherent loads (values
// written by other work-groups of the same launch with store_coherent).
// R: values thread 0 holds in registers per group (three groups at once);
// LOADS: loads in flight per thread, at most.  Kernels that carry the fold
// beside other work (1 pass) pass smaller ones, so that the fold does not
// raise their register count.
// fold_values continues the fold from (acc, acc64) over partials[0 .. G);
// the results are thread 0's.  final_fold folds from the literal 0 and
// writes the strategy's result.
template <class A, int FINAL, bool COHERENT = false,
          int R = (sizeof(typename A::T) > 4 ? 8 : 16), int LOADS = 8>
__device__ void fold_values(const typename A::T* partials, int64_t G, typename A::T* buf,
                            typename A::T& acc, double& acc64) {
  using T = typename A::T;
  constexpr int kHalf = kFoldBlock / 2;
  constexpr int kLoads = LOADS;
  auto fold1 = [&](const T& e) {
    if constexpr (FINAL == kFinalKahan64)
      acc64 = (static_cast<double>(e.s) - static_cast<double>(e.c)) + acc64;
    else if constexpr (FINAL == kFinalSum2_64)
      acc64 = (static_cast<double>(e.s) + static_cast<double>(e.c)) + acc64;
    else
      acc = A::add(e, acc);
  };
  const int nt = static_cast<int>(blockDim.x);
  const int step = nt * kLoads < kHalf ? nt * kLoads : kHalf;   // values per half
  const int mine = (step + nt - 1) / nt;                        // loads per thread
  T reg[kLoads];
  // this thread's values of [b, b + step), clamped into [0, G) (uniform
  // trip count: every load is issued before any is waited for)
  auto fetch = [&](int64_t b) {
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
      if (k < mine) {
        int64_t i = b + threadIdx.x + static_cast<int64_t>(k) * nt;
        i = i < G ? i : G - 1;
        reg[k] = COHERENT ? load_coherent(partials + i) : partials[i];
      }
    }
  };
  auto put = [&](T* half, int64_t b) {
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
      const int i = static_cast<int>(threadIdx.x) + k * nt;
      if (k < mine && i < step && b + i < G) half[i] = reg[k];
    }
  };
  // thread 0: the fold of half[0 .. cnt) in index order, in unrolled blocks
  // of kBlock groups of R values.  Within a block the LDS reads of the next
  // two groups are in flight while the current group is added (straight-line
  // code, so the compiler waits for exactly the group it adds); the
  // scheduling barrier keeps the reads from being sunk down to their uses.
  auto fold_half = [&](const T* half, int cnt) {
    constexpr int kBlock = 16;
    T r[3][R];
    auto read = [&](T (&dst)[R], int at) {
#pragma unroll
      for (int j = 0; j < R; ++j) dst[j] = half[at + j];
      __builtin_amdgcn_sched_barrier(0);
    };
    int i = 0;
    if constexpr (std::is_integral_v<T>) {
      // addition modulo 2^32 is associative: any order gives the same
      // bits, and the compiler would reorder an unrolled block anyway
      for (; i < cnt; ++i) fold1(half[i]);
      return;
    }
    for (; i + kBlock * R <= cnt; i += kBlock * R) {
      read(r[0], i);
      read(r[1], i + R);
#pragma unroll
      for (int grp = 0; grp < kBlock; ++grp) {
        if (grp + 2 < kBlock) read(r[(grp + 2) % 3], i + (grp + 2) * R);
#pragma unroll
        for (int j = 0; j < R; ++j) fold1(r[grp % 3][j]);
      }
    }
    for (; i + R <= cnt; i += R) {
      read(r[0], i);
#pragma unroll
      for (int j = 0; j < R; ++j) fold1(r[0][j]);
    }
    for (; i < cnt; ++i) fold1(half[i]);
  };
  if (G > 0) {
    fetch(0);
    put(buf, 0);
  }
  __syncthreads();
  int h = 0;
  for (int64_t b = 0; b < G; b += step, h ^= 1) {
    const int cnt = static_cast<int>(G - b < step ? G - b : step);
    const bool more = b + step < G;
    if (more) fetch(b + step);
    if (threadIdx.x == 0) fold_half(buf + h * kHalf, cnt);
    if (more) put(buf + (h ^ 1) * kHalf, b + step);
    __syncthreads();
  }
}

// The strategy's result from the fold's accumulator (thread 0 writes it).
template <class A, int FINAL>
__device__ void write_fold(const typename A::T& acc, double acc64, void* out, int out_f64) {
  using T = typename A::T;
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

template <class A, int FINAL, bool COHERENT = false,
          int R = (sizeof(typename A::T) > 4 ? 8 : 16), int LOADS = 8>
__device__ void final_fold(const typename A::T* partials, int64_t G, void* out, int out_f64,
                           typename A::T* buf) {
  typename A::T acc = A::zero();
  double acc64 = 0.0;
  fold_values<A, FINAL, COHERENT, R, LOADS>(partials, G, buf, acc, acc64);
  write_fold<A, FINAL>(acc, acc64, out, out_f64);
}

}  // namespace dpia
