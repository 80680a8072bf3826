// dot and asum under a DPIA strategy (blocked dot product, Sec. 2.1 eq. (2);
// asum and dot are benchmarks of Sec. 7.1).
//
// Kernel 1 evaluates the mapWorkgroup level: every chunk of W = L*C elements
// is reduced by one team (lane folds, then the work-group combine) and its
// value is written to the workspace, partial[g] (the hoisted newGlobal
// temporary of Sec. 6.3: one slot per parforWorkgroup iteration).  The outer
// reduceSeq over partial[0..G) from +0 in chunk order then runs either in a
// second kernel (2 passes) or in the last work-group to finish (1 pass:
// device-coherent chunk-value stores, an integer arrival counter, coherent
// loads in the last work-group).  Both evaluate the same expression and give
// the same bits.
#include <mutex>

#include "device.h"
#include "fed.h"
#include "fold.h"
#include "ops.h"
#include "host.h"
#include "plan.h"

namespace dpia {

struct ReduceArgs {
  int64_t items;          // G chunks
  int64_t values;         // values the outer fold reads (G * values per chunk)
  int64_t n;              // elements; the last chunk may be partly beyond n
  int64_t W;
  int L, C, team, teams_per_wg;
  int team_lds_elems;     // LDS elements of T per team
  int stage_off;          // byte offset of the LDS staging region, -1: none
  int one_pass;
  int out_f64;            // Kahan 64 only: write a double
  void* partials;
  unsigned int* counter;
  void* nodes;            // split teams: kSplitMax nodes per chunk, or nullptr
  unsigned int* node_cnt; // split teams: one arrival count per chunk
  void* out;
};

// MAXT: the largest work-group it is launched with (256 or 1024); the
// 256-thread build may use more registers than the 1024-thread one.
template <class Op, int ORDER, int NV, int COMBINE, int FINAL, int VEC, int MAXT>
__global__ void __launch_bounds__(MAXT) reduce_kernel(Op op, ReduceArgs a) {
  using T = typename Op::T;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int is_last;
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int team_id = threadIdx.x / a.team;
  const int t = threadIdx.x - team_id * a.team;
  T* scratch = lds + team_id * a.team_lds_elems;
  float* stage = a.stage_off < 0 ? nullptr
                                 : reinterpret_cast<float*>(lds_raw + a.stage_off) +
                                       (threadIdx.x / kWave) * stage_floats(kWave);
  T* partials = static_cast<T*>(a.partials);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * a.teams_per_wg;
  // parforWorkgroup as a grid-stride loop: every thread of a work-group
  // runs the same iterations, so the barriers inside are uniform
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * a.teams_per_wg; base < a.items;
       base += stride) {
    const int64_t g = base + team_id;
    const bool active = g < a.items;
    const auto view = op.chunk(active ? g : 0, a.W);
    const int64_t rest = a.n - g * a.W;
    const int limit = static_cast<int>(rest < a.W ? rest : a.W);
    if constexpr (VEC == 1 && COMBINE != kNone) {
      const T v = chunk_value<Op, ORDER, NV, COMBINE>(view, active, t, a.team, a.L, a.C, limit,
                                                      scratch, stage);
      if (active && t == 0) store_coherent(partials + g, v);
    } else {
      chunk_values_wide<Op, ORDER, NV, COMBINE, VEC>(view, active, t, a.team, a.L, a.C, limit,
                                                     scratch, partials, g, stage);
    }
  }
  if (a.one_pass) {
    // Chunk values were written with device-coherent stores; each thread
    // waits for its own to complete, the barrier then puts all of this
    // work-group's before the arrival counter, and the last work-group to
    // arrive reads them back with device-coherent loads.  No L2 write-back
    // per work-group.
    wait_memory();
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned prev =
          __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (is_last) {
      final_fold<typename Op::Arith, FINAL, true, (sizeof(T) > 4 ? 4 : 8), 4>(
          partials, a.values, a.out, a.out_f64, lds);
      if (threadIdx.x == 0)   // leave the counter at zero for the next call
        __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

#ifndef DPIA_FED
#define DPIA_FED 1
#endif

// The mapWorkgroup level of a strategy with few chunks, fed by loader
// wavefronts (fed.h): staged contiguous lanes (teams of 64, 128 or 256 lanes,
// one per thread) or scalar strided lanes.  Each work-group takes ROWS lanes
// of one chunk (a slice; L / ROWS slices per chunk), its wave 0 folds them,
// one lane per thread, and waves 1 .. kFedLoaders load.  Uncombined slices store their lanes' values.  A tree
// combine over a split team: each slice reduces its ROWS lanes with the
// team's butterfly levels below ROWS and stores that node (device-coherent);
// the slice whose arrival completes the chunk's count applies the levels
// from ROWS up to the team over the nodes in lane order, which is the same
// tree (the levels are hierarchical), and stores the chunk value.  Lane rows
// that are not whole (the last chunk, when W does not divide n) are folded
// by wave 0 alone, as reduce_kernel folds them.  The same chunk values, the
// same 1-pass arrival and fold as reduce_kernel.
template <class Op, int ORDER, int COMBINE, int FINAL, int VEC, int ROWS>
__global__ void __launch_bounds__(kWave*(1 + kFedLoaders)) fed_reduce_kernel(Op op,
                                                                               ReduceArgs a) {
  using T = typename Op::T;
  using A = typename Op::Arith;
  static_assert(COMBINE != kSeq, "a sequential combine has barriers of the team alone");
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ int is_last;
  T* lds = reinterpret_cast<T*>(lds_raw);
  float* ring = reinterpret_cast<float*>(lds_raw + a.stage_off);
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  T* partials = static_cast<T*>(a.partials);
  static_assert(ORDER == kContiguous || VEC == 1, "strided slices are scalar lanes");
  const int Cel = a.C * VEC;
  const int S = a.L / ROWS;   // slices per chunk
  for (int64_t w = blockIdx.x; w < a.items * S; w += gridDim.x) {
    const int64_t g = w / S;
    const int s = static_cast<int>(w % S);
    const int row0 = s * ROWS;
    const auto view = op.chunk(g, a.W);
    const int64_t rest = a.n - g * a.W;
    const int limit = static_cast<int>(rest < a.W ? rest : a.W);
    T acc[VEC];
    if constexpr (ORDER == kStrided) {
      if (limit == a.W)
        fed_fold_strided<Op, ROWS>(view, a.L, a.C, wave, lane, row0, ring, acc[0]);
      else if (wave == 0)
        lane_folds<Op, kStrided, 1>(view, lane < ROWS, row0 + lane, a.L, a.C, limit, acc);
    } else {
      if (limit == a.W)
        fed_fold<Op, VEC, ROWS>(view, Cel, wave, lane, row0, ring, acc);
      else if (wave == 0)
        contiguous_staged<Op, VEC>(view, lane < ROWS, row0 + lane, a.C, limit, acc, ring);
    }
    if (wave == 0) {
      if constexpr (COMBINE == kNone) {
        if (lane < ROWS) {
          const int64_t l = g * a.L + row0 + lane;
#pragma unroll
          for (int j = 0; j < VEC; ++j) store_coherent(partials + l * VEC + j, acc[j]);
        }
      } else if (S == 1) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
          T one[1] = {acc[j]};
          const T c = combine_lanes<A, 1, COMBINE>(one, lane, kWave, a.L, lds);
          if (lane == 0) store_coherent(partials + g * VEC + j, c);
        }
      } else if constexpr (VEC == 1) {
        T one[1] = {acc[0]};
        const T node = combine_lanes<A, 1, COMBINE>(one, lane, ROWS, a.L, lds);
        T* nodes = static_cast<T*>(a.nodes) + g * kSplitMax;
        unsigned last = 0;
        if (lane == 0) {
          store_coherent(nodes + s, node);
          wait_memory();
          last = __hip_atomic_fetch_add(a.node_cnt + g, 1u, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) == static_cast<unsigned>(S - 1);
        }
        if (__shfl(last, 0)) {   // every slice's node is stored
          T v = lane < S ? load_coherent(nodes + lane) : A::zero();
          butterfly_levels<A>(v, lane, S);
          if (lane == 0) {
            store_coherent(partials + g, v);
            __hip_atomic_store(a.node_cnt + g, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
    }
    __syncthreads();   // the ring may be written for the next slice
  }
  if (a.one_pass) {
    wait_memory();
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned prev =
          __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (is_last) {
      final_fold<typename Op::Arith, FINAL, true, (sizeof(T) > 4 ? 4 : 8), 4>(
          partials, a.values, a.out, a.out_f64, lds);
      if (threadIdx.x == 0)
        __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <class A, int FINAL>
__global__ void __launch_bounds__(256) final_kernel(const typename A::T* partials, int64_t G,
                                                    void* out, int out_f64) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  final_fold<A, FINAL>(partials, G, out, out_f64, reinterpret_cast<typename A::T*>(lds_raw));
}

template <class Op>
ReduceArgs reduce_args(const Plan& p, void* partials, void* counter, void* out, int out_f64,
                       bool one_pass) {
  ReduceArgs a{};
  a.items = p.items;
  a.values = p.values;
  a.n = p.n;
  a.W = p.W;
  a.L = static_cast<int>(p.L);
  a.C = static_cast<int>(p.C);
  a.team = p.team;
  a.teams_per_wg = p.teams_per_wg;
  a.team_lds_elems = (p.combine == DPIA_COMBINE_SEQ) ? static_cast<int>(p.L)
                                                     : (p.team > 64 ? p.team / 64 : 1);
  a.stage_off = p.stage ? static_cast<int>(p.stage_off) : -1;
  a.out_f64 = out_f64;
  a.partials = partials;
  a.counter = static_cast<unsigned int*>(counter);
  a.out = out;
  a.one_pass = one_pass ? 1 : 0;
  return a;
}

// Calls f(order, combine, nv, vec constants) for a plan.  Vector and
// uncombined shapes exist for the plain operations only (WIDE).
template <bool WIDE, class F>
hipError_t with_reduce_shape(const Plan& p, F&& f) {
  constexpr int MAXNV = kVecBytes / static_cast<int>(sizeof(float));
  if (p.V == 1 && p.combine != DPIA_COMBINE_NONE) {
    return with_order_combine(p.order, p.combine, [&](auto ord, auto comb) {
      return with_nv<MAXNV>(p.nv, [&](auto nvc) { return f(ord, comb, nvc, ic<1>{}); });
    });
  }
  if constexpr (WIDE) {
    auto by_order = [&](auto comb, auto nvc, auto vec) {
      if (p.order == DPIA_ORDER_STRIDED) return f(ic<kStrided>{}, comb, nvc, vec);
      return f(ic<kContiguous>{}, comb, nvc, vec);
    };
    if (p.V == 1)
      return with_nv<MAXNV>(p.nv, [&](auto nvc) { return by_order(ic<kNone>{}, nvc, ic<1>{}); });
    auto by_combine = [&](auto vec) {
      if (p.combine == DPIA_COMBINE_TREE) return by_order(ic<kTree>{}, vec, vec);
      if (p.combine == DPIA_COMBINE_SEQ) return by_order(ic<kSeq>{}, vec, vec);
      return by_order(ic<kNone>{}, vec, vec);
    };
    if (p.V == 2) return by_combine(ic<2>{});
    if (p.V == 4) return by_combine(ic<4>{});
  }
  return hipErrorInvalidValue;
}

// Lane rows per work-group when a plan's chunks are folded by
// fed_reduce_kernel (0: they are not): staged contiguous lanes, one lane per
// thread, fewer chunks than compute units (otherwise the launch has
// wavefronts enough), and a chunk's tiles a multiple of the loaders' depth
// for that row count.  A compute unit streams at most about 37 GB/s, so the
// chunks' lanes are split over as many work-groups as the compute units
// allow: uncombined lanes into 2 or 4 slices of a 64-lane team, tree-combined
// teams of 64, 128 or 256 lanes into up to kSplitMax slices when the call
// brings the workspace's split region (`can_split`); a 64-lane tree team may
// also stay whole.
template <int NOPS>
int fed_rows_strided(const Plan& p, bool can_split) {
  // scalar strided lanes, L a power of two from 16 to 512, whole tiles of
  // kFedStrideRows steps; a tree needs the split region beyond one slice
  if (p.V != 1 || p.combine == DPIA_COMBINE_SEQ) return 0;
  if (p.L < 16 || p.L > 512 || (p.L & (p.L - 1)) || p.C % kFedStrideRows) return 0;
  const int64_t cus = device_cus();
  if (p.items >= cus) return 0;
  const bool split = can_split && p.split_off;
  const int64_t ntiles = p.C / kFedStrideRows;
  auto fits = [&](int depth) { return ntiles >= depth && ntiles % depth == 0; };
  auto ok = [&](int rows, int depth) {
    const int64_t per = p.L / rows;
    if (rows > p.L || p.items * per > cus || !fits(depth)) return false;
    if (p.combine == DPIA_COMBINE_TREE && per > 1 && (!split || per > kSplitMax)) return false;
    return true;
  };
  if (ok(16, fed_depth<16, NOPS>())) return 16;
  if (ok(32, fed_depth<32, NOPS>())) return 32;
  if (ok(kWave, fed_depth<kWave, NOPS>())) return kWave;
  return 0;
}

template <int NOPS>
int fed_rows(const Plan& p, bool can_split) {
  if (!DPIA_FED) return 0;
  if (p.op != DPIA_OP_DOT && p.op != DPIA_OP_ASUM) return 0;
  if (p.order == DPIA_ORDER_STRIDED) return fed_rows_strided<NOPS>(p, can_split);
  if (!p.stage || p.order != DPIA_ORDER_CONTIGUOUS) return 0;
  if (p.teams_per_wg != 1 || p.combine == DPIA_COMBINE_SEQ) return 0;
  if (p.V != 1 && p.V != 4) return 0;
  const bool split = can_split && p.split_off && p.combine == DPIA_COMBINE_TREE && p.V == 1;
  if (p.team != kWave && !(split && (p.team == 128 || p.team == 256))) return 0;
  const int64_t cus = device_cus();
  if (p.items >= cus || (p.C * p.V) % kFedStage) return 0;
  const int64_t ntiles = p.C * p.V / kFedStage;
  auto fits = [&](int depth) { return ntiles >= depth && ntiles % depth == 0; };
  if (p.combine == DPIA_COMBINE_NONE || split) {
    const int64_t per16 = p.team / 16, per32 = p.team / 32;   // slices per chunk
    if (per16 <= kSplitMax && p.items * per16 <= cus && fits(fed_depth<16, NOPS>())) return 16;
    if (per32 <= kSplitMax && p.items * per32 <= cus && fits(fed_depth<32, NOPS>())) return 32;
    if (p.items * (p.team / kWave) <= cus && fits(fed_depth<kWave, NOPS>())) return kWave;
    return 0;
  }
  return fits(fed_depth<kWave, NOPS>()) ? kWave : 0;
}

template <class Op, int FINAL>
hipError_t launch_fed(const Plan& p, const Op& op, const ReduceArgs& a, int rows,
                      hipStream_t stream) {
  const int64_t grid = p.items * (p.L / rows);
  // the ring from the start of the LDS: the kernel's combines within one
  // wavefront need no LDS, and the 1-pass fold uses it after the chunks
  size_t lds = static_cast<size_t>(fed_ring_floats()) * sizeof(float);
  const size_t fold = static_cast<size_t>(kFoldBlock) * sizeof(typename Op::T);
  if (fold > lds) lds = fold;
  lds = (lds + 16 + 15) / 16 * 16;
  Op op_copy = op;
  ReduceArgs a_copy = a;
  a_copy.stage_off = 0;
  void* args[] = {&op_copy, &a_copy};
  const bool strided = p.order == DPIA_ORDER_STRIDED;
  auto go = [&](auto comb, auto vec, auto nrows) {
    constexpr int COMBINE = decltype(comb)::value;
    constexpr int VEC = decltype(vec)::value;
    constexpr int ROWS = decltype(nrows)::value;
    auto kern = strided && VEC == 1
                    ? fed_reduce_kernel<Op, (VEC == 1 ? kStrided : kContiguous), COMBINE, FINAL,
                                        VEC, ROWS>
                    : fed_reduce_kernel<Op, kContiguous, COMBINE, FINAL, VEC, ROWS>;
    return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid),
                           dim3(kWave * (1 + kFedLoaders)), args, lds, stream);
  };
  auto by_rows = [&](auto comb, auto vec) {
    if (rows == 16) return go(comb, vec, ic<16>{});
    if (rows == 32) return go(comb, vec, ic<32>{});
    return go(comb, vec, ic<kWave>{});
  };
  if constexpr (FINAL != kFinalPlain) {
    return by_rows(ic<kTree>{}, ic<1>{});   // compensated: scalar, combined lanes
  } else {
    if (p.combine == DPIA_COMBINE_TREE)
      return p.V == 4 ? go(ic<kTree>{}, ic<4>{}, ic<kWave>{}) : by_rows(ic<kTree>{}, ic<1>{});
    return p.V == 4 ? by_rows(ic<kNone>{}, ic<4>{}) : by_rows(ic<kNone>{}, ic<1>{});
  }
}

// The mapWorkgroup level: chunk values into `partials`; with one_pass the
// last work-group also folds them into `out`.
template <class Op, int FINAL>
hipError_t launch_chunks(const Plan& p, const Op& op, const ReduceArgs& a, hipStream_t stream) {
  if (p.items == 0) return hipSuccess;
  // (the loaders keep the tiles in flight, so the deeper load batches of
  // DotF32Deep and DotF32Deeper would only add registers)
  const bool can_split = a.nodes != nullptr;
  if constexpr (std::is_same<Op, DotF32Deeper>::value || std::is_same<Op, DotF32Deep>::value) {
    if (const int rows = fed_rows<2>(p, can_split))
      return launch_fed<DotF32, FINAL>(p, DotF32{op.x, op.y}, a, rows, stream);
  } else if constexpr (Op::View::kStageable) {
    const int rows = fed_rows<Op::View::kOps>(p, can_split);
    if (rows && (FINAL == kFinalPlain || (p.V == 1 && p.combine == DPIA_COMBINE_TREE)))
      return launch_fed<Op, FINAL>(p, op, a, rows, stream);
  }
  const int64_t grid = grid_size(p);
  return with_reduce_shape<FINAL == kFinalPlain>(p, [&](auto ord, auto comb, auto nvc, auto vec) {
    constexpr int ORDER = decltype(ord)::value;
    constexpr int COMBINE = decltype(comb)::value;
    constexpr int NV = decltype(nvc)::value;
    constexpr int VEC = decltype(vec)::value;
    auto kern = p.wg_threads <= 256 ? reduce_kernel<Op, ORDER, NV, COMBINE, FINAL, VEC, 256>
                                    : reduce_kernel<Op, ORDER, NV, COMBINE, FINAL, VEC, 1024>;
    Op op_copy = op;
    ReduceArgs a_copy = a;
    void* args[] = {&op_copy, &a_copy};
    return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(p.wg_threads),
                           args, p.lds_bytes, stream);
  });
}

// The outer reduceSeq over G chunk values, as a kernel of its own.
template <class Op, int FINAL>
hipError_t launch_fold(int64_t G, const void* partials, void* out, int out_f64,
                       hipStream_t stream) {
  using T = typename Op::T;
  const T* pp = static_cast<const T*>(partials);
  void* args[] = {&pp, &G, &out, &out_f64};
  auto kern = final_kernel<typename Op::Arith, FINAL>;
  return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(1), dim3(256), args,
                         kFoldBlock * sizeof(T), stream);
}

// Both passes of a reduction: chunk values into `partials`, then the outer
// fold (1 pass: in the last work-group, which needs `counter` at zero and
// leaves it at zero; 2 passes: a second kernel).  `split`: the workspace's
// split region (p.split_off), or nullptr where the call has none.
template <class Op, int FINAL>
hipError_t launch_reduce(const Plan& p, const Op& op, void* out, int out_f64, void* partials,
                         void* counter, hipStream_t stream, void* split = nullptr) {
  const bool two_pass = p.passes == 2 || p.items == 0;
  ReduceArgs a = reduce_args<Op>(p, partials, counter, out, out_f64, !two_pass);
  if (split && p.split_off) {
    a.nodes = split;
    a.node_cnt = reinterpret_cast<unsigned int*>(
        static_cast<char*>(split) +
        (static_cast<size_t>(p.items) * kSplitMax * p.acc_bytes + kWsAlign - 1) / kWsAlign *
            kWsAlign);
  }
  hipError_t e = launch_chunks<Op, FINAL>(p, op, a, stream);
  if (e != hipSuccess || !two_pass) return e;
  return launch_fold<Op, FINAL>(p.values, partials, out, out_f64, stream);
}

#ifndef DPIA_DEEPER_DOT
#define DPIA_DEEPER_DOT 1
#endif

// Plain binary32 dots whose strided lanes form teams narrower than 1024
// lanes use a deeper load batch: DotF32Deep, or DotF32Deeper when the whole
// launch has fewer than two wavefronts per compute unit.  Contiguous dots
// staged through LDS whose launch has fewer wavefronts than compute units
// use DotF32Deeper too (two staged tiles in flight); unstaged contiguous
// dots keep the default batch (a deeper one would need 128 registers of
// loads in flight).
inline int dot_depth(const Plan& p) {
  const int64_t waves = p.items * ((p.team + 63) / 64);
  const int64_t cus = device_cus();
  if (p.order != DPIA_ORDER_STRIDED)
    return (DPIA_DEEPER_DOT && p.stage && waves < cus) ? 2 : 0;
  if (p.L >= 1024) return 0;
  return (DPIA_DEEPER_DOT && waves < 2 * cus) ? 2 : 1;
}

// Calls f(op, final-kind constant) for the operation and accumulation of a plan.
template <class F>
hipError_t with_reduction(const Plan& p, const void* x, const void* y, F&& f) {
  if (p.op == DPIA_OP_ASUM)
    return f(AsumF32{static_cast<const float*>(x)}, ic<kFinalPlain>{});
  if (p.dt == DPIA_I32)
    return f(DotU32{static_cast<const uint32_t*>(x), static_cast<const uint32_t*>(y)},
             ic<kFinalPlain>{});
  if (p.accum == DPIA_ACCUM_KAHAN) {
    KahanDotF32 op{static_cast<const float*>(x), static_cast<const float*>(y)};
    if (p.final_f64) return f(op, ic<kFinalKahan64>{});
    return f(op, ic<kFinalKahan32>{});
  }
  if (p.accum == DPIA_ACCUM_SUM2) {
    Sum2DotF32 op{static_cast<const float*>(x), static_cast<const float*>(y)};
    if (p.final_f64) return f(op, ic<kFinalSum2_64>{});
    return f(op, ic<kFinalSum2_32>{});
  }
  const int depth = dot_depth(p);
  if (depth == 2)
    return f(DotF32Deeper{{static_cast<const float*>(x), static_cast<const float*>(y)}},
             ic<kFinalPlain>{});
  if (depth == 1)
    return f(DotF32Deep{{static_cast<const float*>(x), static_cast<const float*>(y)}},
             ic<kFinalPlain>{});
  return f(DotF32{static_cast<const float*>(x), static_cast<const float*>(y)},
           ic<kFinalPlain>{});
}

namespace {

dpia_status check_ws(const Plan& p, void* ws, size_t ws_bytes) {
  if (ws_bytes < p.ws_bytes) {
    return bad(DPIA_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) +
                                       " bytes is smaller than the required " +
                                       std::to_string(p.ws_bytes));
  }
  if (p.ws_bytes && !ws) return bad(DPIA_ERR_WORKSPACE, "workspace is NULL");
  if (ws && (reinterpret_cast<uintptr_t>(ws) % kWsAlign))
    return bad(DPIA_ERR_SHAPE, "workspace must be 256-byte aligned");
  return DPIA_OK;
}

}  // namespace
}  // namespace dpia

using namespace dpia;

namespace {

// Shared body of dpia_dot and dpia_dot_noalloc after validation: the launches
// of a dot with its chunk values in `partials` and the 1-pass arrival
// counter at `counter`.
dpia_status dot_launch(const Plan& p, dpia_dtype dt, const void* x, const void* y, void* out,
                       dpia_dtype out_dt, void* partials, void* counter, hipStream_t hs,
                       const char* name, void* split = nullptr) {
  hipError_t e;
  if (dt == DPIA_I32) {
    e = launch_reduce<DotU32, kFinalPlain>(
        p, DotU32{static_cast<const uint32_t*>(x), static_cast<const uint32_t*>(y)}, out, 0,
        partials, counter, hs, split);
  } else if (p.accum == DPIA_ACCUM_KAHAN || p.accum == DPIA_ACCUM_SUM2) {
    const float* xf = static_cast<const float*>(x);
    const float* yf = static_cast<const float*>(y);
    const int f64 = out_dt == DPIA_F64;
    if (p.accum == DPIA_ACCUM_KAHAN) {
      KahanDotF32 op{xf, yf};
      e = p.final_f64 ? launch_reduce<KahanDotF32, kFinalKahan64>(p, op, out, f64, partials,
                                                                  counter, hs, split)
                      : launch_reduce<KahanDotF32, kFinalKahan32>(p, op, out, 0, partials,
                                                                  counter, hs, split);
    } else {
      Sum2DotF32 op{xf, yf};
      e = p.final_f64 ? launch_reduce<Sum2DotF32, kFinalSum2_64>(p, op, out, f64, partials,
                                                                 counter, hs, split)
                      : launch_reduce<Sum2DotF32, kFinalSum2_32>(p, op, out, 0, partials,
                                                                 counter, hs, split);
    }
  } else {
    const float* xf = static_cast<const float*>(x);
    const float* yf = static_cast<const float*>(y);
    const int depth = dot_depth(p);
    e = depth == 2 ? launch_reduce<DotF32Deeper, kFinalPlain>(p, DotF32Deeper{{xf, yf}}, out, 0,
                                                               partials, counter, hs, split)
        : depth == 1 ? launch_reduce<DotF32Deep, kFinalPlain>(p, DotF32Deep{{xf, yf}}, out, 0,
                                                              partials, counter, hs, split)
                     : launch_reduce<DotF32, kFinalPlain>(p, DotF32{xf, yf}, out, 0, partials,
                                                          counter, hs, split);
  }
  if (e != hipSuccess) return hip_fail(e, name);
  clear_detail();
  return DPIA_OK;
}

// Everything dpia_dot checks apart from the workspace.
dpia_status dot_validate(const dpia_strategy* s, dpia_dtype dt, int64_t n, const void* x,
                         const void* y, const void* out, dpia_dtype out_dt, Plan* p) {
  std::string detail;
  dpia_status st = make_plan(s, DPIA_OP_DOT, dt, 0, n, p, &detail);
  if (st != DPIA_OK) return bad(st, detail);
  if (!out || (n > 0 && (!x || !y))) return bad(DPIA_ERR_NULL, "x, y and out must be non-NULL");
  if (n > 0 && (!aligned16(x) || !aligned16(y)))
    return bad(DPIA_ERR_SHAPE, "x and y must be 16-byte aligned");
  if (dt == DPIA_I32) {
    if (out_dt != DPIA_I32) return bad(DPIA_ERR_DTYPE, "an I32 dot writes an I32 result");
  } else if (p->accum == DPIA_ACCUM_KAHAN || p->accum == DPIA_ACCUM_SUM2) {
    if (out_dt != DPIA_F32 && !(out_dt == DPIA_F64 && p->final_f64))
      return bad(DPIA_ERR_DTYPE, "a compensated dot writes F32, or F64 with final_f64");
  } else if (out_dt != DPIA_F32) {
    return bad(DPIA_ERR_DTYPE, "an F32 dot writes an F32 result");
  }
  return DPIA_OK;
}

}  // namespace

extern "C" dpia_status dpia_dot(const dpia_strategy* s, dpia_dtype dt, int64_t n, const void* x,
                                const void* y, void* out, dpia_dtype out_dt, void* ws,
                                size_t ws_bytes, dpia_stream_t stream) {
  Plan p;
  dpia_status st = dot_validate(s, dt, n, x, y, out, out_dt, &p);
  if (st != DPIA_OK) return st;
  st = check_ws(p, ws, ws_bytes);
  if (st != DPIA_OK) return st;
  void* split = p.split_off ? static_cast<char*>(ws) + p.split_off : nullptr;
  return dot_launch(p, dt, x, y, out, out_dt, ws, static_cast<char*>(ws) + p.partial_bytes,
                    reinterpret_cast<hipStream_t>(stream), "dpia_dot launch", split);
}

// ------------------------------------------------------------ no-alloc dot
// dpia_dot_noalloc keeps the chunk values and the arrival counter of a call
// in this file-scope device array instead of a caller workspace: bytes
// [0, kWsAlign) hold the counter (at a fixed place, so that 1-pass calls of
// any size find it at zero), the chunk values start at kWsAlign.  Every GPU
// the library runs on has its own copy, at its own address.
constexpr size_t kScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

__global__ void scratch_clear_kernel(unsigned int* counter) {
  // the whole 256-byte block of the arrival counter
  if (threadIdx.x < kWsAlign / sizeof(unsigned int)) counter[threadIdx.x] = 0u;
}

namespace {

constexpr int kMaxDevices = 64;

struct ScratchSlot {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchSlot g_scratch[kMaxDevices];

// The current device's copy of `scratch` (set up on the first call on that
// device: its address, and the counter cleared by a kernel on `hs`).
dpia_status scratch_for_current_device(hipStream_t hs, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "dpia_dot_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return bad(DPIA_ERR_HIP, "dpia_dot_noalloc: device id beyond the supported 64");
  ScratchSlot& slot = g_scratch[dev];
  std::call_once(slot.once, [&] {
    void* ptr = nullptr;
    slot.err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (slot.err != hipSuccess) return;
    unsigned int* counter = static_cast<unsigned int*>(ptr);
    void* args[] = {&counter};
    slot.err = hipLaunchKernel(reinterpret_cast<const void*>(scratch_clear_kernel), dim3(1),
                               dim3(64), args, 0, hs);
    if (slot.err == hipSuccess) slot.ptr = ptr;
  });
  if (slot.err != hipSuccess) return hip_fail(slot.err, "dpia_dot_noalloc: scratch set-up");
  *out = slot.ptr;
  return DPIA_OK;
}

}  // namespace

extern "C" dpia_status dpia_dot_noalloc(const dpia_strategy* s, dpia_dtype dt, int64_t n,
                                        const void* x, const void* y, void* out,
                                        dpia_dtype out_dt, dpia_stream_t stream) {
  Plan p;
  dpia_status st = dot_validate(s, dt, n, x, y, out, out_dt, &p);
  if (st != DPIA_OK) return st;
  if (p.partial_bytes > kScratchBytes - kWsAlign)
    return bad(DPIA_ERR_WORKSPACE,
               "the strategy's " + std::to_string(p.partial_bytes) +
                   " bytes of chunk values exceed the no-alloc scratch of " +
                   std::to_string(kScratchBytes - kWsAlign) + " bytes");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  void* base = nullptr;
  st = scratch_for_current_device(hs, &base);
  if (st != DPIA_OK) return st;
  unsigned char* b = static_cast<unsigned char*>(base);
  return dot_launch(p, dt, x, y, out, out_dt, b + kWsAlign, b, hs, "dpia_dot_noalloc launch");
}

extern "C" dpia_status dpia_asum(const dpia_strategy* s, dpia_dtype dt, int64_t n, const void* x,
                                 void* out, dpia_dtype out_dt, void* ws, size_t ws_bytes,
                                 dpia_stream_t stream) {
  Plan p;
  std::string detail;
  dpia_status st = make_plan(s, DPIA_OP_ASUM, dt, 0, n, &p, &detail);
  if (st != DPIA_OK) return bad(st, detail);
  if (out_dt != DPIA_F32) return bad(DPIA_ERR_DTYPE, "asum writes an F32 result");
  if (!out || (n > 0 && !x)) return bad(DPIA_ERR_NULL, "x and out must be non-NULL");
  if (n > 0 && !aligned16(x)) return bad(DPIA_ERR_SHAPE, "x must be 16-byte aligned");
  st = check_ws(p, ws, ws_bytes);
  if (st != DPIA_OK) return st;
  void* split = p.split_off ? static_cast<char*>(ws) + p.split_off : nullptr;
  hipError_t e = launch_reduce<AsumF32, kFinalPlain>(p, AsumF32{static_cast<const float*>(x)},
                                                     out, 0, ws,
                                                     static_cast<char*>(ws) + p.partial_bytes,
                                                     reinterpret_cast<hipStream_t>(stream), split);
  if (e != hipSuccess) return hip_fail(e, "dpia_asum launch");
  clear_detail();
  return DPIA_OK;
}

// The two stages of a 2-pass strategy as separate calls (see dpia.h).
extern "C" dpia_status dpia_chunks(const dpia_strategy* s, dpia_op op, dpia_dtype dt, int64_t n,
                                   const void* x, const void* y, void* chunks,
                                   size_t chunks_bytes, dpia_stream_t stream) {
  if (op != DPIA_OP_DOT && op != DPIA_OP_ASUM)
    return bad(DPIA_ERR_STRATEGY, "dpia_chunks takes DPIA_OP_DOT or DPIA_OP_ASUM");
  Plan p;
  std::string detail;
  dpia_status st = make_plan(s, op, dt, 0, n, &p, &detail);
  if (st != DPIA_OK) return bad(st, detail);
  const bool dot = op == DPIA_OP_DOT;
  if (n > 0 && (!x || (dot && !y))) return bad(DPIA_ERR_NULL, "input vectors must be non-NULL");
  if (n > 0 && (!aligned16(x) || (dot && !aligned16(y))))
    return bad(DPIA_ERR_SHAPE, "input vectors must be 16-byte aligned");
  const size_t need = static_cast<size_t>(p.values) * p.acc_bytes;
  if (p.items > 0 && !chunks) return bad(DPIA_ERR_NULL, "chunks must be non-NULL");
  if (chunks_bytes < need)
    return bad(DPIA_ERR_WORKSPACE, "chunks holds " + std::to_string(chunks_bytes) +
                                       " bytes, the strategy writes " + std::to_string(need));
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = with_reduction(p, x, y, [&](auto op_v, auto fin) {
    using Op = decltype(op_v);
    constexpr int FINAL = decltype(fin)::value;
    ReduceArgs a = reduce_args<Op>(p, chunks, nullptr, nullptr, 0, false);
    return launch_chunks<Op, FINAL>(p, op_v, a, hs);
  });
  if (e != hipSuccess) return hip_fail(e, "dpia_chunks launch");
  clear_detail();
  return DPIA_OK;
}

extern "C" dpia_status dpia_fold(const dpia_strategy* s, dpia_op op, dpia_dtype dt, int64_t n,
                                 const void* chunks, void* out, dpia_dtype out_dt,
                                 dpia_stream_t stream) {
  if (op != DPIA_OP_DOT && op != DPIA_OP_ASUM)
    return bad(DPIA_ERR_STRATEGY, "dpia_fold takes DPIA_OP_DOT or DPIA_OP_ASUM");
  Plan p;
  std::string detail;
  dpia_status st = make_plan(s, op, dt, 0, n, &p, &detail);
  if (st != DPIA_OK) return bad(st, detail);
  if (!out || (p.items > 0 && !chunks)) return bad(DPIA_ERR_NULL, "chunks and out must be non-NULL");
  const dpia_dtype want = (dt == DPIA_I32) ? DPIA_I32 : DPIA_F32;
  if (!(out_dt == want || (out_dt == DPIA_F64 && p.final_f64)))
    return bad(DPIA_ERR_DTYPE, "output type does not match the strategy");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = with_reduction(p, nullptr, nullptr, [&](auto op_v, auto fin) {
    using Op = decltype(op_v);
    constexpr int FINAL = decltype(fin)::value;
    return launch_fold<Op, FINAL>(p.values, chunks, out, out_dt == DPIA_F64, hs);
  });
  if (e != hipSuccess) return hip_fail(e, "dpia_fold launch");
  clear_detail();
  return DPIA_OK;
}
