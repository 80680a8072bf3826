// y = A x under a DPIA strategy (gemv benchmark, Sec. 7.1):
//   join (mapWorkgroup (lam rows. map (lam row. ROWRED (zip row x)) rows)
//         (split R A))
// where ROWRED is the chunk reduction of the dot-product strategy (lane folds
// of C elements, then the combine of the L lanes).  With two row parts each
// half row is a chunk of its own and the halves are folded as (0 + h0) + h1.
// bf16 and fp8-e4m3 matrices are decoded exactly to binary32 before the
// multiply; fp8 rows are scaled after the reduction: y[r] = scale[r] * sum.
// No cross-work-group step: each team owns whole rows of y.
#include "device.h"
#include "fed.h"
#include "ops.h"
#include "host.h"
#include "plan.h"

namespace dpia {

struct GemvArgs {
  int64_t m;
  int64_t k;
  int64_t lda;
  int W, L, C, team, teams_per_wg, team_lds_elems, parts;
  int stage_off;          // byte offset of the LDS staging region, -1: none
};

// Strided lane folds of RB rows at once: thread t holds lanes t*NV ..
// t*NV + NV-1 of each of the RB rows, so every x load serves RB rows.  Each
// row's lanes fold their own elements in increasing index, exactly as with
// one row per team.  `limit`: elements of the row part that exist.
// Row-blocked folds load their batch as two halves, one in flight while the
// other is folded.  With 4 rows per team the fp8 launch has one wavefront
// per SIMD, so a batch's decodes, products and sums otherwise ran with no
// loads of that SIMD in flight (measured at 16384^2, cache evicted, C=64
// L=256: 53.1 -> 50.6-50.9 us; bf16 C=32 L=512 98.5 -> 97.3 us).
#ifndef DPIA_ROW_BLOCK_PIPELINE
#define DPIA_ROW_BLOCK_PIPELINE 1
#endif

template <class Op, int NV, int RB>
__device__ __forceinline__ void row_block_folds(const Op& op, const int64_t (&row)[RB],
                                                const bool (&act)[RB], int64_t lda, int64_t col0,
                                                int t, int L, int C, int limit,
                                                float (&acc)[RB][NV]) {
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[b][v] = 0.0f;
  bool any = false;
#pragma unroll
  for (int b = 0; b < RB; ++b) any = any || act[b];
  if (!any) return;
  constexpr int U = Batch<NV, OpBatch<Op>::E>::U;
  const int rows = limit / L;
  const int nfull = rows < C ? rows : C;
  const int start = t * NV;
  int k = 0;
#if DPIA_ROW_BLOCK_PIPELINE
  if constexpr (U >= 2 && U % 2 == 0) {
    // two half batches: one in flight while the other is folded
    constexpr int H = U / 2;
    float xa[H][NV], xb[H][NV];
    typename Op::Code ca[H][RB][NV], cb[H][RB][NV];
    auto load_half = [&](int k0, float (&xv)[H][NV], typename Op::Code (&cc)[H][RB][NV]) {
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const int64_t c = col0 + start + static_cast<int64_t>(k0 + u) * L;
        op.template load_x<NV>(c, xv[u]);
#pragma unroll
        for (int b = 0; b < RB; ++b) op.template load_codes<NV>(row[b], lda, c, cc[u][b]);
      }
    };
    auto fold_half = [&](const float (&xv)[H][NV], const typename Op::Code (&cc)[H][RB][NV]) {
#pragma unroll
      for (int u = 0; u < H; ++u)
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          float av[NV];
          Op::template decode<NV>(cc[u][b], av);
#pragma unroll
          for (int v = 0; v < NV; ++v)
            acc[b][v] = Op::step(typename Op::Term{av[v], xv[u][v]}, acc[b][v]);
        }
    };
    if (k + U <= nfull) {
      load_half(k, xa, ca);
      for (; k + U <= nfull; k += U) {
        load_half(k + H, xb, cb);
        __builtin_amdgcn_sched_barrier(0);
        fold_half(xa, ca);
        __builtin_amdgcn_sched_barrier(0);
        if (k + U + H <= nfull) load_half(k + U, xa, ca);
        __builtin_amdgcn_sched_barrier(0);
        fold_half(xb, cb);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (k + H <= nfull) {   // the half batch loaded last
        fold_half(xa, ca);
        k += H;
      }
    }
  }
#endif
  for (; k + U <= nfull; k += U) {
    float xv[U][NV];
    typename Op::Code ca[U][RB][NV];   // codes: decoded only when folded
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t c = col0 + start + static_cast<int64_t>(k + u) * L;
      op.template load_x<NV>(c, xv[u]);
#pragma unroll
      for (int b = 0; b < RB; ++b) op.template load_codes<NV>(row[b], lda, c, ca[u][b]);
    }
    __builtin_amdgcn_sched_barrier(0);   // issue the whole batch first
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        float av[NV];
        Op::template decode<NV>(ca[u][b], av);
#pragma unroll
        for (int v = 0; v < NV; ++v)
          acc[b][v] = Op::step(typename Op::Term{av[v], xv[u][v]}, acc[b][v]);
      }
  }
  for (; k < nfull; ++k) {
    const int64_t c = col0 + start + static_cast<int64_t>(k) * L;
    float xv[NV];
    op.template load_x<NV>(c, xv);
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      float av[NV];
      op.template load_a<NV>(row[b], lda, c, av);
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[b][v] = Op::step(typename Op::Term{av[v], xv[v]}, acc[b][v]);
    }
  }
  if (nfull < C) {   // the last, partly existing row of the part
    const int o = start + nfull * L;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (o + v < limit) {
        const float xv = op.x[col0 + o + v];
#pragma unroll
        for (int b = 0; b < RB; ++b)
          acc[b][v] = Op::step(typename Op::Term{op.load_a1(row[b], lda, col0 + o + v), xv},
                               acc[b][v]);
      }
    }
  }
}

template <class Op, int NV, int COMBINE, int RB>
__global__ void __launch_bounds__(256) gemv_block_kernel(Op op, GemvArgs a) {
  using T = float;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int team_id = threadIdx.x / a.team;
  const int t = threadIdx.x - team_id * a.team;
  T* scratch = lds + team_id * a.team_lds_elems;
  const int64_t per_wg = static_cast<int64_t>(a.teams_per_wg) * RB;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * per_wg; base < a.m;
       base += static_cast<int64_t>(gridDim.x) * per_wg) {
    int64_t row[RB];
    bool act[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int64_t r = base + static_cast<int64_t>(team_id) * RB + b;
      act[b] = r < a.m;
      row[b] = act[b] ? r : 0;
    }
    float acc[RB][NV];
    T v[RB];
    const int lim0 = static_cast<int>(a.k < a.W ? a.k : a.W);
    row_block_folds<Op, NV, RB>(op, row, act, a.lda, 0, t, a.L, a.C, lim0, acc);
#pragma unroll
    for (int b = 0; b < RB; ++b) v[b] = combine_lanes<PlainF32, NV, COMBINE>(acc[b], t, a.team, a.L, scratch);
    if (a.parts == 2) {
      const int lim1 = static_cast<int>(a.k - a.W);
      row_block_folds<Op, NV, RB>(op, row, act, a.lda, a.W, t, a.L, a.C, lim1 > 0 ? lim1 : 0, acc);
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const T h1 = combine_lanes<PlainF32, NV, COMBINE>(acc[b], t, a.team, a.L, scratch);
        v[b] = tree_node<PlainF32>(v[b], h1);   // reduceSeq (+) 0 [h0, h1]
      }
    }
    if (t == 0) {
#pragma unroll
      for (int b = 0; b < RB; ++b)
        if (act[b]) op.store(row[b], v[b]);
    }
  }
}

// MAXT: the largest work-group it is launched with (256 or 1024); the
// 256-thread build may use twice the registers of the 1024-thread one.
// SS: strided rows of one thread each, staged through LDS (a build of its
// own: the staged fold's registers would lower every other strided launch's
// occupancy).
template <class Op, int ORDER, int NV, int COMBINE, int MAXT, bool SS = false>
__global__ void __launch_bounds__(MAXT) gemv_kernel(Op op, GemvArgs a) {
  using T = typename Op::T;
  using A = typename Op::Arith;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int team_id = threadIdx.x / a.team;
  const int t = threadIdx.x - team_id * a.team;
  T* scratch = lds + team_id * a.team_lds_elems;
  // (staging needs work-groups of at most 256 threads: none in the 1024 build)
  float* stage = MAXT > 256 || a.stage_off < 0
                     ? nullptr
                     : reinterpret_cast<float*>(lds_raw + a.stage_off) +
                           (threadIdx.x / kWave) * stage_floats(kWave);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * a.teams_per_wg;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * a.teams_per_wg; base < a.m;
       base += stride) {
    const int64_t row = base + team_id;
    const bool active = row < a.m;
    const int64_t r = active ? row : 0;
    // elements of each row part that exist (k may stop short of W * parts:
    // the row is zero-extended)
    const int lim0 = static_cast<int>(a.k < a.W ? a.k : a.W);
    T v = chunk_value<Op, ORDER, NV, COMBINE, SS>(op.part(r, 0, a.lda, a.W), active, t, a.team,
                                                  a.L, a.C, lim0, scratch, stage);
    if (a.parts == 2) {
      const int lim1 = static_cast<int>(a.k - a.W);
      const T h1 = chunk_value<Op, ORDER, NV, COMBINE, SS>(op.part(r, 1, a.lda, a.W), active, t,
                                                           a.team, a.L, a.C, lim1 > 0 ? lim1 : 0,
                                                           scratch, stage);
      v = tree_node<A>(v, h1);   // reduceSeq (+) 0 [h0, h1]
    }
    if (active && t == 0) op.store(row, v);
  }
}

// Binary32 rows fed by loader wavefronts: teams of one thread (the strided
// order with L = NL lanes held as that thread's components, or one
// contiguous lane), strided teams of two threads (TPR below) and contiguous
// teams of L threads (one lane each), row parts of whole tiles.  The strategy's work-groups of R rows give each busy
// compute unit a wavefront or two (16384 rows of R = 128: 128 work-groups),
// too few loads in flight to stream A.  The rows are independent, so a
// hardware work-group here takes ROWS lane rows of its own, ROWS / team
// consecutive matrix rows: wave 0 folds them (lane q the Cel = W / team
// elements of lane q % team of its row, element e into component e % NL, in
// increasing e, as chunk_value's staged folds do), kFedLoaders wavefronts
// load A and x into the LDS ring.  The lanes are combined by combine_lanes
// over teams of `team` adjacent lanes of wave 0 and the parts by tree_node,
// as in gemv_kernel: every row's association is the strategy's.
// TPR = 2: strided teams of 2 threads holding 4 lanes each (L = 8);
// the ROWS ring rows are whole matrix row parts, and the team's threads fold
// their own 16-byte pieces of every step of the shared row (fed_fold).
// XR: x rows of a ring slot, 1 where a matrix row is one ring row (every
// team but the contiguous teams of L > 1 lanes), L for contiguous teams of
// L = 2 or 4 lanes (lane l reads x row l), 0: one x row per ring row.
template <class Op, int NL, int COMBINE, int ROWS, int TPR = 1, int XR = 0>
__global__ void __launch_bounds__(kWave * (1 + kFedLoaders)) gemv_fed_kernel(Op op, GemvArgs a) {
  using T = typename Op::T;
  using A = typename Op::Arith;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* ring = reinterpret_cast<float*>(lds_raw);
  const int team = TPR > 1 ? TPR : a.team;
  const int t = static_cast<int>(threadIdx.x) % team;
  // each team's combine region (its team * NL lane values)
  T* scratch = reinterpret_cast<T*>(ring + fed_ring_floats()) +
               (static_cast<int>(threadIdx.x) - t) * NL;
  const int wave = static_cast<int>(threadIdx.x) / kWave;
  const int lane = static_cast<int>(threadIdx.x) % kWave;
  const int row_lanes = TPR > 1 ? 1 : team;   // ring rows per matrix row
  const int cel = a.W / row_lanes;
  const int rows_per_wg = ROWS / row_lanes;
  for (int64_t row0 = static_cast<int64_t>(blockIdx.x) * rows_per_wg; row0 < a.m;
       row0 += static_cast<int64_t>(gridDim.x) * rows_per_wg) {
    T acc[NL];
    fed_fold<Op, NL, ROWS, true, TPR, XR>(op.part(row0, 0, a.lda, a.W), cel, wave, lane, 0,
                                            ring, acc, static_cast<int>(a.lda), row_lanes);
    T v = combine_lanes<A, NL, COMBINE>(acc, t, team, a.L, scratch);
    if (a.parts == 2) {
      fed_fold<Op, NL, ROWS, true, TPR, XR>(op.part(row0, 1, a.lda, a.W), cel, wave, lane, 0,
                                              ring, acc, static_cast<int>(a.lda), row_lanes);
      const T h1 = combine_lanes<A, NL, COMBINE>(acc, t, team, a.L, scratch);
      v = tree_node<A>(v, h1);   // reduceSeq (+) 0 [h0, h1]
    }
    if (wave == 0 && lane < ROWS * TPR && t == 0) op.store(row0 + lane / team, v);
  }
}

// Lane rows per work-group of gemv_fed_kernel for this plan, or 0 where it
// does not apply: teams of one thread, strided teams of two, or contiguous
// teams of at most 64 threads, binary32 A (the caller's check), every row part whole (k = W *
// parts) with lanes of at least 64 tiles of 64 elements, and m a multiple
// of the matrix rows per work-group.  The most lane rows that still give
// every compute unit a work-group.
template <int ROWS>
constexpr bool fed_gemv_fits(int64_t tiles) {
  // (a multiple of every depth fed_fold uses for these rows: 4 to 16 tiles)
  return tiles % fed_depth<ROWS, 1>() == 0;
}
// Strided teams of 2 threads of 4 lanes each (L = 8): ring rows are matrix
// rows, 16 or 32 of them (at most 64 folding lanes).  (Teams of 4 threads,
// 16 rows of 4 KB per round, measured no faster this way at 16384^2:
// strided C=1024 L=16 177.9 -> 175.1 us, C=512 L=16 with two parts 174.6
// -> 176.0 us; teams of 2: C=1024 L=8 with two parts 235.5 -> 181.8 us.)
static int fed_gemv_rows(const Plan& p, int64_t m, int64_t lda) {
  if (m <= 0 || lda % 4 || lda > (int64_t(1) << 24)) return 0;
  if (p.order == DPIA_ORDER_STRIDED && p.nv == 4 && p.team == 2 && p.L == 8) {
    if (p.W % kFedStage || p.k != p.W * p.row_parts || p.W / kFedStage < 64) return 0;
    const int64_t tiles = p.W / kFedStage;
    if (m % 32 == 0 && m / 32 >= device_cus() && fed_gemv_fits<32>(tiles)) return 32;
    if (m % 16 == 0 && fed_gemv_fits<16>(tiles)) return 16;
    return 0;
  }
  const bool lanes = p.order == DPIA_ORDER_STRIDED
                         ? (p.team == 1 && p.nv == p.L && (p.L == 1 || p.L == 2 || p.L == 4))
                         : p.team == p.L && p.L <= 64 && (p.L & (p.L - 1)) == 0;
  if (!lanes || p.W % (int64_t(kFedStage) * p.team) || p.k != p.W * p.row_parts) return 0;
  // (lanes of 16 tiles measured slower than gemv_kernel: 16384^2 contiguous
  // C=1024 L=16 234.9 -> 248.3 us, L=8 with two parts 191.6 -> 251.0 us; a
  // work-group's pipeline fills and drains every 16 rounds)
  const int64_t tiles = p.W / p.team / kFedStage;
  if (tiles < 64) return 0;
  const int64_t cus = device_cus();
  const int64_t lane_rows = m * p.team;
  auto fits = [&](int rows, bool fill) {
    return rows % p.team == 0 && m % (rows / p.team) == 0 && (!fill || lane_rows / rows >= cus);
  };
  if (fits(64, true) && fed_gemv_fits<64>(tiles)) return 64;
  if (fits(32, true) && fed_gemv_fits<32>(tiles)) return 32;
  if (fits(16, false) && fed_gemv_fits<16>(tiles)) return 16;
  if (fits(64, false) && fed_gemv_fits<64>(tiles)) return 64;
  return 0;
}

template <class Op>
hipError_t launch_gemv_fed(const Plan& p, const Op& op, int64_t m, int64_t lda, int rows,
                           hipStream_t stream) {
  GemvArgs a{};
  a.m = m;
  a.k = p.k;
  a.lda = lda;
  a.W = static_cast<int>(p.W);
  a.L = static_cast<int>(p.L);
  a.C = static_cast<int>(p.C);
  // threads per row: strided teams of 1, 2 or 4 threads, contiguous teams of L
  a.team = p.order == DPIA_ORDER_STRIDED ? p.team : static_cast<int>(p.L);
  // matrix rows per work-group (ring rows are matrix rows for strided teams)
  a.teams_per_wg = p.order == DPIA_ORDER_STRIDED ? rows : rows / a.team;
  a.parts = p.row_parts;
  a.stage_off = -1;
  const int nl = p.order == DPIA_ORDER_STRIDED ? p.nv : 1;
  const int64_t need = m / a.teams_per_wg;
  const int64_t grid = p.max_grid && need > static_cast<int64_t>(p.max_grid)
                           ? static_cast<int64_t>(p.max_grid) : need;
  const size_t lds = sizeof(float) * fed_ring_floats() +
                     sizeof(typename Op::T) * kWave * (1 + kFedLoaders) * 4;
  auto go = [&](auto nlc, auto comb, auto rc) {
    constexpr int NL = decltype(nlc)::value;
    constexpr int COMBINE = decltype(comb)::value;
    constexpr int ROWS = decltype(rc)::value;
    auto kern = gemv_fed_kernel<Op, NL, COMBINE, ROWS, 1, 1>;
    if constexpr (NL == 1) {
      if (a.team == 2) kern = gemv_fed_kernel<Op, NL, COMBINE, ROWS, 1, 2>;
      else if (a.team == 4) kern = gemv_fed_kernel<Op, NL, COMBINE, ROWS, 1, 4>;
      else if (a.team > 4) kern = gemv_fed_kernel<Op, NL, COMBINE, ROWS, 1, 0>;
    }
    Op op_copy = op;
    void* args[] = {&op_copy, &a};
    return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid),
                           dim3(kWave * (1 + kFedLoaders)), args, lds, stream);
  };
  auto by_rows = [&](auto nlc, auto comb) {
    return rows == 64 ? go(nlc, comb, ic<64>{})
                      : (rows == 32 ? go(nlc, comb, ic<32>{}) : go(nlc, comb, ic<16>{}));
  };
  auto by_combine = [&](auto nlc) {
    return p.combine == DPIA_COMBINE_TREE ? by_rows(nlc, ic<kTree>{}) : by_rows(nlc, ic<kSeq>{});
  };
  auto team_go = [&](auto comb, auto rc, auto tc) {
    auto kern = gemv_fed_kernel<Op, 4, decltype(comb)::value, decltype(rc)::value,
                                decltype(tc)::value, 1>;
    Op op_copy = op;
    void* args[] = {&op_copy, &a};
    return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid),
                           dim3(kWave * (1 + kFedLoaders)), args, lds, stream);
  };
  auto team_rows = [&](auto comb) {
    return rows == 32 ? team_go(comb, ic<32>{}, ic<2>{}) : team_go(comb, ic<16>{}, ic<2>{});
  };
  if (p.order == DPIA_ORDER_STRIDED && a.team > 1)
    return p.combine == DPIA_COMBINE_TREE ? team_rows(ic<kTree>{}) : team_rows(ic<kSeq>{});
  return nl == 4 ? by_combine(ic<4>{}) : (nl == 2 ? by_combine(ic<2>{}) : by_combine(ic<1>{}));
}

template <class Op, int MAXNV>
hipError_t launch_gemv(const Plan& p, const Op& op, int64_t m, int64_t lda, hipStream_t stream,
                       int rb = 1) {
  GemvArgs a{};
  a.m = m;
  a.k = p.k;
  a.lda = lda;
  a.W = static_cast<int>(p.W);
  a.L = static_cast<int>(p.L);
  a.C = static_cast<int>(p.C);
  a.team = p.team;
  a.teams_per_wg = p.teams_per_wg;
  a.team_lds_elems = (p.combine == DPIA_COMBINE_SEQ) ? static_cast<int>(p.L)
                                                     : (p.team > 64 ? p.team / 64 : 1);
  a.parts = p.row_parts;
  a.stage_off = p.stage ? static_cast<int>(p.stage_off) : -1;
  if constexpr (Op::kRowBlockable) {
  if (rb > 1 && p.order == DPIA_ORDER_STRIDED && p.nv == MAXNV && p.wg_threads <= 256) {
    // row blocking: each team reduces rb rows at once (see row_block_folds)
    const int64_t per_wg = static_cast<int64_t>(p.teams_per_wg) * rb;
    const int64_t need = (m + per_wg - 1) / per_wg;
    const int64_t cap = p.max_grid ? static_cast<int64_t>(p.max_grid)
                                   : static_cast<int64_t>(device_cus()) *
                                         (2048 / p.wg_threads > 0 ? 2048 / p.wg_threads : 1);
    const int64_t grid = need < cap ? need : cap;
    auto go = [&](auto comb, auto rbc) {
      constexpr int COMBINE = decltype(comb)::value;
      constexpr int RB = decltype(rbc)::value;
      auto kern = gemv_block_kernel<Op, MAXNV, COMBINE, RB>;
      Op op_copy = op;
      void* args[] = {&op_copy, &a};
      return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid),
                             dim3(p.wg_threads), args, p.lds_bytes, stream);
    };
    if (p.combine == DPIA_COMBINE_TREE)
      return rb == 4 ? go(ic<0>{}, ic<4>{}) : go(ic<0>{}, ic<2>{});
    return rb == 4 ? go(ic<1>{}, ic<4>{}) : go(ic<1>{}, ic<2>{});
  }
  }
  const int64_t grid = grid_size(p);
  return with_order_combine(p.order, p.combine, [&](auto ord, auto comb) {
    constexpr int ORDER = decltype(ord)::value;
    constexpr int COMBINE = decltype(comb)::value;
    return with_nv<MAXNV>(p.nv, [&](auto nvc) {
      constexpr int NV = decltype(nvc)::value;
      auto kern = p.wg_threads <= 256 ? gemv_kernel<Op, ORDER, NV, COMBINE, 256>
                                      : gemv_kernel<Op, ORDER, NV, COMBINE, 1024>;
      if constexpr (ORDER == kStrided && NV <= 4) {
        // (the staged fold loads 16-byte pieces of every row)
        if (p.stage && p.wg_threads <= 256 && lda % 4 == 0)
          kern = gemv_kernel<Op, ORDER, NV, COMBINE, 256, true>;
      }
      Op op_copy = op;
      void* args[] = {&op_copy, &a};
      return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid),
                             dim3(p.wg_threads), args, p.lds_bytes, stream);
    });
  });
}

}  // namespace dpia

using namespace dpia;

#ifndef DPIA_ROW_BLOCK
#define DPIA_ROW_BLOCK 2
#endif
// Rows one team reduces at once for bf16 / fp8 matrices (1 = no blocking):
// with narrow A elements the x operand, reloaded per row, would otherwise
// dominate the traffic through the vector caches.
static constexpr int kRowBlock = DPIA_ROW_BLOCK;

// fp8 rows: 4 rows per team where that still gives one or two work-groups
// per compute unit, else 2.  Measured at 16384^2 (cache evicted), 4 rows
// per team: C=64 L=256 66.0 -> 52.8 us, C=32 L=512 68.4 -> 58.8 us (256
// and 512 work-groups); slower where it leaves 128 work-groups (C=128
// L=128: 57.4 -> 67.9 us) or 1024 (C=16 L=1024: 58.6 -> 68.5 us).
static int fp8_row_block(const Plan& p, int64_t m) {
  const int64_t wgs4 = (m + int64_t(p.teams_per_wg) * 4 - 1) / (int64_t(p.teams_per_wg) * 4);
  const int64_t cus = device_cus();
  return (wgs4 >= cus && wgs4 <= 2 * cus) ? 4 : kRowBlock;
}

namespace {

// Shared body of dpia_gemv (blas = false) and dpia_gemv_blas.
dpia_status gemv_impl(const char* name, const dpia_strategy* s, dpia_dtype a_dt, int64_t m,
                      int64_t k, int64_t lda, const void* A, const float* row_scale, bool blas,
                      float alpha, const void* x, float beta, void* y, dpia_stream_t stream) {
  Plan p;
  std::string detail;
  dpia_status st = make_plan(s, DPIA_OP_GEMV, a_dt, m, k, &p, &detail);
  if (st != DPIA_OK) return bad(st, detail);
  if (lda < k) return bad(DPIA_ERR_SHAPE, "lda must be >= k");
  if (lda % p.nv)
    return bad(DPIA_ERR_SHAPE, "lda must keep every row aligned for the strategy's vector loads");
  if (a_dt == DPIA_FP8_E4M3 && !row_scale && m > 0)
    return bad(DPIA_ERR_NULL, "an FP8 matrix needs row_scale");
  if (a_dt != DPIA_FP8_E4M3 && row_scale)
    return bad(DPIA_ERR_DTYPE, "row_scale applies to FP8 matrices only");
  if (blas && a_dt == DPIA_I32)
    return bad(DPIA_ERR_DTYPE, "the alpha / beta form takes F32, BF16 or FP8 matrices");
  if (m == 0) {
    clear_detail();
    return DPIA_OK;
  }
  if (!A || !x || !y) return bad(DPIA_ERR_NULL, "A, x and y must be non-NULL");
  if (!aligned16(A) || !aligned16(x))
    return bad(DPIA_ERR_SHAPE, "A and x must be 16-byte aligned");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipErrorInvalidValue;
  auto with_epilogue = [&](auto op) {
    op.blas = blas;
    op.alpha = alpha;
    op.beta = beta;
    op.beta_zero = beta == 0.0f;
    return op;
  };
  switch (a_dt) {
    case DPIA_F32:
      if (const int rows = fed_gemv_rows(p, m, lda))
        e = launch_gemv_fed(
            p, with_epilogue(GemvF32{static_cast<const float*>(A), static_cast<const float*>(x),
                                     nullptr, static_cast<float*>(y)}),
            m, lda, rows, hs);
      else if (p.order == DPIA_ORDER_STRIDED && p.team < 4)
        e = launch_gemv<GemvF32Cached, 4>(
            p, with_epilogue(GemvF32Cached{static_cast<const float*>(A),
                                           static_cast<const float*>(x), nullptr,
                                           static_cast<float*>(y)}),
            m, lda, hs);
      else
        e = launch_gemv<GemvF32, 4>(
            p, with_epilogue(GemvF32{static_cast<const float*>(A), static_cast<const float*>(x),
                                     nullptr, static_cast<float*>(y)}),
            m, lda, hs);
      break;
    case DPIA_BF16:
      e = launch_gemv<GemvBF16, 8>(
          p, with_epilogue(GemvBF16{static_cast<const uint16_t*>(A),
                                    static_cast<const float*>(x), nullptr,
                                    static_cast<float*>(y)}),
          m, lda, hs, kRowBlock);
      break;
    case DPIA_FP8_E4M3:
      if (p.C >= 64)
        e = launch_gemv<GemvFP8Long, 16>(
            p, with_epilogue(GemvFP8Long{static_cast<const uint8_t*>(A),
                                         static_cast<const float*>(x), row_scale,
                                         static_cast<float*>(y)}),
            m, lda, hs, fp8_row_block(p, m));
      else
        e = launch_gemv<GemvFP8, 16>(
            p, with_epilogue(GemvFP8{static_cast<const uint8_t*>(A),
                                     static_cast<const float*>(x), row_scale,
                                     static_cast<float*>(y)}),
            m, lda, hs, fp8_row_block(p, m));
      break;
    case DPIA_I32:
      e = launch_gemv<GemvU32, 4>(
          p, GemvU32{static_cast<const uint32_t*>(A), static_cast<const uint32_t*>(x), nullptr,
                     static_cast<uint32_t*>(y)},
          m, lda, hs);
      break;
    default:
      return bad(DPIA_ERR_DTYPE, "unsupported matrix type");
  }
  if (e != hipSuccess) return hip_fail(e, name);
  clear_detail();
  return DPIA_OK;
}

}  // namespace

extern "C" dpia_status dpia_gemv(const dpia_strategy* s, dpia_dtype a_dt, int64_t m, int64_t k,
                                 int64_t lda, const void* A, const float* row_scale,
                                 const void* x, void* y, void* ws, size_t ws_bytes,
                                 dpia_stream_t stream) {
  (void)ws;
  (void)ws_bytes;
  return gemv_impl("dpia_gemv launch", s, a_dt, m, k, lda, A, row_scale, false, 1.0f, x, 0.0f,
                   y, stream);
}

extern "C" dpia_status dpia_gemv_blas(const dpia_strategy* s, dpia_dtype a_dt, int64_t m,
                                      int64_t k, int64_t lda, float alpha, const void* A,
                                      const float* row_scale, const float* x, float beta,
                                      float* y, dpia_stream_t stream) {
  return gemv_impl("dpia_gemv_blas launch", s, a_dt, m, k, lda, A, row_scale, true, alpha, x,
                   beta, y, stream);
}
