// Contiguous lanes staged through LDS and fed by loader wavefronts.
//
// A strategy with one 64-lane team per chunk and fewer chunks than compute
// units (the Sec. 6.2 form: 128 chunks of 64 vector lanes) gives each busy
// compute unit a single wavefront, and one wavefront can keep only a couple
// of staged tiles of loads in flight.  Here the work-group carries
// kFedLoaders loader wavefronts beside the wavefront that folds.  The loaders
// split every tile of the lane rows between them (each issues the same
// 16-byte loads of its own rows, so all of them run the same straight-line
// code), keep several tiles in flight, and write each tile into a two-slot
// LDS ring one round ahead of the fold; one work-group barrier per tile
// separates the rounds.  Which elements each lane folds, and in which order,
// is exactly what contiguous_staged folds: the loaders only move data.
#pragma once

#include "device.h"

namespace dpia {

#ifndef DPIA_FED_LOADERS
#define DPIA_FED_LOADERS 4
#endif
#ifndef DPIA_FED_STAGE
#define DPIA_FED_STAGE 64
#endif
constexpr int kFedLoaders = DPIA_FED_LOADERS;
// Elements of a lane row per tile, and the LDS row stride in floats (an odd
// number of 16-byte units): 256 contiguous bytes of a row per load
// instruction, and half the rounds of 32-element tiles (measured equal to
// them on the Sec. 6.2 form; the bursts below are what the rows' DRAM pages
// needed).
constexpr int kFedStage = DPIA_FED_STAGE;
constexpr int kFedRow = kFedStage + 4;
constexpr int kFedVec = kFedStage / 4;                // 16-byte parts of a row tile
static_assert(kWave % kFedVec == 0, "a load instruction covers whole row tiles");
constexpr int kFedRowsPerLoad = kWave / kFedVec;
// The deepest pipeline (tiles in flight) of any row count.
constexpr int kFedMaxDepth = 16;
// Tiles each loader requests back to back: consecutive pieces of its rows.
// The lane rows lie C * V elements apart, so every row is a stream of its
// own, and requesting kFedBurst tiles of a row together lets a DRAM page
// serve kFedBurst * 256 bytes of it rather than 256 (measured on the Sec. 6.2
// form at 2^26, kernel trace medians: 1, 2 and 4 tiles 103.8, 99.4 and 90.7
// us on one box; 8 tiles, the pipeline emptying before each burst, 108.2
// against 97.8 us for 4 on another).  At most the depth.
#ifndef DPIA_FED_BURST
#define DPIA_FED_BURST 4
#endif
constexpr int kFedBurst = DPIA_FED_BURST;

// LDS floats of the ring: two slots, each two operands x 64 rows (also the
// staging region of contiguous_staged for a ragged chunk).
constexpr int fed_ring_floats() { return 2 * 2 * kWave * kFedRow; }
static_assert(fed_ring_floats() >= stage_floats(kWave), "the ring holds a staging region");

// ROWS lane rows (row0 .. row0 + ROWS - 1) of one chunk whose 64 lane rows
// are whole: Cel elements each, Cel / kFedStage tiles, a multiple of the
// depth.  Every thread of the work-group calls this; wave 0 folds (lane l <
// ROWS folds row row0 + l into acc), waves 1 .. kFedLoaders load.  Local row
// r of operand o in ring slot s starts at ((s * NOPS + o) * 64 + r) *
// kFedRow floats.  An uncombined strategy may split a chunk's rows over
// several work-groups (ROWS < 64): its lanes' values are independent.
// Rows lie `rstride` elements apart (0: Cel, the lane rows of a chunk).
// SHARED1 (a gemv: operand 0 is A, operand 1 is x): lane row q is lane
// q % lanes of matrix row q / lanes, Cel elements at (q % lanes) * Cel of
// that row (rows of A `rstride` apart) and of x.  x is read with cached
// loads, since every row and every work-group reads it again.
// TPR > 1 (strided teams of TPR threads holding 4 lanes each, L = 4 * TPR):
// folding lane l reads row l / TPR, whose every step of L elements gives
// thread t = l % TPR the 4 elements at 4 t, in increasing step: its lanes'
// elements in index order (VEC = 4, element 4 t + i of a step into
// component i).  The ROWS rows then feed ROWS * TPR folding lanes.
template <int ROWS, int NOPS>
constexpr int fed_per() { return ROWS / kFedRowsPerLoad / kFedLoaders; }
// Tiles in flight: every loader keeps 32 sixteen-byte loads outstanding, up
// to kFedMaxDepth tiles.
template <int ROWS, int NOPS>
constexpr int fed_depth() {
  return 32 / (NOPS * fed_per<ROWS, NOPS>()) < kFedMaxDepth ? 32 / (NOPS * fed_per<ROWS, NOPS>())
                                                            : kFedMaxDepth;
}

// XR > 0 (with SHARED1, lanes = XR = 1, 2 or 4): x is XR rows for all lane
// rows of a tile, lane row q reading row q % XR.  Each loader fetches them
// with one cached load per tile (lane l: piece l % 16 of row (l / 16) % XR)
// and loader 1's first 16 XR lanes write them to rows 0 .. XR - 1 of the x
// part of the slot, which the folding lanes read (LDS broadcasts).
template <class Op, int VEC, int ROWS, bool SHARED1 = false, int TPR = 1, int XR = 0,
          class View>
__device__ __forceinline__ void fed_fold(const View& view, int Cel, int wave, int lane, int row0,
                                         float* ring, typename Op::T (&acc)[VEC],
                                         int rstride = 0, int lanes = 1) {
  constexpr int NOPS = View::kOps;
  constexpr int kPer = fed_per<ROWS, NOPS>();       // load instructions per operand per tile
  // One x row: a loader's loads in flight are A's (one x load per tile
  // aside), 8 tiles deep.  Measured at 16384^2: rows of one thread (64 rows
  // per work-group) 4 -> 8 tiles 199.6 -> 155.6 us (C=8192 L=2); teams of
  // two (32 rows) 8 -> 16 tiles 180.6 -> 190.6 us (C=1024 L=8, two parts).
  constexpr int kXoneDepth = fed_depth<ROWS, 1>() < 8 ? fed_depth<ROWS, 1>() : 8;
  constexpr int D = XR > 0 ? kXoneDepth : fed_depth<ROWS, NOPS>();
  static_assert(kPer >= 1 && kPer * kFedLoaders * kFedRowsPerLoad == ROWS,
                "the loaders split a tile's loads evenly");
  static_assert(D % 2 == 0 && D <= kFedMaxDepth, "a round's ring slot is the parity of its tile");
  constexpr int B = kFedBurst < D ? kFedBurst : D;
  static_assert(D % B == 0, "whole bursts of tiles");
#pragma unroll
  for (int j = 0; j < VEC; ++j) acc[j] = Op::Arith::zero();
  const int part = lane % kFedVec;
  // loader q = wave - 1 takes the tile's load instructions q*kPer .. q*kPer +
  // kPer - 1; instruction i covers local rows i * kFedRowsPerLoad + lane / kFedVec
  const int q = wave - 1;
  const float* rowp[NOPS][kPer];
  int rofs[kPer];
  const int64_t rs = rstride > 0 ? rstride : Cel;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int r = (q * kPer + k) * kFedRowsPerLoad + lane / kFedVec;
    rofs[k] = r * kFedRow + part * 4;
    if constexpr (SHARED1) {
      const int mr = (row0 + r) / lanes, ml = (row0 + r) - mr * lanes;
      rowp[0][k] = view.operand(0) + mr * rs + static_cast<int64_t>(ml) * Cel + part * 4;
      rowp[1][k] = view.operand(1) + static_cast<int64_t>(ml) * Cel + part * 4;
    } else {
#pragma unroll
      for (int o = 0; o < NOPS; ++o) rowp[o][k] = view.operand(o) + (row0 + r) * rs + part * 4;
    }
  }
  f32x4 regs[D][NOPS][kPer];
  static_assert(XR == 0 || (SHARED1 && NOPS == 2 && (XR == 1 || XR == 2 || XR == 4)),
                "x rows: a gemv's, one per lane of a matrix row");
  const float* xpiece = view.operand(NOPS - 1) +
                        static_cast<int64_t>(XR > 0 ? (lane / kFedVec) % XR : 0) * Cel +
                        (lane % kFedVec) * 4;
  auto gload = [&](f32x4 (&rg)[NOPS][kPer], int tile) {
#pragma unroll
    for (int k = 0; k < kPer; ++k)
#pragma unroll
      for (int o = 0; o < NOPS; ++o) {
        if (XR > 0 && o == 1) {
          if (k == 0)
            rg[1][0] = ld<false>(reinterpret_cast<const f32x4*>(xpiece + tile * kFedStage));
          continue;
        }
        const f32x4* g = reinterpret_cast<const f32x4*>(rowp[o][k] + tile * kFedStage);
        rg[o][k] = SHARED1 && o == 1 ? ld<false>(g) : ld<DPIA_NT_LOADS != 0>(g);
      }
    // tiles are requested in round order, so that each round waits for its
    // own tile only (the scheduler would interleave the sets' loads)
    __builtin_amdgcn_sched_barrier(0);
  };
  auto put = [&](const f32x4 (&rg)[NOPS][kPer], int slot) {
#pragma unroll
    for (int k = 0; k < kPer; ++k)
#pragma unroll
      for (int o = 0; o < NOPS; ++o) {
        if (XR > 0 && o == 1) continue;
        *reinterpret_cast<f32x4*>(ring + (slot * NOPS + o) * kWave * kFedRow + rofs[k]) =
            rg[o][k];
      }
    if constexpr (XR > 0) {
      if (q == 0 && lane < kFedVec * XR)
        *reinterpret_cast<f32x4*>(ring + ((slot * NOPS + 1) * kWave + lane / kFedVec) * kFedRow +
                                  (lane % kFedVec) * 4) = rg[1][0];
    }
  };
  // row `lane` of a slot, in increasing element index; element e of the
  // row belongs to component e % VEC
  static_assert(TPR == 1 || (VEC == 4 && ROWS * TPR <= kWave && kFedVec % TPR == 0),
                "teams sharing a row hold 4 lanes per thread and fit the folding wavefront");
  auto fold_slot = [&](int slot) {
    if (ROWS * TPR < kWave && lane >= ROWS * TPR) return;
    const int row = lane / TPR, t = lane % TPR;
#pragma unroll
    for (int j = 0; j < kFedVec / TPR; ++j) {
      f32x4 v[NOPS];
#pragma unroll
      for (int o = 0; o < NOPS; ++o)
        v[o] = *reinterpret_cast<const f32x4*>(
            ring + ((slot * NOPS + o) * kWave + (XR > 0 && o == 1 ? row % (XR > 0 ? XR : 1) : row)) *
                       kFedRow +
            (j * TPR + t) * 4);
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i % VEC] = Op::step(View::term(v, i), acc[i % VEC]);
    }
  };
  // Round r (0 .. ntiles - 1, each ending with a work-group barrier): the
  // loaders put tile r into slot r % 2 (register set r % D) and load tile
  // r + D into that set; the folding wavefront folds tile r - 1.  One more
  // round folds the last tile.  The two roles run in loops of their own, with
  // the same ntiles + 1 barriers, so that the loaders' D register sets stay
  // live in the loaders' loop alone (in a shared loop the compiler staged the
  // loads through registers of the fold and waited for each one).
  const int ntiles = Cel / kFedStage;
  if (wave > 0) {
#pragma unroll
    for (int d = 0; d < D; ++d) gload(regs[d], d);
    int r0 = 0;
    for (; r0 + D < ntiles; r0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        put(regs[d], d & 1);
        if (d % B == B - 1) {
          // the last B sets are free: their next tiles, back to back
#pragma unroll
          for (int b = d - B + 1; b <= d; ++b) gload(regs[b], r0 + b + D);
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {   // the last D tiles: nothing more to load
      put(regs[d], d & 1);
      __syncthreads();
    }
    __syncthreads();
  } else {
    __syncthreads();
    for (int r = 1; r < ntiles; ++r) {
      fold_slot((r - 1) & 1);
      __syncthreads();
    }
    fold_slot((ntiles - 1) & 1);
    __syncthreads();   // the ring is free for the next chunk
  }
}

// The strided order, ROWS lanes (lane0 .. lane0 + ROWS - 1) of one chunk
// whose elements all exist: lane l takes elements l, l + L, l + 2L, ...
// (Cj of them), so step j of every lane is one contiguous row of L elements.
// A tile is kFedStrideRows consecutive steps of the slice's ROWS lanes; the
// loaders fetch each step's ROWS * 4 bytes (ROWS / 4 threads per step, 256 /
// ROWS steps per load instruction), and the folding wavefront, one lane per
// thread, reads its lane's element of each step in increasing j.  Ring rows
// are steps, ROWS + 4 floats apart.  Cj / kFedStrideRows tiles, a multiple of
// the depth.
constexpr int kFedStrideRows = 64;
static_assert(2 * kWave * (kWave + 4) <= fed_ring_floats() / 2,
              "a strided slot of 64 lanes fits a ring slot");

template <class Op, int ROWS, class View>
__device__ __forceinline__ void fed_fold_strided(const View& view, int L, int Cj, int wave,
                                                 int lane, int lane0, float* ring,
                                                 typename Op::T& acc) {
  constexpr int NOPS = View::kOps;
  constexpr int RS = ROWS + 4;                      // ring row stride (floats)
  constexpr int kThreadsPerStep = ROWS / 4;
  constexpr int kStepsPerLoad = kWave / kThreadsPerStep;
  constexpr int kPer = fed_per<ROWS, NOPS>();       // load instructions per operand per tile
  constexpr int D = fed_depth<ROWS, NOPS>();
  constexpr int B = kFedBurst < D ? kFedBurst : D;
  static_assert(kPer * kFedLoaders * kStepsPerLoad == kFedStrideRows,
                "the loaders split a tile's loads evenly");
  static_assert(D % 2 == 0 && D % B == 0, "whole bursts; a round's slot is its tile's parity");
  acc = Op::Arith::zero();
  const int part = lane % kThreadsPerStep;
  const int q = wave - 1;
  // element offsets within the chunk (below 2^31: W is), added to the
  // chunk's base pointers, which are the same for the whole work-group; 32-
  // bit offsets keep the loads from holding a 64-bit address per tile set
  uint32_t gofs[kPer];
  int rofs[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int r = (q * kPer + k) * kStepsPerLoad + lane / kThreadsPerStep;   // step in the tile
    rofs[k] = r * RS + part * 4;
    gofs[k] = static_cast<uint32_t>(r * L + lane0 + part * 4);
  }
  f32x4 regs[D][NOPS][kPer];
  const uint32_t tile_elems = static_cast<uint32_t>(kFedStrideRows) * static_cast<uint32_t>(L);
  auto gload = [&](f32x4 (&rg)[NOPS][kPer], int tile) {
    const uint32_t t0 = static_cast<uint32_t>(tile) * tile_elems;
#pragma unroll
    for (int k = 0; k < kPer; ++k)
#pragma unroll
      for (int o = 0; o < NOPS; ++o)
        rg[o][k] = ld<DPIA_NT_LOADS != 0>(
            reinterpret_cast<const f32x4*>(view.operand(o) + (t0 + gofs[k])));
    __builtin_amdgcn_sched_barrier(0);
  };
  auto put = [&](const f32x4 (&rg)[NOPS][kPer], int slot) {
#pragma unroll
    for (int k = 0; k < kPer; ++k)
#pragma unroll
      for (int o = 0; o < NOPS; ++o)
        *reinterpret_cast<f32x4*>(ring + (slot * NOPS + o) * kFedStrideRows * RS + rofs[k]) =
            rg[o][k];
  };
  // (blocks of 16 steps: the whole tile's reads at once would spill)
  auto fold_slot = [&](int slot) {
    if (lane >= ROWS) return;
#pragma unroll 1
    for (int r0 = 0; r0 < kFedStrideRows; r0 += 16)
#pragma unroll
    for (int r = r0; r < r0 + 16; r += 4) {
      f32x4 v[NOPS];
#pragma unroll
      for (int o = 0; o < NOPS; ++o)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          v[o][i] = ring[((slot * NOPS + o) * kFedStrideRows + r + i) * RS + lane];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc = Op::step(View::term(v, i), acc);
    }
  };
  // the same rounds as fed_fold
  const int ntiles = Cj / kFedStrideRows;
  if (wave > 0) {
#pragma unroll
    for (int d = 0; d < D; ++d) gload(regs[d], d);
    int r0 = 0;
    for (; r0 + D < ntiles; r0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        put(regs[d], d & 1);
        if (d % B == B - 1) {
#pragma unroll
          for (int b = d - B + 1; b <= d; ++b) gload(regs[b], r0 + b + D);
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      put(regs[d], d & 1);
      __syncthreads();
    }
    __syncthreads();
  } else {
    __syncthreads();
    for (int r = 1; r < ntiles; ++r) {
      fold_slot((r - 1) & 1);
      __syncthreads();
    }
    fold_slot((ntiles - 1) & 1);
    __syncthreads();
  }
}

}  // namespace dpia
