// Internal launch plan shared by the validation unit (plan.cpp, no HIP) and
// the kernel dispatch (dpia_kernels.hip).  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "dpia.h"

namespace dpia {

// Bytes of one 16-byte vector load, the widest global load used.
constexpr int kVecBytes = 16;
// Chunk results staged through LDS per block by the final sequential fold.
constexpr int kFoldBlock = 2048;
// Alignment of the sections of a workspace.
constexpr size_t kWsAlign = 256;
// LDS staging of the contiguous order: elements per lane per tile, and the
// LDS row stride in floats (144 bytes: an odd number of 16-byte units).  A
// tile of 32 binary32 elements is one 128-byte line of each lane's row:
// measured on the contiguous dot at 2^26 (L=256, C=64..1024), 32 runs at
// 65-75% of peak, 16 at 39-46% and 64 at 51-77% (needing 256 registers).
#ifndef DPIA_STAGE
#define DPIA_STAGE 32
#endif
constexpr int kStage = DPIA_STAGE;
constexpr int kStageRow = kStage + 4;
// LDS floats one team needs for staging: two operands x L rows.
constexpr int stage_floats(int L) { return 2 * L * kStageRow; }

struct Plan {
  dpia_op op;
  dpia_dtype dt;          // input element type (gemv: type of A)
  uint32_t order;         // dpia_order
  uint32_t combine;       // dpia_combine (already SEQ when L == 1)
  uint32_t accum;         // dpia_accum
  bool final_f64;
  uint32_t passes;

  int64_t L, C, W;        // lanes, elements (vectors) per lane, elements per chunk
  int V;                  // vector width of the asVector view (1: scalar)
  int64_t items;          // dot/asum: chunks G = ceil(n / W); gemv: rows m
  int64_t cv;             // dot/asum: values per chunk (V, times L uncombined)
  int64_t values;         // dot/asum: values the outer fold reads, items * cv
  int64_t n;              // dot/asum: vector length
  int64_t k, lda;         // gemv only
  int row_parts, R;       // gemv only

  int nv;                 // strided: lanes per thread; contiguous: elements
                          // per vector load of one lane; V > 1: V (a thread
                          // is one vector lane)
  int team;               // threads cooperating on one chunk (P)
  int teams_per_wg;       // chunks (rows) a hardware work-group holds at once
  int wg_threads;         // teams_per_wg * team
  uint32_t max_grid;      // 0 = automatic

  size_t acc_bytes;       // bytes of one chunk result (8 for a Kahan pair)
  size_t partial_bytes;   // workspace bytes for the chunk results (aligned)
  size_t ws_bytes;        // total workspace: partials + arrival counter
  size_t lds_bytes;       // dynamic LDS per work-group
  bool stage;             // contiguous order staged through LDS
  int scal_tile;          // scal staged: elements of a row per tile (16, 32, 64)
  size_t stage_off;       // byte offset of the staging region in the LDS
  size_t split_off;       // dot/asum: byte offset in the workspace of the nodes and
                          // per-chunk arrival counts of teams split over work-groups
                          // (0: the workspace has none)
};

// Teams whose lanes the loader-wavefront kernel may split over work-groups
// (tree combine, one lane per thread, at most kSplitMaxItems chunks) keep up
// to kSplitMax nodes per chunk in the workspace.
constexpr int kSplitMax = 8;
constexpr int64_t kSplitMaxItems = 1024;

size_t elem_bytes(dpia_dtype dt);

// Validates and fills `p`.  On error returns the status and sets `detail`.
dpia_status make_plan(const dpia_strategy* s, dpia_op op, dpia_dtype dt, int64_t m,
                      int64_t n, Plan* p, std::string* detail);

// Thread-local error detail (set by every failing entry point).
void set_detail(const std::string& d);
void clear_detail();
const char* detail_cstr();

}  // namespace dpia
