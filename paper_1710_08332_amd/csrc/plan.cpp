// Strategy validation and launch planning.  Pure host C++: no HIP call, so
// it also runs on machines without a GPU.
#include "plan.h"

#include <sstream>

#ifndef DPIA_MIN_WORKGROUPS
#define DPIA_MIN_WORKGROUPS 256   // the MI355X's compute units
#endif
// gemv rows spread down to this many work-groups (four per compute unit;
// measured at 16384^2, back to back, 256 / 512 / 1024: contiguous C=1024
// L=8 with two parts 190.8 / 191.2 / 182.0 us, strided C=1024 L=16 179.6 /
// 174.7 / 176.9 us, strided C=1024 L=8 with two parts 239.1 / 234.3 / 235.5)
#ifndef DPIA_GEMV_MIN_WORKGROUPS
#define DPIA_GEMV_MIN_WORKGROUPS 1024
#endif

namespace dpia {

namespace {

thread_local std::string g_detail;

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Largest power of two <= cap that divides every value in `vals`.
int widest_vector(int cap, std::initializer_list<int64_t> vals) {
  int v = cap;
  while (v > 1) {
    bool ok = true;
    for (int64_t x : vals) ok = ok && (x % v == 0);
    if (ok) break;
    v >>= 1;
  }
  return v;
}

dpia_status fail(std::string* detail, dpia_status st, const std::string& msg) {
  if (detail) *detail = msg;
  return st;
}

}  // namespace

void set_detail(const std::string& d) { g_detail = d; }
void clear_detail() { g_detail.clear(); }
const char* detail_cstr() { return g_detail.c_str(); }

size_t elem_bytes(dpia_dtype dt) {
  switch (dt) {
    case DPIA_F32: return 4;
    case DPIA_F64: return 8;
    case DPIA_I32: return 4;
    case DPIA_BF16: return 2;
    case DPIA_FP8_E4M3: return 1;
  }
  return 0;
}

dpia_status make_plan(const dpia_strategy* s, dpia_op op, dpia_dtype dt, int64_t m,
                      int64_t n, Plan* p, std::string* detail) {
  std::ostringstream os;
  if (!s) return fail(detail, DPIA_ERR_NULL, "strategy descriptor is NULL");
  if (s->abi_version != DPIA_ABI_VERSION) {
    os << "descriptor abi_version " << s->abi_version << " != library " << DPIA_ABI_VERSION;
    return fail(detail, DPIA_ERR_ABI, os.str());
  }
  if (op != DPIA_OP_DOT && op != DPIA_OP_ASUM && op != DPIA_OP_GEMV && op != DPIA_OP_SCAL)
    return fail(detail, DPIA_ERR_STRATEGY, "unknown operation");
  if (s->seq_len < 1 || s->local_size < 1)
    return fail(detail, DPIA_ERR_STRATEGY, "seq_len and local_size must be >= 1");
  if (s->order > DPIA_ORDER_STRIDED) return fail(detail, DPIA_ERR_STRATEGY, "unknown order");
  if (s->wg_combine > DPIA_COMBINE_NONE)
    return fail(detail, DPIA_ERR_STRATEGY, "unknown wg_combine");
  const int V = s->vec_width == 0 ? 1 : static_cast<int>(s->vec_width);
  if (V != 1 && V != 2 && V != 4)
    return fail(detail, DPIA_ERR_STRATEGY, "vec_width must be 0, 1, 2 or 4");
  if ((V > 1 || s->wg_combine == DPIA_COMBINE_NONE) && op != DPIA_OP_DOT && op != DPIA_OP_ASUM)
    return fail(detail, DPIA_ERR_STRATEGY,
                "vector and uncombined strategies apply to dot and asum only");
  if ((V > 1 || s->wg_combine == DPIA_COMBINE_NONE) && s->accum != DPIA_ACCUM_PLAIN)
    return fail(detail, DPIA_ERR_STRATEGY,
                "vector and uncombined strategies use plain accumulation");
  if (s->passes != 1 && s->passes != 2)
    return fail(detail, DPIA_ERR_STRATEGY, "passes must be 1 or 2");
  if (s->accum > DPIA_ACCUM_SUM2) return fail(detail, DPIA_ERR_STRATEGY, "unknown accum");
  if (s->final_f64 > 1) return fail(detail, DPIA_ERR_STRATEGY, "final_f64 must be 0 or 1");
  const bool compensated = s->accum == DPIA_ACCUM_KAHAN || s->accum == DPIA_ACCUM_SUM2;
  if (s->final_f64 && !compensated)
    return fail(detail, DPIA_ERR_STRATEGY,
                "final_f64 applies to the compensated accumulations only");
  // (scal is a map: it has no combine, whatever the descriptor says)
  if (s->wg_combine == DPIA_COMBINE_TREE && !is_pow2(s->local_size) && op != DPIA_OP_SCAL)
    return fail(detail, DPIA_ERR_STRATEGY, "a tree combine needs a power-of-two local_size");
  if (s->rows_per_wg < 1) return fail(detail, DPIA_ERR_STRATEGY, "rows_per_wg must be >= 1");
  if (s->row_parts != 1 && s->row_parts != 2)
    return fail(detail, DPIA_ERR_STRATEGY, "row_parts must be 1 or 2");

  // element types
  if (op == DPIA_OP_DOT) {
    if (dt != DPIA_F32 && dt != DPIA_I32)
      return fail(detail, DPIA_ERR_DTYPE, "dot takes F32 or I32 vectors");
    if (compensated && dt != DPIA_F32)
      return fail(detail, DPIA_ERR_DTYPE, "compensated accumulation is defined for F32 only");
  } else if (op == DPIA_OP_SCAL) {
    if (dt != DPIA_F32) return fail(detail, DPIA_ERR_DTYPE, "scal takes F32 vectors");
    if (s->accum != DPIA_ACCUM_PLAIN)
      return fail(detail, DPIA_ERR_STRATEGY, "scal has no accumulation");
  } else if (op == DPIA_OP_ASUM) {
    if (dt != DPIA_F32) return fail(detail, DPIA_ERR_DTYPE, "asum takes F32 vectors");
    if (s->accum != DPIA_ACCUM_PLAIN)
      return fail(detail, DPIA_ERR_STRATEGY, "asum supports plain accumulation only");
  } else {
    if (dt != DPIA_F32 && dt != DPIA_BF16 && dt != DPIA_FP8_E4M3 && dt != DPIA_I32)
      return fail(detail, DPIA_ERR_DTYPE, "gemv takes an F32, BF16, FP8_E4M3 or I32 matrix");
    if (s->accum != DPIA_ACCUM_PLAIN)
      return fail(detail, DPIA_ERR_STRATEGY, "gemv supports plain accumulation only");
  }
  if (op != DPIA_OP_GEMV && (s->rows_per_wg != 1 || s->row_parts != 1))
    return fail(detail, DPIA_ERR_STRATEGY, "rows_per_wg and row_parts apply to gemv only");

  Plan q{};
  q.op = op;
  q.dt = dt;
  q.order = s->order;
  q.L = s->local_size;
  q.C = s->seq_len;
  q.V = V;
  q.W = q.L * q.C * V;
  q.combine = (q.L == 1 && s->wg_combine != DPIA_COMBINE_NONE)
                  ? static_cast<uint32_t>(DPIA_COMBINE_SEQ)
                  : s->wg_combine;
  q.accum = s->accum;
  q.final_f64 = s->final_f64 != 0;
  q.passes = s->passes;
  q.max_grid = s->max_grid;
  q.row_parts = static_cast<int>(s->row_parts);
  q.R = static_cast<int>(s->rows_per_wg);
  q.acc_bytes = compensated ? 8 : 4;

  const int cap = kVecBytes / static_cast<int>(elem_bytes(dt));
  if (op == DPIA_OP_GEMV) {
    int64_t k = n;
    if (m < 0 || k < 0) return fail(detail, DPIA_ERR_SHAPE, "negative gemv size");
    if (m % q.R) {
      os << "m = " << m << " is not a multiple of rows_per_wg = " << q.R;
      return fail(detail, DPIA_ERR_SHAPE, os.str());
    }
    // rows shorter than W * row_parts are zero-extended (no partial
    // product of a missing element changes a fold from +0)
    if (k < 1 || k > q.W * q.row_parts) {
      os << "k = " << k << " must be in [1, seq_len * local_size * row_parts = "
         << q.W * q.row_parts << "]";
      return fail(detail, DPIA_ERR_SHAPE, os.str());
    }
    q.k = k;
    q.items = m;
  } else {
    if (n < 0) return fail(detail, DPIA_ERR_SHAPE, "negative length");
    // A length that is not a multiple of W is zero-extended to the next
    // multiple; that leaves plain folds unchanged but not compensated ones.
    if (n % q.W && compensated) {
      os << "n = " << n << " is not a multiple of the chunk W = seq_len * local_size = " << q.W
         << " (required for compensated accumulation)";
      return fail(detail, DPIA_ERR_SHAPE, os.str());
    }
    q.n = n;
    q.items = (n + q.W - 1) / q.W;
  }
  if (q.W >= (int64_t(1) << 31)) {
    os << "chunk W = seq_len * local_size = " << q.W << " must be below 2^31";
    return fail(detail, DPIA_ERR_STRATEGY, os.str());
  }

  // Vector width (semantics-free: it decides which lanes or elements one
  // thread loads at once, never the order of any operation).
  if (V > 1) {
    // a thread is one vector lane and loads its V components at once
    if (V > cap) return fail(detail, DPIA_ERR_STRATEGY, "vec_width exceeds a 16-byte load");
    q.nv = V;
    q.team = static_cast<int>(q.L);
  } else if (q.order == DPIA_ORDER_STRIDED) {
    q.nv = widest_vector(cap, {q.L});
    q.team = static_cast<int>(q.L / q.nv);
  } else {
    q.nv = widest_vector(cap, {q.C});
    q.team = static_cast<int>(q.L);
  }
  if (q.team > 1024) {
    os << "one chunk would need " << q.team << " threads (> 1024); reduce local_size";
    return fail(detail, DPIA_ERR_STRATEGY, os.str());
  }
  if (op == DPIA_OP_GEMV) {
    if (static_cast<int64_t>(q.team) * q.R > 1024) {
      os << "rows_per_wg * threads per row = " << int64_t(q.team) * q.R << " > 1024";
      return fail(detail, DPIA_ERR_STRATEGY, os.str());
    }
    int lg = 256 / (q.team * q.R);
    if (lg < 1) lg = 1;
    q.teams_per_wg = lg * q.R;
#if DPIA_MIN_WORKGROUPS
    // few rows per compute unit (R rows of many threads each): fewer rows per
    // hardware work-group, down to one wavefront.  Rows are independent, so
    // which work-group reduces a row does not change its association.
    while (q.teams_per_wg > 1 && (q.teams_per_wg / 2) * q.team >= 64 &&
           (q.items + q.teams_per_wg - 1) / q.teams_per_wg < DPIA_GEMV_MIN_WORKGROUPS)
      q.teams_per_wg /= 2;
#endif
  } else {
    q.teams_per_wg = q.team >= 256 ? 1 : 256 / q.team;
#if DPIA_MIN_WORKGROUPS
    // few chunks: fewer chunks per work-group, down to one wavefront per
    // work-group, so that they spread over more compute units (which
    // work-group evaluates a chunk is free; measured on the Sec. 6.2 form,
    // 128 chunks of 64 lanes: 3.4% -> 7.8% of peak)
    while (q.teams_per_wg > 1 && (q.teams_per_wg / 2) * q.team >= 64 &&
           (q.items + q.teams_per_wg - 1) / q.teams_per_wg < DPIA_MIN_WORKGROUPS)
      q.teams_per_wg /= 2;
#endif
  }
  q.wg_threads = q.teams_per_wg * q.team;

  // LDS: lane values for a sequential combine, one value per wave for a
  // tree wider than a wavefront, and the staging block of the final fold.
  size_t lds = 0;
  if (q.combine == DPIA_COMBINE_NONE) {
    lds = 0;
  } else if (q.combine == DPIA_COMBINE_SEQ) {
    lds = static_cast<size_t>(q.teams_per_wg) * q.L * q.acc_bytes;
  } else if (q.team > 64) {
    lds = static_cast<size_t>(q.teams_per_wg) * (q.team / 64) * q.acc_bytes;
  }
  // The contiguous order with binary32 operands is staged through LDS, one
  // wavefront at a time, when every lane's row (C elements, or C vectors of
  // 4) holds whole tiles and the work-group is whole wavefronts, at most 256
  // threads.
  q.stage = q.order == DPIA_ORDER_CONTIGUOUS && dt == DPIA_F32 && q.nv == 4 &&
            (V == 1 || V == 4) && (q.C * V) % kStage == 0 && q.wg_threads <= 256 &&
            q.wg_threads % 64 == 0;
  // gemv rows of bf16 / fp8 codes: the codes' and x's row tiles, each row
  // stride an odd number of 16-byte units, fit the same region
  if (op == DPIA_OP_GEMV && (dt == DPIA_BF16 || dt == DPIA_FP8_E4M3))
    q.stage = q.order == DPIA_ORDER_CONTIGUOUS && q.C % kStage == 0 &&
              q.wg_threads <= 256 && q.wg_threads % 64 == 0;
  // binary32 gemv rows in the strided order with one thread per row (L = 1,
  // 2 or 4 lanes, all in that thread): the thread walks its row part
  // contiguously, lane l taking elements l, l + L, ..., which is the staged
  // contiguous fold with L components; without staging every load
  // instruction of a wavefront touched 64 rows
  if (op == DPIA_OP_GEMV && dt == DPIA_F32 && q.order == DPIA_ORDER_STRIDED && q.team == 1 &&
      (q.C * q.L) % kStage == 0 && q.wg_threads <= 256 && q.wg_threads % 64 == 0)
    q.stage = true;
  q.stage_off = 0;
  if (q.stage) {
    q.stage_off = round_up(lds, 16);
    lds = q.stage_off + static_cast<size_t>(q.wg_threads / 64) * stage_floats(64) * sizeof(float);
  }
  if (op == DPIA_OP_SCAL) {
    // a map: no combine and no fold; the contiguous order is staged through
    // LDS per wavefront (one operand) under the same conditions as above
    // in tiles of up to 64 elements of a row (whole rows when C allows)
    q.stage = q.order == DPIA_ORDER_CONTIGUOUS && q.nv == 4 && q.C % 16 == 0 &&
              q.wg_threads <= 256 && q.wg_threads % 64 == 0;
    q.scal_tile = q.C % 64 == 0 ? 64 : (q.C % 32 == 0 ? 32 : 16);
    q.stage_off = 0;
    lds = q.stage ? static_cast<size_t>(q.wg_threads / 64) * 64 * (q.scal_tile + 4) * sizeof(float)
                  : 0;
  }
  if ((op == DPIA_OP_DOT || op == DPIA_OP_ASUM) && q.passes == 1) {
    // the last work-group of a 1-pass launch runs the final fold
    size_t fold = static_cast<size_t>(kFoldBlock) * q.acc_bytes;
    if (fold > lds) lds = fold;
  }
  lds = round_up(lds + 16, 16);
#ifndef DPIA_LDS_CAP
#define DPIA_LDS_CAP (160 * 1024)   // gfx950: 160 KB of LDS per compute unit
#endif
  if (lds > DPIA_LDS_CAP) {
    os << "strategy needs " << lds << " bytes of LDS per work-group (> " << DPIA_LDS_CAP << ")";
    return fail(detail, DPIA_ERR_STRATEGY, os.str());
  }
  q.lds_bytes = lds;

  if (op == DPIA_OP_GEMV || op == DPIA_OP_SCAL) {
    q.partial_bytes = 0;
    q.ws_bytes = 0;
  } else {
    q.cv = (q.combine == DPIA_COMBINE_NONE ? q.L : 1) * V;
    q.values = q.items * q.cv;
    q.partial_bytes = round_up(static_cast<size_t>(q.values) * q.acc_bytes, kWsAlign);
    q.ws_bytes = q.partial_bytes + kWsAlign;   // + the arrival counter
    // staged contiguous teams of 64, 128 or 256 lanes, and scalar strided
    // teams of 16 to 512 lanes, with a tree combine and few chunks: room for
    // the nodes of their lanes split over work-groups, and one arrival count
    // per chunk (zero between calls)
    q.split_off = 0;
    const bool split_contiguous = q.stage && q.order == DPIA_ORDER_CONTIGUOUS &&
                                  q.teams_per_wg == 1 &&
                                  (q.team == 64 || q.team == 128 || q.team == 256);
    const bool split_strided = q.order == DPIA_ORDER_STRIDED && dt == DPIA_F32 &&
                               q.accum == DPIA_ACCUM_PLAIN && q.L >= 16 && q.L <= 512 &&
                               (q.L & (q.L - 1)) == 0 && q.C % 64 == 0;
    if ((split_contiguous || split_strided) && q.combine == DPIA_COMBINE_TREE && V == 1 &&
        q.items > 0 && q.items <= kSplitMaxItems) {
      q.split_off = q.ws_bytes;
      q.ws_bytes += round_up(static_cast<size_t>(q.items) * kSplitMax * q.acc_bytes, kWsAlign) +
                    round_up(static_cast<size_t>(q.items) * sizeof(uint32_t), kWsAlign);
    }
  }
  *p = q;
  return DPIA_OK;
}

}  // namespace dpia

extern "C" {

dpia_status dpia_strategy_check(const dpia_strategy* s, dpia_op op, dpia_dtype dt, int64_t m,
                                int64_t n, size_t* ws_bytes_out) {
  dpia::Plan p;
  std::string detail;
  dpia_status st = dpia::make_plan(s, op, dt, m, n, &p, &detail);
  if (st != DPIA_OK) {
    dpia::set_detail(detail);
    return st;
  }
  dpia::clear_detail();
  if (ws_bytes_out) *ws_bytes_out = p.ws_bytes;
  return DPIA_OK;
}

const char* dpia_status_str(dpia_status st) {
  switch (st) {
    case DPIA_OK: return "ok";
    case DPIA_ERR_NULL: return "null pointer";
    case DPIA_ERR_SHAPE: return "shape does not fit the strategy";
    case DPIA_ERR_STRATEGY: return "invalid strategy";
    case DPIA_ERR_DTYPE: return "unsupported dtype";
    case DPIA_ERR_WORKSPACE: return "workspace too small";
    case DPIA_ERR_HIP: return "HIP error";
    case DPIA_ERR_ABI: return "ABI version mismatch";
  }
  return "unknown status";
}

const char* dpia_last_error_detail(void) { return dpia::detail_cstr(); }

uint32_t dpia_abi_version(void) { return DPIA_ABI_VERSION; }

}  // extern "C"
