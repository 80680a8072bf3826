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
#include "host.h"
#include "plan.h"

namespace dpia {

struct GTerm { float a, b; };
struct GTermU { uint32_t a, b; };

__device__ __forceinline__ float bf16_to_f32(uint16_t c) {
  return __uint_as_float(static_cast<uint32_t>(c) << 16);
}

// Decode NV fp8-e4m3 codes with the hardware converter (OCP E4M3 on gfx950;
// checked against the format definition over all 256 codes by the tests).
template <int NV>
__device__ __forceinline__ void fp8_to_f32(const uint8_t (&c)[NV], float (&f)[NV]) {
  if constexpr (NV == 1) {
    f[0] = __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(c[0]), 0);
  } else {
#pragma unroll
    for (int i = 0; i < NV; i += 4) {
      int w = 0;
      __builtin_memcpy(&w, &c[i], (NV - i) < 4 ? (NV - i) : 4);
      auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
      f[i] = lo[0];
      f[i + 1] = lo[1];
      if constexpr (NV >= 4) {
        auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
        f[i + 2] = hi[0];
        f[i + 3] = hi[1];
      }
    }
  }
}

template <typename E, class Decode>
struct GemvF32Acc {
  using Arith = PlainF32;
  using T = float;
  using Term = GTerm;
  struct View {
    const E* a;
    const float* x;
    template <int NV>
    __device__ __forceinline__ void load(int off, Term (&z)[NV]) const {
      E ca[NV];
      float fa[NV], b[NV];
      vload<E, NV>(a + off, ca);
      vload<float, NV, false>(x + off, b);   // x is reused by every row: cached
      Decode::template run<NV>(ca, fa);
#pragma unroll
      for (int i = 0; i < NV; ++i) z[i] = Term{fa[i], b[i]};
    }
  };
  const E* A;
  const float* x;
  const float* scale;   // fp8 only
  float* y;
  __device__ View part(int64_t r, int p, int64_t lda, int W) const {
    return View{A + r * lda + static_cast<int64_t>(p) * W, x + static_cast<int64_t>(p) * W};
  }
  __device__ static T step(const Term& z, T acc) { return z.a * z.b + acc; }
  __device__ void store(int64_t r, T v) const { y[r] = scale ? scale[r] * v : v; }
};

struct DecodeF32 {
  template <int NV>
  __device__ static void run(const float (&c)[NV], float (&f)[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) f[i] = c[i];
  }
};
struct DecodeBF16 {
  template <int NV>
  __device__ static void run(const uint16_t (&c)[NV], float (&f)[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) f[i] = bf16_to_f32(c[i]);
  }
};
struct DecodeFP8 {
  template <int NV>
  __device__ static void run(const uint8_t (&c)[NV], float (&f)[NV]) {
    fp8_to_f32<NV>(c, f);
  }
};

using GemvF32 = GemvF32Acc<float, DecodeF32>;
using GemvBF16 = GemvF32Acc<uint16_t, DecodeBF16>;
using GemvFP8 = GemvF32Acc<uint8_t, DecodeFP8>;

struct GemvU32 {
  using Arith = PlainU32;
  using T = uint32_t;
  using Term = GTermU;
  struct View {
    const uint32_t* a;
    const uint32_t* x;
    template <int NV>
    __device__ __forceinline__ void load(int off, Term (&z)[NV]) const {
      uint32_t ca[NV], b[NV];
      vload<uint32_t, NV>(a + off, ca);
      vload<uint32_t, NV, false>(x + off, b);
#pragma unroll
      for (int i = 0; i < NV; ++i) z[i] = Term{ca[i], b[i]};
    }
  };
  const uint32_t* A;
  const uint32_t* x;
  const float* scale;
  uint32_t* y;
  __device__ View part(int64_t r, int p, int64_t lda, int W) const {
    return View{A + r * lda + static_cast<int64_t>(p) * W, x + static_cast<int64_t>(p) * W};
  }
  __device__ static T step(const Term& z, T acc) { return z.a * z.b + acc; }
  __device__ void store(int64_t r, T v) const { y[r] = v; }
};

struct GemvArgs {
  int64_t m;
  int64_t k;
  int64_t lda;
  int W, L, C, team, teams_per_wg, team_lds_elems, parts;
};

template <class Op, int ORDER, int NV, int COMBINE>
__global__ void __launch_bounds__(1024) gemv_kernel(Op op, GemvArgs a) {
  using T = typename Op::T;
  using A = typename Op::Arith;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  const int team_id = threadIdx.x / a.team;
  const int t = threadIdx.x - team_id * a.team;
  T* scratch = lds + team_id * a.team_lds_elems;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * a.teams_per_wg;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * a.teams_per_wg; base < a.m;
       base += stride) {
    const int64_t row = base + team_id;
    const bool active = row < a.m;
    const int64_t r = active ? row : 0;
    // elements of each row part that exist (k may stop short of W * parts:
    // the row is zero-extended)
    const int lim0 = static_cast<int>(a.k < a.W ? a.k : a.W);
    T v = chunk_value<Op, ORDER, NV, COMBINE>(op.part(r, 0, a.lda, a.W), active, t, a.team,
                                              a.L, a.C, lim0, scratch);
    if (a.parts == 2) {
      const int lim1 = static_cast<int>(a.k - a.W);
      const T h1 = chunk_value<Op, ORDER, NV, COMBINE>(op.part(r, 1, a.lda, a.W), active, t,
                                                       a.team, a.L, a.C, lim1 > 0 ? lim1 : 0,
                                                       scratch);
      v = tree_node<A>(v, h1);   // reduceSeq (+) 0 [h0, h1]
    }
    if (active && t == 0) op.store(row, v);
  }
}

template <class Op, int MAXNV>
hipError_t launch_gemv(const Plan& p, const Op& op, int64_t m, int64_t lda, hipStream_t stream) {
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
  const int64_t grid = grid_size(p);
  return with_order_combine(p.order, p.combine, [&](auto ord, auto comb) {
    constexpr int ORDER = decltype(ord)::value;
    constexpr int COMBINE = decltype(comb)::value;
    return with_nv<MAXNV>(p.nv, [&](auto nvc) {
      constexpr int NV = decltype(nvc)::value;
      auto kern = gemv_kernel<Op, ORDER, NV, COMBINE>;
      Op op_copy = op;
      void* args[] = {&op_copy, &a};
      return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid),
                             dim3(p.wg_threads), args, p.lds_bytes, stream);
    });
  });
}

}  // namespace dpia

using namespace dpia;

extern "C" dpia_status dpia_gemv(const dpia_strategy* s, dpia_dtype a_dt, int64_t m, int64_t k,
                                 int64_t lda, const void* A, const float* row_scale,
                                 const void* x, void* y, void* ws, size_t ws_bytes,
                                 dpia_stream_t stream) {
  (void)ws;
  (void)ws_bytes;
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
  if (m == 0) {
    clear_detail();
    return DPIA_OK;
  }
  if (!A || !x || !y) return bad(DPIA_ERR_NULL, "A, x and y must be non-NULL");
  if (!aligned16(A) || !aligned16(x))
    return bad(DPIA_ERR_SHAPE, "A and x must be 16-byte aligned");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipErrorInvalidValue;
  switch (a_dt) {
    case DPIA_F32:
      e = launch_gemv<GemvF32, 4>(
          p, GemvF32{static_cast<const float*>(A), static_cast<const float*>(x), nullptr,
                     static_cast<float*>(y)},
          m, lda, hs);
      break;
    case DPIA_BF16:
      e = launch_gemv<GemvBF16, 8>(
          p, GemvBF16{static_cast<const uint16_t*>(A), static_cast<const float*>(x), nullptr,
                      static_cast<float*>(y)},
          m, lda, hs);
      break;
    case DPIA_FP8_E4M3:
      e = launch_gemv<GemvFP8, 16>(
          p, GemvFP8{static_cast<const uint8_t*>(A), static_cast<const float*>(x), row_scale,
                     static_cast<float*>(y)},
          m, lda, hs);
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
  if (e != hipSuccess) return hip_fail(e, "dpia_gemv launch");
  clear_detail();
  return DPIA_OK;
}
