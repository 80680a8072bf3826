// The operations a strategy can fold: each provides the lane operator
// (step), the accumulator arithmetic (Arith) and a view of one chunk or row
// part of its operands (element loads relative to the chunk start).
#pragma once

#include <type_traits>

#include "device.h"

namespace dpia {

// ---------------------------------------------------------------- dot, asum

struct TermF { float a, b; };
struct TermA { float a; };
struct TermU { uint32_t a, b; };

// zip xs ys with lane operator lam z a. (fst z * snd z) + a
struct DotF32 {
  using Arith = PlainF32;
  using T = float;
  using Term = TermF;
  struct View {
    static constexpr bool kStageable = true;
    static constexpr int kOps = 2;
    const float* x;
    const float* y;
    __device__ const float* operand(int o) const { return o == 0 ? x : y; }
    __device__ static Term term(const f32x4 (&v)[2], int i) { return Term{v[0][i], v[1][i]}; }
    template <int NV>
    __device__ __forceinline__ void load(int off, Term (&z)[NV]) const {
      float a[NV], b[NV];
      vload<float, NV>(x + off, a);
      vload<float, NV>(y + off, b);
#pragma unroll
      for (int i = 0; i < NV; ++i) z[i] = Term{a[i], b[i]};
    }
  };
  const float* x;
  const float* y;
  __device__ View chunk(int64_t g, int64_t W) const { return View{x + g * W, y + g * W}; }
  __device__ static T step(const Term& z, T acc) { return z.a * z.b + acc; }
};

// integers modulo 2^32, same expression
struct DotU32 {
  using Arith = PlainU32;
  using T = uint32_t;
  using Term = TermU;
  struct View {
    static constexpr bool kStageable = false;
    const uint32_t* x;
    const uint32_t* y;
    template <int NV>
    __device__ __forceinline__ void load(int off, Term (&z)[NV]) const {
      uint32_t a[NV], b[NV];
      vload<uint32_t, NV>(x + off, a);
      vload<uint32_t, NV>(y + off, b);
#pragma unroll
      for (int i = 0; i < NV; ++i) z[i] = Term{a[i], b[i]};
    }
  };
  const uint32_t* x;
  const uint32_t* y;
  __device__ View chunk(int64_t g, int64_t W) const { return View{x + g * W, y + g * W}; }
  __device__ static T step(const Term& z, T acc) { return z.a * z.b + acc; }
};

// The dot with twice the load batch, for strided lanes in teams narrower
// than 1024 lanes: a batch then spans as many contiguous bytes of each
// operand as the default batch does with 1024 lanes (measured at 2^26: C=128
// L=256 58.7% -> 67.1% of peak, C=256 L=512 81% -> 84.5%; with 1024 lanes the
// default batch stays faster).
struct DotF32Deep : DotF32 {
  static constexpr int kBatchElems = 2 * DPIA_BATCH_ELEMS;
};
// Four times the batch, for strategies with too few wavefronts to keep the
// memory system busy otherwise (fewer than two per compute unit); staged
// contiguous folds keep two tiles in flight.
struct DotF32Deeper : DotF32 {
  static constexpr int kBatchElems = 4 * DPIA_BATCH_ELEMS;
  static constexpr int kStageDepth = 2;
};

// xs with lane operator lam x a. abs x + a.  One operand: twice the dot's
// batch keeps the same bytes in flight (measured at 2^26, C=256 L=1024:
// 69% -> 83% of peak).
struct AsumF32 {
  static constexpr int kBatchElems = 2 * DPIA_BATCH_ELEMS;
  using Arith = PlainF32;
  using T = float;
  using Term = TermA;
  struct View {
    static constexpr bool kStageable = true;
    static constexpr int kOps = 1;
    const float* x;
    __device__ const float* operand(int) const { return x; }
    __device__ static Term term(const f32x4 (&v)[1], int i) { return Term{v[0][i]}; }
    template <int NV>
    __device__ __forceinline__ void load(int off, Term (&z)[NV]) const {
      float a[NV];
      vload<float, NV>(x + off, a);
#pragma unroll
      for (int i = 0; i < NV; ++i) z[i] = Term{a[i]};
    }
  };
  const float* x;
  __device__ View chunk(int64_t g, int64_t W) const { return View{x + g * W}; }
  __device__ static T step(const Term& z, T acc) { return fabsf(z.a) + acc; }
};

// zip xs ys with Kahan's step on acc = (s, c):
//   y' = x*y - c ; t = s + y' ; new acc = (t, (t - s) - y')
struct KahanDotF32 {
  using Arith = KahanF32;
  using T = KPair;
  using Term = TermF;
  using View = DotF32::View;
  const float* x;
  const float* y;
  __device__ View chunk(int64_t g, int64_t W) const { return View{x + g * W, y + g * W}; }
  __device__ static T step(const Term& z, T acc) {
    const float yk = z.a * z.b - acc.c;
    const float t = acc.s + yk;
    return KPair{t, (t - acc.s) - yk};
  }
};


// zip xs ys with Sum2's step on acc = (s, c), value s + c:
//   p = x*y ; t = s + p ; bp = t - s ; new acc = (t, c + ((s - (t - bp)) + (p - bp)))
struct Sum2DotF32 {
  using Arith = Sum2F32;
  using T = KPair;
  using Term = TermF;
  using View = DotF32::View;
  const float* x;
  const float* y;
  __device__ View chunk(int64_t g, int64_t W) const { return View{x + g * W, y + g * W}; }
  __device__ static T step(const Term& z, T acc) {
    const float p = z.a * z.b;
    const float t = acc.s + p;
    const float bp = t - acc.s;
    return KPair{t, acc.c + ((acc.s - (t - bp)) + (p - bp))};
  }
};


// ---------------------------------------------------------------- gemv rows

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

#ifndef DPIA_BF16_BATCH_ELEMS
#define DPIA_BF16_BATCH_ELEMS 16
#endif
#ifndef DPIA_F32_GEMV_BATCH_ELEMS
#define DPIA_F32_GEMV_BATCH_ELEMS 32
#endif
#ifndef DPIA_F32_GEMV_STREAM_A
#define DPIA_F32_GEMV_STREAM_A 1
#endif
#ifndef DPIA_FP8_BATCH_ELEMS
#define DPIA_FP8_BATCH_ELEMS 16
#endif

// BATCH: elements per load batch (0: the format's default).  STREAM: 1 or 0
// to load A with non-temporal or cached loads (-1: the format's default).
template <typename E, class Decode, int BATCH = 0, int STREAM = -1>
struct GemvF32Acc {
  using Arith = PlainF32;
  using T = float;
  using Term = GTerm;
  // Measured on MI355X for binary32 rows, with the last-level cache evicted
  // before every call: 32-element load batches and non-temporal loads of A
  // (16384^2, C=32 L=512: 172.4 us with cached loads of A, 158.5 us
  // non-temporal, 97.7% of the read-stream ceiling on A's bytes; 16- and
  // 64-element batches 162.9 and 158.2 us; 8192^2 headline strategy 46.7 ->
  // 43.3 us).  The narrow formats stream A with 16-element batches
  // (row-blocked kernel).  x is reused by every row and stays cached.
  static constexpr bool kF32 = std::is_same<E, float>::value;
  static constexpr int kBatchElems =
      BATCH ? BATCH
            : (kF32 ? DPIA_F32_GEMV_BATCH_ELEMS
                    : (sizeof(E) == 2 ? DPIA_BF16_BATCH_ELEMS : DPIA_FP8_BATCH_ELEMS));
  static constexpr bool kStreamA = STREAM >= 0 ? STREAM != 0 : (!kF32 || DPIA_F32_GEMV_STREAM_A);
  struct View {
    static constexpr bool kStageable = std::is_same<E, float>::value;
    // 1- and 2-byte codes: staged by contiguous_staged_codes
    static constexpr bool kStageableCodes = !std::is_same<E, float>::value;
    using Code = E;
    static constexpr int kOps = 2;
    const E* a;
    const float* x;
    __device__ const float* operand(int o) const {
      return o == 0 ? reinterpret_cast<const float*>(a) : x;
    }
    __device__ static Term term(const f32x4 (&v)[2], int i) { return Term{v[0][i], v[1][i]}; }
    // NV elements as loaded: A's codes and x's values.  A batch of loads in
    // flight holds these (1 or 2 bytes per element for the narrow formats)
    // and decodes each group just before it is folded (expand).
    static constexpr bool kRaw = true;
    template <int NV>
    struct Raw {
      E a[NV];
      float x[NV];
    };
    template <int NV>
    __device__ __forceinline__ void load_raw(int off, Raw<NV>& r) const {
      vload<E, NV, kStreamA>(a + off, r.a);
      vload<float, NV, false>(x + off, r.x);   // x is reused by every row: cached
    }
    template <int NV>
    __device__ __forceinline__ static void expand(const Raw<NV>& r, Term (&z)[NV]) {
      float fa[NV];
      Decode::template run<NV>(r.a, fa);
#pragma unroll
      for (int i = 0; i < NV; ++i) z[i] = Term{fa[i], r.x[i]};
    }
    template <int NV>
    __device__ __forceinline__ void load(int off, Term (&z)[NV]) const {
      Raw<NV> r;
      load_raw<NV>(off, r);
      expand<NV>(r, z);
    }
  };
  static constexpr bool kRowBlockable = true;
  // Row blocking: NV decoded elements of row `r` (part p, offset off), and
  // NV elements of x at the same offset, loaded separately so that one x
  // load can serve several rows.
  // (The codes are loaded and decoded separately, so that a batch of loads
  // in flight holds codes, not decoded binary32 values.)
  using Code = E;
  template <int NV>
  __device__ __forceinline__ void load_codes(int64_t r, int64_t lda, int64_t col,
                                             E (&c)[NV]) const {
    vload<E, NV, kStreamA>(A + r * lda + col, c);
  }
  template <int NV>
  __device__ __forceinline__ static void decode(const E (&c)[NV], float (&f)[NV]) {
    Decode::template run<NV>(c, f);
  }
  template <int NV>
  __device__ __forceinline__ void load_a(int64_t r, int64_t lda, int64_t col,
                                         float (&f)[NV]) const {
    E c[NV];
    load_codes<NV>(r, lda, col, c);
    decode<NV>(c, f);
  }
  template <int NV>
  __device__ __forceinline__ void load_x(int64_t col, float (&f)[NV]) const {
    vload<float, NV, false>(x + col, f);
  }
  __device__ float load_a1(int64_t r, int64_t lda, int64_t col) const {
    float f[1];
    load_a<1>(r, lda, col, f);
    return f[0];
  }
  const E* A;
  const float* x;
  const float* scale;   // fp8 only
  float* y;
  // BLAS form y := alpha * v + beta * y (off: y := v).  With beta == 0 the
  // old y is never read.
  bool blas = false;
  bool beta_zero = true;
  float alpha = 1.0f, beta = 0.0f;
  __device__ View part(int64_t r, int p, int64_t lda, int W) const {
    return View{A + r * lda + static_cast<int64_t>(p) * W, x + static_cast<int64_t>(p) * W};
  }
  __device__ static T step(const Term& z, T acc) { return z.a * z.b + acc; }
  __device__ void store(int64_t r, T v) const {
    float w = scale ? scale[r] * v : v;
    if (blas) w = beta_zero ? alpha * w : alpha * w + beta * y[r];
    y[r] = w;
  }
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
// binary32 rows read by strided teams of fewer than 4 threads: each load
// instruction of a team covers under 64 bytes of its row, and the rest of the
// line is read by the team's next loads, so A stays cached (measured at
// 16384^2: C=8192 L=2 1294 us cached, 3947 us non-temporal; C=1024 L=8 with
// two row parts 252 against 524 us; teams of 4 and more gain or break even)
using GemvF32Cached = GemvF32Acc<float, DecodeF32, 0, 0>;
using GemvBF16 = GemvF32Acc<uint16_t, DecodeBF16>;
using GemvFP8 = GemvF32Acc<uint8_t, DecodeFP8>;
// fp8 rows with long lanes: four 16-byte loads per row in flight (measured
// faster from C = 64 up, slower for short lanes)
using GemvFP8Long = GemvF32Acc<uint8_t, DecodeFP8, 64>;

struct GemvU32 {
  static constexpr bool kRowBlockable = false;
  using Arith = PlainU32;
  using T = uint32_t;
  using Term = GTermU;
  struct View {
    static constexpr bool kStageable = false;
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

}  // namespace dpia
