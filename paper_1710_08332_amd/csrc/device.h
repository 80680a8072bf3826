// Device building blocks shared by the reduction and gemv kernels.
//
// A strategy (blocked dot product, Sec. 2.1 eq. (2)) is run as follows.
// A "team" of threads evaluates one chunk (one mapWorkgroup iteration): each
// of the chunk's L lanes (mapLocal iterations) folds its C elements with
// reduceSeq in registers (toPrivate), then the team combines the L lane
// values (tree or sequential).  Which hardware thread holds which lane, and
// how many lanes or elements one load brings in, changes no operation and no
// operand order: every lane still folds its own elements in increasing
// index, and every combine node is (0 + left) + right on the same operands.
//
// Compiled with -ffp-contract=off (and the pragma below): every product and
// every sum is rounded on its own, as the expression says.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

#pragma clang fp contract(off)

namespace dpia {

enum : int { kContiguous = 0, kStrided = 1 };
enum : int { kTree = 0, kSeq = 1, kNone = 2 };

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

#ifndef DPIA_NT_LOADS
#define DPIA_NT_LOADS 1
#endif
#ifndef DPIA_BATCH_ELEMS
#define DPIA_BATCH_ELEMS 16
#endif

template <bool NT, typename V>
__device__ __forceinline__ V ld(const V* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// Load NV consecutive elements of type E from an address aligned to
// min(16, NV * sizeof(E)) bytes, with the widest loads that fit.  STREAM
// marks data read once (non-temporal loads: streamed past the caches).
template <typename E, int NV, bool STREAM = true>
__device__ __forceinline__ void vload(const E* __restrict__ p, E (&out)[NV]) {
  constexpr bool NT = STREAM && DPIA_NT_LOADS;
  constexpr int B = static_cast<int>(sizeof(E)) * NV;
  const char* src = reinterpret_cast<const char*>(p);
  char* dst = reinterpret_cast<char*>(out);
  if constexpr (B >= 16) {
#pragma unroll
    for (int i = 0; i < B / 16; ++i) {
      u32x4 r = ld<NT>(reinterpret_cast<const u32x4*>(src + 16 * i));
      __builtin_memcpy(dst + 16 * i, &r, 16);
    }
  } else if constexpr (B == 8) {
    u32x2 r = ld<NT>(reinterpret_cast<const u32x2*>(src));
    __builtin_memcpy(dst, &r, 8);
  } else if constexpr (B == 4) {
    unsigned int r = ld<NT>(reinterpret_cast<const unsigned int*>(src));
    __builtin_memcpy(dst, &r, 4);
  } else if constexpr (B == 2) {
    unsigned short r = ld<NT>(reinterpret_cast<const unsigned short*>(src));
    __builtin_memcpy(dst, &r, 2);
  } else {
    static_assert(B == 1, "unsupported vector width");
    out[0] = ld<NT>(p);
  }
}

// Device-coherent accesses to chunk values that another work-group (on
// another XCD, whose L2 is not kept coherent with this one's) wrote or will
// read within the same launch: a relaxed agent-scope atomic store goes
// through to memory (global_store ... sc1) and a relaxed agent-scope atomic
// load is served coherently (global_load ... sc1).  A writer makes its stores
// complete (s_waitcnt) before it raises an arrival counter, so no L2
// write-back (an agent-scope release) is needed per work-group.
template <class T>
__device__ __forceinline__ void store_coherent(T* p, const T& v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte values");
  if constexpr (sizeof(T) == 4) {
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    __hip_atomic_store(reinterpret_cast<uint32_t*>(p), u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  } else {
    uint64_t u;
    __builtin_memcpy(&u, &v, 8);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <class T>
__device__ __forceinline__ T load_coherent(const T* p) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte values");
  T v;
  if constexpr (sizeof(T) == 4) {
    const uint32_t u = __hip_atomic_load(reinterpret_cast<const uint32_t*>(p), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    __builtin_memcpy(&v, &u, 4);
  } else {
    const uint64_t u = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    __builtin_memcpy(&v, &u, 8);
  }
  return v;
}

// Waits until every memory access this thread issued has completed (its
// coherent stores included).
__device__ __forceinline__ void wait_memory() { __builtin_amdgcn_s_waitcnt(0); }

// ------------------------------------------------------------ lane exchange
// The 32-bit value of the butterfly partner at distance D (1, 2, ..., 32)
// within the wavefront, for the levels of the tree combine, without the LDS
// crossbar: DPP quad permutations swap neighbours (D = 1) and pairs (D = 2);
// from D = 4 on, every aligned group of D lanes already holds one value (the
// node of the levels below), so the half-row and row mirrors (lane i reads
// lane 7 - i, or 15 - i, within its 8 or 16 lanes) fetch the partner group's
// value as an exchange with lane i ^ D would; gfx950's permlane swaps
// exchange the 16-lane rows (D = 16) and the 32-lane halves (D = 32).  Every
// lane of the wavefront must execute it.
template <int D>
__device__ __forceinline__ uint32_t butterfly_partner(uint32_t v) {
  const int x = static_cast<int>(v);
  if constexpr (D == 1) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));
  } else if constexpr (D == 2) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));
  } else if constexpr (D == 4) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false));
  } else if constexpr (D == 8) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false));
  } else if constexpr (D == 16) {
    // {old vdst, old vsrc} = {v, v}: vdst then holds rows 0,0,2,2 of v and
    // vsrc rows 1,1,3,3
    const auto s = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (threadIdx.x & 16) ? s[0] : s[1];
  } else {
    static_assert(D == 32, "butterfly distances are powers of two up to 32");
    // vdst then holds halves 0,0 of v and vsrc halves 1,1
    const auto s = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? s[0] : s[1];
  }
}

template <int D>
__device__ __forceinline__ float butterfly_partner(float v) {
  return __uint_as_float(butterfly_partner<D>(__float_as_uint(v)));
}

// ------------------------------------------------------------ accumulators
// Each accumulator type provides zero() (the literal 0 of the expression,
// +0 for binary32) and add(e, acc) = the reduceSeq operator (+) applied to an
// element e and the accumulator acc (element first, as in the paper's
// reduce), plus the butterfly exchange for the tree.

struct PlainF32 {
  using T = float;
  __device__ static T zero() { return 0.0f; }
  __device__ static T add(T e, T acc) { return e + acc; }
  template <int D>
  __device__ static T partner(T v) { return butterfly_partner<D>(v); }
};

struct PlainU32 {
  using T = uint32_t;
  __device__ static T zero() { return 0u; }
  __device__ static T add(T e, T acc) { return e + acc; }
  template <int D>
  __device__ static T partner(T v) { return butterfly_partner<D>(v); }
};

// Compensated pair (s, c), value s - c.  add(r, l) merges a later pair r
// into an earlier accumulator l with Knuth's TwoSum:
//   s = l.s + r.s ; bp = s - l.s ; e = (l.s - (s - bp)) + (r.s - bp) ;
//   result (s, (l.c + r.c) - e).
struct KPair {
  float s, c;
};

struct KahanF32 {
  using T = KPair;
  __device__ static T zero() { return KPair{0.0f, 0.0f}; }
  __device__ static T add(T r, T l) {
    const float s = l.s + r.s;
    const float bp = s - l.s;
    const float e = (l.s - (s - bp)) + (r.s - bp);
    return KPair{s, (l.c + r.c) - e};
  }
  template <int D>
  __device__ static T partner(T v) {
    return KPair{butterfly_partner<D>(v.s), butterfly_partner<D>(v.c)};
  }
};

// Sum2 pair (s, c), value s + c (Ogita, Rump, Oishi 2005).  add(r, l)
// merges a later pair r into an earlier accumulator l: TwoSum of the s
// parts, whose exact error joins the c parts:
//   s = l.s + r.s ; bp = s - l.s ; e = (l.s - (s - bp)) + (r.s - bp) ;
//   result (s, (l.c + r.c) + e).
struct Sum2F32 {
  using T = KPair;
  __device__ static T zero() { return KPair{0.0f, 0.0f}; }
  __device__ static T add(T r, T l) {
    const float s = l.s + r.s;
    const float bp = s - l.s;
    const float e = (l.s - (s - bp)) + (r.s - bp);
    return KPair{s, (l.c + r.c) + e};
  }
  template <int D>
  __device__ static T partner(T v) {
    return KPair{butterfly_partner<D>(v.s), butterfly_partner<D>(v.c)};
  }
};

// One node of the pairwise tree: reduceSeq (+) 0 over [left, right].
template <class A>
__device__ __forceinline__ typename A::T tree_node(typename A::T left, typename A::T right) {
  return A::add(right, A::add(left, A::zero()));
}

// ------------------------------------------------------------ team combine
// The tree levels over `width` adjacent threads (a power of two up to 64,
// uniform across the wavefront): level d pairs thread t with t ^ d, and both
// compute the node (0 + left) + right with the lower thread's value on the
// left.  Every thread of the wavefront takes part.
template <class A, int D>
__device__ __forceinline__ void butterfly_level(typename A::T& v, int t, int width) {
  if (width > D) {
    const typename A::T other = A::template partner<D>(v);
    v = (t & D) ? tree_node<A>(other, v) : tree_node<A>(v, other);
  }
}

template <class A>
__device__ __forceinline__ void butterfly_levels(typename A::T& v, int t, int width) {
  butterfly_level<A, 1>(v, t, width);
  butterfly_level<A, 2>(v, t, width);
  butterfly_level<A, 4>(v, t, width);
  butterfly_level<A, 8>(v, t, width);
  butterfly_level<A, 16>(v, t, width);
  butterfly_level<A, 32>(v, t, width);
}

// Combine the lane values of one chunk.  `acc` holds the NL lane values of
// this thread (NL = lanes per thread: NV for the strided order, 1 for the
// contiguous order), lanes t*NL .. t*NL + NL-1 of the team.  Returns the
// chunk value in team thread 0.  `scratch` is this team's LDS region.  All
// threads of the work-group must call this together (it has barriers).
template <class A, int NL, int COMBINE>
__device__ __forceinline__ typename A::T combine_lanes(typename A::T (&acc)[NL], int t, int team,
                                                       int L, typename A::T* scratch) {
  using T = typename A::T;
  if constexpr (COMBINE == kSeq) {
#pragma unroll
    for (int v = 0; v < NL; ++v) scratch[t * NL + v] = acc[v];
    __syncthreads();
    T r = A::zero();
    if (t == 0) {
      for (int l = 0; l < L; ++l) r = A::add(scratch[l], r);
    }
    __syncthreads();
    return r;
  } else {
    // levels inside the thread: adjacent lane pairs
#pragma unroll
    for (int w = NL; w > 1; w >>= 1) {
#pragma unroll
      for (int i = 0; i < w / 2; ++i) acc[i] = tree_node<A>(acc[2 * i], acc[2 * i + 1]);
    }
    T v = acc[0];
    // levels across the threads of one wavefront: butterfly over ascending
    // distances pairs thread t with t^d, the lower one holding the left node
    const int in_wave = team < 64 ? team : 64;
    butterfly_levels<A>(v, t, in_wave);
    if (team > 64) {
      // levels across wavefronts, through LDS
      const int waves = team / 64;
      if ((t & 63) == 0) scratch[t >> 6] = v;
      __syncthreads();
      if (t < 64) {
        v = (t < waves) ? scratch[t] : A::zero();
        butterfly_levels<A>(v, t, waves);
      }
      __syncthreads();
    }
    return v;
  }
}

// ------------------------------------------------------------ lane folds
// Fold the lanes of one chunk.  `view` gives element access relative to the
// chunk start: view.template load<NV>(off, terms) loads elements off ..
// off+NV-1 and Op::step(term, acc) is the lane operator.
//
// Loads are issued in batches of U steps before any of them is folded, so
// every wavefront keeps U vector loads per operand in flight; the folds then
// consume the batch in increasing index order.  U * NV is kept near 16
// elements per batch: a second, alternating batch was measured slower
// (register pressure lowered occupancy).
template <int NV, int E = DPIA_BATCH_ELEMS>
struct Batch {
  static constexpr int U = (E / NV) < 1 ? 1 : ((E / NV) > 16 ? 16 : (E / NV));
};

// Elements per lane group that one batch of loads covers: operations may
// choose their own (Op::kBatchElems); the default is DPIA_BATCH_ELEMS.
template <class Op, class = void>
struct OpBatch {
  static constexpr int E = DPIA_BATCH_ELEMS;
};
template <class Op>
struct OpBatch<Op, decltype(void(Op::kBatchElems))> {
  static constexpr int E = Op::kBatchElems;
};

// Views whose loads can be kept as loaded until the fold (kRaw: Raw<NV>,
// load_raw, expand), so that a batch in flight holds narrow codes.
template <class V, class = void>
struct HasRaw {
  static constexpr bool value = false;
};
template <class V>
struct HasRaw<V, decltype(void(V::kRaw))> {
  static constexpr bool value = V::kRaw;
};

// `limit` is the number of chunk elements that exist (W for a full chunk).
// A chunk past the end of the data is the zero-extended chunk of the
// expression; a missing element would contribute (0 * 0) + acc = acc (or
// |0| + acc), which leaves every accumulator unchanged because folds from
// +0 never hold -0, so missing elements are simply not folded.
template <class Op, int ORDER, int NV, class View>
__device__ __forceinline__ void lane_folds(const View& view, bool active, int t, int L, int C,
                                           int limit,
                                           typename Op::T (&acc)[ORDER == kStrided ? NV : 1]) {
  using Term = typename Op::Term;
  constexpr int U = Batch<NV, OpBatch<Op>::E>::U;
  constexpr int NL = (ORDER == kStrided) ? NV : 1;
#pragma unroll
  for (int v = 0; v < NL; ++v) acc[v] = Op::Arith::zero();
  if (!active) return;
  auto fold_vec = [&](Term (&z)[NV], int nvalid) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (ORDER == kStrided) {
        if (v < nvalid) acc[v] = Op::step(z[v], acc[v]);
      } else {
        if (v < nvalid) acc[0] = Op::step(z[v], acc[0]);
      }
    }
  };
  // element offsets: strided lane l = t*NV + v takes l + k*L (one vector
  // load covers NV lanes at the same k); contiguous lane l = t takes
  // l*C + k (one vector load covers NV consecutive k)
  int start, step, nfull;
  if constexpr (ORDER == kStrided) {
    start = t * NV;
    step = L;
    const int rows = limit / L;                 // rows k whose L elements all exist
    nfull = rows < C ? rows : C;
  } else {
    start = t * C;
    step = NV;
    int have = limit - t * C;                   // elements of this lane that exist
    have = have < 0 ? 0 : (have > C ? C : have);
    nfull = have / NV;
  }
  const int nb = nfull / U;
  for (int j = 0; j < nb; ++j) {
    const int o = start + j * U * step;
    if constexpr (HasRaw<View>::value) {
      // the batch holds operands as loaded; each group is expanded (decoded)
      // just before its fold
      typename View::template Raw<NV> r[U];
#pragma unroll
      for (int u = 0; u < U; ++u) view.template load_raw<NV>(o + u * step, r[u]);
      __builtin_amdgcn_sched_barrier(0);   // issue the whole batch first
#pragma unroll
      for (int u = 0; u < U; ++u) {
        Term z[NV];
        View::template expand<NV>(r[u], z);
        fold_vec(z, NV);
      }
    } else {
      Term z[U][NV];
#pragma unroll
      for (int u = 0; u < U; ++u) view.template load<NV>(o + u * step, z[u]);
      __builtin_amdgcn_sched_barrier(0);   // issue the whole batch first
#pragma unroll
      for (int u = 0; u < U; ++u) fold_vec(z[u], NV);
    }
  }
  for (int i = nb * U; i < nfull; ++i) {
    Term z[NV];
    view.template load<NV>(start + i * step, z);
    fold_vec(z, NV);
  }
  // the last, partly existing row (strided) or the last elements of a lane
  // (contiguous), one element at a time
  if constexpr (ORDER == kStrided) {
    if (nfull < C) {
      const int o = start + nfull * step;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (o + v < limit) {
          Term z[1];
          view.template load<1>(o + v, z);
          acc[v] = Op::step(z[0], acc[v]);
        }
      }
    }
  } else {
    int have = limit - t * C;
    have = have < 0 ? 0 : (have > C ? C : have);
    for (int k = nfull * NV; k < have; ++k) {
      Term z[1];
      view.template load<1>(start + k, z);
      acc[0] = Op::step(z[0], acc[0]);
    }
  }
}

// ------------------------------------------------------------ LDS staging
// Contiguous order through LDS, one wavefront at a time.  In the contiguous
// order lane l folds the elements l*C .. l*C + C-1 of its chunk, so the 64
// lanes of a wavefront read 64 different rows at once.  Here each wavefront
// instead loads a tile of kStage elements of each of its own 64 lanes' rows
// with 16-byte loads, kStage / 4 work-items covering one row's contiguous
// bytes, writes the tile to the wavefront's own LDS region, and every lane
// reads its kStage elements back and folds them in increasing index: the
// same operands in the same order as the direct path.  A wavefront's LDS
// accesses complete in program order, so the region needs no barrier
// between the writes and the reads, or before the next tile overwrites it:
// only a compiler fence keeps the accesses in that order.  Elements at or
// past a row's end are read as zeros, which fold as the identity (see
// lane_folds).
#ifndef DPIA_STAGE_DEPTH
#define DPIA_STAGE_DEPTH 1
#endif
constexpr int kStageVec = kStage / 4;            // 16-byte parts per row tile
constexpr int kWave = 64;
static_assert(kWave % kStageVec == 0, "a load instruction covers whole row tiles");
constexpr int kStageRowsPerLoad = kWave / kStageVec;

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 load4_masked(const float* p, int rem) {
  if (rem >= 4) return ld<DPIA_NT_LOADS != 0>(reinterpret_cast<const f32x4*>(p));
  f32x4 r = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int i = 0; i < rem; ++i) r[i] = p[i];
  return r;
}

__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// `stage`: this wavefront's region of 2 * 64 rows of kStageRow floats.  Every
// work-item of the wavefront calls this (inactive lanes fold nothing but
// still load their share of the other rows).  VEC > 1: the lane is a vector
// lane whose row holds C vectors (C * VEC elements); element e of the row
// belongs to component e % VEC, and each component folds its elements in
// increasing index (kStage is a multiple of VEC).
// Tiles a staged fold keeps in flight: Op::kStageDepth where the operation
// declares it (launches with fewer wavefronts than compute units), else
// DPIA_STAGE_DEPTH.
template <class Op, class = void>
struct StageDepth {
  static constexpr int value = DPIA_STAGE_DEPTH;
};
template <class Op>
struct StageDepth<Op, decltype(void(Op::kStageDepth))> {
  static constexpr int value = Op::kStageDepth;
};

template <class Op, int VEC = 1, class View>
__device__ __forceinline__ void contiguous_staged(const View& view, bool active, int t, int C,
                                                  int limit, typename Op::T (&acc)[VEC],
                                                  float* stage) {
  static_assert(4 % VEC == 0, "a staged 16-byte part holds whole vectors");
  constexpr int NOPS = View::kOps;
#pragma unroll
  for (int j = 0; j < VEC; ++j) acc[j] = Op::Arith::zero();
  C *= VEC;                                     // elements per lane row
  const int lane = threadIdx.x & (kWave - 1);
  int have = limit - t * C;                     // elements of this lane's row that exist
  have = active ? (have < 0 ? 0 : (have > C ? C : have)) : 0;
  // this work-item loads part `part` of rows i * kStageRowsPerLoad + lane / kStageVec
  const int part = lane % kStageVec;
  const float* rowp[NOPS][kStageVec];
  int rowhave[kStageVec];
#pragma unroll
  for (int i = 0; i < kStageVec; ++i) {
    const int r = i * kStageRowsPerLoad + lane / kStageVec;
    rowhave[i] = __shfl(have, r, kWave);
#pragma unroll
    for (int o = 0; o < NOPS; ++o) {
      const unsigned long long mine =
          reinterpret_cast<unsigned long long>(view.operand(o) + static_cast<int64_t>(t) * C);
      rowp[o][i] = reinterpret_cast<const float*>(__shfl(mine, r, kWave));
    }
  }
  const int ntiles = C / kStage;
  auto gload = [&](f32x4 (&regs)[NOPS][kStageVec], int tile) {
#pragma unroll
    for (int i = 0; i < kStageVec; ++i) {
      const int e = tile * kStage + part * 4;
#pragma unroll
      for (int o = 0; o < NOPS; ++o) regs[o][i] = load4_masked(rowp[o][i] + e, rowhave[i] - e);
    }
  };
  // tile `regs` -> this wavefront's LDS region, then `next` (the loads of a
  // later tile, in flight while this one is folded), then every lane folds
  // its row's elements of the tile in increasing index
  auto stage_fold = [&](const f32x4 (&regs)[NOPS][kStageVec], auto&& next) {
#pragma unroll
    for (int i = 0; i < kStageVec; ++i) {
      const int r = i * kStageRowsPerLoad + lane / kStageVec;
#pragma unroll
      for (int o = 0; o < NOPS; ++o)
        *reinterpret_cast<f32x4*>(stage + (o * kWave + r) * kStageRow + part * 4) = regs[o][i];
    }
    wave_lds_order();
    next();
    if (active) {
#pragma unroll
      for (int j = 0; j < kStageVec; ++j) {
        f32x4 v[NOPS];
#pragma unroll
        for (int o = 0; o < NOPS; ++o)
          v[o] = *reinterpret_cast<const f32x4*>(stage + (o * kWave + lane) * kStageRow + j * 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i % VEC] = Op::step(View::term(v, i), acc[i % VEC]);
      }
    }
    wave_lds_order();
  };
  if constexpr (StageDepth<Op>::value >= 2) {
    // two tiles in flight: tiles alternate between two register sets
    f32x4 ra[NOPS][kStageVec], rb[NOPS][kStageVec];
    gload(ra, 0);
    if (ntiles > 1) gload(rb, 1);
    for (int tile = 0; tile < ntiles; tile += 2) {
      stage_fold(ra, [&] { if (tile + 2 < ntiles) gload(ra, tile + 2); });
      if (tile + 1 < ntiles)
        stage_fold(rb, [&] { if (tile + 3 < ntiles) gload(rb, tile + 3); });
    }
  } else {
    f32x4 regs[NOPS][kStageVec];
    gload(regs, 0);
    for (int tile = 0; tile < ntiles; ++tile)
      stage_fold(regs, [&] { if (tile + 1 < ntiles) gload(regs, tile + 1); });
  }
}

// The contiguous order staged through LDS for rows of 1- or 2-byte codes
// (gemv with bf16 / fp8 A; View::kStageableCodes): as contiguous_staged,
// with the codes' row tiles (kStage codes, 2 or 4 16-byte parts) and x's
// row tiles (kStage binary32, 8 parts) loaded by their own work-item
// layouts.  Each lane decodes its kStage codes and folds them with its x
// values in increasing index.  Parts at or past a row's end hold zero
// codes and zero x, which fold as the identity.
template <class E>
__device__ __forceinline__ u32x4 load_codes_masked(const E* p, int rem) {
  constexpr int N = 16 / static_cast<int>(sizeof(E));
  if (rem >= N) return ld<false>(reinterpret_cast<const u32x4*>(p));
  E c[N];
#pragma unroll
  for (int i = 0; i < N; ++i) c[i] = (i < rem) ? p[i] : E(0);
  u32x4 r;
  __builtin_memcpy(&r, c, 16);
  return r;
}

template <class Op, class View>
__device__ __forceinline__ void contiguous_staged_codes(const View& view, bool active, int t,
                                                        int C, int limit, typename Op::T& acc,
                                                        float* stage) {
  using E = typename View::Code;
  constexpr int ES = static_cast<int>(sizeof(E));
  constexpr int PA = kStage * ES / 16;          // 16-byte parts of a code row tile
  constexpr int PX = kStage / 4;                // 16-byte parts of an x row tile
  constexpr int RA = kWave / PA, RX = kWave / PX;
  constexpr int SA = (PA + 1) * 16, SX = (PX + 1) * 16;   // row strides: odd 16-byte units
  static_assert(PA >= 1 && kWave % PA == 0, "whole code row tiles per load instruction");
  unsigned char* la = reinterpret_cast<unsigned char*>(stage);
  unsigned char* lx = la + kWave * SA;
  acc = Op::Arith::zero();
  const int lane = threadIdx.x & (kWave - 1);
  int have = limit - t * C;                     // elements of this lane's row that exist
  have = active ? (have < 0 ? 0 : (have > C ? C : have)) : 0;
  const int pa = lane % PA, px = lane % PX;
  const E* rowa[PA];
  const float* rowx[PX];
  int hava[PA], havx[PX];
  const unsigned long long mya =
      reinterpret_cast<unsigned long long>(view.a + static_cast<int64_t>(t) * C);
  const unsigned long long myx =
      reinterpret_cast<unsigned long long>(view.x + static_cast<int64_t>(t) * C);
#pragma unroll
  for (int i = 0; i < PA; ++i) {
    const int r = i * RA + lane / PA;
    hava[i] = __shfl(have, r, kWave);
    rowa[i] = reinterpret_cast<const E*>(__shfl(mya, r, kWave));
  }
#pragma unroll
  for (int i = 0; i < PX; ++i) {
    const int r = i * RX + lane / PX;
    havx[i] = __shfl(have, r, kWave);
    rowx[i] = reinterpret_cast<const float*>(__shfl(myx, r, kWave));
  }
  const int ntiles = C / kStage;
  u32x4 ca[PA];
  f32x4 cx[PX];
  auto gload = [&](int tile) {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      const int e = tile * kStage + pa * (16 / ES);
      ca[i] = load_codes_masked(rowa[i] + e, hava[i] - e);
    }
#pragma unroll
    for (int i = 0; i < PX; ++i) {
      const int e = tile * kStage + px * 4;
      cx[i] = load4_masked(rowx[i] + e, havx[i] - e);
    }
  };
  gload(0);
  for (int tile = 0; tile < ntiles; ++tile) {
#pragma unroll
    for (int i = 0; i < PA; ++i)
      *reinterpret_cast<u32x4*>(la + (i * RA + lane / PA) * SA + pa * 16) = ca[i];
#pragma unroll
    for (int i = 0; i < PX; ++i)
      *reinterpret_cast<f32x4*>(lx + (i * RX + lane / PX) * SX + px * 16) = cx[i];
    wave_lds_order();
    if (tile + 1 < ntiles) gload(tile + 1);   // in flight while this tile is folded
    if (active) {
#pragma unroll
      for (int j = 0; j < PA; ++j) {
        E c[16 / ES];
        const u32x4 u = *reinterpret_cast<const u32x4*>(la + lane * SA + j * 16);
        __builtin_memcpy(c, &u, 16);
        float f[16 / ES];
        Op::template decode<16 / ES>(c, f);
#pragma unroll
        for (int q = 0; q < 16 / ES / 4; ++q) {
          const f32x4 xv =
              *reinterpret_cast<const f32x4*>(lx + lane * SX + (j * (16 / ES / 4) + q) * 16);
#pragma unroll
          for (int i = 0; i < 4; ++i)
            acc = Op::step(typename Op::Term{f[4 * q + i], xv[i]}, acc);
        }
      }
    }
    wave_lds_order();
  }
}

template <class V, class = void>
struct StageableCodes {
  static constexpr bool value = false;
};
template <class V>
struct StageableCodes<V, decltype(void(V::kStageableCodes))> {
  static constexpr bool value = V::kStageableCodes;
};

// `stage`: this wavefront's LDS staging region (contiguous order, stageable
// views; with SS, also the strided order with one thread per chunk) or
// nullptr for direct loads.  The choice is uniform per launch.
template <class Op, int ORDER, int NV, int COMBINE, bool SS = false, class View>
__device__ __forceinline__ typename Op::T chunk_value(const View& view, bool active, int t,
                                                      int team, int L, int C, int limit,
                                                      typename Op::T* scratch,
                                                      float* stage = nullptr) {
  constexpr int NL = (ORDER == kStrided) ? NV : 1;
  typename Op::T acc[NL];
  if constexpr (ORDER == kContiguous && View::kStageable) {
    if (stage != nullptr) {
      contiguous_staged<Op, 1>(view, active, t, C, limit, acc, stage);
      return combine_lanes<typename Op::Arith, NL, COMBINE>(acc, t, team, L, scratch);
    }
  } else if constexpr (ORDER == kStrided && SS && View::kStageable && 4 % NV == 0) {
    // one thread holds all NV = L lanes of its chunk (team 1; the plan
    // stages only then): its chunk is C * NV contiguous elements, element e
    // belonging to lane e % NV, which contiguous_staged folds as components
    if (stage != nullptr) {
      contiguous_staged<Op, NV>(view, active, 0, C, limit, acc, stage);
      return combine_lanes<typename Op::Arith, NL, COMBINE>(acc, t, team, L, scratch);
    }
  } else if constexpr (ORDER == kContiguous && StageableCodes<View>::value) {
    if (stage != nullptr) {
      contiguous_staged_codes<Op>(view, active, t, C, limit, acc[0], stage);
      return combine_lanes<typename Op::Arith, NL, COMBINE>(acc, t, team, L, scratch);
    }
  }
  lane_folds<Op, ORDER, NV>(view, active, t, L, C, limit, acc);
  return combine_lanes<typename Op::Arith, NL, COMBINE>(acc, t, team, L, scratch);
}

}  // namespace dpia

namespace dpia {

// A view whose element offsets start `base` elements into another view.
template <class View>
struct ShiftedView {
  View v;
  int base;
  template <int NV, class Term>
  __device__ __forceinline__ void load(int off, Term (&z)[NV]) const {
    v.template load<NV>(base + off, z);
  }
};

// Chunk values of vector strategies (VEC > 1: the view is read as vectors of
// VEC consecutive elements, asVector VEC) and of uncombined ones (COMBINE ==
// kNone: every lane's value is a chunk value).  Writes the chunk's values to
// out[g * cv ...], cv = VEC, or L * VEC uncombined, in lane then component
// order (asScalar VEC of the join), with device-coherent stores.  All threads of the work-group call this
// together (the combine has barriers).
// `stage`: as for chunk_value (the contiguous order, staged per wavefront).
template <class Op, int ORDER, int NV, int COMBINE, int VEC, class View>
__device__ __forceinline__ void chunk_values_wide(const View& view, bool active, int t, int team,
                                                  int L, int C, int limit,
                                                  typename Op::T* scratch, typename Op::T* out,
                                                  int64_t g, float* stage = nullptr) {
  using T = typename Op::T;
  constexpr bool kStaged = ORDER == kContiguous && View::kStageable;
  if constexpr (VEC == 1) {
    static_assert(COMBINE == kNone, "scalar combined chunks use chunk_value");
    constexpr int NL = (ORDER == kStrided) ? NV : 1;
    T acc[NL];
    if constexpr (kStaged) {
      if (stage != nullptr)
        contiguous_staged<Op, 1>(view, active, t, C, limit, acc, stage);
      else
        lane_folds<Op, ORDER, NV>(view, active, t, L, C, limit, acc);
    } else {
      lane_folds<Op, ORDER, NV>(view, active, t, L, C, limit, acc);
    }
    if (active) {
      const int64_t lane0 = g * L + (ORDER == kStrided ? t * NV : t);
#pragma unroll
      for (int v = 0; v < NL; ++v) store_coherent(out + lane0 + v, acc[v]);
    }
  } else {
    static_assert(NV == VEC, "a thread is one vector lane");
    T acc[VEC];
    if constexpr (ORDER == kStrided) {
      // vector lane t takes vectors t, t + L, ...: element VEC*(k*L + t) + j
      // is scalar lane VEC*t + j of the strided order over VEC*L lanes
      lane_folds<Op, kStrided, VEC>(view, active, t, L * VEC, C, limit, acc);
    } else {
      // vector lane t takes vectors t*C .. t*C + C-1: within the lane's row of
      // VEC*C elements, component j takes elements j, j + VEC, ..., the
      // strided order over VEC lanes
      bool staged = false;
      if constexpr (kStaged) {
        if (stage != nullptr) {
          contiguous_staged<Op, VEC>(view, active, t, C, limit, acc, stage);
          staged = true;
        }
      }
      if (!staged) {
        const int base = t * VEC * C;
        int have = limit - base;
        have = have < 0 ? 0 : (have > VEC * C ? VEC * C : have);
        lane_folds<Op, kStrided, VEC>(ShiftedView<View>{view, base}, active, 0, VEC, C, have,
                                      acc);
      }
    }
    if constexpr (COMBINE == kNone) {
      if (active) {
#pragma unroll
        for (int j = 0; j < VEC; ++j) store_coherent(out + (g * L + t) * VEC + j, acc[j]);
      }
    } else {
      // the combine acts on each component
#pragma unroll
      for (int j = 0; j < VEC; ++j) {
        T one[1] = {acc[j]};
        const T c = combine_lanes<typename Op::Arith, 1, COMBINE>(one, t, team, L, scratch);
        if (active && t == 0) store_coherent(out + g * VEC + j, c);
      }
    }
  }
}

}  // namespace dpia
