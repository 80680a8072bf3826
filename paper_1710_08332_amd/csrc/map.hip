// scal: y[i] = alpha * x[i] (the scal benchmark of Sec. 7.1), under the same
// strategy descriptor as the reductions.  A map has no association: the
// strategy only decides which work-group (chunk of W elements) and which
// lane (its C elements, contiguous or strided) produces each element, and
// every element is one binary32 product.  y may be x (in place): each
// element is read and written by the same thread.
#include "device.h"
#include "host.h"
#include "plan.h"

namespace dpia {

struct MapArgs {
  int64_t n, W, items;
  int L, C, team, teams_per_wg;
};

template <int NV>
__device__ __forceinline__ void scal_vec(float alpha, const float* x, float* y,
                                         int64_t off, int64_t limit) {
  if (off + NV <= limit) {
    float v[NV];
    vload<float, NV>(x + off, v);
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = alpha * v[i];
    if constexpr (NV == 4) {
      f32x4 w = {v[0], v[1], v[2], v[3]};
      __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(y + off));
    } else {
#pragma unroll
      for (int i = 0; i < NV; ++i) y[off + i] = v[i];
    }
  } else {
    for (int64_t i = off; i < limit && i < off + NV; ++i) y[i] = alpha * x[i];
  }
}

// U vectors of one thread at offsets off0 + u * stride: all loads first,
// then the products and stores (whole chunks only: every offset exists).
template <int NV, int U>
__device__ __forceinline__ void scal_batch(float alpha, const float* x, float* y, int64_t off0,
                                           int64_t stride) {
  float v[U][NV];
#pragma unroll
  for (int u = 0; u < U; ++u) vload<float, NV>(x + off0 + u * stride, v[u]);
  __builtin_amdgcn_sched_barrier(0);   // issue the whole batch first
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t off = off0 + u * stride;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[u][i] = alpha * v[u][i];
    if constexpr (NV == 4) {
      f32x4 w = {v[u][0], v[u][1], v[u][2], v[u][3]};
      __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(y + off));
    } else {
#pragma unroll
      for (int i = 0; i < NV; ++i) y[off + i] = v[u][i];
    }
  }
}

template <int ORDER, int NV>
__global__ void __launch_bounds__(1024) scal_kernel(float alpha, const float* x, float* y,
                                                    MapArgs a) {
  constexpr int U = (32 / NV) < 1 ? 1 : (32 / NV);   // 32 elements per batch
  const int team_id = threadIdx.x / a.team;
  const int t = threadIdx.x - team_id * a.team;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * a.teams_per_wg;
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * a.teams_per_wg; base < a.items;
       base += stride) {
    const int64_t g = base + team_id;
    if (g >= a.items) continue;       // no barriers in this kernel
    const int64_t c0 = g * a.W;
    const int64_t rest = a.n - c0;
    const bool whole = rest >= a.W;
    const int64_t limit = c0 + (whole ? a.W : rest);
    if constexpr (ORDER == kStrided) {
      // lane l = t*NV + v maps elements l, l + L, ...
      int k = 0;
      if (whole)
        for (; k + U <= a.C; k += U)
          scal_batch<NV, U>(alpha, x, y, c0 + static_cast<int64_t>(k) * a.L + t * NV, a.L);
      for (; k < a.C; ++k)
        scal_vec<NV>(alpha, x, y, c0 + static_cast<int64_t>(k) * a.L + t * NV, limit);
    } else {
      // lane l = t maps elements l*C .. l*C + C-1
      const int64_t s = c0 + static_cast<int64_t>(t) * a.C;
      int k = 0;
      if (whole)
        for (; k + U * NV <= a.C; k += U * NV) scal_batch<NV, U>(alpha, x, y, s + k, NV);
      for (; k < a.C; k += NV) scal_vec<NV>(alpha, x, y, s + k, limit);
    }
  }
}

__device__ __forceinline__ void store4_masked(float* p, f32x4 v, int rem) {
  if (rem >= 4) {
    __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p));
    return;
  }
  for (int i = 0; i < rem; ++i) p[i] = v[i];
}

// The contiguous order through LDS, one wavefront at a time (as for the
// contiguous reductions): the wavefront loads a tile of S elements of each
// of its 64 lanes' rows with 16-byte loads, every lane multiplies its own S
// elements in the wavefront's LDS region, and the wavefront stores the tile
// with 16-byte stores.  Each product is still made by the lane that owns the
// element.  Elements past a row's end are neither loaded nor stored.  A
// wavefront's LDS accesses complete in program order, so compiler fences
// suffice between the phases.  With S = C a wavefront's tile is its 64
// rows, one contiguous block.
template <int S>
__global__ void __launch_bounds__(256) scal_staged_kernel(float alpha, const float* x, float* y,
                                                          MapArgs a) {
  constexpr int P = S / 4;                 // 16-byte parts per row tile
  constexpr int RPL = kWave / P;           // rows one load instruction covers
  constexpr int ROW = S + 4;               // LDS row stride in floats
  static_assert(kWave % P == 0, "a load instruction covers whole row tiles");
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* stage = reinterpret_cast<float*>(lds_raw) + (threadIdx.x / kWave) * kWave * ROW;
  const int lane = threadIdx.x & (kWave - 1);
  const int team_id = threadIdx.x / a.team;
  const int t = threadIdx.x - team_id * a.team;
  const int part = lane % P;
  const int ntiles = a.C / S;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * a.teams_per_wg;
  // the loop bounds depend on the work-group only: every wavefront runs them
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * a.teams_per_wg; base < a.items;
       base += stride) {
    const int64_t g = base + team_id;
    const bool active = g < a.items;
    const int64_t row0 = (active ? g : 0) * a.W + static_cast<int64_t>(t) * a.C;
    const int64_t left = a.n - row0;
    const int have = active ? static_cast<int>(left < 0 ? 0 : (left > a.C ? a.C : left)) : 0;
    int64_t rowoff[P];
    int rowhave[P], rowslot[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int r = i * RPL + lane / P;
      rowoff[i] = __shfl(row0, r, kWave);
      rowhave[i] = __shfl(have, r, kWave);
      rowslot[i] = r * ROW + part * 4;
    }
    f32x4 regs[P];
    auto gload = [&](int tile) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int e = tile * S + part * 4;
        regs[i] = load4_masked(x + rowoff[i] + e, rowhave[i] - e);
      }
    };
    gload(0);
    for (int tile = 0; tile < ntiles; ++tile) {
#pragma unroll
      for (int i = 0; i < P; ++i) *reinterpret_cast<f32x4*>(stage + rowslot[i]) = regs[i];
      wave_lds_order();
      if (tile + 1 < ntiles) gload(tile + 1);   // in flight during this tile
#pragma unroll
      for (int j = 0; j < P; ++j) {             // this lane's own elements
        f32x4* q = reinterpret_cast<f32x4*>(stage + lane * ROW + j * 4);
        f32x4 v = *q;
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = alpha * v[i];
        *q = v;
      }
      wave_lds_order();
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int e = tile * S + part * 4;
        store4_masked(y + rowoff[i] + e, *reinterpret_cast<const f32x4*>(stage + rowslot[i]),
                      rowhave[i] - e);
      }
      wave_lds_order();
    }
  }
}

}  // namespace dpia

using namespace dpia;

extern "C" dpia_status dpia_scal(const dpia_strategy* s, dpia_dtype dt, int64_t n, float alpha,
                                 const void* x, void* y, dpia_stream_t stream) {
  Plan p;
  std::string detail;
  dpia_status st = make_plan(s, DPIA_OP_SCAL, dt, 0, n, &p, &detail);
  if (st != DPIA_OK) return bad(st, detail);
  if (n > 0 && (!x || !y)) return bad(DPIA_ERR_NULL, "x and y must be non-NULL");
  if (n > 0 && (!aligned16(x) || !aligned16(y)))
    return bad(DPIA_ERR_SHAPE, "x and y must be 16-byte aligned");
  if (p.items == 0) {
    clear_detail();
    return DPIA_OK;
  }
  MapArgs a{p.n, p.W, p.items, static_cast<int>(p.L), static_cast<int>(p.C), p.team,
            p.teams_per_wg};
  const int64_t grid = grid_size(p);
  const float* xp = static_cast<const float*>(x);
  float* yp = static_cast<float*>(y);
  if (p.stage) {
    void* args[] = {&alpha, &xp, &yp, &a};
    const void* kern = p.scal_tile == 64   ? reinterpret_cast<const void*>(scal_staged_kernel<64>)
                       : p.scal_tile == 32 ? reinterpret_cast<const void*>(scal_staged_kernel<32>)
                                           : reinterpret_cast<const void*>(scal_staged_kernel<16>);
    hipError_t e = hipLaunchKernel(kern, dim3(grid), dim3(p.wg_threads), args, p.lds_bytes,
                                   reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "dpia_scal launch");
    clear_detail();
    return DPIA_OK;
  }
  hipError_t e = with_order_combine(p.order, DPIA_COMBINE_TREE, [&](auto ord, auto) {
    constexpr int ORDER = decltype(ord)::value;
    return with_nv<4>(p.nv, [&](auto nvc) {
      constexpr int NV = decltype(nvc)::value;
      auto kern = scal_kernel<ORDER, NV>;
      void* args[] = {&alpha, &xp, &yp, &a};
      return hipLaunchKernel(reinterpret_cast<const void*>(kern), dim3(grid),
                             dim3(p.wg_threads), args, 0,
                             reinterpret_cast<hipStream_t>(stream));
    });
  });
  if (e != hipSuccess) return hip_fail(e, "dpia_scal launch");
  clear_detail();
  return DPIA_OK;
}
