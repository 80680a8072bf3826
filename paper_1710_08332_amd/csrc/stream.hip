// Read-bandwidth ceiling: the plainest kernel that reads a buffer once from
// HBM.  It is the yardstick the reductions' bandwidth is compared with, not
// an operation of the method.  Every 32-bit word is XORed into its
// work-group's value, so that no load is dead and the result can be checked
// against the host.  Each work-group stores its value with one plain store:
// atomics on one shared word serialise (about 9 ns each measured, which at
// thousands of wavefronts costs as much as the stream itself).
#include "device.h"
#include "host.h"

namespace dpia {

constexpr int kStreamThreads = 256;
constexpr int kStreamBatch = 8;   // 16-byte loads in flight per thread

// Work-group b, thread t reads the 16-byte units
// (b + j * gridDim.x) * 256 * U + u * 256 + t for u < U: each load
// instruction of a wavefront covers 1 KiB in one piece.
template <int U>
__global__ void __launch_bounds__(kStreamThreads) read_stream_kernel(const u32x4* x,
                                                                     int64_t nvec,
                                                                     unsigned* sink) {
  constexpr int64_t kStep = static_cast<int64_t>(kStreamThreads) * U;
  const int64_t stride = kStep * gridDim.x;
  u32x4 acc = {0u, 0u, 0u, 0u};
  int64_t base = static_cast<int64_t>(blockIdx.x) * kStep + threadIdx.x;
  for (; base + (U - 1) * kStreamThreads < nvec; base += stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(x + base + u * kStreamThreads);
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u];
  }
  // The step at `base` is partial; the next one (base + stride, with
  // stride >= U * 256) starts past the end.
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = base + u * kStreamThreads;
    if (i < nvec) acc ^= x[i];
  }
  unsigned w = acc[0] ^ acc[1] ^ acc[2] ^ acc[3];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) w ^= __shfl_xor(w, off, kWave);
  __shared__ unsigned wave_value[kStreamThreads / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) wave_value[threadIdx.x / kWave] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned r = 0;
#pragma unroll
    for (int i = 0; i < kStreamThreads / kWave; ++i) r ^= wave_value[i];
    sink[blockIdx.x] = r;
  }
}

}  // namespace dpia

using namespace dpia;

extern "C" dpia_status dpia_read_stream(const void* x, int64_t bytes, int32_t grid,
                                        uint32_t* sink, dpia_stream_t stream) {
  if (bytes < 0 || bytes % 16 != 0)
    return bad(DPIA_ERR_SHAPE, "bytes must be a non-negative multiple of 16");
  if (grid < 1 || grid > 65536) return bad(DPIA_ERR_SHAPE, "grid must be in [1, 65536]");
  if (!sink || (bytes > 0 && !x)) return bad(DPIA_ERR_NULL, "x and sink must be non-NULL");
  if (bytes > 0 && !aligned16(x)) return bad(DPIA_ERR_SHAPE, "x must be 16-byte aligned");
  if (bytes == 0) {
    clear_detail();
    return DPIA_OK;
  }
  const u32x4* xp = static_cast<const u32x4*>(x);
  int64_t nvec = bytes / 16;
  unsigned* sp = sink;
  void* args[] = {&xp, &nvec, &sp};
  hipError_t e = hipLaunchKernel(reinterpret_cast<const void*>(read_stream_kernel<kStreamBatch>),
                                 dim3(static_cast<unsigned>(grid)), dim3(kStreamThreads), args, 0,
                                 reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "dpia_read_stream launch");
  clear_detail();
  return DPIA_OK;
}
