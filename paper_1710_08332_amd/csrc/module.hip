// Loading and launching generated kernels (code objects built by hipcc from
// the HIP source that the expression generator emits).  Host code only.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "host.h"
#include "plan.h"

struct dpia_module {
  hipModule_t mod = nullptr;
  std::mutex mu;
  std::map<std::string, hipFunction_t> fns;
};

using namespace dpia;

extern "C" dpia_status dpia_module_load(const char* path, dpia_module** out) {
  if (!path || !out) return bad(DPIA_ERR_NULL, "path and out must be non-NULL");
  hipModule_t m = nullptr;
  hipError_t e = hipModuleLoad(&m, path);
  if (e != hipSuccess) return hip_fail(e, std::string("hipModuleLoad ") + path);
  dpia_module* d = new (std::nothrow) dpia_module;
  if (!d) {
    (void)hipModuleUnload(m);
    return bad(DPIA_ERR_HIP, "out of host memory");
  }
  d->mod = m;
  *out = d;
  clear_detail();
  return DPIA_OK;
}

extern "C" dpia_status dpia_module_launch(dpia_module* m, const char* kernel, uint32_t grid,
                                          uint32_t block, void* const* args, int32_t nargs,
                                          dpia_stream_t stream) {
  if (!m || !kernel || (nargs > 0 && !args))
    return bad(DPIA_ERR_NULL, "module, kernel and args must be non-NULL");
  if (grid < 1 || block < 1 || block > 1024)
    return bad(DPIA_ERR_SHAPE, "grid must be >= 1 and block in [1, 1024]");
  constexpr int kMaxArgs = 64;
  if (nargs < 0 || nargs > kMaxArgs) return bad(DPIA_ERR_SHAPE, "at most 64 kernel arguments");
  for (int i = 0; i < nargs; ++i)
    if (!args[i]) return bad(DPIA_ERR_NULL, "kernel argument " + std::to_string(i) + " is NULL");
  hipFunction_t f = nullptr;
  {
    std::lock_guard<std::mutex> lock(m->mu);
    auto it = m->fns.find(kernel);
    if (it == m->fns.end()) {
      hipError_t e = hipModuleGetFunction(&f, m->mod, kernel);
      if (e != hipSuccess) return hip_fail(e, std::string("kernel ") + kernel);
      m->fns.emplace(kernel, f);
    } else {
      f = it->second;
    }
  }
  // every generated kernel takes device pointers only
  void* vals[kMaxArgs];
  void* params[kMaxArgs];
  for (int i = 0; i < nargs; ++i) {
    vals[i] = args[i];
    params[i] = &vals[i];
  }
  hipError_t e = hipModuleLaunchKernel(f, grid, 1, 1, block, 1, 1, 0,
                                       reinterpret_cast<hipStream_t>(stream), params, nullptr);
  if (e != hipSuccess) return hip_fail(e, std::string("launch of ") + kernel);
  clear_detail();
  return DPIA_OK;
}

extern "C" dpia_status dpia_module_unload(dpia_module* m) {
  if (!m) return DPIA_OK;
  hipError_t e = hipModuleUnload(m->mod);
  delete m;
  if (e != hipSuccess) return hip_fail(e, "hipModuleUnload");
  clear_detail();
  return DPIA_OK;
}
