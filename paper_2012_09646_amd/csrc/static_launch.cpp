// dag_launch_static: one built-in task kernel launched directly on a caller's
// stream, with no device allocation anywhere on the call path.  The kernel's
// scratch (reduction ticket and partials, SpMV tile partition and carries,
// dense-layer partials) is the fixed device array below instead of the
// per-stream scratch that a context allocates.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>

#include "../../include/dagrt.h"
#include "kernels.hpp"

namespace dagrt {
namespace {

constexpr size_t kStaticScratchBytes = DAG_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr uint32_t kMaxStaticArgs = 16;

// One copy per GPU, alive until the process ends.  In host code this name
// stands for the variable, not for a device address: kernels get the address
// that hipGetSymbolAddress returned for the current device (g_scratch_ptr).
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

void* g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

thread_local char t_err[512];

dag_status static_fail(dag_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_err, sizeof(t_err), fmt, ap);
  va_end(ap);
  return st;
}

// Zero the ticket counter and header in front of the partials: every
// reduction-style kernel expects it at zero when it starts (a completed
// launch leaves it so, but the array keeps whatever the last call left).
__global__ __launch_bounds__(64) void k_zero_header(uint32_t* p) {
  p[threadIdx.x] = 0u;  // 64 words = the 256-byte header
}
static_assert(kScratchPartialsOffset == 64 * sizeof(uint32_t), "header is 64 words");

// Device address of this GPU's array, looked up once per device with that
// device current.
dag_status scratch_ptr(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return static_fail(DAG_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                         hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DAG_OK;
}

}  // namespace

const char* static_launch_error() { return t_err; }

}  // namespace dagrt

using namespace dagrt;

extern "C" dag_status dag_launch_static(uint32_t kernel_id, const void* params, size_t params_bytes,
                                        void* const* ptrs, const size_t* bytes, uint32_t nargs,
                                        const dag_launch* cfg, void* stream) {
  t_err[0] = '\0';
  const KernelDesc* kd = builtin_kernel(kernel_id);
  if (!kd) return static_fail(DAG_E_INVAL, "unknown built-in kernel id %u", kernel_id);
  if (params_bytes != kd->params_bytes)
    return static_fail(DAG_E_INVAL, "%s: parameter block must be %zu bytes", kd->name, kd->params_bytes);
  if (kd->params_bytes && !params) return static_fail(DAG_E_INVAL, "%s: params is NULL", kd->name);
  if (kd->nargs && nargs != kd->nargs)
    return static_fail(DAG_E_INVAL, "%s takes %u arguments", kd->name, kd->nargs);
  if (nargs > kMaxStaticArgs) return static_fail(DAG_E_INVAL, "at most %u arguments", kMaxStaticArgs);
  if (nargs && (!ptrs || !bytes)) return static_fail(DAG_E_INVAL, "ptrs or bytes is NULL");
  for (uint32_t i = 0; i < nargs; ++i)
    if (!ptrs[i]) return static_fail(DAG_E_INVAL, "argument %u is NULL", i);
  LaunchCfg lc = kd->def;
  if (cfg) lc = LaunchCfg{cfg->block, cfg->grid_cap, cfg->variant};
  if (const char* msg = kd->check_cfg(lc)) return static_fail(DAG_E_INVAL, "%s: %s", kd->name, msg);
  // Argument errors first (as if scratch were unlimited), then the limit.
  if (const char* msg = kd->validate(params, bytes, nargs, lc, SIZE_MAX))
    return static_fail(DAG_E_INVAL, "%s: %s", kd->name, msg);
  if (const char* msg = kd->validate(params, bytes, nargs, lc, kStaticScratchBytes))
    return static_fail(DAG_E_RANGE, "%s: %s (the static scratch holds %zu bytes)", kd->name, msg,
                       kStaticScratchBytes);

  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return static_fail(DAG_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return static_fail(DAG_E_UNSUPPORTED, "device %d out of range", dev);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (s) {
    hipDevice_t sdev = -1;
    e = hipStreamGetDevice(s, &sdev);
    if (e != hipSuccess) return static_fail(DAG_E_HIP, "hipStreamGetDevice failed: %s", hipGetErrorString(e));
    if (sdev != dev)
      return static_fail(DAG_E_INVAL, "the stream belongs to device %d, the current device is %d", sdev, dev);
  }
  void* scr = nullptr;
  if (dag_status st = scratch_ptr(dev, &scr)) return st;

  hipLaunchKernelGGL(k_zero_header, dim3(1), dim3(64), 0, s, static_cast<uint32_t*>(scr));
  e = hipGetLastError();
  if (e == hipSuccess) e = kd->launch(s, ptrs, params, lc, scr, kStaticScratchBytes);
  if (e != hipSuccess) return static_fail(DAG_E_HIP, "%s launch failed: %s", kd->name, hipGetErrorString(e));
  return DAG_OK;
}
