// Built-in task kernels: host-side descriptors (argument checks + launch).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace dagrt {

struct LaunchCfg {
  uint32_t block;
  uint32_t grid_cap;
  uint32_t variant;
};

struct KernelDesc {
  const char* name;
  uint32_t nargs;       // exact argument count (0 = any number)
  uint32_t write_mask;  // bit i: argument i is modified by the kernel
  size_t params_bytes;
  LaunchCfg def;
  // nullptr when the call is valid; otherwise a static message.
  const char* (*validate)(const void* params, const size_t* sizes, uint32_t nargs,
                          const LaunchCfg& cfg, size_t scratch_bytes);
  hipError_t (*launch)(hipStream_t s, void* const* ptrs, const void* params,
                       const LaunchCfg& cfg, void* scratch, size_t scratch_bytes);
  const char* (*check_cfg)(const LaunchCfg& cfg);
};

// Built-in kernel ids are 1..kNumBuiltin-1; nullptr for unknown ids.
constexpr uint32_t kNumBuiltin = 21;
const KernelDesc* builtin_kernel(uint32_t id);

// Timing events for the next built-in launch call (both null = none): the
// first kernel dispatch takes `start`, every dispatch `stop`.
void set_launch_events(hipEvent_t start, hipEvent_t stop);

// Merge-path SpMV (kernel 9) in two parts, for callers that keep a matrix's
// tile partition while its row pointers stay unchanged: the partition needs
// spmv_plan_ints() ints of device memory and depends only on row_ptr, nrows,
// nnz and the launch variant; spmv_planned() runs the SpMV proper with it.
// Arguments as for the kernel's launch; the call must have been validated.
uint64_t spmv_plan_ints(const void* params, const LaunchCfg& cfg);
hipError_t spmv_plan(hipStream_t s, const int* row_ptr, const void* params, const LaunchCfg& cfg, int* coord);
hipError_t spmv_planned(hipStream_t s, void* const* ptrs, const void* params, const LaunchCfg& cfg,
                        const int* coord, void* scratch);

// Host<->device copy of `bytes` by a copy kernel on 128 workgroups (both
// pointers device-accessible; pinned host memory is).
hipError_t copy_by_kernel(hipStream_t s, void* dst, const void* src, size_t bytes);

// A kernel whose workgroups write back the dirty lines of every XCD's L2
// (system-scope release on each XCD): the final node of region graphs.
hipError_t release_l2(hipStream_t s);

// Completion signals between streams: one 64-bit word per stream, kSignalStride
// words apart.  signal_raise queues a one-wave kernel that stores value into
// word once the work queued before it on s has finished; signal_wait queues a
// one-wave kernel that returns once every listed word has reached its value
// (or, after max_ticks of the device's constant-rate clock, stores 1 into
// *timed_out, host memory, and returns).
constexpr uint32_t kMaxSignalWaits = 8;
constexpr uint32_t kSignalStride = 16;  // words: one 128-byte line per stream
struct SignalWaits {
  const uint64_t* words;
  uint32_t* timed_out;
  uint64_t max_ticks;
  uint32_t n;
  uint32_t slot[kMaxSignalWaits];
  uint64_t value[kMaxSignalWaits];
};
hipError_t signal_raise(hipStream_t s, uint64_t* word, uint64_t value);
hipError_t signal_wait(hipStream_t s, const SignalWaits& w);
uint64_t wall_clock_ticks_per_ms();

// Message of the calling thread's last failing dag_launch_static call.
const char* static_launch_error();

// Device wall-clock frequency in kHz (for the spin kernel); set once.
void set_wall_clock_khz(uint64_t khz);

// Scratch layout shared by the reduction kernels: a 32-bit ticket counter at
// offset 0 (zero between launches: the last workgroup resets it) and
// per-workgroup partials from offset 256.
constexpr size_t kScratchPartialsOffset = 256;

}  // namespace dagrt
