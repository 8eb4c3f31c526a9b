// Internal: the execution context shared by the C-ABI translation units
// (dagrt.cpp: scheduler and executor; serve.cpp: serving loop).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dagrt.h"
#include "kernels.hpp"
#include "tracker.hpp"

namespace dagrt {

using Clock = std::chrono::steady_clock;

inline double us_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
}

struct Buffer {
  void* ptr = nullptr;
  size_t bytes = 0;
  uint32_t loc = 0;
  bool owned = false;
  bool live = false;
  // Tile partition of a CSR matrix whose row pointers are this buffer (the
  // merge-path SpMV's first step), kept until the buffer is next written.
  int* plan = nullptr;
  uint64_t plan_cap = 0;  // ints allocated
  bool plan_valid = false;
  bool plan_ready = false;  // plan_ev known to have completed
  uint32_t plan_variant = 0;
  uint64_t plan_nrows = 0, plan_nnz = 0;
  int32_t plan_stream = -1;  // pool stream the partition ran on
  hipEvent_t plan_ev = nullptr;
  uint32_t pins = 0;  // serving shapes that use it (release is refused while > 0)
};

struct UserKernel {
  std::string name;
  dag_launch_fn fn;
  void* user;
};

// One recorded call of a region.
struct RegionTask {
  uint32_t kind = 0;  // TK_KERNEL or TK_COPY
  uint32_t kernel_id = 0;
  std::vector<char> params;
  std::vector<void*> ptrs;
  LaunchCfg cfg{};
  void* cdst = nullptr;
  const void* csrc = nullptr;
  size_t cbytes = 0;
  hipMemcpyKind ckind = hipMemcpyDefault;
  uint64_t id = 0;         // task id of the eager run
  std::vector<dag_arg> args;  // kernel arguments as submitted (handles, modes)
  dag_buf cdst_h = 0, csrc_h = 0;  // copy ends as submitted
  size_t cdst_off = 0, csrc_off = 0;
  int32_t rstream = 0;     // region-local stream
  std::vector<uint32_t> rwaits;    // region-local task indices waited on
  std::vector<uint32_t> rparents;  // every intra-region parent (region-local indices)
  bool waited_on = false;
};

struct Region {
  std::vector<RegionTask> tasks;
  std::vector<Access> accs;  // union of accesses, MUTABLE wins
  uint32_t nstreams = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* scratch = nullptr;  // nstreams * scratch_bytes (graph mode)
  std::vector<hipEvent_t> evs;  // replay-mode events (per task)
  bool dead = false;  // a buffer it uses was released: it can no longer be launched
  uint32_t pins = 0;  // serving shapes built on it (re-recording and dropping are refused while > 0)
};

constexpr uint32_t kMaxArgs = 16;
// Wait mode 0: signal words (streams with a larger index end their tasks
// with events) and the longest a device-side wait polls before giving up.
constexpr uint32_t kSignalSlots = 128;
constexpr uint32_t kAuxSlotBase = 96;  // words of the capture / replay streams (pool streams and lanes stay below)
constexpr uint64_t kSignalTimeoutMs = 10000;
constexpr size_t kStagingBytes = 64 << 10;

}  // namespace dagrt

struct dag_ctx_s {
  dag_config cfg{};
  bool serial = false;
  bool dry = false;
  bool poisoned = false;
  std::string err;
  dagrt::Tracker tr;
  std::vector<dagrt::Buffer> bufs;        // slot = handle - 1
  std::vector<void*> dead_plans;          // SpMV partitions replaced while possibly in use
  std::map<uintptr_t, uint32_t> ranges;   // live buffers: base -> slot
  uintptr_t fake_next = uintptr_t(1) << 44;
  std::vector<hipStream_t> streams;
  std::vector<void*> scratch;             // per pool stream
  hipStream_t io = nullptr;
  void* staging = nullptr;                // pinned, for small host reads
  hipEvent_t read_ev = nullptr;
  std::vector<hipEvent_t> ev;             // per task (GPU tasks), completion; ev[id - ev_base]
  uint64_t ev_base = 0;                   // first task id of ev (records before it were compacted)
  // Wait mode 0: completion signals between streams (kernels.hpp).  sig_dev
  // holds one word per stream.  A task that ends with a signal takes the
  // next value of its stream, sig_next[s]; tsig[id - ev_base] keeps it (0:
  // the task has an event instead).  The value is raised on the device
  // lazily: sig_raised[s] is the last value queued for raising on stream s.
  // mark_ev[s] is recorded on stream s when the host must wait for a
  // signalled task of it.
  bool signals = false;
  uint64_t* sig_dev = nullptr;
  uint32_t* sig_timed_out = nullptr;      // pinned host word raised by a wait that gave up
  std::vector<uint64_t> sig_next, sig_raised;
  std::vector<std::vector<uint32_t>> tail_writes;  // per stream: buffers its last signalled task wrote
  std::vector<std::pair<uint32_t, uint64_t>> tmp_sig;  // replay: (word, value) raised after each waited-on task
  std::vector<uint64_t> tsig;
  std::vector<hipEvent_t> mark_ev;
  uint64_t n_signals = 0, n_signal_waits = 0;
  uint64_t sig_timeout_ms = dagrt::kSignalTimeoutMs;  // DAGRT_SIGNAL_TIMEOUT_MS overrides (tests)
  std::vector<hipEvent_t> ev0;            // per task, start (trace mode)
  std::vector<hipEvent_t> ev1;            // per task, kernel end (trace mode 2, built-in kernels)
  std::vector<hipEvent_t> free_ev;
  hipEvent_t trace_ref = nullptr;
  std::vector<uint64_t> tmp_wait, tmp_retired;
  std::vector<dagrt::Access> tmp_acc;
  std::vector<dagrt::UserKernel> user_kernels;
  dagrt::LaunchCfg launch_cfg[dagrt::kNumBuiltin]{};  // indexed by built-in kernel id
  // regions
  std::unordered_map<uint64_t, std::unique_ptr<dagrt::Region>> regions;
  bool recording = false;
  uint64_t rec_key = 0;
  // dag_region_run_*: calls compared with the recording of match_key instead
  // of being run; match_pos calls have matched so far
  bool matching = false;
  uint64_t match_key = 0;
  size_t match_pos = 0;
  // the calls diverged from a recording that a serving shape uses: the rest
  // of this run is eager and nothing is recorded
  bool eager_run = false;
  bool in_region() const { return recording || matching || eager_run; }
  std::unique_ptr<dagrt::Region> rec;
  std::vector<hipStream_t> aux;           // capture / replay streams
  std::vector<void*> aux_scratch;
  // failure injection (tests): the fault_at-th kernel launch reports an error
  // instead of launching; 0 = off
  uint64_t fault_at = 0, n_launches = 0;
  // DAGRT_ROCTX=1: each GPU task's submission is a roctx range (profiler
  // marker trace); the functions come from the roctx library, loaded at
  // context creation
  int (*roctx_push)(const char*) = nullptr;
  int (*roctx_pop)() = nullptr;
  hipEvent_t gate_ev = nullptr;  // trace mode 3
  // stats
  uint64_t n_waits = 0, n_host_waits = 0, n_plans = 0;
  double submit_us = 0.0, launch_us = 0.0;

  dag_ctx_s(uint32_t ms, uint32_t lanes) : tr(ms, lanes) {}
};

namespace dagrt {
// Error helpers (dagrt.cpp).
dag_status fail(dag_ctx c, dag_status st, const char* fmt, ...);
// An asynchronous copy as the context is configured to run it: host<->device
// copies by the SDMA engines (hipMemcpyAsync) or, with cfg.copy_engine = 1,
// by a copy kernel on the CUs; device-to-device copies always by HIP.
hipError_t copy_async(dag_ctx c, void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
// A new non-blocking stream of the context, default priority.
hipError_t new_stream(dag_ctx c, hipStream_t* st);
dag_status hip_fail(dag_ctx c, hipError_t e, const char* what);
Buffer* get_buf(dag_ctx c, dag_buf h);
hipError_t launch_region_task(dag_ctx c, const RegionTask& t, hipStream_t s, void* scratch);
}  // namespace dagrt

#define HIP_TRY(c, call)                                            \
  do {                                                              \
    hipError_t e_ = (call);                                         \
    if (e_ != hipSuccess) return ::dagrt::hip_fail((c), e_, #call); \
  } while (0)

#define CHECK_CTX(c)                                                                                     \
  do {                                                                                                   \
    if (!(c)) return DAG_E_INVAL;                                                                        \
    if ((c)->poisoned) return ::dagrt::fail((c), DAG_E_POISONED, "context poisoned: %s", (c)->err.c_str()); \
  } while (0)
