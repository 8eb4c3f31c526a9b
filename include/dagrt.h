/*
 * dagrt.h -- C ABI of a runtime DAG scheduler for GPU kernel and copy calls.
 *
 * The scheduler receives GPU computations one call at a time, infers the data
 * dependencies between them from the buffers each call reads and modifies,
 * and executes them asynchronously: independent calls run concurrently on
 * separate HIP streams (space-sharing), events are waited on only where a
 * real read-after-write, write-after-read or write-after-write dependency
 * crosses streams, and host<->device copies overlap with kernels.  A host
 * read of a buffer is the point where the host waits.
 *
 * Paper: A. Parravicini, A. Delamare, M. Arnaboldi, M. D. Santambrogio,
 * "DAG-based Scheduling with Resource Sharing for Multi-task Applications in
 * a Polyglot GPU Runtime" (arXiv:2012.09646).  Each declaration cites the
 * section that defines the operation:
 *   Sec. IV-A  computation DAG, dependency sets, read-only arguments, host
 *              accesses as computational elements
 *   Sec. IV-B  execution context, one event per computation, activity until
 *              the host needs a result
 *   Sec. IV-C  serial/parallel x synchronous/asynchronous policies, stream
 *              manager (FIFO reuse, first child on the parent's stream)
 *   Sec. IV-D  argument annotations (read-only vs modifiable)
 *   Sec. V-D   comparison with graph-based APIs (graph capture here)
 *   Sec. V-E   contention-free (critical-path) bound
 *
 * Conventions
 *   - Every call returns a dag_status; DAG_OK (0) on success, a negative code
 *     otherwise.  dag_last_error(ctx) returns a message for the last failure.
 *   - Argument errors (DAG_E_INVAL, DAG_E_ALIAS, DAG_E_RANGE, ...) leave the
 *     context usable.  A failing HIP call poisons the context: that call
 *     returns DAG_E_HIP and every later call except dag_destroy,
 *     dag_last_error and the introspection calls returns DAG_E_POISONED.
 *   - A context is used by one host thread at a time (not thread-safe).
 *   - Testing hook: if the environment variable DAGRT_FAULT_LAUNCH=N is set
 *     when a context is created, its N-th kernel launch fails with DAG_E_HIP
 *     (without launching anything) and poisons the context.
 *   - Profiling hook: with DAGRT_ROCTX=1 set when a context is created (and
 *     the roctx library of the ROCm profiler present), the host-side
 *     submission of every GPU task is a roctx range named
 *     "dagrt task <id> <kernel|copy|region> stream <s> waits <n>", which
 *     rocprofv3 --marker-trace records beside the kernel and copy traces.
 *   - Pointers are plain host or device addresses; sizes are in bytes unless
 *     stated.  Nothing in this header refers to a framework type.
 *   - Task ids are 1-based positions in program order (every submit, host
 *     access and sync call takes the next id) and are never reused.
 */
#ifndef DAGRT_H
#define DAGRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dag_ctx_s* dag_ctx;
typedef uint32_t dag_buf;  /* buffer handle; 0 is never a valid handle */
typedef uint64_t dag_task; /* task id; 0 = none */
typedef int32_t dag_status;

#define DAG_OK 0
#define DAG_E_INVAL (-1)       /* bad argument (handle, size, mode, params) */
#define DAG_E_ALIAS (-2)       /* registration overlaps a registered buffer */
#define DAG_E_NOMEM (-3)       /* allocation failed */
#define DAG_E_HIP (-4)         /* a HIP call failed; the context is poisoned */
#define DAG_E_POISONED (-5)    /* an earlier HIP failure poisoned the context */
#define DAG_E_BUSY (-6)        /* call not allowed in the current state */
#define DAG_E_UNSUPPORTED (-7) /* operation not available in this mode */
#define DAG_E_NOTFOUND (-8)    /* unknown region key / kernel id */
#define DAG_E_RANGE (-9)       /* size beyond a fixed library limit */

/* Argument access modes (Sec. IV-D): a read-only ("input"/"const") argument
 * or a modifiable one.  An argument without annotation must be passed as
 * DAG_MUTABLE; MUTABLE means read-write.  The same buffer passed twice in one
 * call counts as MUTABLE if either use is. */
#define DAG_CONST 0u
#define DAG_MUTABLE 1u

/* Buffer locations: device memory, or page-locked host memory that the copy
 * engines can read and write asynchronously. */
#define DAG_DEVICE 0u
#define DAG_PINNED_HOST 1u

/* Scheduling policies (Sec. IV-C).  SERIAL_SYNC: every call runs on one
 * stream and the host waits for it before returning (no dependency
 * computation).  PARALLEL_ASYNC: the DAG scheduler. */
#define DAG_SERIAL_SYNC 0u
#define DAG_PARALLEL_ASYNC 1u

/* Dependency kinds on an edge. */
#define DAG_EDGE_RAW 0u
#define DAG_EDGE_WAR 1u
#define DAG_EDGE_WAW 2u

/* Task kinds. */
#define DAG_TASK_KERNEL 0u
#define DAG_TASK_COPY 1u
#define DAG_TASK_HOST_READ 2u
#define DAG_TASK_HOST_WRITE 3u
#define DAG_TASK_SYNC 4u
#define DAG_TASK_REGION 5u  /* one replay of a captured region */
#define DAG_TASK_RELEASE 6u /* buffer release (waits like a host write) */

/* Upper bound of max_streams. */
#define DAG_MAX_STREAMS 64u

typedef struct {
  uint32_t policy;        /* DAG_SERIAL_SYNC or DAG_PARALLEL_ASYNC */
  uint32_t max_streams;   /* stream pool bound, 1..DAG_MAX_STREAMS (0 = 8) */
  uint32_t trace;         /* 1 = timing events for every GPU task, 2 = for
                             kernels and region replays only; built-in
                             kernels are timed by events attached to their
                             dispatch packets, other tasks by markers.
                             3 = markers around every GPU task, each task
                             first held behind a 50 us delay kernel on a
                             side stream so its start marker and its work
                             are queued together (without it a marker on an
                             idle stream also times the host's launch
                             latency); meant for the serial policy */
  uint32_t dry_run;       /* 1 = schedule only: infer edges, streams and
                             waits, make no HIP call and touch no memory */
  int32_t device;         /* HIP device ordinal */
  uint32_t graph_mode;    /* region replays: 0 = hipGraph, 1 = recorded
                             multi-stream replay without dependency work,
                             2 = hipGraph unless the region has host<->device
                             copies (which a graph runs as blit kernels on
                             the CUs rather than on the SDMA engines), then
                             recorded replay */
  uint64_t scratch_bytes; /* per-stream device scratch for reductions and
                             SpMV carries (0 = 4 MiB) */
  uint32_t copy_streams;  /* 0 = host->device and device->host copies each
                             run on one FIFO stream of their own, outside
                             the pool (concurrent copies in one direction
                             share one link, so issue order finishes them
                             soonest); 1 = copies are placed by the stream
                             policy like kernels */
  uint32_t spin_wait;     /* 1 = host waits spin instead of sleeping (asks
                             HIP for hipDeviceScheduleSpin; effective only if
                             no HIP context exists yet in the process) */
  uint32_t copy_lanes;    /* copy_streams = 0: FIFO streams per copy
                             direction, copies rotating over them (0 = 1,
                             at most 4); more than one hides per-copy gaps
                             at the price of later first completions */
  uint32_t own_queues;    /* must be 0: streams come from the runtime's
                             shared pool of GPU_MAX_HW_QUEUES hardware
                             queues (two streams on one queue run in each
                             other's order).  1 (a hardware queue per
                             stream, via CU-masked streams) is refused with
                             DAG_E_UNSUPPORTED: it hung in testing */
  uint32_t copy_engine;   /* host<->device copies: 0 = the SDMA engines
                             (hipMemcpyAsync); 1 = a copy kernel on 128
                             workgroups of the CUs reading or writing the
                             page-locked host memory over PCIe; 2 = host->
                             device by SDMA, device->host by the copy
                             kernel; 3 = the reverse.  With 2 and 3 the two
                             directions never share an SDMA engine.
                             Device-to-device copies always use HIP. */
  uint32_t wait_mode;     /* how a task on one stream waits for a parent on
                             another (the event waits of Sec. IV-B):
                             DAG_WAIT_SIGNALS (0) = a task on the CUs takes
                             the next value of a per-stream counter in device
                             memory, which a one-wave kernel queued behind it
                             raises (lazily: before the next task on that
                             stream when the pool has several streams, else
                             when a task elsewhere first waits for it), and
                             the child's stream is held by a one-wave kernel
                             that polls the counter (about 2 us per edge
                             against about 12 us for a HIP event wait; SDMA
                             copies, hipGraph launches and recorded replays
                             that contain SDMA copies still end with an
                             event; a
                             poll that has not seen its value after 10 s
                             gives up, and the next host wait or sync of the
                             context then fails with DAG_E_HIP and poisons
                             it); DAG_WAIT_EVENTS (1) = a HIP event recorded
                             after every task and hipStreamWaitEvent.  The
                             serial policy uses neither.  The environment
                             variable DAGRT_SIGNAL_TIMEOUT_MS, read at
                             dag_create, lowers the 10 s bound (tests of the
                             failure path). */
} dag_config;

/* dag_config.wait_mode */
#define DAG_WAIT_SIGNALS 0u
#define DAG_WAIT_EVENTS 1u

/* One argument of a call: a buffer and its access mode. */
typedef struct {
  dag_buf buf;
  uint32_t mode; /* DAG_CONST or DAG_MUTABLE */
} dag_arg;

/* One dependency edge, labelled with the buffer that causes it (Sec. IV-A;
 * two calls linked through several buffers give one record per buffer). */
typedef struct {
  dag_task src;
  dag_task dst;
  dag_buf buf;
  uint32_t kind; /* DAG_EDGE_* */
} dag_edge;

typedef struct {
  uint32_t kind;      /* DAG_TASK_* */
  int32_t stream;     /* pool stream index, -1 for host accesses / sync */
  uint32_t vertex;    /* 1 if the task is a DAG vertex (host accesses
                         without a conflict are not) */
  uint32_t active;    /* 1 until a host access retires it (Sec. IV-B) */
  uint32_t nparents;  /* distinct tasks it depends on */
  uint32_t nwaits;    /* event waits placed for it */
  uint32_t kernel_id; /* kernel id for kernel tasks, else 0 */
  uint32_t reserved;
  double t_start_ms;  /* trace mode: start/end on the device, in ms after the
                         last dag_trace_reset (or context creation); -1 when
                         not traced */
  double t_end_ms;
} dag_task_info;

typedef struct {
  uint64_t tasks;        /* ids handed out */
  uint64_t vertices;     /* tasks that are DAG vertices */
  uint64_t edges;        /* edge records (per buffer) */
  uint64_t waits;        /* cross-stream waits placed (event waits and
                            signal polls) */
  uint64_t host_waits;   /* host blocking waits */
  uint32_t streams;      /* streams created so far */
  uint32_t active;       /* currently active tasks */
  double submit_host_us; /* host time spent inside submit calls, excluding
                            the HIP launch/copy calls themselves */
  double launch_host_us; /* host time spent in HIP launch/copy/event calls */
  uint64_t spmv_plans;   /* merge-path SpMV partitions computed; an SpMV
                            whose row-pointer buffer was not written since
                            its partition was computed (same sizes) reuses
                            it */
  uint64_t signals;      /* signal kernels queued (wait mode 0); one raise
                            covers every task queued before it on its
                            stream */
  uint64_t signal_waits; /* of `waits`, those placed as device-side polls of
                            a signal rather than event waits */
} dag_stats;

/* ---- context ------------------------------------------------------------
 * The execution context of Sec. IV-B: it tracks every call, owns the DAG,
 * the stream pool and the events.  cfg may be NULL (defaults).  On success
 * *out owns HIP streams and device scratch (none in dry-run mode). */
dag_status dag_create(const dag_config* cfg, dag_ctx* out);
/* Waits for all outstanding work, then frees everything the context owns
 * (library-allocated buffers included).  ctx may be NULL. */
dag_status dag_destroy(dag_ctx ctx);
/* Message of the last failing call on ctx (ctx NULL: of the calling thread's
 * last failing dag_launch_static call). */
const char* dag_last_error(dag_ctx ctx);
const char* dag_status_string(dag_status st);

/* ---- buffers ------------------------------------------------------------
 * Buffers are the unit of dependency tracking (Sec. IV-A relies on managed
 * objects to exclude aliasing; here a registration that overlaps a
 * registered buffer is rejected with DAG_E_ALIAS).  Any sub-range access
 * counts as an access to the whole buffer. */
/* Register caller-owned memory [ptr, ptr+bytes) (bytes > 0).  The memory
 * must stay valid until dag_buffer_release returns. */
dag_status dag_buffer_register(dag_ctx ctx, void* ptr, size_t bytes, uint32_t loc,
                               dag_buf* out);
/* Allocate and register library-owned memory (hipMalloc / hipHostMalloc,
 * 256-byte aligned, not initialised). */
dag_status dag_buffer_alloc(dag_ctx ctx, size_t bytes, uint32_t loc, dag_buf* out);
/* Wait for every active task that uses the buffer (as a host write would),
 * then drop the handle; library-owned memory is freed.  Recorded regions
 * that use the buffer can no longer be launched (dag_region_launch returns
 * DAG_E_INVAL).  DAG_E_BUSY while a serving shape uses the buffer. */
dag_status dag_buffer_release(dag_ctx ctx, dag_buf buf);
/* Address and size of a registered buffer (the managed object behind a
 * handle, Sec. IV-A), e.g. to hand it to code outside the scheduler. */
dag_status dag_buffer_ptr(dag_ctx ctx, dag_buf buf, void** ptr, size_t* bytes);

/* ---- kernels --------------------------------------------------------------
 * Built-in task kernels (hand-written for gfx950).  Arguments are passed in
 * the order listed; "c" arguments may be DAG_CONST, "m" arguments must be
 * DAG_MUTABLE (DAG_E_INVAL otherwise).  All kernel arguments must be
 * DAG_DEVICE buffers large enough for the sizes in params (checked on the
 * host before launch).  fp32 data, fp64 arithmetic, one rounding to fp32. */
#define DAG_K_VEC_SQUARE 1u      /* x:m                 x_i <- x_i*x_i (fp32) */
#define DAG_K_VEC_SUM_DIFF 2u    /* x:c y:c r:m         r[0] = sum(x_i - y_i) */
#define DAG_K_BS_CALL 3u         /* S:c C:m             Black-Scholes call (spots >= 0; S = 0 prices at 0) */
#define DAG_K_GAUSS_BLUR 4u      /* in:c out:m          Gaussian blur, clamp */
#define DAG_K_SOBEL 5u           /* in:c out:m          Sobel magnitude */
#define DAG_K_MINMAX 6u          /* in:c M:m            M = [max, min] */
#define DAG_K_NORMALISE 7u       /* S:c M:c N:m         (S-min)/(max-min) */
#define DAG_K_UNSHARP_COMBINE 8u /* img B3 B7 B15 N3 N7 N15:c out:m */
#define DAG_K_SPMV 9u            /* row_ptr col val x:c y:m   y = A x (CSR),
                                    merge-path: any row lengths */
#define DAG_K_SPMV_ROWS 10u      /* row_ptr col val x:c y:m   y = A x (CSR),
                                    lanes per row: for short rows only */
#define DAG_K_SUMSQ 11u          /* v:c s:m             s (fp64) = sum v_i^2 */
#define DAG_K_SCALE_L2 12u       /* t:c s:c v:m         v_i = t_i / sqrt(s) */
#define DAG_K_SPIN 13u           /* (any args)          busy-wait, no data */
#define DAG_K_COPY_F32 14u       /* src:c dst:m         dst_i = src_i */
/* ML ensemble (Sec. V-B): X holds n rows of F fp32 category codes 0..V-1,
 * stored feature-major (feature f of row r at X[f*n + r]); P* are n x C
 * row-major fp32 probabilities. */
#define DAG_K_NB_PROBA 15u       /* X lt lp:c P:m       categorical naive Bayes:
                                    P[r] = softmax_c(lp[c] + sum_f lt[c][f][X[f*n+r]]),
                                    lt = log P(x_f = v | c) as C x F x V,
                                    lp = log P(c); codes are truncated and
                                    clamped to [0, V-1]; C*F*V <= 32768 */
#define DAG_K_RIDGE_PROBA 16u    /* X mean scale W b:c P:m  ridge classifier:
                                    P[r] = softmax_c(sum_f (X[f*n+r] - mean_f) /
                                    scale_f * W[c][f] + b[c]), W is C x F;
                                    F*(C+1) <= 8192 */
#define DAG_K_ENSEMBLE 17u       /* Pnb Prr:c avg:m label:m  avg = (Pnb + Prr)/2,
                                    label[r] (int32) = first index of the
                                    largest average (lowest class on ties) */
/* DL (Sec. V-B, a Siamese convolutional network); tensors channel-major
 * (C, H, W) fp32. */
#define DAG_K_CONV3X3_RELU_POOL 18u /* x w b:c y:m   y[o] = maxpool2x2(relu(b[o] +
                                    sum_c corr3x3(x[c], w[o][c]))), zero
                                    padding; x: cin x h x w, w: cout x cin x
                                    3 x 3, y: cout x h/2 x w/2 (h, w even);
                                    launch variant 2 keeps an fp64 copy of w
                                    in the stream's scratch (variant 1 runs
                                    where it does not fit) */
#define DAG_K_DENSE 19u          /* x W b:c y:m         y[j] = sum_i W[i][j] x[i] + b[j],
                                    W: n x m row-major (input-major: the m
                                    weights of input i adjacent), m <= 16
                                    (uses the stream's scratch for
                                    per-workgroup partials; launch variants
                                    3 and 4 add them in a second kernel on
                                    the same stream) */
#define DAG_K_SIAMESE_COMBINE 20u /* e1 e2 w b:c p:m     p[0] = sigmoid(w . [e1; e2]
                                    + b[0]), e1, e2: m <= 32, w: 2m */
#define DAG_K_USER_BASE 1000u    /* ids of dag_kernel_register */

/* Parameter blocks (passed by pointer + size to dag_submit_kernel). */
typedef struct { uint64_t n; } dag_p_n; /* VEC_SQUARE, VEC_SUM_DIFF, MINMAX,
                                           NORMALISE, UNSHARP_COMBINE, SUMSQ,
                                           SCALE_L2, COPY_F32: element count */
typedef struct {
  uint64_t n;      /* options priced */
  double strike;   /* K */
  double rate;     /* r, continuously compounded */
  double vol;      /* sigma */
  double years;    /* T */
} dag_p_bs;
typedef struct {
  uint32_t w, h;  /* image width, height (row-major, w contiguous) */
  uint32_t ksize; /* GAUSS_BLUR: odd kernel size 1..31, sigma = ksize/6 */
  uint32_t reserved;
} dag_p_img;
typedef struct {
  uint32_t nrows, ncols; /* y has nrows, x has ncols entries */
  uint64_t nnz;          /* row_ptr: nrows+1 int32; col: nnz int32; val:
                            nnz fp32.  row_ptr must be non-decreasing from 0
                            to nnz and col < ncols (kernels clamp indices
                            so that malformed input cannot fault) */
} dag_p_csr;
typedef struct { uint64_t ns; } dag_p_spin; /* delay in ns (<= 1 s) */
typedef struct {
  uint64_t n;          /* rows */
  uint32_t features;   /* F >= 1 */
  uint32_t classes;    /* C, 1..16 */
  uint32_t categories; /* V >= 1 (naive Bayes codes; unused by the others) */
  uint32_t reserved;   /* 0 */
} dag_p_ml;            /* NB_PROBA, RIDGE_PROBA, ENSEMBLE */
typedef struct { uint32_t cin, cout, h, w; } dag_p_conv;       /* CONV3X3_RELU_POOL: input h x w */
typedef struct { uint64_t n; uint32_t m, reserved; } dag_p_dense; /* DENSE: n inputs, m outputs */
typedef struct { uint32_t m, reserved; } dag_p_combine;        /* SIAMESE_COMBINE: embedding size */

/* Launch configuration of a built-in kernel (used by the autotuner). */
typedef struct {
  uint32_t block;    /* threads per workgroup (multiple of 64, <= 1024) */
  uint32_t grid_cap; /* max workgroups for grid-stride kernels and for the
                        resident grids (row-window SpMV 0x504/0x508, blur
                        and Sobel 9/11), which otherwise take as many as fit
                        on the GPU at once; 0 = none */
  uint32_t variant;  /* kernel-specific (SpMV items per thread, ...); the
                        library's error message for a refused one lists the
                        kernel's accepted values */
  uint32_t reserved;
} dag_launch;
dag_status dag_kernel_get_launch(dag_ctx ctx, uint32_t kernel_id, dag_launch* out);
/* Validated against the kernel's supported set (DAG_E_INVAL otherwise). */
dag_status dag_kernel_set_launch(dag_ctx ctx, uint32_t kernel_id, const dag_launch* cfg);

/* Autotuning (the paper keeps each kernel's history to guide later
 * scheduling, Sec. IV-A, and tunes launch parameters for serial execution,
 * Sec. V-A): time every candidate configuration of a built-in kernel on the
 * given arguments, alone on the GPU (reps launches back to back between two
 * timing events, three batches, median), install the fastest as the kernel's
 * launch configuration and return its index.  us[i] receives candidate i's
 * time per launch in microseconds (-1 for a candidate the kernel rejects).
 * This is a host synchronisation point: it first waits for and retires all
 * tasks.  The launches overwrite the kernel's outputs, so pass scratch
 * buffers (or data that may be clobbered).  The merge-path SpMV is timed as
 * dag_submit_kernel runs it: with the tile partition kept with its row-pointer
 * buffer (built by two untimed warm-up launches per candidate).  Not
 * available in dry-run mode. */
dag_status dag_tune_kernel(dag_ctx ctx, uint32_t kernel_id, const void* params, size_t params_bytes,
                           const dag_arg* args, uint32_t nargs, const dag_launch* candidates,
                           uint32_t ncand, uint32_t reps, uint32_t* best, double* us);

/* User kernels: fn enqueues its work on the given hipStream_t (passed as
 * void*) using the device pointers of its arguments, in order; it returns
 * 0 on success.  The scheduler treats the call like any other. */
typedef int (*dag_launch_fn)(void* stream, void* const* ptrs, uint32_t nptrs,
                             const void* params, void* user);
dag_status dag_kernel_register(dag_ctx ctx, const char* name, dag_launch_fn fn,
                               void* user, uint32_t* kernel_id);

/* ---- calls ------------------------------------------------------------------
 * Submit one computational element (Sec. IV-A): the scheduler adds it to the
 * DAG with an edge from every active task it conflicts with (RAW, WAR, WAW
 * through the read-only rule of Sec. IV-A), picks a stream (Sec. IV-C),
 * makes that stream wait on the events of parents on other streams that are
 * not already ordered before it, enqueues the work and returns without
 * waiting.  params is copied; nargs <= 16. */
dag_status dag_submit_kernel(dag_ctx ctx, uint32_t kernel_id, const void* params,
                             size_t params_bytes, const dag_arg* args, uint32_t nargs,
                             dag_task* out);
/* Asynchronous copy of bytes from src+src_off to dst+dst_off: src is read
 * (DAG_CONST), dst modified (DAG_MUTABLE).  Direction follows the buffer
 * locations; pinned host memory makes host<->device copies asynchronous. */
dag_status dag_submit_copy(dag_ctx ctx, dag_buf dst, size_t dst_off, dag_buf src,
                           size_t src_off, size_t bytes, dag_task* out);
/* Host read (Sec. IV-A): if an active task writes buf, the host waits for
 * it, and that task and all its ancestors stop being active (Sec. IV-B);
 * otherwise the read happens immediately and is not a DAG vertex.  Then
 * copies bytes at off into host_dst (NULL = wait only).  out (optional)
 * receives the task id. */
dag_status dag_host_read(dag_ctx ctx, dag_buf buf, size_t off, void* host_dst,
                         size_t bytes, dag_task* out);
/* Host write: waits for the active tasks that read or write buf (WAR/WAW),
 * retires them with their ancestors, then copies host_src into the buffer. */
dag_status dag_host_write(dag_ctx ctx, dag_buf buf, size_t off, const void* host_src,
                          size_t bytes, dag_task* out);
/* Wait for every submitted task and retire all of them. */
dag_status dag_sync(dag_ctx ctx);

/* ---- launch without allocating ----------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc.  The built-in
 * kernel kernel_id runs directly on `stream` (a hipStream_t of the current
 * device; NULL = its null stream) with the same parameters, arguments and
 * results as dag_submit_kernel, but outside any context: no dependency
 * tracking, no stream choice, no events, and no allocation on the call path
 * (no hipMalloc, hipFree or other allocating routine).  The scratch that a
 * context allocates per stream (reduction ticket and partials, SpMV tile
 * partition and carries, dense-layer partials) is instead a fixed array of
 * DAG_STATIC_SCRATCH_BYTES in device memory, one per GPU, held until the
 * process ends; its 256-byte header is cleared by a small kernel on `stream`
 * before each launch (no memset node under capture).
 *   ptrs[i]: device-accessible address of argument i (the dag_submit_kernel
 *     argument order of the kernel); bytes[i]: its size in bytes, checked
 *     like a registered buffer's.  cfg: launch configuration (NULL = the
 *     kernel's default; a context's tuned one comes from
 *     dag_kernel_get_launch).  The call returns after enqueueing; the caller
 *     owns every pointer and orders its own accesses on `stream`.
 *   Every call on a GPU shares that GPU's array: calls that can overlap on
 *   the device (other streams, other threads, other processes' contexts
 *   do not share it) race and must be serialised by the caller, e.g. by
 *   issuing them on one stream.
 *   Errors: DAG_E_INVAL for a bad id, parameter block, argument count, NULL
 *   pointer, size or configuration, or a stream of another device;
 *   DAG_E_RANGE when the work needs more scratch than the array holds (e.g.
 *   a merge-path SpMV of more than 149,787 tiles, i.e. nrows + nnz above
 *   ~306 M at 8 items per thread); DAG_E_HIP if a launch fails.  Argument
 *   and range errors enqueue nothing.  dag_last_error(NULL) returns
 *   the calling thread's message for its last failing call. */
#define DAG_STATIC_SCRATCH_BYTES (4u << 20)
dag_status dag_launch_static(uint32_t kernel_id, const void* params, size_t params_bytes,
                             void* const* ptrs, const size_t* bytes, uint32_t nargs,
                             const dag_launch* cfg, void* stream);

/* Batched submission: ops are processed in order exactly as the equivalent
 * sequence of single calls (same ids, edges, streams and waits).  Stops at
 * the first failing op; *done (optional) = number of ops completed. */
typedef struct {
  uint32_t kind;         /* DAG_TASK_KERNEL/COPY/HOST_READ/HOST_WRITE/SYNC */
  uint32_t kernel_id;    /* KERNEL */
  const void* params;    /* KERNEL */
  size_t params_bytes;   /* KERNEL */
  const dag_arg* args;   /* KERNEL */
  uint32_t nargs;        /* KERNEL */
  dag_buf dst;           /* COPY destination; HOST_READ/WRITE buffer */
  dag_buf src;           /* COPY source */
  uint32_t reserved;
  size_t dst_off;        /* COPY / HOST_READ / HOST_WRITE offset in dst */
  size_t src_off;        /* COPY */
  size_t bytes;          /* COPY / HOST_READ / HOST_WRITE */
  void* host;            /* HOST_READ destination / HOST_WRITE source */
} dag_op;
dag_status dag_submit_batch(dag_ctx ctx, const dag_op* ops, uint32_t nops,
                            dag_task* ids, uint32_t* done);

/* ---- recurring DAG shapes (graph capture; Sec. V-D compares the scheduler
 * with graphs built once and replayed) -----------------------------------------
 * dag_region_begin(key) ... kernel/copy submissions ... dag_region_end():
 * the calls run eagerly as usual and are also recorded; region_end builds a
 * replayable graph of them (intra-region dependencies only) under key.
 * Host accesses and sync are not allowed inside a region (DAG_E_BUSY).
 * dag_region_launch(key) replays it as ONE task whose access set is the
 * union of the region's accesses (MUTABLE wins), with its dependencies on
 * earlier tasks inferred like any call.  Re-recording an existing key
 * replaces it; both are refused (DAG_E_BUSY) while a serving shape uses the
 * key, as is dag_region_drop. */
dag_status dag_region_begin(dag_ctx ctx, uint64_t key);
dag_status dag_region_end(dag_ctx ctx);
dag_status dag_region_launch(dag_ctx ctx, uint64_t key, dag_task* out);
/* Recurring shapes replayed automatically.  The program brackets the
 * region's calls with dag_region_run_begin(key) / dag_region_run_end every
 * time it runs them.  The first time (no recording under key) the calls run
 * eagerly and are recorded, as between dag_region_begin/end.  Later, each
 * call is only compared with the recording (kernel id, parameter bytes,
 * launch configuration, argument handles and modes; copy ends, offsets and
 * size) and nothing is enqueued; the submit calls return task id 0.  If every
 * recorded call matched, dag_region_run_end launches the recording as one
 * task (as dag_region_launch; *out = its id, *replayed = 1).  At the first
 * call that differs, or at the end when only a prefix matched, the calls so
 * far are submitted eagerly, the rest of the region runs eagerly, and the new
 * sequence replaces the recording at dag_region_run_end (*out = 0,
 * *replayed = 0); if a serving shape uses the recording, it is kept and the
 * run is only eager.  A recording whose buffer was released is recorded
 * anew.  Host accesses, sync and release are refused inside (DAG_E_BUSY).
 * out and replayed may be NULL. */
dag_status dag_region_run_begin(dag_ctx ctx, uint64_t key);
dag_status dag_region_run_end(dag_ctx ctx, dag_task* out, uint32_t* replayed);
/* Hand-written schedules (the paper compares its scheduler with
 * hand-optimized multi-stream code and CUDA Graphs, Sec. V-D): replace the
 * stream assignment and event waits of a recorded region with the caller's.
 * sched[k] belongs to the region's k-th recorded call: its stream (0..63)
 * and the earlier calls (indices < k) it waits for through events; calls on
 * one stream run in recording order.  The schedule must order every
 * dependency the region's calls have among themselves (checked against the
 * inferred edges: DAG_E_INVAL names the first call that is not ordered after
 * one of its parents).  The region is then rebuilt as the context's graph
 * mode says (hipGraph or multi-stream replay) and launched with
 * dag_region_launch as before.  n must equal the region's call count. */
typedef struct {
  uint32_t stream;
  uint32_t nwaits;
  const uint32_t* waits;
} dag_sched;
dag_status dag_region_set_schedule(dag_ctx ctx, uint64_t key, const dag_sched* sched, uint32_t n);
/* Number of recorded tasks and distinct streams of a region. */
dag_status dag_region_info(dag_ctx ctx, uint64_t key, uint32_t* ntasks, uint32_t* nstreams);
dag_status dag_region_drop(dag_ctx ctx, uint64_t key);

/* ---- introspection ------------------------------------------------------- */
/* The computation DAG (Sec. IV-A: one edge per dependency, labelled with the
 * argument that causes it).  Edge records in order of (dst, src, buf); *n =
 * total count even when it exceeds cap (then only cap records are
 * written). */
dag_status dag_edges(dag_ctx ctx, dag_edge* out, size_t cap, size_t* n);
/* Parents a task waited on through events (ascending ids): the
 * synchronisation events of Sec. IV-B, placed only for parents on other
 * streams (Sec. IV-C). */
dag_status dag_task_waits(dag_ctx ctx, dag_task t, dag_task* out, uint32_t cap, uint32_t* n);
/* A task's kind, stream (Sec. IV-C), activity (Sec. IV-B) and parent and
 * wait counts; trace times (the per-computation timing the contention-free
 * bound of Sec. V-E and the overlap figures of Sec. V-F use) need the task
 * to have completed; this call waits for it. */
dag_status dag_task_get_info(dag_ctx ctx, dag_task t, dag_task_info* out);
/* Counters of the context (Sec. IV-B: tasks, vertices, edges, event waits,
 * host waits, streams of the pool; host time spent scheduling). */
dag_status dag_get_stats(dag_ctx ctx, dag_stats* out);
/* Wait for all work, then restart the trace clock (trace mode only): the
 * time origin of the intervals the overlap figures of Sec. V-F use. */
dag_status dag_trace_reset(dag_ctx ctx);
/* HIP stream of pool stream index i (as void*; the stream manager of
 * Sec. IV-C), e.g. to time on it. */
dag_status dag_stream_handle(dag_ctx ctx, uint32_t i, void** stream);

/* ---- serving loop ------------------------------------------------------------
 * Requests are DAGs of recorded shapes (a region recorded with
 * dag_region_begin/end on template buffers).  They arrive over time (open
 * loop) and are admitted while the sum of the device footprints of the
 * requests in flight stays within budget_bytes: each admitted request gets
 * private copies of its shape's PRIVATE and INIT buffers, sub-allocated from
 * arenas the server keeps resident (device arena for device buffers, pinned
 * host arena for pinned ones and for staging device results), replays the
 * shape's calls in recorded order on one of `lanes` HIP streams (the lane
 * with the fewest requests in flight among those its class may use, see
 * transfer_lanes), and is retired when its completion
 * event fires, which frees its memory for queued requests.  Requests in
 * flight on different lanes run concurrently (space-sharing, Sec. IV-B/C
 * applied across independent requests).  Requests are queued FIFO; up to
 * `bypass` queued requests are examined per admission pass, so small requests
 * can pass a large one that does not fit yet.
 *
 * The server uses the context's regions and kernel launch configurations;
 * while it runs, the context must not record, drop or re-record those
 * regions, and nothing may modify SHARED buffers.  Not thread-safe. */
typedef struct dag_server_s* dag_server;

#define DAG_ROLE_SHARED 0u  /* every request uses the template buffer itself;
                               the region must only read it */
#define DAG_ROLE_PRIVATE 1u /* each request gets its own, uninitialised */
#define DAG_ROLE_INIT 2u    /* each request gets its own, first filled from
                               init_src (same size or larger) */

typedef struct {
  dag_buf buf;      /* a buffer the shape's region uses */
  uint32_t role;    /* DAG_ROLE_* */
  dag_buf init_src; /* DAG_ROLE_INIT: source of the initial contents */
  uint32_t reserved;
} dag_shape_buf;

typedef struct {
  uint64_t budget_bytes;       /* device bytes in flight at most (the
                                  admission budget); <= device_arena_bytes */
  uint64_t device_arena_bytes; /* device memory the server allocates */
  uint64_t host_arena_bytes;   /* pinned host memory the server allocates */
  uint32_t lanes;              /* HIP streams requests are spread over */
  uint32_t bypass;             /* queued requests examined per pass (>= 1) */
  uint32_t copy_lanes;         /* concurrent mode, 0..4: N >= 1 = the
                                  host<->device copies of all requests run on
                                  N FIFO streams per direction, request i
                                  using stream i mod N of each (kernels stay
                                  on the request's lane, with event waits on
                                  the request's own recorded dependencies);
                                  0 = a request runs wholly on its lane */
  uint32_t transfer_lanes;     /* concurrent mode: N >= 1 = requests whose
                                  shape copies between host and device use
                                  lanes 0..N-1 only and all other requests
                                  lanes N..lanes-1 only (lanes > N), so that
                                  requests bound by the host link never hold
                                  up compute-bound ones queued on the same
                                  lane; 0 = any request may use any lane */
} dag_serve_config;

typedef struct {
  uint32_t shape;      /* from dag_serve_add_shape */
  uint32_t reserved;
  uint64_t arrival_ns; /* scheduled arrival after the start of the run;
                          non-decreasing over the request array */
  void* result;        /* host memory for result_bytes, or NULL */
} dag_request;

/* One completed request. */
typedef struct {
  uint64_t id;         /* dag_serve_submit's id: 0, 1, ... in submission
                          order within the session (dag_serve_run: the
                          request's index) */
  uint64_t arrival_ns; /* scheduled (or stamped) arrival, ns after the start
                          of the session */
  uint64_t admit_ns;   /* enqueued on the GPU */
  uint64_t done_ns;    /* completion observed */
  uint32_t shape;
  uint32_t lane;
} dag_serve_done;

typedef struct {
  double p50_ms, p99_ms, mean_ms, max_ms; /* latency = done - arrival
                                             (nearest-rank percentiles) */
  double req_per_s;          /* completed / (last completion - first arrival) */
  double wall_ms;            /* session start to last completion */
  uint64_t peak_device_bytes; /* max footprint in flight */
  uint32_t max_inflight;
  uint32_t max_queued;
  uint64_t completed;        /* requests completed in the session */
} dag_serve_summary;

#define DAG_SERVE_CONCURRENT 0u /* continuous admission, lanes in parallel */
#define DAG_SERVE_SERIAL 1u     /* one request at a time on one lane, the
                                   host waiting after every call (baseline) */
#define DAG_SERVE_NOW UINT64_MAX /* dag_serve_submit: arrival = now */

dag_status dag_serve_create(dag_ctx ctx, const dag_serve_config* cfg, dag_server* out);
/* Waits for the lanes, frees the arenas, unpins the shapes' regions and
 * buffers.  Destroy every server before its context. */
dag_status dag_serve_destroy(dag_server s);
/* Register a shape: the region recorded under region_key, the role of every
 * buffer it uses (all must be listed), and the buffer whose first
 * result_bytes are returned per request (0 = none).  sim_ns is the service
 * time assumed by schedule-only contexts (dry_run), which simulate the loop
 * on a virtual clock instead of running it.  While the shape exists its
 * region cannot be re-recorded or dropped and its buffers (and INIT sources)
 * cannot be released (DAG_E_BUSY).  Not allowed while a session runs. */
dag_status dag_serve_add_shape(dag_server s, uint64_t region_key, const dag_shape_buf* bufs,
                               uint32_t nbufs, dag_buf result_buf, size_t result_bytes,
                               uint64_t sim_ns, uint32_t* shape_id);
/* Per-request footprint of a shape (device arena bytes, pinned arena bytes). */
dag_status dag_serve_shape_info(dag_server s, uint32_t shape, uint64_t* device_bytes,
                                uint64_t* host_bytes);

/* Online serving.  A session starts with dag_serve_start (its clock starts
 * there) and accepts requests until dag_serve_close.  dag_serve_submit and
 * dag_serve_close may be called from any thread, also while another thread
 * is inside dag_serve_poll (they only hand the request over, without a HIP
 * call, and return a status without setting the context's message); every
 * other call on the server or its context must come from the one thread
 * that polls.  dag_serve_poll runs the loop: it moves requests whose arrival
 * time has come into the admission queue, retires requests whose completion
 * event has fired (copying their results to the caller's memory), and admits
 * queued requests while they fit, as described above.  It returns once at
 * least one completion is ready to be reported, once every submitted
 * request of a closed session has been reported, or after wait_us, and
 * writes up to cap completions into done (in completion order; *n = count).
 * *outstanding (optional) = requests submitted and not yet reported.
 * Schedule-only contexts advance a virtual clock; it never passes the
 * arrival of the latest submission until the session is closed, so a
 * producer that submits in arrival order gets exactly the admissions and
 * completions of a run that knew every request from the start. */
dag_status dag_serve_start(dag_server s, uint32_t mode);
/* arrival_ns: scheduled arrival in ns after dag_serve_start, non-decreasing
 * over the submissions of a session (DAG_E_INVAL otherwise), or
 * DAG_SERVE_NOW (not in schedule-only contexts).  result: host memory for
 * the shape's result_bytes (or NULL), written before the completion is
 * reported.  *id (optional) = the request's id.  DAG_E_BUSY: no session, or
 * the session is closed. */
dag_status dag_serve_submit(dag_server s, uint32_t shape, uint64_t arrival_ns, void* result,
                            uint64_t* id);
/* No more submissions in this session. */
dag_status dag_serve_close(dag_server s);
dag_status dag_serve_poll(dag_server s, uint64_t wait_us, dag_serve_done* done, uint32_t cap,
                          uint32_t* n, uint64_t* outstanding);
/* Latency percentiles, throughput and occupancy over the requests the
 * session has completed so far. */
dag_status dag_serve_stats(dag_server s, dag_serve_summary* out);
/* A whole arrival trace as one session: starts it, submits every request
 * with its scheduled arrival, closes it and polls until every request has
 * completed (blocks).  done[i] receives request i's record; stats may be
 * NULL. */
dag_status dag_serve_run(dag_server s, const dag_request* reqs, uint32_t n, uint32_t mode,
                         dag_serve_done* done, dag_serve_summary* stats);

#ifdef __cplusplus
}
#endif
#endif /* DAGRT_H */
