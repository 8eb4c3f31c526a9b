// Serving loop: request DAGs of uneven sizes arrive over time (open loop)
// and are admitted while their device footprint fits a memory budget; each
// admitted request gets private buffers sub-allocated from resident arenas,
// replays its shape's recorded calls on one of several lanes (HIP streams),
// and is retired when its completion event fires, which frees its memory for
// the requests waiting behind it.  Requests in flight on different lanes
// space-share the GPU.  The paper schedules one application's computations
// (Sec. IV); serving applies the same space-sharing across independent
// requests, each of which is a DAG recorded like a recurring region.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "context.hpp"

namespace dagrt {
namespace {

constexpr uint64_t kAlign = 256;
inline uint64_t align_up(uint64_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit sub-allocator over [0, size) with coalescing free ranges.
class Arena {
 public:
  explicit Arena(uint64_t size = 0) { reset(size); }
  void reset(uint64_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(uint64_t bytes, uint64_t* off) {
    bytes = align_up(std::max<uint64_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const uint64_t o = it->first, rem = it->second - bytes;
      free_.erase(it);
      if (rem) free_[o + bytes] = rem;
      *off = o;
      return true;
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = align_up(std::max<uint64_t>(bytes, 1));
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<uint64_t, uint64_t> free_;
};

struct ShapeBuf {
  uint32_t role;
  void* tmpl;        // template buffer the region was recorded on
  size_t bytes;
  uint32_t loc;
  void* init_src;    // DAG_ROLE_INIT
  uint32_t init_loc;
  uint64_t off;      // offset inside the request's block (private roles)
};

struct PtrRef {
  int32_t buf;   // shape buffer index, -1 = not remapped
  uint64_t off;  // offset inside that buffer
  void* raw;     // pointer as recorded
};

struct ShapeTask {
  const RegionTask* t;
  std::vector<PtrRef> refs;  // kernel arguments
  PtrRef cdst, csrc;         // copy ends
};

// Where a request's call runs when copies have lanes of their own.
enum : uint8_t { kOnLane = 0, kOnH2D = 1, kOnD2H = 2 };

struct Shape {
  Region* region;
  std::vector<ShapeBuf> bufs;
  std::vector<ShapeTask> tasks;
  // copy-lane plan: per call its stream class, the calls it waits for on
  // other streams (newest recorded parent per stream), whether a later call
  // or the request's final join waits for it, and the last call per class
  std::vector<uint8_t> cls;
  std::vector<std::vector<uint32_t>> waits;
  std::vector<uint8_t> needs_ev;
  int32_t last_of[3] = {-1, -1, -1};
  bool has_init = false;
  bool host_io = false;  // the recorded calls copy between host and device
  int32_t result_buf;
  size_t result_bytes;
  uint64_t dev_bytes = 0, host_bytes = 0;  // per-request block sizes
  uint64_t result_off = 0;                 // in the host block (device results)
  uint64_t sim_ns;
  std::vector<uint32_t> pinned;  // buffer slots pinned while the shape exists
};

struct Flight {
  uint64_t req;       // request id
  uint32_t lane;
  hipEvent_t ev;
  uint64_t dev_off, host_off;
  uint64_t sim_done;  // schedule-only contexts
  std::vector<hipEvent_t> evs;  // copy-lane mode: events of the request's calls
};

// A submitted request (the caller's view: shape, arrival, result memory).
struct Req {
  uint64_t id;
  uint32_t shape;
  uint64_t arrival_ns;
  void* result;
};

}  // namespace
}  // namespace dagrt

using namespace dagrt;

struct dag_server_s {
  dag_ctx ctx;
  dag_serve_config cfg;
  void* dev_base = nullptr;
  void* host_base = nullptr;
  Arena dev, host;
  std::vector<Shape> shapes;
  std::vector<hipStream_t> lanes;
  std::vector<void*> lane_scratch;
  std::vector<hipStream_t> copy_st[3];  // [kOnH2D], [kOnD2H]: copy lanes per direction
  uint64_t launched = 0;                // requests launched (rotates the copy lanes)
  std::vector<hipEvent_t> free_ev;

  // ---- session (dag_serve_start .. end of the last request) ----
  bool started = false;
  bool serial = false;
  Clock::time_point t0;
  // shared with submitting threads (guarded by mu)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req> incoming;  // submitted, not yet taken by the polling thread
  uint64_t next_id = 0;
  uint64_t horizon = 0;      // arrival of the last submission (schedule-only clock bound)
  bool closed = false;
  // owned by the polling thread
  std::deque<Req> pending;   // submitted, arrival still in the future
  std::deque<Req> queue;     // arrived, waiting for admission (FIFO, bounded bypass)
  std::vector<std::deque<Flight>> flights;  // per lane, in launch order
  std::vector<uint64_t> lane_free;          // schedule-only: virtual time a lane drains
  std::unordered_map<uint64_t, Req> live;   // admitted requests by id
  std::unordered_map<uint64_t, dag_serve_done> admitted;  // admission records by id
  std::deque<dag_serve_done> unreported;    // completions not yet returned by poll
  std::vector<double> lat_ms;               // latencies of completed requests
  uint64_t used = 0, peak = 0, vclock = 0, taken = 0, ndone = 0;
  uint64_t first_arrival = UINT64_MAX, last_done = 0;
  uint32_t inflight = 0, max_inflight = 0, max_queued = 0;
};

namespace {

dag_status ev_get(dag_server s, hipEvent_t* e) {
  if (!s->free_ev.empty()) {
    *e = s->free_ev.back();
    s->free_ev.pop_back();
    return DAG_OK;
  }
  HIP_TRY(s->ctx, hipEventCreateWithFlags(e, hipEventDisableTiming));
  return DAG_OK;
}

void* resolve(const dag_server_s* s, const Shape& sh, const PtrRef& r, uint64_t dev_off, uint64_t host_off) {
  if (r.buf < 0) return r.raw;
  const ShapeBuf& b = sh.bufs[r.buf];
  if (b.role == DAG_ROLE_SHARED) return static_cast<char*>(b.tmpl) + r.off;
  char* base = b.loc == DAG_PINNED_HOST ? static_cast<char*>(s->host_base) + host_off
                                        : static_cast<char*>(s->dev_base) + dev_off;
  return base + b.off + r.off;
}

hipMemcpyKind kind_of(uint32_t dst_loc, uint32_t src_loc) {
  if (src_loc == DAG_PINNED_HOST)
    return dst_loc == DAG_PINNED_HOST ? hipMemcpyHostToHost : hipMemcpyHostToDevice;
  return dst_loc == DAG_PINNED_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
}

hipError_t launch_task(dag_server s, const Shape& sh, const ShapeTask& t, uint64_t dev_off, uint64_t host_off,
                       hipStream_t st, void* scratch) {
  if (t.t->kind == TK_COPY)
    return copy_async(s->ctx, resolve(s, sh, t.cdst, dev_off, host_off), resolve(s, sh, t.csrc, dev_off, host_off),
                      t.t->cbytes, t.t->ckind, st);
  void* ptrs[kMaxArgs];
  for (size_t i = 0; i < t.refs.size(); ++i) ptrs[i] = resolve(s, sh, t.refs[i], dev_off, host_off);
  const KernelDesc* kd = builtin_kernel(t.t->kernel_id);
  return kd->launch(st, ptrs, t.t->params.data(), t.t->cfg, scratch, s->ctx->cfg.scratch_bytes);
}

// Enqueue one request: its INIT copies and kernels on lane stream `st`, its
// host<->device copies on the server's copy streams when those exist (not in
// serial mode), with event waits for the request's own recorded
// dependencies; the lane then joins the copy streams, so an event recorded on
// the lane afterwards marks the whole request.  serial = wait after every
// call.  Events used are appended to *evs (recycled when the request retires).
dag_status launch_request(dag_server s, const Shape& sh, uint64_t dev_off, uint64_t host_off, hipStream_t st,
                          void* scratch, bool serial, std::vector<hipEvent_t>* evs) {
  dag_ctx c = s->ctx;
  for (const ShapeBuf& b : sh.bufs) {
    if (b.role != DAG_ROLE_INIT) continue;
    PtrRef r{static_cast<int32_t>(&b - sh.bufs.data()), 0, nullptr};
    void* dst = resolve(s, sh, r, dev_off, host_off);
    HIP_TRY(c, hipMemcpyAsync(dst, b.init_src, b.bytes, kind_of(b.loc, b.init_loc), st));
    if (serial) HIP_TRY(c, hipStreamSynchronize(st));
  }
  const bool split = !serial && !s->copy_st[kOnH2D].empty();
  const size_t cl_ix = split ? s->launched % s->copy_st[kOnH2D].size() : 0;
  ++s->launched;
  if (!split) {
    for (const ShapeTask& t : sh.tasks) {
      hipError_t e = launch_task(s, sh, t, dev_off, host_off, st, scratch);
      if (e != hipSuccess) return hip_fail(c, e, "serving launch");
      if (serial) HIP_TRY(c, hipStreamSynchronize(st));
    }
  } else {
    hipEvent_t init_ev = nullptr;
    if (sh.has_init) {
      dag_status e = ev_get(s, &init_ev);
      if (e) return e;
      evs->push_back(init_ev);
      HIP_TRY(c, hipEventRecord(init_ev, st));
    }
    bool init_seen[3] = {true, false, false};
    std::vector<hipEvent_t> tev(sh.tasks.size(), nullptr);
    for (size_t k = 0; k < sh.tasks.size(); ++k) {
      const uint8_t cl = sh.cls[k];
      hipStream_t ts = cl == kOnLane ? st : s->copy_st[cl][cl_ix];
      if (init_ev && !init_seen[cl]) {
        HIP_TRY(c, hipStreamWaitEvent(ts, init_ev, 0));
        init_seen[cl] = true;
      }
      for (uint32_t w : sh.waits[k]) HIP_TRY(c, hipStreamWaitEvent(ts, tev[w], 0));
      hipError_t e = launch_task(s, sh, sh.tasks[k], dev_off, host_off, ts, scratch);
      if (e != hipSuccess) return hip_fail(c, e, "serving launch");
      if (sh.needs_ev[k]) {
        dag_status es = ev_get(s, &tev[k]);
        if (es) return es;
        evs->push_back(tev[k]);
        HIP_TRY(c, hipEventRecord(tev[k], ts));
      }
    }
    for (int cl = kOnH2D; cl <= kOnD2H; ++cl)
      if (sh.last_of[cl] >= 0) HIP_TRY(c, hipStreamWaitEvent(st, tev[sh.last_of[cl]], 0));
  }
  if (sh.result_buf >= 0 && sh.result_bytes && sh.bufs[sh.result_buf].loc == DAG_DEVICE) {
    PtrRef r{sh.result_buf, 0, nullptr};
    void* src = resolve(s, sh, r, dev_off, host_off);
    void* dst = static_cast<char*>(s->host_base) + host_off + sh.result_off;
    HIP_TRY(c, hipMemcpyAsync(dst, src, sh.result_bytes, hipMemcpyDeviceToHost, st));
    if (serial) HIP_TRY(c, hipStreamSynchronize(st));
  }
  return DAG_OK;
}

// The copy-lane plan of a shape (see Shape).
void plan_copy_lanes(Shape* sh) {
  const size_t n = sh->tasks.size();
  sh->cls.assign(n, kOnLane);
  sh->waits.assign(n, {});
  sh->needs_ev.assign(n, 0);
  for (size_t k = 0; k < n; ++k) {
    const RegionTask& t = *sh->tasks[k].t;
    if (t.kind == TK_COPY && t.ckind == hipMemcpyHostToDevice) sh->cls[k] = kOnH2D;
    if (t.kind == TK_COPY && t.ckind == hipMemcpyDeviceToHost) sh->cls[k] = kOnD2H;
    int32_t newest[3] = {-1, -1, -1};
    for (uint32_t p : t.rparents)
      if (sh->cls[p] != sh->cls[k]) newest[sh->cls[p]] = std::max<int32_t>(newest[sh->cls[p]], static_cast<int32_t>(p));
    for (int cl = 0; cl < 3; ++cl) {
      if (newest[cl] < 0) continue;
      sh->waits[k].push_back(static_cast<uint32_t>(newest[cl]));
      sh->needs_ev[newest[cl]] = 1;
    }
    sh->last_of[sh->cls[k]] = static_cast<int32_t>(k);
  }
  for (int cl = kOnH2D; cl <= kOnD2H; ++cl)
    if (sh->last_of[cl] >= 0) sh->needs_ev[sh->last_of[cl]] = 1;
  for (const ShapeBuf& b : sh->bufs)
    if (b.role == DAG_ROLE_INIT) sh->has_init = true;
  for (size_t k = 0; k < n; ++k)
    if (sh->cls[k] != kOnLane) sh->host_io = true;
}

void copy_result(const dag_server_s* s, const Shape& sh, uint64_t dev_off, uint64_t host_off, void* out) {
  if (!out || sh.result_buf < 0 || !sh.result_bytes) return;
  const ShapeBuf& b = sh.bufs[sh.result_buf];
  const char* src;
  if (b.loc == DAG_PINNED_HOST) {
    PtrRef r{sh.result_buf, 0, nullptr};
    src = static_cast<const char*>(resolve(s, sh, r, dev_off, host_off));
  } else {
    src = static_cast<const char*>(s->host_base) + host_off + sh.result_off;
  }
  std::memcpy(out, src, sh.result_bytes);
}

// ---- the polling thread's loop ---------------------------------------------

uint64_t now_ns(const dag_server_s* s) {
  if (s->ctx->dry) return s->vclock;
  return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - s->t0).count());
}

// Take what submitting threads have handed over; *closed and *horizon
// receive the submission state seen at that moment.
void take_incoming(dag_server s, bool* closed, uint64_t* horizon) {
  std::lock_guard<std::mutex> lk(s->mu);
  while (!s->incoming.empty()) {
    s->pending.push_back(s->incoming.front());
    s->incoming.pop_front();
  }
  s->taken = s->next_id;
  *closed = s->closed;
  *horizon = s->horizon;
}

// Retire the request at the head of a lane.
void complete(dag_server s, uint32_t lane, uint64_t when) {
  Flight f = std::move(s->flights[lane].front());
  s->flights[lane].pop_front();
  auto it = s->live.find(f.req);
  const Req rq = it->second;
  s->live.erase(it);
  const Shape& sh = s->shapes[rq.shape];
  copy_result(s, sh, f.dev_off, f.host_off, rq.result);
  dag_serve_done d = s->admitted[f.req];
  s->admitted.erase(f.req);
  d.done_ns = when;
  s->unreported.push_back(d);
  s->lat_ms.push_back((static_cast<double>(when) - static_cast<double>(rq.arrival_ns)) * 1e-6);
  s->last_done = std::max(s->last_done, when);
  if (sh.dev_bytes) s->dev.release(f.dev_off, sh.dev_bytes);
  if (sh.host_bytes) s->host.release(f.host_off, sh.host_bytes);
  s->used -= sh.dev_bytes;
  if (f.ev) s->free_ev.push_back(f.ev);
  for (hipEvent_t e : f.evs) s->free_ev.push_back(e);
  --s->inflight;
  ++s->ndone;
}

// One pass at the current time: arrivals into the queue, finished requests
// retired (each lane completes in order), queued requests admitted while
// their footprint fits (FIFO with a bounded bypass).  *progress = whether
// anything changed.
dag_status step(dag_server s, uint64_t now, bool* progress) {
  dag_ctx c = s->ctx;
  const bool dry = c->dry;
  *progress = false;
  while (!s->pending.empty() && s->pending.front().arrival_ns <= now) {
    s->queue.push_back(s->pending.front());
    s->pending.pop_front();
  }
  s->max_queued = std::max<uint32_t>(s->max_queued, static_cast<uint32_t>(s->queue.size()));
  const uint32_t nl = static_cast<uint32_t>(s->flights.size());
  for (uint32_t l = 0; l < nl; ++l) {
    while (!s->flights[l].empty()) {
      const Flight& f = s->flights[l].front();
      bool fin;
      if (dry) {
        fin = f.sim_done <= now;
      } else {
        const hipError_t q = hipEventQuery(f.ev);
        if (q != hipSuccess && q != hipErrorNotReady) return hip_fail(c, q, "hipEventQuery");
        if (q == hipErrorNotReady) (void)hipGetLastError();
        fin = q == hipSuccess;
      }
      if (!fin) break;
      complete(s, l, dry ? f.sim_done : now);
      *progress = true;
    }
  }
  uint32_t scanned = 0;
  for (auto it = s->queue.begin(); it != s->queue.end() && scanned < std::max<uint32_t>(s->cfg.bypass, 1);) {
    ++scanned;
    if (s->serial && s->inflight) break;
    const Req rq = *it;
    const Shape& sh = s->shapes[rq.shape];
    uint64_t doff = 0, hoff = 0;
    bool ok = s->used + sh.dev_bytes <= s->cfg.budget_bytes;
    if (ok && sh.dev_bytes) ok = s->dev.alloc(sh.dev_bytes, &doff);
    if (ok && sh.host_bytes && !s->host.alloc(sh.host_bytes, &hoff)) {
      if (sh.dev_bytes) s->dev.release(doff, sh.dev_bytes);
      ok = false;
    }
    if (!ok) {
      ++it;
      continue;
    }
    // the lane with the fewest requests in flight (lowest index on ties)
    // among the lanes of the request's class
    uint32_t lo = 0, hi = nl;
    if (!s->serial && s->cfg.transfer_lanes) {
      if (sh.host_io)
        hi = s->cfg.transfer_lanes;
      else
        lo = s->cfg.transfer_lanes;
    }
    uint32_t lane = lo;
    for (uint32_t l = lo + 1; l < hi; ++l)
      if (s->flights[l].size() < s->flights[lane].size()) lane = l;
    Flight f{rq.id, lane, nullptr, doff, hoff, 0, {}};
    if (dry) {
      const uint64_t start = std::max(now, s->lane_free[lane]);
      s->lane_free[lane] = f.sim_done = start + sh.sim_ns;
    } else {
      dag_status st = launch_request(s, sh, doff, hoff, s->lanes[lane], s->lane_scratch[lane], s->serial, &f.evs);
      if (st) return st;
      st = ev_get(s, &f.ev);
      if (st) return st;
      HIP_TRY(c, hipEventRecord(f.ev, s->lanes[lane]));
    }
    dag_serve_done d{};
    d.id = rq.id;
    d.arrival_ns = rq.arrival_ns;
    d.admit_ns = now;
    d.shape = rq.shape;
    d.lane = lane;
    s->admitted[rq.id] = d;
    s->live[rq.id] = rq;
    s->flights[lane].push_back(std::move(f));
    s->used += sh.dev_bytes;
    s->peak = std::max(s->peak, s->used);
    ++s->inflight;
    s->max_inflight = std::max(s->max_inflight, s->inflight);
    it = s->queue.erase(it);
    *progress = true;
  }
  return DAG_OK;
}

bool all_done(dag_server s, bool closed) {
  return closed && s->pending.empty() && s->queue.empty() && s->inflight == 0 && s->ndone == s->taken;
}

// Advance the loop until a completion is available to report, everything is
// done, or (GPU contexts) wait_us has passed.  Schedule-only contexts run on
// a virtual clock that jumps to the next arrival or completion; it never
// passes the arrival of the last submission until the session is closed, so
// requests submitted later in arrival order are seen exactly as if they had
// all been known from the start.
dag_status advance(dag_server s, uint64_t wait_us) {
  dag_ctx c = s->ctx;
  const bool dry = c->dry;
  const auto w0 = Clock::now();
  for (;;) {
    bool closed;
    uint64_t horizon;
    take_incoming(s, &closed, &horizon);
    if (all_done(s, closed) || !s->unreported.empty()) return DAG_OK;
    const uint64_t now = now_ns(s);
    if (dry && !closed && now >= horizon) return DAG_OK;  // wait for the next submission
    bool progress = false;
    dag_status st = step(s, now, &progress);
    if (st) return st;
    if (progress) continue;
    if (dry) {
      uint64_t t = UINT64_MAX;
      if (!s->pending.empty()) t = s->pending.front().arrival_ns;
      for (const auto& fl : s->flights)
        if (!fl.empty()) t = std::min(t, fl.front().sim_done);
      if (t == UINT64_MAX) {
        if (!s->queue.empty()) return fail(c, DAG_E_RANGE, "a queued request can never be admitted");
        return DAG_OK;  // nothing to do until a submission
      }
      if (!closed && t >= horizon) return DAG_OK;
      s->vclock = std::max(s->vclock, t);
      continue;
    }
    if (s->inflight == 0 && !s->queue.empty())
      return fail(c, DAG_E_RANGE, "a queued request can never be admitted (arena fragmentation)");
    const double waited = us_since(w0);
    if (waited >= static_cast<double>(wait_us)) return DAG_OK;
    if (s->inflight == 0 && s->queue.empty()) {
      // idle: sleep until shortly before the next known arrival, or up to
      // 1 ms when none is known; a submission or the close wakes it
      const double left_ns = (static_cast<double>(wait_us) - waited) * 1e3;
      uint64_t sleep_ns = 0;
      if (!s->pending.empty()) {
        const uint64_t a = s->pending.front().arrival_ns;
        sleep_ns = a > now + 200000 ? a - now - 100000 : 0;
      } else if (!closed) {
        sleep_ns = 1000000;
      }
      sleep_ns = std::min<uint64_t>(sleep_ns, static_cast<uint64_t>(std::max(left_ns, 0.0)));
      if (sleep_ns) {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv.wait_for(lk, std::chrono::nanoseconds(sleep_ns), [&] { return !s->incoming.empty() || s->closed; });
      }
    }
  }
}

}  // namespace

extern "C" {

dag_status dag_serve_create(dag_ctx c, const dag_serve_config* cfg, dag_server* out) {
  CHECK_CTX(c);
  if (!cfg || !out) return fail(c, DAG_E_INVAL, "cfg and out are required");
  if (cfg->lanes == 0 || cfg->lanes > DAG_MAX_STREAMS) return fail(c, DAG_E_INVAL, "lanes must be 1..64");
  if (cfg->copy_lanes > 4) return fail(c, DAG_E_INVAL, "copy_lanes must be 0..4");
  if (cfg->transfer_lanes && cfg->transfer_lanes >= cfg->lanes)
    return fail(c, DAG_E_INVAL, "transfer_lanes must be 0 or less than lanes");
  if (cfg->budget_bytes == 0 || cfg->budget_bytes > cfg->device_arena_bytes)
    return fail(c, DAG_E_INVAL, "budget must be in (0, device_arena_bytes]");
  auto* s = new (std::nothrow) dag_server_s();
  if (!s) return fail(c, DAG_E_NOMEM, "server");
  s->ctx = c;
  s->cfg = *cfg;
  s->dev.reset(cfg->device_arena_bytes);
  s->host.reset(cfg->host_arena_bytes);
  if (!c->dry) {
    hipError_t e = hipMalloc(&s->dev_base, cfg->device_arena_bytes);
    if (e == hipSuccess && cfg->host_arena_bytes)
      e = hipHostMalloc(&s->host_base, cfg->host_arena_bytes, hipHostMallocDefault);
    for (int cl = kOnH2D; cl <= kOnD2H; ++cl)
      for (uint32_t i = 0; e == hipSuccess && i < cfg->copy_lanes; ++i) {
        hipStream_t cs;
        e = new_stream(c, &cs);
        if (e == hipSuccess) s->copy_st[cl].push_back(cs);
      }
    for (uint32_t i = 0; e == hipSuccess && i < cfg->lanes; ++i) {
      hipStream_t st;
      void* scr = nullptr;
      e = new_stream(c, &st);
      if (e == hipSuccess) s->lanes.push_back(st);
      if (e == hipSuccess) e = hipMalloc(&scr, c->cfg.scratch_bytes);
      if (e == hipSuccess) s->lane_scratch.push_back(scr);
      if (e == hipSuccess) e = hipMemsetAsync(scr, 0, c->cfg.scratch_bytes, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess) {
      dag_status st = (e == hipErrorOutOfMemory) ? fail(c, DAG_E_NOMEM, "server allocation failed")
                                                 : hip_fail(c, e, "server setup");
      dag_serve_destroy(s);
      return st;
    }
  } else {
    s->lanes.assign(cfg->lanes, nullptr);
    s->lane_scratch.assign(cfg->lanes, nullptr);
  }
  *out = s;
  return DAG_OK;
}

dag_status dag_serve_destroy(dag_server s) {
  if (!s) return DAG_OK;
  if (!s->ctx->dry) {
    for (hipStream_t st : s->lanes)
      if (st) (void)hipStreamSynchronize(st);
    for (auto& v : s->copy_st)
      for (hipStream_t st : v) (void)hipStreamSynchronize(st);
    for (const auto& fl : s->flights)
      for (const Flight& f : fl) {
        if (f.ev) (void)hipEventDestroy(f.ev);
        for (hipEvent_t e : f.evs) (void)hipEventDestroy(e);
      }
    for (hipStream_t st : s->lanes)
      if (st) (void)hipStreamDestroy(st);
    for (auto& v : s->copy_st)
      for (hipStream_t st : v) (void)hipStreamDestroy(st);
    for (void* p : s->lane_scratch)
      if (p) (void)hipFree(p);
    for (hipEvent_t e : s->free_ev) (void)hipEventDestroy(e);
    if (s->dev_base) (void)hipFree(s->dev_base);
    if (s->host_base) (void)hipHostFree(s->host_base);
  }
  // unpin the regions and buffers the shapes use
  for (Shape& sh : s->shapes) {
    if (sh.region->pins) --sh.region->pins;
    for (uint32_t slot : sh.pinned)
      if (slot < s->ctx->bufs.size() && s->ctx->bufs[slot].pins) --s->ctx->bufs[slot].pins;
  }
  delete s;
  return DAG_OK;
}

dag_status dag_serve_add_shape(dag_server s, uint64_t key, const dag_shape_buf* bufs, uint32_t nbufs,
                               dag_buf result_buf, size_t result_bytes, uint64_t sim_ns, uint32_t* shape_id) {
  if (!s) return DAG_E_INVAL;
  dag_ctx c = s->ctx;
  CHECK_CTX(c);
  if (s->started) return fail(c, DAG_E_BUSY, "shapes cannot be added while a session runs");
  auto it = c->regions.find(key);
  if (it == c->regions.end()) return fail(c, DAG_E_NOTFOUND, "unknown region key");
  if (it->second->dead) return fail(c, DAG_E_INVAL, "region uses a released buffer");
  if (!bufs || nbufs == 0 || !shape_id) return fail(c, DAG_E_INVAL, "shape buffers required");
  Shape sh;
  sh.region = it->second.get();
  sh.result_buf = -1;
  sh.result_bytes = result_bytes;
  sh.sim_ns = sim_ns;
  std::vector<int32_t> slot_to_buf(c->bufs.size(), -1);
  for (uint32_t i = 0; i < nbufs; ++i) {
    Buffer* b = get_buf(c, bufs[i].buf);
    if (!b) return fail(c, DAG_E_INVAL, "shape buffer %u: invalid handle", i);
    if (bufs[i].role > DAG_ROLE_INIT) return fail(c, DAG_E_INVAL, "shape buffer %u: bad role", i);
    if (slot_to_buf[bufs[i].buf - 1] >= 0) return fail(c, DAG_E_INVAL, "shape buffer %u listed twice", i);
    slot_to_buf[bufs[i].buf - 1] = static_cast<int32_t>(i);
    ShapeBuf sb{bufs[i].role, b->ptr, b->bytes, b->loc, nullptr, 0, 0};
    sh.pinned.push_back(bufs[i].buf - 1);
    if (bufs[i].role == DAG_ROLE_INIT) {
      Buffer* src = get_buf(c, bufs[i].init_src);
      if (!src || src->bytes < b->bytes) return fail(c, DAG_E_INVAL, "shape buffer %u: bad init source", i);
      sb.init_src = src->ptr;
      sb.init_loc = src->loc;
      sh.pinned.push_back(bufs[i].init_src - 1);
    }
    if (bufs[i].role != DAG_ROLE_SHARED) {
      uint64_t& total = b->loc == DAG_PINNED_HOST ? sh.host_bytes : sh.dev_bytes;
      sb.off = total;
      total += align_up(b->bytes);
    }
    sh.bufs.push_back(sb);
    if (bufs[i].buf == result_buf) sh.result_buf = static_cast<int32_t>(i);
  }
  if (result_buf && sh.result_buf < 0) return fail(c, DAG_E_INVAL, "result buffer is not a shape buffer");
  if (sh.result_buf >= 0 && result_bytes > sh.bufs[sh.result_buf].bytes)
    return fail(c, DAG_E_INVAL, "result_bytes beyond the result buffer");
  if (sh.result_buf >= 0 && sh.result_bytes && sh.bufs[sh.result_buf].loc == DAG_DEVICE) {
    sh.result_off = sh.host_bytes;
    sh.host_bytes += align_up(result_bytes);
  }
  // every buffer the region touches must be a shape buffer; shared ones read-only
  for (const Access& a : sh.region->accs) {
    const int32_t bi = a.buf < slot_to_buf.size() ? slot_to_buf[a.buf] : -1;
    if (bi < 0) return fail(c, DAG_E_INVAL, "region uses buffer %u that the shape does not list", a.buf + 1);
    if (sh.bufs[bi].role == DAG_ROLE_SHARED && a.acc == ACC_W)
      return fail(c, DAG_E_INVAL, "shared buffer %u is modified by the region", a.buf + 1);
  }
  auto ref = [&](const void* p) {
    const uintptr_t u = reinterpret_cast<uintptr_t>(p);
    for (size_t i = 0; i < sh.bufs.size(); ++i) {
      const uintptr_t b0 = reinterpret_cast<uintptr_t>(sh.bufs[i].tmpl);
      if (u >= b0 && u < b0 + sh.bufs[i].bytes) return PtrRef{static_cast<int32_t>(i), u - b0, const_cast<void*>(p)};
    }
    return PtrRef{-1, 0, const_cast<void*>(p)};
  };
  for (const RegionTask& t : sh.region->tasks) {
    ShapeTask st;
    st.t = &t;
    if (t.kind == TK_COPY) {
      st.cdst = ref(t.cdst);
      st.csrc = ref(t.csrc);
    } else {
      for (void* p : t.ptrs) st.refs.push_back(ref(p));
    }
    sh.tasks.push_back(std::move(st));
  }
  plan_copy_lanes(&sh);
  if (sh.dev_bytes > s->cfg.budget_bytes) return fail(c, DAG_E_RANGE, "shape needs more than the budget");
  if (sh.host_bytes > s->cfg.host_arena_bytes) return fail(c, DAG_E_RANGE, "shape needs more than the host arena");
  // the region and the buffers stay as recorded while the shape exists
  ++sh.region->pins;
  std::sort(sh.pinned.begin(), sh.pinned.end());
  sh.pinned.erase(std::unique(sh.pinned.begin(), sh.pinned.end()), sh.pinned.end());
  for (uint32_t slot : sh.pinned) ++c->bufs[slot].pins;
  s->shapes.push_back(std::move(sh));
  *shape_id = static_cast<uint32_t>(s->shapes.size() - 1);
  return DAG_OK;
}

dag_status dag_serve_shape_info(dag_server s, uint32_t shape, uint64_t* device_bytes, uint64_t* host_bytes) {
  if (!s || shape >= s->shapes.size()) return DAG_E_INVAL;
  if (device_bytes) *device_bytes = s->shapes[shape].dev_bytes;
  if (host_bytes) *host_bytes = s->shapes[shape].host_bytes;
  return DAG_OK;
}

dag_status dag_serve_start(dag_server s, uint32_t mode) {
  if (!s) return DAG_E_INVAL;
  dag_ctx c = s->ctx;
  CHECK_CTX(c);
  if (mode > DAG_SERVE_SERIAL) return fail(c, DAG_E_INVAL, "bad mode");
  bool closed;
  {
    std::lock_guard<std::mutex> lk(s->mu);  // dag_serve_close may run on another thread
    closed = s->closed;
  }
  if (s->started && !all_done(s, closed))
    return fail(c, DAG_E_BUSY, "the previous session has requests outstanding");
  s->started = true;
  s->serial = mode == DAG_SERVE_SERIAL;
  const uint32_t nl = s->serial ? 1u : static_cast<uint32_t>(s->lanes.size());
  s->flights.assign(nl, {});
  s->lane_free.assign(nl, 0);
  s->pending.clear();
  s->queue.clear();
  s->live.clear();
  s->admitted.clear();
  s->unreported.clear();
  s->lat_ms.clear();
  s->used = s->peak = s->vclock = s->taken = s->ndone = 0;
  s->last_done = 0;
  s->inflight = s->max_inflight = s->max_queued = 0;
  std::lock_guard<std::mutex> lk(s->mu);
  s->first_arrival = UINT64_MAX;
  s->incoming.clear();
  s->next_id = 0;
  s->horizon = 0;
  s->closed = false;
  s->t0 = Clock::now();
  return DAG_OK;
}

dag_status dag_serve_submit(dag_server s, uint32_t shape, uint64_t arrival_ns, void* result, uint64_t* id) {
  if (!s) return DAG_E_INVAL;
  dag_ctx c = s->ctx;
  if (c->poisoned) return DAG_E_POISONED;
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->started || s->closed) return DAG_E_BUSY;
  if (shape >= s->shapes.size()) return DAG_E_INVAL;
  if (arrival_ns == DAG_SERVE_NOW) {
    if (c->dry) return DAG_E_INVAL;  // a virtual clock has no "now" for other threads
    arrival_ns =
        static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - s->t0).count());
    arrival_ns = std::max(arrival_ns, s->horizon);
  } else if (arrival_ns < s->horizon) {
    return DAG_E_INVAL;  // arrivals are submitted in non-decreasing order
  }
  Req r{s->next_id++, shape, arrival_ns, result};
  s->horizon = arrival_ns;
  s->first_arrival = std::min(s->first_arrival, arrival_ns);
  s->incoming.push_back(r);
  if (id) *id = r.id;
  s->cv.notify_all();
  return DAG_OK;
}

dag_status dag_serve_close(dag_server s) {
  if (!s) return DAG_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->started) return DAG_E_BUSY;
  s->closed = true;
  s->cv.notify_all();
  return DAG_OK;
}

dag_status dag_serve_poll(dag_server s, uint64_t wait_us, dag_serve_done* done, uint32_t cap, uint32_t* n,
                          uint64_t* outstanding) {
  if (n) *n = 0;
  if (!s) return DAG_E_INVAL;
  dag_ctx c = s->ctx;
  CHECK_CTX(c);
  if (!s->started) return fail(c, DAG_E_BUSY, "no session: call dag_serve_start first");
  if (cap && !done) return fail(c, DAG_E_INVAL, "done is NULL");
  dag_status st = advance(s, wait_us);
  if (st) return st;
  uint32_t k = 0;
  while (k < cap && !s->unreported.empty()) {
    done[k++] = s->unreported.front();
    s->unreported.pop_front();
  }
  if (n) *n = k;
  if (outstanding) {
    std::lock_guard<std::mutex> lk(s->mu);
    *outstanding = (s->next_id - s->ndone) + s->unreported.size();
  }
  return DAG_OK;
}

dag_status dag_serve_stats(dag_server s, dag_serve_summary* out) {
  if (!s || !out) return DAG_E_INVAL;
  std::vector<double> lat(s->lat_ms);
  std::sort(lat.begin(), lat.end());
  const size_t n = lat.size();
  auto pct = [&](double q) {
    if (lat.empty()) return 0.0;
    size_t k = static_cast<size_t>(std::ceil(q / 100.0 * n));
    k = std::max<size_t>(k, 1);
    return lat[k - 1];
  };
  double sum = 0.0;
  for (double v : lat) sum += v;
  std::memset(out, 0, sizeof(*out));
  out->p50_ms = pct(50);
  out->p99_ms = pct(99);
  out->mean_ms = n ? sum / n : 0.0;
  out->max_ms = n ? lat.back() : 0.0;
  uint64_t first_arrival;
  {
    std::lock_guard<std::mutex> lk(s->mu);  // dag_serve_submit updates it from producer threads
    first_arrival = s->first_arrival;
  }
  const double span_s =
      n ? (static_cast<double>(s->last_done) - static_cast<double>(first_arrival)) * 1e-9 : 0.0;
  out->req_per_s = span_s > 0 ? n / span_s : 0.0;
  out->wall_ms = static_cast<double>(s->last_done) * 1e-6;
  out->peak_device_bytes = s->peak;
  out->max_inflight = s->max_inflight;
  out->max_queued = s->max_queued;
  out->completed = n;
  return DAG_OK;
}

dag_status dag_serve_run(dag_server s, const dag_request* reqs, uint32_t n, uint32_t mode, dag_serve_done* done,
                         dag_serve_summary* stats) {
  if (!s) return DAG_E_INVAL;
  dag_ctx c = s->ctx;
  CHECK_CTX(c);
  if (mode > DAG_SERVE_SERIAL) return fail(c, DAG_E_INVAL, "bad mode");
  if (n && (!reqs || !done)) return fail(c, DAG_E_INVAL, "reqs and done are required");
  for (uint32_t i = 0; i < n; ++i) {
    if (reqs[i].shape >= s->shapes.size()) return fail(c, DAG_E_INVAL, "request %u: unknown shape", i);
    if (reqs[i].arrival_ns == DAG_SERVE_NOW) return fail(c, DAG_E_INVAL, "request %u: arrival must be a time", i);
    if (i && reqs[i].arrival_ns < reqs[i - 1].arrival_ns)
      return fail(c, DAG_E_INVAL, "requests must be sorted by arrival");
  }
  dag_status st = dag_serve_start(s, mode);
  if (st) return st;
  for (uint32_t i = 0; i < n; ++i) {
    st = dag_serve_submit(s, reqs[i].shape, reqs[i].arrival_ns, reqs[i].result, nullptr);
    if (st) return fail(c, st, "request %u: submission failed", i);
  }
  dag_serve_close(s);
  std::vector<dag_serve_done> buf(256);
  uint64_t left = n;
  while (left) {
    uint32_t got = 0;
    uint64_t outstanding = 0;
    st = dag_serve_poll(s, 1000000, buf.data(), static_cast<uint32_t>(buf.size()), &got, &outstanding);
    if (st) return st;
    for (uint32_t k = 0; k < got; ++k) done[buf[k].id] = buf[k];
    left -= got;
    if (!got && !outstanding) break;
  }
  if (left) return fail(c, DAG_E_RANGE, "%llu requests never completed", (unsigned long long)left);
  if (stats) dag_serve_stats(s, stats);
  return DAG_OK;
}

}  // extern "C"
