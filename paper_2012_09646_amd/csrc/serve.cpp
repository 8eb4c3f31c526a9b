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
#include <cmath>
#include <cstring>
#include <new>
#include <deque>
#include <map>
#include <thread>
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
};

struct Flight {
  uint32_t req;
  uint32_t lane;
  hipEvent_t ev;
  uint64_t dev_off, host_off;
  uint64_t sim_done;  // schedule-only contexts
  std::vector<hipEvent_t> evs;  // copy-lane mode: events of the request's calls
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
  delete s;
  return DAG_OK;
}

dag_status dag_serve_add_shape(dag_server s, uint64_t key, const dag_shape_buf* bufs, uint32_t nbufs,
                               dag_buf result_buf, size_t result_bytes, uint64_t sim_ns, uint32_t* shape_id) {
  if (!s) return DAG_E_INVAL;
  dag_ctx c = s->ctx;
  CHECK_CTX(c);
  auto it = c->regions.find(key);
  if (it == c->regions.end()) return fail(c, DAG_E_NOTFOUND, "unknown region key");
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
    if (bufs[i].role == DAG_ROLE_INIT) {
      Buffer* src = get_buf(c, bufs[i].init_src);
      if (!src || src->bytes < b->bytes) return fail(c, DAG_E_INVAL, "shape buffer %u: bad init source", i);
      sb.init_src = src->ptr;
      sb.init_loc = src->loc;
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

dag_status dag_serve_run(dag_server s, const dag_request* reqs, uint32_t n, uint32_t mode, dag_request_done* done,
                         dag_serve_stats* stats) {
  if (!s) return DAG_E_INVAL;
  dag_ctx c = s->ctx;
  CHECK_CTX(c);
  if (mode > DAG_SERVE_SERIAL) return fail(c, DAG_E_INVAL, "bad mode");
  if (n && (!reqs || !done)) return fail(c, DAG_E_INVAL, "reqs and done are required");
  for (uint32_t i = 0; i < n; ++i) {
    if (reqs[i].shape >= s->shapes.size()) return fail(c, DAG_E_INVAL, "request %u: unknown shape", i);
    if (i && reqs[i].arrival_ns < reqs[i - 1].arrival_ns)
      return fail(c, DAG_E_INVAL, "requests must be sorted by arrival");
  }
  const bool dry = c->dry;
  const bool serial = mode == DAG_SERVE_SERIAL;
  const uint32_t nl = serial ? 1u : static_cast<uint32_t>(s->lanes.size());
  std::vector<std::deque<Flight>> flights(nl);
  std::vector<uint64_t> lane_free(nl, 0);  // schedule-only: virtual time a lane drains
  std::deque<uint32_t> queue;
  uint32_t next = 0, ndone = 0, inflight = 0;
  uint64_t used = 0, peak = 0, vclock = 0;
  uint32_t max_inflight = 0, max_queued = 0;
  const auto t0 = Clock::now();
  auto now_ns = [&]() -> uint64_t {
    if (dry) return vclock;
    return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count());
  };
  auto complete = [&](uint32_t lane, uint64_t when) {
    Flight f = flights[lane].front();
    flights[lane].pop_front();
    const Shape& sh = s->shapes[reqs[f.req].shape];
    copy_result(s, sh, f.dev_off, f.host_off, reqs[f.req].result);
    done[f.req].done_ns = when;
    if (sh.dev_bytes) s->dev.release(f.dev_off, sh.dev_bytes);
    if (sh.host_bytes) s->host.release(f.host_off, sh.host_bytes);
    used -= sh.dev_bytes;
    if (f.ev) s->free_ev.push_back(f.ev);
    for (hipEvent_t e : f.evs) s->free_ev.push_back(e);
    --inflight;
    ++ndone;
  };
  while (ndone < n) {
    uint64_t now = now_ns();
    while (next < n && reqs[next].arrival_ns <= now) queue.push_back(next++);
    max_queued = std::max<uint32_t>(max_queued, static_cast<uint32_t>(queue.size()));
    bool progress = false;
    // retire finished requests (lanes complete in order)
    for (uint32_t l = 0; l < nl; ++l) {
      while (!flights[l].empty()) {
        const Flight& f = flights[l].front();
        bool fin;
        if (dry) {
          fin = f.sim_done <= now;
        } else {
          const hipError_t q = hipEventQuery(f.ev);
          if (q != hipSuccess && q != hipErrorNotReady) return hip_fail(c, q, "hipEventQuery");
          fin = q == hipSuccess;
        }
        if (!fin) break;
        complete(l, dry ? f.sim_done : now);
        progress = true;
      }
    }
    // admit queued requests whose footprint fits (FIFO, bounded bypass)
    uint32_t scanned = 0;
    for (auto it = queue.begin(); it != queue.end() && scanned < std::max<uint32_t>(s->cfg.bypass, 1);) {
      ++scanned;
      if (serial && inflight) break;
      const uint32_t r = *it;
      const Shape& sh = s->shapes[reqs[r].shape];
      uint64_t doff = 0, hoff = 0;
      bool ok = used + sh.dev_bytes <= s->cfg.budget_bytes;
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
      if (!serial && s->cfg.transfer_lanes) {
        if (sh.host_io)
          hi = s->cfg.transfer_lanes;
        else
          lo = s->cfg.transfer_lanes;
      }
      uint32_t lane = lo;
      for (uint32_t l = lo + 1; l < hi; ++l)
        if (flights[l].size() < flights[lane].size()) lane = l;
      Flight f{r, lane, nullptr, doff, hoff, 0};
      done[r].admit_ns = now;
      done[r].lane = lane;
      done[r].reserved = 0;
      if (dry) {
        const uint64_t start = std::max(now, lane_free[lane]);
        lane_free[lane] = f.sim_done = start + sh.sim_ns;
      } else {
        dag_status st = launch_request(s, sh, doff, hoff, s->lanes[lane], s->lane_scratch[lane], serial, &f.evs);
        if (st) return st;
        st = ev_get(s, &f.ev);
        if (st) return st;
        HIP_TRY(c, hipEventRecord(f.ev, s->lanes[lane]));
      }
      flights[lane].push_back(std::move(f));
      used += sh.dev_bytes;
      peak = std::max(peak, used);
      ++inflight;
      max_inflight = std::max(max_inflight, inflight);
      it = queue.erase(it);
      progress = true;
    }
    if (!progress) {
      if (dry) {
        // advance the virtual clock to the next arrival or completion
        uint64_t t = UINT64_MAX;
        if (next < n) t = reqs[next].arrival_ns;
        for (uint32_t l = 0; l < nl; ++l)
          if (!flights[l].empty()) t = std::min(t, flights[l].front().sim_done);
        if (t == UINT64_MAX) return fail(c, DAG_E_RANGE, "a queued request can never be admitted");
        vclock = std::max(vclock, t);
      } else if (inflight == 0 && next < n && queue.empty()) {
        const uint64_t wait = reqs[next].arrival_ns > now ? reqs[next].arrival_ns - now : 0;
        if (wait > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(wait - 100000));
      } else if (inflight == 0 && !queue.empty()) {
        return fail(c, DAG_E_RANGE, "a queued request can never be admitted (arena fragmentation)");
      }
    }
  }
  if (stats) {
    std::vector<double> lat(n);
    double sum = 0.0;
    uint64_t last = 0;
    for (uint32_t i = 0; i < n; ++i) {
      lat[i] = (static_cast<double>(done[i].done_ns) - static_cast<double>(reqs[i].arrival_ns)) * 1e-6;
      sum += lat[i];
      last = std::max(last, done[i].done_ns);
    }
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double q) {
      if (lat.empty()) return 0.0;
      size_t k = static_cast<size_t>(std::ceil(q / 100.0 * lat.size()));
      k = std::max<size_t>(k, 1);
      return lat[k - 1];
    };
    stats->p50_ms = pct(50);
    stats->p99_ms = pct(99);
    stats->mean_ms = n ? sum / n : 0.0;
    stats->max_ms = n ? lat.back() : 0.0;
    const double span_s = n ? (static_cast<double>(last) - static_cast<double>(reqs[0].arrival_ns)) * 1e-9 : 0.0;
    stats->req_per_s = span_s > 0 ? n / span_s : 0.0;
    stats->wall_ms = static_cast<double>(last) * 1e-6;
    stats->peak_device_bytes = peak;
    stats->max_inflight = max_inflight;
    stats->max_queued = max_queued;
  }
  return DAG_OK;
}

}  // extern "C"
