// Dependency tracker and stream manager of the runtime DAG scheduler.
//
// HIP-free: it decides edges, activity, streams and event waits; the
// executor (dagrt.cpp) turns those decisions into HIP calls.
//
// Dependency sets (paper Sec. IV-A) are kept per buffer instead of per
// computation, which yields the same edges in O(#args + #readers):
//   W(b)  the last computation that modified b,
//   R(b)  the computations that read b since W(b) (only active ones are
//         kept; a flag remembers that some read happened).
// A call that reads b depends on W(b) (read-after-write); a call that
// modifies b depends on the readers since W(b) (write-after-read) or, when
// nobody read b since, on W(b) itself (write-after-write).  A later writer
// therefore never depends on both a writer and its readers, and a later
// reader shares the writer with the earlier readers (the read-only cases of
// Sec. IV-A).  Only active computations create edges; a host access that
// waits on computations retires them and all their ancestors (Sec. IV-B).
//
// Streams (Sec. IV-C): the first child of a computation goes on its parent's
// stream; otherwise an empty stream is reused in FIFO order; otherwise a new
// stream is created while the pool is below its bound, and beyond it the
// stream whose last task is oldest is reused.  Optionally, host<->device
// copies bypass the pool and go to one FIFO stream per direction (a copy
// lane): concurrent copies in one direction share the single PCIe link, so
// running them one after the other in issue order finishes the first ones
// early and lets their consumers start while later copies still stream.  A call waits only on parents
// on other streams (Sec. IV-B: one event per computation), and among those
// only on the newest per stream that is not already ordered before it;
// per-stream vector clocks decide that in O(#streams).
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <vector>

namespace dagrt {

constexpr uint8_t ACC_R = 1;
constexpr uint8_t ACC_W = 2;

enum TaskKind : uint8_t {
  TK_KERNEL = 0,
  TK_COPY = 1,
  TK_HOST_READ = 2,
  TK_HOST_WRITE = 3,
  TK_SYNC = 4,
  TK_REGION = 5,
  TK_RELEASE = 6,
};

constexpr uint8_t kLaneH2D = 1;  // copy directions with lanes of their own
constexpr uint8_t kLaneD2H = 2;
constexpr uint32_t kMaxLanesPerDir = 4;

inline bool is_gpu_kind(uint8_t k) { return k == TK_KERNEL || k == TK_COPY || k == TK_REGION; }

struct Access {
  uint32_t buf;  // buffer slot (handle - 1)
  uint8_t acc;   // ACC_R or ACC_W
};

struct EdgeRec {
  uint64_t src, dst;
  uint32_t buf;  // buffer slot
  uint32_t kind; // 0 RAW, 1 WAR, 2 WAW
};

struct TaskRec {
  uint8_t kind = 0;
  bool active = false;
  bool vertex = false;
  int32_t stream = -1;
  uint32_t pos = 0;  // 1-based position on its stream
  uint32_t kernel_id = 0;
  uint32_t par_off = 0, par_n = 0;
  uint32_t wait_off = 0, wait_n = 0;
  uint32_t vc_off = 0, vc_n = 0;  // vector clock of its stream right after it
};

struct BufTrack {
  uint64_t W = 0;
  bool read_since_write = false;
  std::vector<uint64_t> R;
};

struct StreamRec {
  uint64_t tail = 0;
  uint32_t nactive = 0;
  uint32_t npos = 0;
  bool in_fifo = false;
  uint8_t lane = 0;  // 0 = pool stream, else the copy lane it serves
  std::vector<uint32_t> vc;  // vc[t]: highest position of stream t ordered before this point
};

class Tracker {
 public:
  explicit Tracker(uint32_t max_streams, uint32_t lanes_per_dir = 1)
      : max_streams_(max_streams), lanes_per_dir_(std::max<uint32_t>(1, std::min<uint32_t>(lanes_per_dir, kMaxLanesPerDir))) {
    tasks_.emplace_back();  // id 0 = none
  }

  // Ids below base_ were dropped by compact(); tasks_[k] is task base_ + k.
  uint64_t last_id() const { return base_ + tasks_.size() - 1; }
  uint64_t first_kept() const { return base_ == 0 ? 1 : base_; }
  bool known(uint64_t id) const { return id >= first_kept() && id <= last_id(); }
  uint64_t base() const { return base_; }
  const TaskRec& task(uint64_t id) const { return tasks_[id - base_]; }
  uint64_t vertices_total() const {
    uint64_t v = dropped_vertices_;
    for (const TaskRec& t : tasks_) v += t.vertex ? 1 : 0;
    return v;
  }
  uint64_t edges_total() const { return dropped_edges_ + edges_.size(); }
  uint32_t num_streams() const { return static_cast<uint32_t>(streams_.size()); }
  bool is_lane(int32_t s) const { return s >= 0 && streams_[s].lane != 0; }
  uint64_t num_active() const { return nactive_total_; }
  const std::vector<EdgeRec>& edges() const { return edges_; }
  const uint64_t* parents(uint64_t id) const { return par_pool_.data() + task(id).par_off; }
  const uint64_t* waits(uint64_t id) const { return wait_pool_.data() + task(id).wait_off; }

  // Drop the records of every task so far (ids stay monotonic): allowed only
  // when no task is active, so none of them can produce an edge or a wait
  // again.  The per-buffer W/R sets are cleared (their tasks are all
  // retired, which yields the same future edges as an empty set).  Edges and
  // task records queried later cover the tasks after this point only.
  void compact() {
    if (nactive_total_ != 0) return;
    for (const TaskRec& t : tasks_) dropped_vertices_ += t.vertex ? 1 : 0;
    dropped_edges_ += edges_.size();
    base_ = last_id() + 1;
    tasks_.clear();
    par_pool_.clear();
    wait_pool_.clear();
    vc_pool_.clear();
    edges_.clear();
    active_list_.clear();
    for (BufTrack& b : bufs_) b = BufTrack();
  }

  void ensure_buffer(uint32_t slot) {
    if (slot >= bufs_.size()) bufs_.resize(slot + 1);
  }
  // Forget a buffer's history (after release: the slot may be reused).
  void reset_buffer(uint32_t slot) {
    if (slot < bufs_.size()) bufs_[slot] = BufTrack();
  }
  // Tasks currently active that access slot (for release-style waits).
  void conflicts_for(uint32_t slot, uint8_t acc, std::vector<uint64_t>* out) const {
    out->clear();
    if (slot >= bufs_.size()) return;
    const BufTrack& b = bufs_[slot];
    if (acc == ACC_W && b.read_since_write) {
      for (uint64_t r : b.R)
        if (T(r).active) out->push_back(r);
    } else if (b.W && T(b.W).active) {
      out->push_back(b.W);
    }
  }

  // Add a GPU call (kernel, copy, region replay).  accs must be deduplicated
  // per buffer (MUTABLE wins).  serial: no dependency work, everything on
  // stream 0 (the serial policy of Sec. IV-C computes no dependencies).
  // Returns the new id; *stream_out, *new_stream_out and the wait list
  // (waits(id), task(id).wait_n) describe what the executor must do.
  // lane: 0 = placed by the policy; kLaneH2D / kLaneD2H = on that copy
  // direction's lanes (FIFO streams outside the pool).
  uint64_t add_gpu(uint8_t kind, uint32_t kernel_id, const Access* accs, uint32_t n,
                   bool serial, int32_t* stream_out, bool* new_stream_out, uint8_t lane = 0) {
    const uint64_t id = base_ + tasks_.size();
    tasks_.emplace_back();
    TaskRec& t = tasks_.back();
    t.kind = kind;
    t.kernel_id = kernel_id;
    t.vertex = true;
    tmp_par_.clear();
    if (!serial) {
      for (uint32_t i = 0; i < n; ++i) collect_edges(id, accs[i], &tmp_par_);
      for (uint32_t i = 0; i < n; ++i) update_buffer(id, accs[i]);
    }
    std::sort(tmp_par_.begin(), tmp_par_.end());
    tmp_par_.erase(std::unique(tmp_par_.begin(), tmp_par_.end()), tmp_par_.end());
    TaskRec& tt = T(id);
    tt.par_off = static_cast<uint32_t>(par_pool_.size());
    tt.par_n = static_cast<uint32_t>(tmp_par_.size());
    par_pool_.insert(par_pool_.end(), tmp_par_.begin(), tmp_par_.end());

    bool created = false;
    int32_t s = serial ? pick_serial(&created) : lane ? pick_lane(lane, &created) : pick_stream(&created);
    place(id, s);
    *stream_out = s;
    *new_stream_out = created;
    return id;
  }

  // Add a host access (TK_HOST_READ with ACC_R, TK_HOST_WRITE / TK_RELEASE
  // with ACC_W).  *wait_on receives the active tasks the host must wait for
  // (empty: not a vertex).  After waiting, the caller calls retire(id).
  uint64_t add_host(uint8_t kind, uint32_t slot, uint8_t acc, bool serial,
                    std::vector<uint64_t>* wait_on) {
    const uint64_t id = base_ + tasks_.size();
    tasks_.emplace_back();
    tasks_.back().kind = kind;
    tmp_par_.clear();
    if (!serial) {
      Access a{slot, acc};
      collect_edges(id, a, &tmp_par_);
      BufTrack& b = bufs_[slot];
      if (acc == ACC_W) {
        b.W = id;  // never active: a host access completes before the next call
        b.R.clear();
        b.read_since_write = false;
      } else {
        b.read_since_write = true;
      }
    }
    std::sort(tmp_par_.begin(), tmp_par_.end());
    tmp_par_.erase(std::unique(tmp_par_.begin(), tmp_par_.end()), tmp_par_.end());
    TaskRec& t = T(id);
    t.vertex = !tmp_par_.empty();
    t.par_off = static_cast<uint32_t>(par_pool_.size());
    t.par_n = static_cast<uint32_t>(tmp_par_.size());
    par_pool_.insert(par_pool_.end(), tmp_par_.begin(), tmp_par_.end());
    *wait_on = tmp_par_;
    return id;
  }

  uint64_t add_sync() {
    const uint64_t id = base_ + tasks_.size();
    tasks_.emplace_back();
    tasks_.back().kind = TK_SYNC;
    return id;
  }

  // Retire the parents of host access `id` and all their ancestors.
  // Retired tasks are appended to *retired (may be null).
  void retire(uint64_t id, std::vector<uint64_t>* retired) {
    stack_.assign(parents(id), parents(id) + task(id).par_n);
    retire_stack(retired);
  }

  // Retire every active task.
  void retire_all(std::vector<uint64_t>* retired) {
    stack_.clear();
    for (uint64_t t : active_list_)
      if (T(t).active) stack_.push_back(t);
    retire_stack(retired);
    active_list_.clear();
  }

 private:
  TaskRec& T(uint64_t id) { return tasks_[id - base_]; }
  const TaskRec& T(uint64_t id) const { return tasks_[id - base_]; }

  void add_edge(uint64_t src, uint64_t dst, uint32_t slot, uint32_t kind,
                std::vector<uint64_t>* par) {
    edges_.push_back(EdgeRec{src, dst, slot, kind});
    par->push_back(src);
  }

  void collect_edges(uint64_t id, const Access& a, std::vector<uint64_t>* par) {
    BufTrack& b = bufs_[a.buf];
    if (a.acc == ACC_W) {
      if (b.read_since_write) {
        for (uint64_t r : b.R)
          if (T(r).active) add_edge(r, id, a.buf, 1u, par);
      } else if (b.W && T(b.W).active) {
        add_edge(b.W, id, a.buf, 2u, par);
      }
    } else if (b.W && T(b.W).active) {
      add_edge(b.W, id, a.buf, 0u, par);
    }
  }

  void update_buffer(uint64_t id, const Access& a) {
    BufTrack& b = bufs_[a.buf];
    if (a.acc == ACC_W) {
      b.W = id;
      b.R.clear();
      b.read_since_write = false;
    } else {
      if (b.R.size() >= 32) {
        size_t k = 0;
        for (uint64_t r : b.R)
          if (T(r).active) b.R[k++] = r;
        b.R.resize(k);
      }
      b.R.push_back(id);
      b.read_since_write = true;
    }
  }

  int32_t new_stream(bool* created, uint8_t lane = 0) {
    streams_.emplace_back();
    streams_.back().lane = lane;
    if (!lane) ++npool_;
    *created = true;
    return static_cast<int32_t>(streams_.size() - 1);
  }

  // Copies of one direction rotate over that direction's lanes.
  int32_t pick_lane(uint8_t dir, bool* created) {
    *created = false;
    const uint32_t k = lane_next_[dir]++ % lanes_per_dir_;
    int32_t& ls = lane_stream_[dir * kMaxLanesPerDir + k];
    if (ls < 0) ls = new_stream(created, dir);
    return ls;
  }

  int32_t pick_serial(bool* created) {
    *created = false;
    if (streams_.empty()) return new_stream(created);
    return 0;
  }

  int32_t pick_stream(bool* created) {
    *created = false;
    int32_t chosen = -1;
    const uint64_t* par = par_pool_.data() + tasks_.back().par_off;
    const uint32_t np = tasks_.back().par_n;
    for (uint32_t i = 0; i < np; ++i) {
      const int32_t s = T(par[i]).stream;
      if (streams_[s].lane) continue;  // calls never join a copy lane
      if (streams_[s].tail == par[i]) {
        chosen = s;
        break;
      }
    }
    if (chosen < 0) {
      while (!fifo_.empty() && !streams_[fifo_.front()].in_fifo) fifo_.pop_front();
      if (!fifo_.empty()) {
        chosen = fifo_.front();
        fifo_.pop_front();
      }
    }
    if (chosen < 0 && npool_ < max_streams_) chosen = new_stream(created);
    if (chosen < 0) {
      for (uint32_t s = 0; s < streams_.size(); ++s) {
        if (streams_[s].lane) continue;
        if (chosen < 0 || streams_[s].tail < streams_[chosen].tail) chosen = static_cast<int32_t>(s);
      }
    }
    streams_[chosen].in_fifo = false;  // lazily dropped from fifo_
    return chosen;
  }

  void place(uint64_t id, int32_t s) {
    StreamRec& st = streams_[s];
    const uint32_t ns = static_cast<uint32_t>(streams_.size());
    if (st.vc.size() < ns) st.vc.resize(ns, 0);
    // event waits: newest parent per other stream, newest first, skipping
    // those already ordered before this point
    TaskRec& t = T(id);
    const uint64_t* par = par_pool_.data() + t.par_off;
    cand_.clear();
    for (uint32_t i = 0; i < t.par_n; ++i) {
      const TaskRec& p = T(par[i]);
      if (p.stream == s) continue;
      bool replaced = false;
      for (uint64_t& c : cand_) {
        if (T(c).stream == p.stream) {
          if (par[i] > c) c = par[i];
          replaced = true;
          break;
        }
      }
      if (!replaced) cand_.push_back(par[i]);
    }
    std::sort(cand_.begin(), cand_.end(), [](uint64_t a, uint64_t b) { return a > b; });
    t.wait_off = static_cast<uint32_t>(wait_pool_.size());
    t.wait_n = 0;
    for (uint64_t c : cand_) {
      const TaskRec& p = T(c);
      if (st.vc[p.stream] >= p.pos) continue;
      wait_pool_.push_back(c);
      ++t.wait_n;
      for (uint32_t k = 0; k < p.vc_n; ++k)
        st.vc[k] = std::max(st.vc[k], vc_pool_[p.vc_off + k]);
    }
    std::sort(wait_pool_.begin() + t.wait_off, wait_pool_.end());
    t.stream = s;
    t.pos = ++st.npos;
    st.vc[s] = t.pos;
    t.vc_off = static_cast<uint32_t>(vc_pool_.size());
    t.vc_n = static_cast<uint32_t>(st.vc.size());
    vc_pool_.insert(vc_pool_.end(), st.vc.begin(), st.vc.end());
    st.tail = id;
    ++st.nactive;
    t.active = true;
    ++nactive_total_;
    active_list_.push_back(id);
    if (active_list_.size() > 64 && active_list_.size() > 2 * nactive_total_) {
      size_t k = 0;
      for (uint64_t a : active_list_)
        if (T(a).active) active_list_[k++] = a;
      active_list_.resize(k);
    }
  }

  void retire_stack(std::vector<uint64_t>* retired) {
    empties_.clear();
    while (!stack_.empty()) {
      const uint64_t x = stack_.back();
      stack_.pop_back();
      TaskRec& t = T(x);
      if (!t.active) continue;
      t.active = false;
      --nactive_total_;
      if (retired) retired->push_back(x);
      StreamRec& st = streams_[t.stream];
      if (--st.nactive == 0 && !st.lane) empties_.push_back(t.stream);
      const uint64_t* par = par_pool_.data() + t.par_off;
      stack_.insert(stack_.end(), par, par + t.par_n);
    }
    std::sort(empties_.begin(), empties_.end());
    for (int32_t s : empties_) {
      if (!streams_[s].in_fifo) {
        streams_[s].in_fifo = true;
        fifo_.push_back(s);
      }
    }
  }

  uint32_t max_streams_;
  uint32_t lanes_per_dir_;
  uint32_t npool_ = 0;
  int32_t lane_stream_[3 * kMaxLanesPerDir] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
  uint32_t lane_next_[3] = {0, 0, 0};
  std::vector<TaskRec> tasks_;
  std::vector<BufTrack> bufs_;
  std::vector<StreamRec> streams_;
  std::deque<int32_t> fifo_;
  std::vector<EdgeRec> edges_;
  std::vector<uint64_t> par_pool_, wait_pool_;
  std::vector<uint32_t> vc_pool_;
  std::vector<uint64_t> active_list_;
  uint64_t nactive_total_ = 0;
  uint64_t base_ = 0;
  uint64_t dropped_vertices_ = 0, dropped_edges_ = 0;
  std::vector<uint64_t> tmp_par_, cand_, stack_;
  std::vector<int32_t> empties_;
};

}  // namespace dagrt
