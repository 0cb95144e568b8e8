// Continuous-batching request loop over the persistent batched launch.
//
// The scheduler is written against a small executor interface so the same
// admission / budget / batching logic drives the GPU (a pooled mtp_batch) or a
// host-only stand-in with synthetic launch durations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mtp.h"
#include "batch.hpp"
#include "plan_internal.hpp"

using namespace mtp;

namespace {

uint64_t now_ns() {
  return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                   std::chrono::steady_clock::now().time_since_epoch())
                                   .count());
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// First-fit allocator over [0, size) with coalescing; 256-byte granules.
class Pool {
 public:
  explicit Pool(size_t size) : size_(size) {
    if (size > 0) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest > 0) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  size_t size_;
  size_t used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct LaunchEntry {
  int robot;
  int k_begin, k_end;
  int shift;
  uint32_t r;
};

// What the scheduler needs from a device.
class Executor {
 public:
  virtual ~Executor() {}
  virtual int max_slots() const = 0;
  virtual void set_slab(int robot, size_t pool_off) = 0;
  virtual void set_x0(int robot, const float* x0) = 0;
  virtual mtp_status launch(int slot, const std::vector<LaunchEntry>& entries) = 0;
  virtual bool ready(int slot) = 0;
  virtual mtp_status wait(int slot, int wait_us, bool* done) = 0;
  virtual mtp_status result(int slot, int robot, float* u) = 0;
  virtual std::string error() const = 0;
};

class GpuExecutor : public Executor {
 public:
  GpuExecutor(mtp_batch* b, const std::vector<mtp_config>& cfgs, float* d_x0, int slots)
      : b_(b), cfgs_(cfgs), d_x0_(d_x0), slots_(slots) {}
  ~GpuExecutor() override {
    for (auto& s : ring_) {
      if (s.ev) (void)hipEventDestroy(s.ev);
      if (s.out) (void)hipHostFree(s.out);
      if (s.x0) (void)hipHostFree(s.x0);
    }
    if (b_) mtp_batch_destroy(b_);
  }
  mtp_status init() {
    x0_off_.resize(cfgs_.size());
    act_off_.resize(cfgs_.size());
    int xo = 0, ao = 0;
    for (size_t i = 0; i < cfgs_.size(); ++i) {
      x0_off_[i] = xo;
      act_off_[i] = ao;
      xo += cfgs_[i].state_dim;
      ao += cfgs_[i].ctrl_dim;
    }
    x0_total_ = xo;
    host_x0_.assign(xo, 0.0f);
    ring_.resize(slots_);
    for (auto& s : ring_) {
      hipError_t e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
      if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s.out), sizeof(float) * (batch_act_total(b_) + 4), hipHostMallocDefault);
      if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s.x0), sizeof(float) * std::max(xo, 1), hipHostMallocDefault);
      if (e != hipSuccess) {
        err_ = hipGetErrorString(e);
        return MTP_ERR_DEVICE;
      }
    }
    return MTP_OK;
  }
  int max_slots() const override { return slots_; }
  void set_slab(int robot, size_t pool_off) override { batch_set_transient(b_, robot, batch_pool_base(b_) + pool_off); }
  void set_x0(int robot, const float* x0) override {
    std::memcpy(host_x0_.data() + x0_off_[robot], x0, sizeof(float) * cfgs_[robot].state_dim);
  }
  mtp_status launch(int slot, const std::vector<LaunchEntry>& es) override {
    Slot& s = ring_[slot];
    // the slot's previous launch has been retired, so its staging buffers are free
    std::memcpy(s.x0, host_x0_.data(), sizeof(float) * x0_total_);
    hipError_t e = hipMemcpyAsync(d_x0_, s.x0, sizeof(float) * x0_total_, hipMemcpyHostToDevice, batch_stream(b_));
    if (e != hipSuccess) {
      err_ = std::string("x0 copy: ") + hipGetErrorString(e);
      return MTP_ERR_DEVICE;
    }
    std::vector<int32_t> act(es.size()), kb(es.size()), ke(es.size()), sh(es.size());
    std::vector<uint32_t> rr(es.size());
    for (size_t a = 0; a < es.size(); ++a) {
      act[a] = es[a].robot;
      kb[a] = es[a].k_begin;
      ke[a] = es[a].k_end;
      sh[a] = es[a].shift;
      rr[a] = es[a].r;
    }
    mtp_status st = mtp_batch_step(b_, static_cast<int32_t>(es.size()), act.data(), kb.data(), ke.data(), sh.data(),
                                   rr.data(), d_x0_);
    if (st == MTP_OK) st = batch_enqueue_readback(b_, s.out, s.ev);
    if (st != MTP_OK) err_ = batch_error(b_);
    s.n_active = static_cast<int>(es.size());
    return st;
  }
  bool ready(int slot) override { return hipEventQuery(ring_[slot].ev) == hipSuccess; }
  mtp_status wait(int slot, int wait_us, bool* done) override {
    const uint64_t t0 = now_ns();
    for (;;) {
      const hipError_t e = hipEventQuery(ring_[slot].ev);
      if (e == hipSuccess) { *done = true; return check(slot); }
      if (e != hipErrorNotReady) {
        err_ = hipGetErrorString(e);
        return MTP_ERR_DEVICE;
      }
      if (now_ns() - t0 > static_cast<uint64_t>(wait_us) * 1000ull) { *done = false; return MTP_OK; }
    }
  }
  mtp_status result(int slot, int robot, float* u) override {
    std::memcpy(u, ring_[slot].out + act_off_[robot], sizeof(float) * cfgs_[robot].ctrl_dim);
    return MTP_OK;
  }
  std::string error() const override { return err_; }

 private:
  mtp_status check(int slot) {
    uint32_t st[3];
    std::memcpy(st, ring_[slot].out + batch_act_total(b_), sizeof(st));
    if (st[0] != 0u || st[1] != static_cast<uint32_t>(ring_[slot].n_active)) {
      err_ = "persistent launch did not complete cleanly";
      return MTP_ERR_DEVICE;
    }
    return MTP_OK;
  }
  struct Slot {
    hipEvent_t ev = nullptr;
    float* out = nullptr;
    float* x0 = nullptr;
    int n_active = 0;
  };
  mtp_batch* b_;
  std::vector<mtp_config> cfgs_;
  float* d_x0_;
  int slots_;
  std::vector<Slot> ring_;
  std::vector<int> x0_off_, act_off_;
  int x0_total_ = 0;
  std::vector<float> host_x0_;
  std::string err_;
};

class SimExecutor : public Executor {
 public:
  SimExecutor(const std::vector<mtp_config>& cfgs, int slots, double ns_per_step)
      : cfgs_(cfgs), slots_(slots), ns_(ns_per_step), end_(slots, 0) {}
  int max_slots() const override { return slots_; }
  void set_slab(int, size_t) override {}
  void set_x0(int, const float*) override {}
  mtp_status launch(int slot, const std::vector<LaunchEntry>& es) override {
    double work = 0.0;
    for (const auto& e : es)
      work += static_cast<double>(cfgs_[e.robot].n_tensor + cfgs_[e.robot].n_gauss) * cfgs_[e.robot].horizon *
              (e.k_end - e.k_begin);
    const uint64_t start = std::max(now_ns(), busy_until_);
    busy_until_ = start + 20000ull + static_cast<uint64_t>(work * ns_);
    end_[slot] = busy_until_;
    return MTP_OK;
  }
  bool ready(int slot) override { return now_ns() >= end_[slot]; }
  mtp_status wait(int slot, int wait_us, bool* done) override {
    const uint64_t t0 = now_ns();
    while (!ready(slot)) {
      if (now_ns() - t0 > static_cast<uint64_t>(wait_us) * 1000ull) { *done = false; return MTP_OK; }
    }
    *done = true;
    return MTP_OK;
  }
  mtp_status result(int, int robot, float* u) override {
    std::fill(u, u + cfgs_[robot].ctrl_dim, 0.0f);
    return MTP_OK;
  }
  std::string error() const override { return ""; }

 private:
  std::vector<mtp_config> cfgs_;
  int slots_;
  double ns_;
  std::vector<uint64_t> end_;
  uint64_t busy_until_ = 0;
};

struct Request {
  uint64_t ticket;
  int robot;
  int shift;
  uint64_t t_arrival;
  std::vector<float> x0;
};

struct ActiveReq {
  uint64_t ticket;
  int robot;
  int shift;
  uint64_t t_arrival, t_admit;
  uint32_t r;
  int k_sched;
  size_t slab;
};

struct InFlight {
  int slot;
  std::vector<LaunchEntry> entries;
  std::vector<uint64_t> finishing;   // tickets whose last iteration is in this launch
};

}  // namespace

struct mtp_server {
  std::vector<mtp_config> cfgs;
  std::vector<std::vector<float>> task, sparams;
  std::unique_ptr<Executor> ex;
  std::unique_ptr<Pool> pool;
  std::vector<size_t> slab_bytes;
  int iters_per_launch = 1;
  size_t resident_bytes = 0;
  // robots
  std::vector<uint32_t> next_r;
  std::vector<char> busy;
  // queues
  std::mutex mu;                       // guards `waiting`, `done`, counters read by stats
  std::deque<Request> waiting;
  std::vector<mtp_completion> done;
  std::map<uint64_t, ActiveReq> active;
  std::deque<InFlight> inflight;
  std::vector<char> slot_used;
  uint64_t next_ticket = 1;
  mtp_server_stats st{};
  bool sticky = false;
  std::string err;
};

static void copy_configs(mtp_server* s, const mtp_config* robots, int32_t n) {
  s->cfgs.assign(robots, robots + n);
  s->task.resize(n);
  s->sparams.resize(n);
  for (int i = 0; i < n; ++i) {
    mtp_config& c = s->cfgs[i];
    s->task[i].assign(c.task_params, c.task_params + c.n_task_params);
    c.task_params = s->task[i].data();
    if (c.dynamics == MTP_DYN_CHAIN_CONTACT) {
      const size_t B = static_cast<size_t>(c.n_tensor) + c.n_gauss;
      s->sparams[i].assign(c.sample_params, c.sample_params + B * (c.ctrl_dim + 1) * static_cast<size_t>(c.n_replicas > 1 ? c.n_replicas : 1));
      c.sample_params = s->sparams[i].data();
    } else {
      c.sample_params = nullptr;
    }
  }
  s->next_r.assign(n, 0u);
  s->busy.assign(n, 0);
  s->slab_bytes.resize(n);
  for (int i = 0; i < n; ++i) s->slab_bytes[i] = compute_layout(s->cfgs[i]).transient;
}

static bool check_robots(const mtp_config* robots, int32_t n, std::string* why, mtp_status* code) {
  if (robots == nullptr || n < 1) {
    *why = "need at least one robot";
    *code = MTP_ERR_INVALID_ARG;
    return false;
  }
  for (int i = 0; i < n; ++i) {
    if (!validate_config(&robots[i], why, code)) {
      *why = "robot " + std::to_string(i) + ": " + *why;
      return false;
    }
    if (robots[i].ctrl_dim > 32) {
      *why = "serving supports ctrl_dim <= 32";
      *code = MTP_ERR_UNSUPPORTED;
      return false;
    }
  }
  return true;
}

// Retire one launch: deliver results of requests that finished in it.
static mtp_status retire(mtp_server* s, int* n_completed) {
  InFlight f = std::move(s->inflight.front());
  s->inflight.pop_front();
  s->slot_used[f.slot] = 0;
  const uint64_t t = now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  for (uint64_t tk : f.finishing) {
    auto it = s->active.find(tk);
    if (it == s->active.end()) continue;
    ActiveReq& a = it->second;
    mtp_completion c{};
    c.ticket = a.ticket;
    c.robot = a.robot;
    c.status = MTP_OK;
    c.t_arrival_ns = a.t_arrival;
    c.t_admit_ns = a.t_admit;
    c.t_done_ns = t;
    c.replan_idx = a.r;
    c.n = s->cfgs[a.robot].ctrl_dim;
    if (s->ex->result(f.slot, a.robot, c.u) != MTP_OK) c.status = MTP_ERR_DEVICE;
    s->done.push_back(c);
    s->pool->release(a.slab, s->slab_bytes[a.robot]);
    s->busy[a.robot] = 0;
    s->active.erase(it);
    s->st.completed += 1;
    if (n_completed) *n_completed += 1;
  }
  return MTP_OK;
}

extern "C" {

uint64_t mtp_server_now_ns(void) { return now_ns(); }

size_t mtp_server_workspace_bytes(const mtp_config* robots, int32_t n_robots, size_t pool_bytes,
                                  int32_t iters_per_launch) {
  std::string why;
  mtp_status code;
  if (!check_robots(robots, n_robots, &why, &code) || iters_per_launch < 1 || pool_bytes == 0) return 0;
  size_t x0 = 0;
  for (int i = 0; i < n_robots; ++i) x0 += robots[i].state_dim;
  const size_t b = batch_workspace_bytes_pooled(robots, n_robots, align256(pool_bytes), iters_per_launch);
  return b == 0 ? 0 : b + align256(x0 * sizeof(float));
}

mtp_status mtp_server_create(const mtp_config* robots, int32_t n_robots, void* d_workspace, size_t ws_bytes,
                             size_t pool_bytes, int32_t iters_per_launch, int32_t max_inflight, void* hip_stream,
                             mtp_server** out) {
  if (out == nullptr) return MTP_ERR_INVALID_ARG;
  *out = nullptr;
  std::string why;
  mtp_status code = MTP_OK;
  if (!check_robots(robots, n_robots, &why, &code)) return code;
  if (iters_per_launch < 1 || max_inflight < 1 || max_inflight > 8 || pool_bytes == 0) return MTP_ERR_INVALID_ARG;
  pool_bytes = align256(pool_bytes);
  const size_t need = mtp_server_workspace_bytes(robots, n_robots, pool_bytes, iters_per_launch);
  if (d_workspace == nullptr || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) != 0)
    return MTP_ERR_WORKSPACE;
  mtp_server* s = new (std::nothrow) mtp_server();
  if (s == nullptr) return MTP_ERR_INVALID_ARG;
  copy_configs(s, robots, n_robots);
  const size_t bbytes = batch_workspace_bytes_pooled(robots, n_robots, pool_bytes, iters_per_launch);
  mtp_batch* b = nullptr;
  code = batch_create_internal(s->cfgs.data(), n_robots, d_workspace, bbytes, hip_stream, pool_bytes,
                               iters_per_launch, &b, &why);
  if (code != MTP_OK) {
    delete s;
    return code;
  }
  s->resident_bytes = batch_resident_bytes(b);
  float* d_x0 = reinterpret_cast<float*>(static_cast<uint8_t*>(d_workspace) + bbytes);
  auto* gx = new (std::nothrow) GpuExecutor(b, s->cfgs, d_x0, max_inflight);
  if (gx == nullptr) {
    mtp_batch_destroy(b);
    delete s;
    return MTP_ERR_INVALID_ARG;
  }
  s->ex.reset(gx);
  if (gx->init() != MTP_OK) {
    delete s;
    return MTP_ERR_DEVICE;
  }
  s->pool.reset(new Pool(pool_bytes));
  s->iters_per_launch = iters_per_launch;
  s->slot_used.assign(max_inflight, 0);
  s->st.pool_bytes = pool_bytes;
  s->st.resident_bytes = s->resident_bytes;
  *out = s;
  return MTP_OK;
}

mtp_status mtp_server_create_simulated(const mtp_config* robots, int32_t n_robots, size_t pool_bytes,
                                       int32_t iters_per_launch, int32_t max_inflight, double ns_per_sample_step,
                                       mtp_server** out) {
  if (out == nullptr) return MTP_ERR_INVALID_ARG;
  *out = nullptr;
  std::string why;
  mtp_status code = MTP_OK;
  if (!check_robots(robots, n_robots, &why, &code)) return code;
  if (iters_per_launch < 1 || max_inflight < 1 || max_inflight > 8 || pool_bytes == 0 || !(ns_per_sample_step >= 0.0))
    return MTP_ERR_INVALID_ARG;
  mtp_server* s = new (std::nothrow) mtp_server();
  if (s == nullptr) return MTP_ERR_INVALID_ARG;
  copy_configs(s, robots, n_robots);
  s->ex.reset(new SimExecutor(s->cfgs, max_inflight, ns_per_sample_step));
  s->pool.reset(new Pool(align256(pool_bytes)));
  s->iters_per_launch = iters_per_launch;
  s->slot_used.assign(max_inflight, 0);
  s->st.pool_bytes = align256(pool_bytes);
  *out = s;
  return MTP_OK;
}

mtp_status mtp_server_submit(mtp_server* s, int32_t robot, const float* h_x0, int32_t shift, uint64_t t_arrival_ns,
                             uint64_t* ticket) {
  if (s == nullptr || h_x0 == nullptr || robot < 0 || robot >= static_cast<int32_t>(s->cfgs.size()) || shift < 0)
    return MTP_ERR_INVALID_ARG;
  if (s->slab_bytes[robot] > s->pool->size()) {
    s->err = "this robot's transient workspace is larger than the whole pool";
    return MTP_ERR_INVALID_ARG;
  }
  Request q;
  q.robot = robot;
  q.shift = shift;
  q.t_arrival = t_arrival_ns;
  q.x0.assign(h_x0, h_x0 + s->cfgs[robot].state_dim);
  std::lock_guard<std::mutex> lk(s->mu);
  q.ticket = s->next_ticket++;
  if (ticket) *ticket = q.ticket;
  s->waiting.push_back(std::move(q));
  s->st.submitted += 1;
  return MTP_OK;
}

mtp_status mtp_server_pump(mtp_server* s, int32_t wait_us, int32_t* n_completed) {
  if (s == nullptr) return MTP_ERR_INVALID_ARG;
  if (n_completed) *n_completed = 0;
  if (s->sticky) return MTP_ERR_DEVICE;
  // 1. retire finished launches in order
  bool retired = false;
  while (!s->inflight.empty() && s->ex->ready(s->inflight.front().slot)) {
    bool done = false;
    mtp_status st = s->ex->wait(s->inflight.front().slot, 0, &done);
    if (st != MTP_OK) { s->sticky = true; s->err = s->ex->error(); return st; }
    retire(s, n_completed);
    retired = true;
  }
  if (!retired && wait_us > 0 && !s->inflight.empty() &&
      static_cast<int>(s->inflight.size()) >= s->ex->max_slots()) {
    bool done = false;
    mtp_status st = s->ex->wait(s->inflight.front().slot, wait_us, &done);
    if (st != MTP_OK) { s->sticky = true; s->err = s->ex->error(); return st; }
    if (done) retire(s, n_completed);
  }
  // 2. admit waiting requests in arrival order while slabs fit
  {
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<char> blocked(s->cfgs.size(), 0);
    bool budget_stop = false;
    for (auto it = s->waiting.begin(); it != s->waiting.end();) {
      const int r = it->robot;
      if (s->busy[r] || blocked[r]) { blocked[r] = 1; ++it; continue; }   // one request per robot, in order
      if (budget_stop) { ++it; continue; }
      size_t off = 0;
      if (!s->pool->alloc(s->slab_bytes[r], &off)) {
        s->st.deferred_for_budget += 1;
        budget_stop = true;      // keep arrival order under memory pressure
        ++it;
        continue;
      }
      ActiveReq a;
      a.ticket = it->ticket;
      a.robot = r;
      a.shift = it->shift;
      a.t_arrival = it->t_arrival;
      a.t_admit = now_ns();
      a.r = s->next_r[r]++;
      a.k_sched = 0;
      a.slab = off;
      s->ex->set_slab(r, off);
      s->ex->set_x0(r, it->x0.data());
      s->busy[r] = 1;
      s->active.emplace(a.ticket, a);
      s->st.admitted += 1;
      it = s->waiting.erase(it);
    }
  }
  // 3. launch the next continuous batch
  if (static_cast<int>(s->inflight.size()) < s->ex->max_slots()) {
    InFlight f;
    for (auto& kv : s->active) {
      ActiveReq& a = kv.second;
      const int K = s->cfgs[a.robot].n_iters;
      if (a.k_sched >= K) continue;
      LaunchEntry e;
      e.robot = a.robot;
      e.k_begin = a.k_sched;
      e.k_end = std::min(K, a.k_sched + s->iters_per_launch);
      e.shift = a.shift;
      e.r = a.r;
      f.entries.push_back(e);
      if (e.k_end == K) f.finishing.push_back(a.ticket);
    }
    if (!f.entries.empty()) {
      int slot = 0;
      while (s->slot_used[slot]) ++slot;
      f.slot = slot;
      const mtp_status st = s->ex->launch(slot, f.entries);
      if (st != MTP_OK) { s->sticky = true; s->err = s->ex->error(); return st; }
      s->slot_used[slot] = 1;
      for (auto& kv : s->active) {
        ActiveReq& a = kv.second;
        const int K = s->cfgs[a.robot].n_iters;
        if (a.k_sched < K) a.k_sched = std::min(K, a.k_sched + s->iters_per_launch);
      }
      s->inflight.push_back(std::move(f));
      s->st.launches += 1;
    }
  }
  return MTP_OK;
}

mtp_status mtp_server_poll(mtp_server* s, mtp_completion* out, int32_t max, int32_t* n_out) {
  if (s == nullptr || n_out == nullptr || (max > 0 && out == nullptr) || max < 0) return MTP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  const int32_t n = std::min<int32_t>(max, static_cast<int32_t>(s->done.size()));
  for (int32_t i = 0; i < n; ++i) out[i] = s->done[i];
  s->done.erase(s->done.begin(), s->done.begin() + n);
  *n_out = n;
  return MTP_OK;
}

mtp_status mtp_server_get_stats(const mtp_server* sc, mtp_server_stats* out) {
  mtp_server* s = const_cast<mtp_server*>(sc);
  if (s == nullptr || out == nullptr) return MTP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->pool_in_use = s->pool->used();
  out->pool_peak = s->pool->peak();
  out->queued = static_cast<int32_t>(s->waiting.size());
  out->in_flight = static_cast<int32_t>(s->active.size());
  return MTP_OK;
}

mtp_status mtp_server_destroy(mtp_server* s) {
  if (s == nullptr) return MTP_ERR_INVALID_ARG;
  delete s;
  return MTP_OK;
}

const char* mtp_server_last_error(const mtp_server* s) { return s ? s->err.c_str() : "no server"; }

}  // extern "C"
