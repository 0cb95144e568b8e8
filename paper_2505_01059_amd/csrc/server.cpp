// Continuous-batching request loop over the persistent batched launch.
//
// The scheduler is written against a small executor interface so the same
// admission / budget / batching logic drives the GPU (a batch whose instances
// are attached as robots are added) or a host-only stand-in with synthetic
// launch durations.
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
  virtual mtp_status attach(int robot, const mtp_config& cfg, size_t res_off) = 0;
  virtual void detach(int robot) = 0;
  virtual void set_slab(int robot, size_t pool_off) = 0;
  virtual void set_x0(int robot, const float* x0) = 0;
  virtual mtp_status launch(int slot, const std::vector<LaunchEntry>& entries) = 0;
  virtual bool ready(int slot) = 0;
  virtual mtp_status wait(int slot, int wait_us, bool* done) = 0;
  virtual mtp_status result(int slot, int robot, float* u) = 0;
  virtual mtp_status state(int robot, float* d_mu, float* d_sigma) = 0;
  virtual std::string error() const = 0;
};

// The device: a batch with one slot per robot; robots' resident buffers and
// the transient slabs of admitted requests both live in the pool.
class GpuExecutor : public Executor {
 public:
  GpuExecutor(mtp_batch* b, float* d_x0, uint8_t* pool, int max_robots, int slots)
      : b_(b), d_x0_(d_x0), pool_(pool), max_robots_(max_robots), slots_(slots) {}
  ~GpuExecutor() override {
    for (auto& s : ring_) {
      if (s.ev) (void)hipEventDestroy(s.ev);
      if (s.out) (void)hipHostFree(s.out);
      if (s.x0) (void)hipHostFree(s.x0);
    }
    if (b_) mtp_batch_destroy(b_);
  }
  mtp_status init() {
    host_x0_.assign(static_cast<size_t>(max_robots_) * kSlotX0, 0.0f);
    ring_.resize(slots_);
    for (auto& s : ring_) {
      hipError_t e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
      if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s.out), sizeof(float) * (batch_act_total(b_) + 4), hipHostMallocDefault);
      if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s.x0), sizeof(float) * host_x0_.size(), hipHostMallocDefault);
      if (e != hipSuccess) {
        err_ = hipGetErrorString(e);
        return MTP_ERR_DEVICE;
      }
    }
    return MTP_OK;
  }
  int max_slots() const override { return slots_; }
  mtp_status attach(int robot, const mtp_config& cfg, size_t res_off) override {
    dims_[robot] = {cfg.state_dim, cfg.ctrl_dim};
    const mtp_status st = batch_attach(b_, robot, cfg, pool_ + res_off);
    if (st != MTP_OK) err_ = batch_error(b_);
    return st;
  }
  void detach(int robot) override {
    batch_detach(b_, robot);
    dims_.erase(robot);
  }
  void set_slab(int robot, size_t pool_off) override { batch_set_transient(b_, robot, pool_ + pool_off); }
  void set_x0(int robot, const float* x0) override {
    std::memcpy(host_x0_.data() + static_cast<size_t>(robot) * kSlotX0, x0, sizeof(float) * dims_[robot].first);
  }
  mtp_status launch(int slot, const std::vector<LaunchEntry>& es) override {
    Slot& s = ring_[slot];
    // the slot's previous launch has been retired, so its staging buffers are free
    std::memcpy(s.x0, host_x0_.data(), sizeof(float) * host_x0_.size());
    hipError_t e = hipMemcpyAsync(d_x0_, s.x0, sizeof(float) * host_x0_.size(), hipMemcpyHostToDevice, batch_stream(b_));
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
    std::memcpy(u, ring_[slot].out + static_cast<size_t>(robot) * kSlotAct, sizeof(float) * dims_[robot].second);
    return MTP_OK;
  }
  mtp_status state(int robot, float* d_mu, float* d_sigma) override {
    const mtp_status st = batch_copy_state(b_, robot, d_mu, d_sigma);
    if (st != MTP_OK) err_ = batch_error(b_);
    return st;
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
  float* d_x0_;
  uint8_t* pool_;
  int max_robots_;
  int slots_;
  std::vector<Slot> ring_;
  std::map<int, std::pair<int, int>> dims_;   // robot -> (state_dim, ctrl_dim)
  std::vector<float> host_x0_;
  std::string err_;
};

// A host-only stand-in: a launch takes 20 us plus a time per candidate-step.
class SimExecutor : public Executor {
 public:
  SimExecutor(int slots, double ns_per_step) : slots_(slots), ns_(ns_per_step), end_(slots, 0) {}
  int max_slots() const override { return slots_; }
  mtp_status attach(int robot, const mtp_config& cfg, size_t) override {
    cfgs_[robot] = cfg;
    return MTP_OK;
  }
  void detach(int robot) override { cfgs_.erase(robot); }
  void set_slab(int, size_t) override {}
  void set_x0(int, const float*) override {}
  mtp_status launch(int slot, const std::vector<LaunchEntry>& es) override {
    double work = 0.0;
    for (const auto& e : es) {
      const mtp_config& c = cfgs_[e.robot];
      work += static_cast<double>(c.n_tensor + c.n_gauss) * c.horizon * (e.k_end - e.k_begin);
    }
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
  mtp_status state(int, float*, float*) override { return MTP_ERR_UNSUPPORTED; }
  std::string error() const override { return ""; }

 private:
  std::map<int, mtp_config> cfgs_;
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

enum RobotState : int { kFree = 0, kLive = 1, kRemoving = 2 };

struct Robot {
  RobotState state = kFree;
  mtp_config cfg{};
  std::vector<float> task, sparams;
  size_t res_off = 0, res_bytes = 0, slab_bytes = 0;
  uint32_t items = 0;      // queue items one launch may need for this robot
  uint32_t next_r = 0;
  bool busy = false;       // a request admitted and not yet retired
};

// Queue items one launch may need for a robot: iters_per_launch iterations in
// the finest item shape (the most items).
uint32_t launch_items(const mtp_config& c, int iters_per_launch) {
  const int B = c.n_tensor + c.n_gauss;
  const bool quad = is_quad_chain(c.dynamics, c.n_links);
  const bool pair = is_pair_chain(c.dynamics, c.n_links);
  uint32_t per = 1u;
  for (uint32_t ph = kPhPaths; ph <= kPhUpd; ++ph)
    per += phase_items(B, c.n_tensor, c.horizon, c.ctrl_dim, ph, quad, pair, c.sample_wor != 0, kShapeFinest);
  return 1u + per * static_cast<uint32_t>(std::min(iters_per_launch, c.n_iters));
}

}  // namespace

struct mtp_server {
  std::vector<Robot> robots;
  std::unique_ptr<Executor> ex;
  std::unique_ptr<Pool> pool;
  int iters_per_launch = 1;
  uint32_t queue_capacity = 0, queue_reserved = 0;
  // queues
  std::mutex mu;                       // guards robots' registry, `waiting`, `done`, counters read by stats
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

static void release_robot(mtp_server* s, int id) {
  Robot& rb = s->robots[id];
  s->pool->release(rb.res_off, rb.res_bytes);
  s->st.resident_bytes -= rb.res_bytes;
  s->queue_reserved -= rb.items;
  s->ex->detach(id);
  rb = Robot{};
}

// Retire one launch: deliver results of requests that finished in it (those of
// robots removed meanwhile are dropped) and free their slabs.
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
    Robot& rb = s->robots[a.robot];
    s->pool->release(a.slab, rb.slab_bytes);
    rb.busy = false;
    if (rb.state == kRemoving) {
      s->st.dropped += 1;
      release_robot(s, a.robot);
    } else {
      mtp_completion c{};
      c.ticket = a.ticket;
      c.robot = a.robot;
      c.status = MTP_OK;
      c.t_arrival_ns = a.t_arrival;
      c.t_admit_ns = a.t_admit;
      c.t_done_ns = t;
      c.replan_idx = a.r;
      c.n = rb.cfg.ctrl_dim;
      if (s->ex->result(f.slot, a.robot, c.u) != MTP_OK) c.status = MTP_ERR_DEVICE;
      s->done.push_back(c);
      s->st.completed += 1;
      if (n_completed) *n_completed += 1;
    }
    s->active.erase(it);
  }
  return MTP_OK;
}

static mtp_server* new_server(size_t budget, int32_t max_robots, uint32_t queue_items, int32_t iters_per_launch,
                              int32_t max_inflight) {
  mtp_server* s = new (std::nothrow) mtp_server();
  if (s == nullptr) return nullptr;
  s->robots.assign(max_robots, Robot{});
  s->pool.reset(new Pool(align256(budget)));
  s->iters_per_launch = iters_per_launch;
  s->queue_capacity = queue_items;
  s->slot_used.assign(max_inflight, 0);
  s->st.pool_bytes = align256(budget);
  return s;
}

static uint32_t queue_items_for(int32_t max_robots, uint32_t queue_items) {
  return queue_items > 0 ? queue_items : static_cast<uint32_t>(max_robots) * 4096u;
}

static bool server_args_ok(size_t budget, int32_t max_robots, int32_t iters_per_launch, int32_t max_inflight) {
  return budget > 0 && max_robots >= 1 && max_robots <= 65536 && iters_per_launch >= 1 && max_inflight >= 1 &&
         max_inflight <= 8;
}

extern "C" {

uint64_t mtp_server_now_ns(void) { return now_ns(); }

size_t mtp_server_workspace_bytes(size_t hbm_budget_bytes, int32_t max_robots, uint32_t queue_items) {
  if (!server_args_ok(hbm_budget_bytes, max_robots, 1, 1)) return 0;
  const size_t tables = batch_dynamic_bytes(max_robots, queue_items_for(max_robots, queue_items));
  if (tables == 0) return 0;
  return tables + align256(static_cast<size_t>(max_robots) * kSlotX0 * sizeof(float)) + align256(hbm_budget_bytes);
}

mtp_status mtp_server_create(size_t hbm_budget_bytes, int32_t max_robots, uint32_t queue_items,
                             int32_t iters_per_launch, int32_t max_inflight, void* d_workspace, size_t ws_bytes,
                             void* hip_stream, mtp_server** out) {
  if (out == nullptr) return MTP_ERR_INVALID_ARG;
  *out = nullptr;
  if (!server_args_ok(hbm_budget_bytes, max_robots, iters_per_launch, max_inflight)) return MTP_ERR_INVALID_ARG;
  const uint32_t cap = queue_items_for(max_robots, queue_items);
  const size_t need = mtp_server_workspace_bytes(hbm_budget_bytes, max_robots, queue_items);
  if (d_workspace == nullptr || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) != 0)
    return MTP_ERR_WORKSPACE;
  mtp_server* s = new_server(hbm_budget_bytes, max_robots, cap, iters_per_launch, max_inflight);
  if (s == nullptr) return MTP_ERR_INVALID_ARG;
  const size_t tables = batch_dynamic_bytes(max_robots, cap);
  mtp_batch* b = nullptr;
  mtp_status code = batch_create_dynamic(max_robots, cap, d_workspace, tables, hip_stream, &b);
  if (code != MTP_OK) {
    delete s;
    return code;
  }
  uint8_t* base = static_cast<uint8_t*>(d_workspace);
  float* d_x0 = reinterpret_cast<float*>(base + tables);
  uint8_t* pool = base + tables + align256(static_cast<size_t>(max_robots) * kSlotX0 * sizeof(float));
  auto* gx = new (std::nothrow) GpuExecutor(b, d_x0, pool, max_robots, max_inflight);
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
  *out = s;
  return MTP_OK;
}

mtp_status mtp_server_create_simulated(size_t hbm_budget_bytes, int32_t max_robots, uint32_t queue_items,
                                       int32_t iters_per_launch, int32_t max_inflight, double ns_per_sample_step,
                                       mtp_server** out) {
  if (out == nullptr) return MTP_ERR_INVALID_ARG;
  *out = nullptr;
  if (!server_args_ok(hbm_budget_bytes, max_robots, iters_per_launch, max_inflight) || !(ns_per_sample_step >= 0.0))
    return MTP_ERR_INVALID_ARG;
  mtp_server* s = new_server(hbm_budget_bytes, max_robots, queue_items_for(max_robots, queue_items),
                             iters_per_launch, max_inflight);
  if (s == nullptr) return MTP_ERR_INVALID_ARG;
  s->ex.reset(new SimExecutor(max_inflight, ns_per_sample_step));
  *out = s;
  return MTP_OK;
}

mtp_status mtp_server_add_robot(mtp_server* s, const mtp_config* cfg, int32_t* robot_id) {
  if (s == nullptr || cfg == nullptr || robot_id == nullptr) return MTP_ERR_INVALID_ARG;
  *robot_id = -1;
  if (s->sticky) return MTP_ERR_DEVICE;
  std::string why;
  mtp_status code = MTP_OK;
  if (!validate_config(cfg, &why, &code)) {
    s->err = why;
    return code;
  }
  if (cfg->ctrl_dim > kSlotAct || cfg->state_dim > kSlotX0) {
    s->err = "serving supports ctrl_dim <= 32 and state_dim <= 64";
    return MTP_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  int id = -1;
  for (int i = 0; i < static_cast<int>(s->robots.size()); ++i)
    if (s->robots[i].state == kFree) { id = i; break; }
  if (id < 0) {
    s->err = "every robot slot is taken";
    return MTP_ERR_BUSY;
  }
  Robot rb;
  rb.cfg = *cfg;
  rb.task.assign(cfg->task_params, cfg->task_params + cfg->n_task_params);
  rb.cfg.task_params = rb.task.data();
  if (cfg->dynamics == MTP_DYN_CHAIN_CONTACT) {
    const size_t B = static_cast<size_t>(cfg->n_tensor) + cfg->n_gauss;
    const size_t R = cfg->n_replicas > 1 ? static_cast<size_t>(cfg->n_replicas) : 1;
    rb.sparams.assign(cfg->sample_params, cfg->sample_params + R * B * (cfg->ctrl_dim + 1));
    rb.cfg.sample_params = rb.sparams.data();
  } else {
    rb.cfg.sample_params = nullptr;
  }
  const Layout lay = compute_layout(rb.cfg);
  rb.res_bytes = lay.resident;
  rb.slab_bytes = lay.transient;
  rb.items = launch_items(rb.cfg, s->iters_per_launch);
  if (rb.slab_bytes + rb.res_bytes > s->pool->size()) {
    s->err = "this robot needs more device memory than the whole budget";
    return MTP_ERR_INVALID_ARG;
  }
  if (s->queue_reserved + rb.items > s->queue_capacity) {
    s->err = "the launch queue is sized for fewer robots of this kind";
    return MTP_ERR_BUSY;
  }
  if (!s->pool->alloc(rb.res_bytes, &rb.res_off)) {
    s->err = "the device-memory budget is used up";
    return MTP_ERR_BUSY;
  }
  const mtp_status st = s->ex->attach(id, rb.cfg, rb.res_off);
  if (st != MTP_OK) {
    s->pool->release(rb.res_off, rb.res_bytes);
    s->err = s->ex->error();
    if (st == MTP_ERR_DEVICE) s->sticky = true;
    return st;
  }
  rb.state = kLive;
  s->queue_reserved += rb.items;
  s->st.resident_bytes += rb.res_bytes;
  s->st.robots += 1;
  s->robots[id] = std::move(rb);
  s->robots[id].cfg.task_params = s->robots[id].task.data();
  if (!s->robots[id].sparams.empty()) s->robots[id].cfg.sample_params = s->robots[id].sparams.data();
  *robot_id = id;
  return MTP_OK;
}

mtp_status mtp_server_remove_robot(mtp_server* s, int32_t robot) {
  if (s == nullptr) return MTP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (robot < 0 || robot >= static_cast<int32_t>(s->robots.size()) || s->robots[robot].state != kLive)
    return MTP_ERR_INVALID_ARG;
  for (auto it = s->waiting.begin(); it != s->waiting.end();) {
    if (it->robot == robot) {
      it = s->waiting.erase(it);
      s->st.dropped += 1;
    } else {
      ++it;
    }
  }
  s->st.robots -= 1;
  if (s->robots[robot].busy)
    s->robots[robot].state = kRemoving;   // memory released when its request's launch retires
  else
    release_robot(s, robot);
  return MTP_OK;
}

mtp_status mtp_server_get_robot_state(mtp_server* s, int32_t robot, float* d_mu, float* d_sigma,
                                      uint32_t* replan_idx) {
  if (s == nullptr) return MTP_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (robot < 0 || robot >= static_cast<int32_t>(s->robots.size()) || s->robots[robot].state != kLive)
      return MTP_ERR_INVALID_ARG;
    if (s->robots[robot].busy) return MTP_ERR_BUSY;
    if (replan_idx) *replan_idx = s->robots[robot].next_r;
  }
  if (d_mu == nullptr && d_sigma == nullptr) return MTP_OK;
  const mtp_status st = s->ex->state(robot, d_mu, d_sigma);
  if (st != MTP_OK) s->err = s->ex->error();
  return st;
}

mtp_status mtp_server_submit(mtp_server* s, int32_t robot, const float* h_x0, int32_t shift, uint64_t t_arrival_ns,
                             uint64_t* ticket) {
  if (s == nullptr || h_x0 == nullptr || shift < 0) return MTP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (robot < 0 || robot >= static_cast<int32_t>(s->robots.size()) || s->robots[robot].state != kLive) {
    s->err = "no such robot";
    return MTP_ERR_INVALID_ARG;
  }
  Request q;
  q.robot = robot;
  q.shift = shift;
  q.t_arrival = t_arrival_ns;
  q.x0.assign(h_x0, h_x0 + s->robots[robot].cfg.state_dim);
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
    std::vector<char> blocked(s->robots.size(), 0);
    bool budget_stop = false;
    for (auto it = s->waiting.begin(); it != s->waiting.end();) {
      const int r = it->robot;
      Robot& rb = s->robots[r];
      if (rb.busy || blocked[r]) { blocked[r] = 1; ++it; continue; }   // one request per robot, in order
      if (budget_stop) { ++it; continue; }
      size_t off = 0;
      if (!s->pool->alloc(rb.slab_bytes, &off)) {
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
      a.r = rb.next_r++;
      a.k_sched = 0;
      a.slab = off;
      s->ex->set_slab(r, off);
      s->ex->set_x0(r, it->x0.data());
      rb.busy = true;
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
      const int K = s->robots[a.robot].cfg.n_iters;
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
        const int K = s->robots[a.robot].cfg.n_iters;
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
