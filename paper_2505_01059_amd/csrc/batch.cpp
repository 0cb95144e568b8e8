// Host side of the persistent batched launch: workspace layout for many
// instances, queue sizing, staging of per-launch parameters through pinned
// memory, hipGraph capture of the persistent kernel, and the schedule
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mtp.h"
#include "batch.hpp"
#include "plan_internal.hpp"

using namespace mtp;

namespace {

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Rough relative work of one CEM iteration, for longest-first ordering.
double work_estimate(const mtp_config& c) {
  const double B = static_cast<double>(c.n_tensor) + c.n_gauss;
  double per_step = 180.0;
  if (c.dynamics != MTP_DYN_POINT_MASS) per_step = 186.0 * c.n_links - 108.0 + 12.0 * c.n_links;
  if (c.dynamics == MTP_DYN_CHAIN_CONTACT) per_step += 96.0 * c.n_links;
  return B * c.horizon * per_step * c.n_iters;
}

uint32_t items_for(const mtp_config& c, int k_begin, int k_end, uint32_t shape) {
  const int B = c.n_tensor + c.n_gauss;
  const bool quad = is_quad_chain(c.dynamics, c.n_links);
  const bool pair = is_pair_chain(c.dynamics, c.n_links);
  const bool wor = c.sample_wor != 0;
  uint32_t per_iter = 0;
  for (uint32_t ph = kPhPaths; ph <= kPhUpd; ++ph)
    per_iter += phase_items(B, c.n_tensor, c.horizon, c.ctrl_dim, ph, quad, pair, wor, shape);
  return 1u + per_iter * static_cast<uint32_t>(k_end - k_begin);
}

uint32_t log2_of(int v) {
  uint32_t l = 0;
  while ((1 << (l + 1)) <= v) ++l;
  return l;
}

// Item shape of a loaded launch under schedule s.
uint32_t coarse_shape(const mtp_batch_schedule& s) {
  return make_shape(log2_of(s.cand_tiles), 0u, log2_of(s.roll_tiles), log2_of(s.refit_outputs));
}

struct BatchLayout {
  size_t ctl, descs, ictl, order, out, queue, ready, inst0;
  std::vector<size_t> res, tr;
  std::vector<Layout> lays;
  uint32_t capacity;
  int32_t x0_total, act_total;
  size_t total;
};

bool batch_layout(const mtp_config* cfgs, int32_t n, BatchLayout* L, std::string* why, mtp_status* code) {
  if (cfgs == nullptr || n < 1 || n > 65536) {
    if (why) *why = "need 1..65536 configs";
    if (code) *code = MTP_ERR_INVALID_ARG;
    return false;
  }
  L->lays.clear();
  L->capacity = 0;
  L->x0_total = 0;
  L->act_total = 0;
  for (int i = 0; i < n; ++i) {
    std::string w;
    if (!validate_config(&cfgs[i], &w, code)) {
      if (why) *why = "config " + std::to_string(i) + ": " + w;
      return false;
    }
    L->lays.push_back(compute_layout(cfgs[i]));
    L->capacity += items_for(cfgs[i], 0, cfgs[i].n_iters, kShapeFinest);   // sized for the most items
    L->x0_total += cfgs[i].state_dim;
    L->act_total += cfgs[i].ctrl_dim;
  }
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
  L->ctl = take(sizeof(BatchCtl));
  L->descs = take(sizeof(PlanDesc) * n);
  L->ictl = take(sizeof(InstCtl) * n);
  L->order = take(sizeof(int32_t) * n);
  L->out = take(sizeof(float) * (L->act_total + 4));
  L->queue = take(sizeof(BatchItem) * L->capacity);
  L->ready = take(sizeof(uint32_t) * L->capacity);
  L->inst0 = off;
  L->res.resize(n);
  L->tr.resize(n);
  for (int i = 0; i < n; ++i) {
    L->res[i] = take(L->lays[i].resident);
    L->tr[i] = take(L->lays[i].transient);
  }
  L->total = off;
  return true;
}

// Tables of a batch whose instances are attached one by one (the server):
// max_inst slots, each with a fixed place in the packed start-state and
// action vectors, and a queue of `capacity` items.  Resident and transient
// memory of the instances comes from the caller (the server's pool).
bool batch_layout_dynamic(int32_t max_inst, uint32_t capacity, BatchLayout* L) {
  if (max_inst < 1 || max_inst > 65536 || capacity < 1) return false;
  L->lays.assign(max_inst, Layout{});
  L->capacity = capacity;
  L->x0_total = max_inst * kSlotX0;
  L->act_total = max_inst * kSlotAct;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
  L->ctl = take(sizeof(BatchCtl));
  L->descs = take(sizeof(PlanDesc) * max_inst);
  L->ictl = take(sizeof(InstCtl) * max_inst);
  L->order = take(sizeof(int32_t) * max_inst);
  L->out = take(sizeof(float) * (L->act_total + 4));
  L->queue = take(sizeof(BatchItem) * capacity);
  L->ready = take(sizeof(uint32_t) * capacity);
  L->inst0 = off;
  L->res.assign(max_inst, 0);
  L->tr.assign(max_inst, 0);
  L->total = off;
  return true;
}

}  // namespace

struct mtp_batch {
  int n = 0;
  std::vector<mtp_config> cfgs;
  std::vector<std::vector<float>> task, sparams;
  BatchLayout lay;
  std::vector<PlanDesc> descs;
  uint8_t* base = nullptr;
  hipStream_t stream = nullptr;
  // device views
  BatchCtl* d_ctl = nullptr;
  PlanDesc* d_descs = nullptr;
  InstCtl* d_ictl = nullptr;
  int32_t* d_order = nullptr;
  float* d_out = nullptr;
  BatchItem* d_queue = nullptr;
  uint32_t* d_ready = nullptr;
  // pinned staging
  InstCtl* h_ictl = nullptr;
  int32_t* h_order = nullptr;
  float* h_out = nullptr;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  // schedule
  int cu_count = 1, max_occ = 1, grid = 1;
  mtp_batch_schedule sched{0, 1, 1, 1, 64, 100};
  std::vector<int32_t> order_natural, order_longest;
  uint64_t wait_ticks = 0;
  bool use_graph = true;
  hipStream_t cap_stream = nullptr;
  // one captured launch per persistent grid size, kept until the batch is
  // destroyed (a schedule change selects another, it never destroys one that
  // may still be executing)
  struct GraphEntry {
    int grid;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  bool dynamic = false;   // instances attached and detached one by one (the server)
  int last_active = 0;
  uint32_t next_r = 0;
  bool descs_dirty = false;
  PlanDesc* h_descs = nullptr;   // pinned staging of the descriptor table (dynamic batches)
  bool sticky = false;
  std::string err;
};

static mtp_status bdev(mtp_batch* b, hipError_t e, const char* where) {
  b->sticky = true;
  b->err = std::string(where) + ": " + hipGetErrorString(e);
  return MTP_ERR_DEVICE;
}

#define BCHK(b, expr, where)                     \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return bdev(b, e_, where); \
  } while (0)

// Only at destroy, after the stream has drained.
static void drop_graphs(mtp_batch* b) {
  for (auto& g : b->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  b->graphs.clear();
}

static BatchLaunch launch_of(mtp_batch* b, int32_t n_active, uint32_t total, const float* x0) {
  BatchLaunch L;
  L.descs = b->d_descs;
  L.ictl = b->d_ictl;
  L.ctl = b->d_ctl;
  L.queue = b->d_queue;
  L.ready = b->d_ready;
  L.order = b->d_order;
  L.n_active = n_active;
  L.total = total;
  L.x0_packed = x0;
  L.wait_ticks = b->wait_ticks;
  return L;
}

static void apply_schedule(mtp_batch* b) {
  const int per_cu = b->sched.wg_per_cu > 0 ? std::min(b->sched.wg_per_cu, b->max_occ) : b->max_occ;
  b->grid = std::max(1, per_cu * b->cu_count);
}

static mtp_status ensure_graph(mtp_batch* b, hipGraphExec_t* exec) {
  for (const auto& g : b->graphs)
    if (g.grid == b->grid) {
      *exec = g.exec;
      return MTP_OK;
    }
  if (!b->cap_stream) BCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "stream create");
  BCHK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  const BatchLaunch L = launch_of(b, 0, 0, nullptr);
  hipError_t e = launch_batch_persistent(L, b->grid, b->cap_stream);
  if (e == hipSuccess) e = launch_batch_pack(L, b->d_out, b->n, b->lay.act_total, b->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
  if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return bdev(b, e, "capture"); }
  if (e2 != hipSuccess) return bdev(b, e2, "end capture");
  hipGraphExec_t x = nullptr;
  const hipError_t e3 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e3 != hipSuccess) {
    (void)hipGraphDestroy(g);
    return bdev(b, e3, "graph instantiate");
  }
  b->graphs.push_back({b->grid, g, x});
  *exec = x;
  return MTP_OK;
}

// Stage per-launch parameters (pinned -> device) and run one persistent launch.
static mtp_status run_launch(mtp_batch* b, int32_t n_active, uint32_t total, const float* d_x0) {
  if (b->staged_pending) BCHK(b, hipEventSynchronize(b->staged), "staging wait");
  if (b->descs_dirty) {
    if (b->h_descs == nullptr)
      BCHK(b, hipHostMalloc(reinterpret_cast<void**>(&b->h_descs), sizeof(PlanDesc) * b->n, hipHostMallocDefault),
           "desc staging");
    std::memcpy(b->h_descs, b->descs.data(), sizeof(PlanDesc) * b->n);
    BCHK(b, hipMemcpyAsync(b->d_descs, b->h_descs, sizeof(PlanDesc) * b->n, hipMemcpyHostToDevice, b->stream),
         "desc copy");
    b->descs_dirty = false;
  }
  BCHK(b, hipMemcpyAsync(b->d_ictl, b->h_ictl, sizeof(InstCtl) * b->n, hipMemcpyHostToDevice, b->stream), "ictl copy");
  BCHK(b, hipMemcpyAsync(b->d_order, b->h_order, sizeof(int32_t) * n_active, hipMemcpyHostToDevice, b->stream),
       "order copy");
  BCHK(b, hipEventRecord(b->staged, b->stream), "event");
  b->staged_pending = true;
  const BatchLaunch L = launch_of(b, n_active, total, d_x0);
  BCHK(b, launch_batch_prepare(L, b->stream), "prepare");
  if (b->use_graph) {
    hipGraphExec_t exec = nullptr;
    const mtp_status s = ensure_graph(b, &exec);
    if (s != MTP_OK) return s;
    BCHK(b, hipGraphLaunch(exec, b->stream), "graph launch");
  } else {
    BCHK(b, launch_batch_persistent(L, b->grid, b->stream), "persistent");
    BCHK(b, launch_batch_pack(L, b->d_out, b->n, b->lay.act_total, b->stream), "pack");
  }
  b->last_active = n_active;
  return MTP_OK;
}

static mtp_status reset_instances(mtp_batch* b) {
  for (int i = 0; i < b->n; ++i) {
    if (b->cfgs[i].horizon == 0) continue;   // an empty slot of a dynamic batch
    const mtp_status s = upload_plan_tables(b->cfgs[i], b->descs[i], b->task[i].data(),
                                            b->sparams[i].empty() ? nullptr : b->sparams[i].data(), b->stream,
                                            &b->err);
    if (s != MTP_OK) {
      b->sticky = true;
      return s;
    }
  }
  b->next_r = 0;
  return MTP_OK;
}

static void set_views(mtp_batch* b) {
  const BatchLayout& lay = b->lay;
  b->d_ctl = reinterpret_cast<BatchCtl*>(b->base + lay.ctl);
  b->d_descs = reinterpret_cast<PlanDesc*>(b->base + lay.descs);
  b->d_ictl = reinterpret_cast<InstCtl*>(b->base + lay.ictl);
  b->d_order = reinterpret_cast<int32_t*>(b->base + lay.order);
  b->d_out = reinterpret_cast<float*>(b->base + lay.out);
  b->d_queue = reinterpret_cast<BatchItem*>(b->base + lay.queue);
  b->d_ready = reinterpret_cast<uint32_t*>(b->base + lay.ready);
}

// Pinned staging, device query, schedule and the zeroed control block and
// ready flags; shared by both ways of creating a batch.
static mtp_status init_common(mtp_batch* b) {
  const int n = b->n;
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&b->h_ictl), sizeof(InstCtl) * n, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->h_order), sizeof(int32_t) * n, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&b->h_out), sizeof(float) * (b->lay.act_total + 4), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
  if (e != hipSuccess) return MTP_ERR_DEVICE;
  int dev = 0;
  e = hipGetDevice(&dev);
  int cus = 0, clk_khz = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return MTP_ERR_DEVICE;
  b->cu_count = std::max(1, cus);
  b->max_occ = std::max(1, batch_max_blocks_per_cu());
  // every wait of the persistent kernel gives up after 10 s of wall clock
  if (clk_khz <= 0) clk_khz = 100000;   // the constant-rate counter runs at 100 MHz on this family
  b->wait_ticks = static_cast<uint64_t>(clk_khz) * 1000ull * 10ull;
  apply_schedule(b);
  BatchCtl ctl{};
  ctl.capacity = b->lay.capacity;
  e = hipMemcpyAsync(b->d_descs, b->descs.data(), sizeof(PlanDesc) * n, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipMemsetAsync(b->d_ready, 0, sizeof(uint32_t) * b->lay.capacity, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return e == hipSuccess ? MTP_OK : MTP_ERR_DEVICE;
}

extern "C" {

size_t mtp_batch_workspace_bytes(const mtp_config* cfgs, int32_t n) {
  BatchLayout L;
  if (!batch_layout(cfgs, n, &L, nullptr, nullptr)) return 0;
  return L.total;
}

}  // extern "C"

static mtp_status batch_create_static(const mtp_config* cfgs, int32_t n, void* d_workspace, size_t ws_bytes,
                                      void* hip_stream, mtp_batch** out) {
  if (out == nullptr) return MTP_ERR_INVALID_ARG;
  *out = nullptr;
  BatchLayout lay;
  std::string why;
  mtp_status code = MTP_OK;
  if (!batch_layout(cfgs, n, &lay, &why, &code)) return code;
  if (d_workspace == nullptr || ws_bytes < lay.total || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) != 0)
    return MTP_ERR_WORKSPACE;
  mtp_batch* b = new (std::nothrow) mtp_batch();
  if (b == nullptr) return MTP_ERR_INVALID_ARG;
  b->n = n;
  b->lay = lay;
  b->base = static_cast<uint8_t*>(d_workspace);
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->cfgs.assign(cfgs, cfgs + n);
  b->task.resize(n);
  b->sparams.resize(n);
  b->descs.resize(n);
  for (int i = 0; i < n; ++i) {
    mtp_config& c = b->cfgs[i];
    b->task[i].assign(c.task_params, c.task_params + c.n_task_params);
    c.task_params = b->task[i].data();
    if (c.dynamics == MTP_DYN_CHAIN_CONTACT) {
      const size_t B = static_cast<size_t>(c.n_tensor) + c.n_gauss;
      b->sparams[i].assign(c.sample_params, c.sample_params + B * (c.ctrl_dim + 1) * static_cast<size_t>(c.n_replicas > 1 ? c.n_replicas : 1));
      c.sample_params = b->sparams[i].data();
    } else {
      c.sample_params = nullptr;
    }
    b->descs[i] = make_desc(c, lay.lays[i], b->base + lay.res[i], b->base + lay.tr[i]);
  }
  set_views(b);
  if (init_common(b) != MTP_OK) {
    mtp_batch_destroy(b);
    return MTP_ERR_DEVICE;
  }
  b->order_natural.resize(n);
  std::iota(b->order_natural.begin(), b->order_natural.end(), 0);
  b->order_longest = b->order_natural;
  std::stable_sort(b->order_longest.begin(), b->order_longest.end(), [&](int a, int c) {
    return work_estimate(b->cfgs[a]) > work_estimate(b->cfgs[c]);
  });
  if (reset_instances(b) != MTP_OK) {
    mtp_batch_destroy(b);
    return MTP_ERR_DEVICE;
  }
  *out = b;
  return MTP_OK;
}

size_t mtp::batch_dynamic_bytes(int32_t max_inst, uint32_t capacity) {
  BatchLayout L;
  return batch_layout_dynamic(max_inst, capacity, &L) ? L.total : 0;
}

mtp_status mtp::batch_create_dynamic(int32_t max_inst, uint32_t capacity, void* d_workspace, size_t ws_bytes,
                                     void* hip_stream, mtp_batch** out) {
  if (out == nullptr) return MTP_ERR_INVALID_ARG;
  *out = nullptr;
  BatchLayout lay;
  if (!batch_layout_dynamic(max_inst, capacity, &lay)) return MTP_ERR_INVALID_ARG;
  if (d_workspace == nullptr || ws_bytes < lay.total || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) != 0)
    return MTP_ERR_WORKSPACE;
  mtp_batch* b = new (std::nothrow) mtp_batch();
  if (b == nullptr) return MTP_ERR_INVALID_ARG;
  b->n = max_inst;
  b->lay = lay;
  b->base = static_cast<uint8_t*>(d_workspace);
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->cfgs.assign(max_inst, mtp_config{});
  b->task.resize(max_inst);
  b->sparams.resize(max_inst);
  b->descs.assign(max_inst, PlanDesc{});
  b->dynamic = true;
  set_views(b);
  if (init_common(b) != MTP_OK) {
    mtp_batch_destroy(b);
    return MTP_ERR_DEVICE;
  }
  *out = b;
  return MTP_OK;
}

mtp_status mtp::batch_attach(mtp_batch* b, int32_t i, const mtp_config& cfg, uint8_t* resident) {
  if (b == nullptr || !b->dynamic || i < 0 || i >= b->n || resident == nullptr) return MTP_ERR_INVALID_ARG;
  if (b->sticky) return MTP_ERR_DEVICE;
  if (cfg.state_dim > kSlotX0 || cfg.ctrl_dim > kSlotAct) {
    b->err = "an attached instance needs state_dim <= 64 and ctrl_dim <= 32";
    return MTP_ERR_UNSUPPORTED;
  }
  mtp_config c = cfg;
  b->task[i].assign(c.task_params, c.task_params + c.n_task_params);
  c.task_params = b->task[i].data();
  if (c.dynamics == MTP_DYN_CHAIN_CONTACT) {
    const size_t B = static_cast<size_t>(c.n_tensor) + c.n_gauss;
    b->sparams[i].assign(c.sample_params, c.sample_params + B * (c.ctrl_dim + 1) *
                                                             static_cast<size_t>(c.n_replicas > 1 ? c.n_replicas : 1));
    c.sample_params = b->sparams[i].data();
  } else {
    b->sparams[i].clear();
    c.sample_params = nullptr;
  }
  b->cfgs[i] = c;
  b->lay.lays[i] = compute_layout(c);
  b->descs[i] = make_desc(c, b->lay.lays[i], resident, nullptr);
  b->descs_dirty = true;
  const mtp_status s = upload_plan_tables(c, b->descs[i], b->task[i].data(),
                                          b->sparams[i].empty() ? nullptr : b->sparams[i].data(), b->stream, &b->err);
  if (s != MTP_OK) b->sticky = true;
  return s;
}

void mtp::batch_detach(mtp_batch* b, int32_t i) {
  if (b == nullptr || !b->dynamic || i < 0 || i >= b->n) return;
  b->cfgs[i] = mtp_config{};
  b->descs[i] = PlanDesc{};
  b->lay.lays[i] = Layout{};
  b->task[i].clear();
  b->sparams[i].clear();
  b->descs_dirty = true;
}

size_t mtp::batch_resident_bytes_of(const mtp_config& c) { return compute_layout(c).resident; }

mtp_status mtp::batch_copy_state(mtp_batch* b, int32_t i, float* d_mu, float* d_sigma) {
  if (b == nullptr || i < 0 || i >= b->n || b->cfgs[i].horizon == 0) return MTP_ERR_INVALID_ARG;
  if (b->sticky) return MTP_ERR_DEVICE;
  const size_t bytes = sizeof(float) * b->cfgs[i].horizon * b->cfgs[i].ctrl_dim;
  if (d_mu) BCHK(b, hipMemcpyAsync(d_mu, b->descs[i].mu, bytes, hipMemcpyDeviceToDevice, b->stream), "mu copy");
  if (d_sigma)
    BCHK(b, hipMemcpyAsync(d_sigma, b->descs[i].sigma, bytes, hipMemcpyDeviceToDevice, b->stream), "sigma copy");
  BCHK(b, hipStreamSynchronize(b->stream), "sync");
  return MTP_OK;
}

void mtp::batch_set_transient(mtp_batch* b, int i, uint8_t* base) {
  set_transient(&b->descs[i], b->cfgs[i], b->lay.lays[i], base);
  b->descs_dirty = true;
}

mtp_status mtp::batch_enqueue_readback(mtp_batch* b, float* h_dst, hipEvent_t done) {
  const size_t bytes = sizeof(float) * (b->lay.act_total + 4);
  BCHK(b, hipMemcpyAsync(h_dst, b->d_out, bytes, hipMemcpyDeviceToHost, b->stream), "readback");
  BCHK(b, hipEventRecord(done, b->stream), "event");
  return MTP_OK;
}

int mtp::batch_act_total(const mtp_batch* b) { return b->lay.act_total; }
const char* mtp::batch_error(const mtp_batch* b) { return b->err.c_str(); }
hipStream_t mtp::batch_stream(const mtp_batch* b) { return b->stream; }

extern "C" {

mtp_status mtp_batch_create(const mtp_config* cfgs, int32_t n, void* d_workspace, size_t ws_bytes, void* hip_stream,
                            mtp_batch** out) {
  return batch_create_static(cfgs, n, d_workspace, ws_bytes, hip_stream, out);
}

mtp_status mtp_batch_step(mtp_batch* b, int32_t n_active, const int32_t* h_active, const int32_t* h_k_begin,
                          const int32_t* h_k_end, const int32_t* h_shift, const uint32_t* h_r,
                          const float* d_x0_packed) {
  if (b == nullptr) return MTP_ERR_INVALID_ARG;
  if (b->sticky) return MTP_ERR_DEVICE;
  if (n_active < 0 || n_active > b->n || (n_active > 0 && (h_active == nullptr || h_k_begin == nullptr ||
                                                           h_k_end == nullptr || h_r == nullptr))) {
    b->err = "bad step arguments";
    return MTP_ERR_INVALID_ARG;
  }
  if (n_active == 0) return MTP_OK;
  if (b->staged_pending) BCHK(b, hipEventSynchronize(b->staged), "staging wait");
  b->staged_pending = false;
  std::vector<char> seen(b->n, 0);
  uint32_t total = 0;
  int x0_off = 0;
  std::vector<int32_t> x0_offsets(b->n);
  std::vector<int32_t> act_offsets(b->n);
  int act_off = 0;
  for (int i = 0; i < b->n; ++i) {
    x0_offsets[i] = b->dynamic ? i * kSlotX0 : x0_off;
    act_offsets[i] = b->dynamic ? i * kSlotAct : act_off;
    x0_off += b->cfgs[i].state_dim;
    act_off += b->cfgs[i].ctrl_dim;
  }
  for (int i = 0; i < b->n; ++i) {
    InstCtl& c = b->h_ictl[i];
    std::memset(&c, 0, sizeof(c));
    c.x0_off = -1;
    c.act_off = act_offsets[i];
  }
  for (int a = 0; a < n_active; ++a) {
    const int i = h_active[a];
    if (i < 0 || i >= b->n || seen[i]) {
      b->err = "active list has a bad or repeated instance";
      return MTP_ERR_INVALID_ARG;
    }
    seen[i] = 1;
    if (b->descs[i].U == nullptr) {
      b->err = "instance has no transient workspace assigned";
      return MTP_ERR_INVALID_ARG;
    }
    const int kb = h_k_begin[a], ke = h_k_end[a];
    if (kb < 0 || ke <= kb || ke > 65535) {
      b->err = "bad iteration range";
      return MTP_ERR_INVALID_ARG;
    }
    const int sh = h_shift ? h_shift[a] : 0;
    if (sh < 0) {
      b->err = "negative shift";
      return MTP_ERR_INVALID_ARG;
    }
    InstCtl& c = b->h_ictl[i];
    c.k_begin = static_cast<uint32_t>(kb);
    c.k_end = static_cast<uint32_t>(ke);
    c.r = h_r[a];
    c.shift = sh;
    c.x0_off = (d_x0_packed != nullptr && kb == 0) ? x0_offsets[i] : -1;
    b->h_order[a] = i;
  }
  // Few active instances leave most workgroups idle while their candidate
  // tiles run, each tile covering all joints one after another, and while
  // their refit items run many outputs each: then every (tile, joint) and
  // every four outputs become items of their own.  With many instances the
  // items stay large (far fewer of them through the one queue counter).
  uint64_t cand_tiles = 0;
  for (int a = 0; a < n_active; ++a) {
    const mtp_config& c = b->cfgs[h_active[a]];
    cand_tiles += static_cast<uint64_t>((c.n_tensor + c.n_gauss + kCandThreads - 1) / kCandThreads);
  }
  const bool light = cand_tiles * 100u < static_cast<uint64_t>(b->sched.split_pct) * static_cast<uint64_t>(b->grid);
  const uint32_t shape = light ? kShapeFinest : coarse_shape(b->sched);
  for (int a = 0; a < n_active; ++a) {
    const int i = h_active[a];
    b->h_ictl[i].shape = shape;
    total += items_for(b->cfgs[i], h_k_begin[a], h_k_end[a], shape);
  }
  if (total > b->lay.capacity) {
    b->err = "step needs more queue items than the batch was sized for";
    return MTP_ERR_INVALID_ARG;
  }
  return run_launch(b, n_active, total, d_x0_packed);
}

mtp_status mtp_batch_replan(mtp_batch* b, const float* d_x0_packed, const int32_t* h_shift) {
  if (b == nullptr) return MTP_ERR_INVALID_ARG;
  if (d_x0_packed == nullptr) {
    b->err = "d_x0_packed is NULL";
    return MTP_ERR_INVALID_ARG;
  }
  const std::vector<int32_t>& ord = b->sched.order == 1 ? b->order_longest : b->order_natural;
  std::vector<int32_t> kb(b->n, 0), ke(b->n), sh(b->n, 0);
  std::vector<uint32_t> rr(b->n, b->next_r);
  for (int a = 0; a < b->n; ++a) {
    const int i = ord[a];
    ke[a] = b->cfgs[i].n_iters;
    sh[a] = h_shift ? h_shift[i] : 0;
  }
  const mtp_status s = mtp_batch_step(b, b->n, ord.data(), kb.data(), ke.data(), sh.data(), rr.data(), d_x0_packed);
  if (s == MTP_OK) b->next_r += 1;
  return s;
}

mtp_status mtp_batch_get_actions(mtp_batch* b, float* h_u_packed) {
  if (b == nullptr || h_u_packed == nullptr) return MTP_ERR_INVALID_ARG;
  if (b->sticky) return MTP_ERR_DEVICE;
  const size_t bytes = sizeof(float) * (b->lay.act_total + 4);
  BCHK(b, hipMemcpyAsync(b->h_out, b->d_out, bytes, hipMemcpyDeviceToHost, b->stream), "actions copy");
  BCHK(b, hipStreamSynchronize(b->stream), "sync");
  uint32_t st[3];
  std::memcpy(st, b->h_out + b->lay.act_total, sizeof(st));
  if (st[0] != 0u) {
    b->sticky = true;
    b->err = st[0] & 2u ? "persistent launch: queue overflow" : "persistent launch: a queue wait timed out";
    return MTP_ERR_DEVICE;
  }
  if (st[1] != static_cast<uint32_t>(b->last_active)) {
    b->sticky = true;
    b->err = "persistent launch: not every instance finished";
    return MTP_ERR_DEVICE;
  }
  std::memcpy(h_u_packed, b->h_out, sizeof(float) * b->lay.act_total);
  return MTP_OK;
}

mtp_status mtp_batch_get_buffers(const mtp_batch* b, int32_t i, mtp_buffers* out) {
  if (b == nullptr || out == nullptr || i < 0 || i >= b->n) return MTP_ERR_INVALID_ARG;
  const PlanDesc& P = b->descs[i];
  out->Z = P.Z; out->I = P.I; out->U = P.U; out->cost = P.cost; out->elite_idx = P.eidx;
  out->elite_cost = P.ecost; out->weights = P.w; out->mu = P.mu; out->sigma = P.sigma; out->x0 = P.x0;
  out->action = P.action; out->X_dbg = P.X; out->entropy = P.entropy; out->ld_U = static_cast<size_t>(P.ldU);
  return MTP_OK;
}

mtp_status mtp_batch_set_state(mtp_batch* b, int32_t i, const float* d_mu, const float* d_sigma) {
  if (b == nullptr || i < 0 || i >= b->n || d_mu == nullptr || d_sigma == nullptr) return MTP_ERR_INVALID_ARG;
  if (b->sticky) return MTP_ERR_DEVICE;
  const size_t bytes = sizeof(float) * b->cfgs[i].horizon * b->cfgs[i].ctrl_dim;
  BCHK(b, hipMemcpyAsync(b->descs[i].mu, d_mu, bytes, hipMemcpyDeviceToDevice, b->stream), "mu copy");
  BCHK(b, hipMemcpyAsync(b->descs[i].sigma, d_sigma, bytes, hipMemcpyDeviceToDevice, b->stream), "sigma copy");
  return MTP_OK;
}

mtp_status mtp_batch_set_schedule(mtp_batch* b, int32_t wg_per_cu, int32_t order) {
  if (b == nullptr) return MTP_ERR_INVALID_ARG;
  mtp_batch_schedule s = b->sched;
  s.wg_per_cu = wg_per_cu;
  s.order = order;
  return mtp_batch_set_schedule_full(b, &s);
}

mtp_status mtp_batch_set_schedule_full(mtp_batch* b, const mtp_batch_schedule* h_schedule) {
  if (b == nullptr || h_schedule == nullptr || !schedule_valid(*h_schedule)) return MTP_ERR_INVALID_ARG;
  b->sched = *h_schedule;
  apply_schedule(b);
  return MTP_OK;
}

mtp_status mtp_batch_get_schedule(const mtp_batch* b, mtp_batch_schedule* h_schedule) {
  if (b == nullptr || h_schedule == nullptr) return MTP_ERR_INVALID_ARG;
  *h_schedule = b->sched;
  return MTP_OK;
}

mtp_status mtp_batch_set_graph_mode(mtp_batch* b, int32_t use_graph) {
  if (b == nullptr) return MTP_ERR_INVALID_ARG;
  b->use_graph = use_graph != 0;
  return MTP_OK;
}

}  // extern "C"

namespace {

// Milliseconds per whole replan of every instance under schedule s: one
// warm-up launch, then reps launches between two HIP events.  The instances'
// iterations run from their current state with replan index 0 (the caller
// resets them afterwards).
mtp_status time_schedule(mtp_batch* b, const mtp_batch_schedule& s, int reps, hipEvent_t e0, hipEvent_t e1,
                         float* ms) {
  mtp_status st = mtp_batch_set_schedule_full(b, &s);
  if (st != MTP_OK) return st;
  const std::vector<int32_t>& ord = s.order == 1 ? b->order_longest : b->order_natural;
  std::vector<int32_t> kb(b->n, 0), ke(b->n), sh(b->n, 0);
  std::vector<uint32_t> rr(b->n, 0);
  for (int a = 0; a < b->n; ++a) ke[a] = b->cfgs[ord[a]].n_iters;
  st = mtp_batch_step(b, b->n, ord.data(), kb.data(), ke.data(), sh.data(), rr.data(), nullptr);
  if (st != MTP_OK) return st;
  BCHK(b, hipEventRecord(e0, b->stream), "event");
  for (int r = 0; r < reps && st == MTP_OK; ++r)
    st = mtp_batch_step(b, b->n, ord.data(), kb.data(), ke.data(), sh.data(), rr.data(), nullptr);
  if (st != MTP_OK) return st;
  BCHK(b, hipEventRecord(e1, b->stream), "event");
  BCHK(b, hipEventSynchronize(e1), "event sync");
  float t = 0.0f;
  BCHK(b, hipEventElapsedTime(&t, e0, e1), "elapsed");
  *ms = t / static_cast<float>(reps);
  // the launches must have completed cleanly for their times to count
  std::vector<float> acts(b->lay.act_total);
  return mtp_batch_get_actions(b, acts.data());
}

struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

}  // namespace

extern "C" {

mtp_status mtp_batch_autotune(mtp_batch* b, int32_t reps, int32_t* h_choice, float* h_ms) {
  if (b == nullptr || reps < 1) return MTP_ERR_INVALID_ARG;
  if (b->sticky) return MTP_ERR_DEVICE;
  Events ev;
  BCHK(b, hipEventCreate(&ev.e0), "event");
  BCHK(b, hipEventCreate(&ev.e1), "event");
  float best = -1.0f;
  mtp_batch_schedule best_s = b->sched;
  for (int order = 0; order <= 1; ++order) {
    for (int wg = 1; wg <= b->max_occ; ++wg) {
      mtp_batch_schedule s = b->sched;
      s.wg_per_cu = wg;
      s.order = order;
      float ms = 0.0f;
      const mtp_status st = time_schedule(b, s, reps, ev.e0, ev.e1, &ms);
      if (st != MTP_OK) return st;
      if (best < 0.0f || ms < best) {
        best = ms;
        best_s = s;
      }
    }
  }
  mtp_batch_set_schedule_full(b, &best_s);
  if (h_choice) {
    h_choice[0] = best_s.wg_per_cu;
    h_choice[1] = best_s.order;
  }
  if (h_ms) *h_ms = best;
  return reset_instances(b);
}

mtp_status mtp_batch_tune(mtp_batch* b, int32_t reps, const char* cache_path, mtp_batch_schedule* h_out,
                          float* h_ms, int32_t* h_from_cache) {
  if (b == nullptr || reps < 1) return MTP_ERR_INVALID_ARG;
  if (b->dynamic) {
    b->err = "a batch without a fixed mix (the server's) cannot be tuned";
    return MTP_ERR_INVALID_ARG;
  }
  if (b->sticky) return MTP_ERR_DEVICE;
  if (h_from_cache) *h_from_cache = 0;
  int dev = 0;
  hipDeviceProp_t prop;
  BCHK(b, hipGetDevice(&dev), "device");
  BCHK(b, hipGetDeviceProperties(&prop, dev), "device properties");
  const std::string arch = prop.gcnArchName;
  const uint64_t mix = mtp_batch_mix_signature(b->cfgs.data(), b->n);
  if (cache_path != nullptr) {
    mtp_batch_schedule s;
    float ms = 0.0f;
    int32_t found = 0;
    if (mtp_schedule_cache_lookup(cache_path, arch.c_str(), b->cu_count, mix, &s, &ms, &found) == MTP_OK && found &&
        mtp_batch_set_schedule_full(b, &s) == MTP_OK) {
      if (h_out) *h_out = s;
      if (h_ms) *h_ms = ms;
      if (h_from_cache) *h_from_cache = 1;
      return MTP_OK;
    }
  }
  Events ev;
  BCHK(b, hipEventCreate(&ev.e0), "event");
  BCHK(b, hipEventCreate(&ev.e1), "event");
  // coordinate descent from the current schedule: one knob at a time, every
  // value of it with the others held; a change must win by 1 %
  mtp_batch_schedule best = b->sched;
  float best_ms = 0.0f;
  mtp_status st = time_schedule(b, best, reps, ev.e0, ev.e1, &best_ms);
  if (st != MTP_OK) return st;
  std::vector<int> wgs;
  for (int w = 1; w <= b->max_occ; ++w) wgs.push_back(w);
  const std::vector<int> orders{0, 1}, tiles{1, 2, 4}, outputs{4, 8, 16, 32, 64}, pcts{0, 25, 100, 400, 1 << 30};
  struct Knob {
    int32_t mtp_batch_schedule::*field;
    const std::vector<int>* values;
  };
  const Knob knobs[] = {{&mtp_batch_schedule::wg_per_cu, &wgs},       {&mtp_batch_schedule::order, &orders},
                        {&mtp_batch_schedule::split_pct, &pcts},      {&mtp_batch_schedule::cand_tiles, &tiles},
                        {&mtp_batch_schedule::roll_tiles, &tiles},    {&mtp_batch_schedule::refit_outputs, &outputs}};
  for (int sweep = 0; sweep < 3; ++sweep) {
    bool changed = false;
    for (const Knob& k : knobs) {
      for (const int v : *k.values) {
        if (best.*(k.field) == v) continue;
        mtp_batch_schedule s = best;
        s.*(k.field) = v;
        float ms = 0.0f;
        st = time_schedule(b, s, reps, ev.e0, ev.e1, &ms);
        if (st != MTP_OK) return st;
        if (ms < 0.99f * best_ms) {
          best = s;
          best_ms = ms;
          changed = true;
        }
      }
    }
    if (!changed) break;
  }
  mtp_batch_set_schedule_full(b, &best);
  if (cache_path != nullptr) {
    st = mtp_schedule_cache_store(cache_path, arch.c_str(), b->cu_count, mix, &best, best_ms);
    if (st != MTP_OK) {
      b->err = std::string("schedule cache not written: ") + cache_path;
      (void)reset_instances(b);
      return st;
    }
  }
  if (h_out) *h_out = best;
  if (h_ms) *h_ms = best_ms;
  return reset_instances(b);
}

mtp_status mtp_batch_destroy(mtp_batch* b) {
  if (b == nullptr) return MTP_ERR_INVALID_ARG;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->staged) (void)hipEventDestroy(b->staged);
  if (b->h_ictl) (void)hipHostFree(b->h_ictl);
  if (b->h_order) (void)hipHostFree(b->h_order);
  if (b->h_out) (void)hipHostFree(b->h_out);
  if (b->h_descs) (void)hipHostFree(b->h_descs);
  delete b;
  return MTP_OK;
}

const char* mtp_batch_last_error(const mtp_batch* b) { return b ? b->err.c_str() : "no batch"; }

}  // extern "C"
