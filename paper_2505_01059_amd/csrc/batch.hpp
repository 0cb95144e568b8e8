// Persistent batched launch: queue items, control blocks and host launchers.
#pragma once

#include <string>

#include "../../include/mtp.h"
#include "mtp_device.hpp"

namespace mtp {

constexpr int kBatchThreads = 256;       // workgroup of the persistent kernel

enum : uint32_t { kPhShift = 0, kPhPaths = 1, kPhCand = 2, kPhRoll = 3, kPhTopk = 4, kPhUpd = 5 };

// Shape of an instance's queue items in one launch (how much work one item
// holds), packed in 16 bits:
//   bits 0-1  log2 of the candidate tiles (kCandThreads candidates each) per item
//   bit  2    a candidate item covers one joint of its tiles instead of all
//   bits 3-4  log2 of the rollout tiles (one workgroup's candidates each) per item
//   bits 5-7  log2 of the refit outputs (t, j) per item, 2..6
// The shape changes only which workgroup computes what: every candidate,
// rollout and refit output is computed by the same code from the same inputs.
__host__ __device__ constexpr uint32_t make_shape(uint32_t cand_lg, uint32_t cand_joint, uint32_t roll_lg,
                                                  uint32_t upd_lg) {
  return cand_lg | (cand_joint << 2) | (roll_lg << 3) | (upd_lg << 5);
}
__host__ __device__ constexpr uint32_t shape_cand_lg(uint32_t s) { return s & 3u; }
__host__ __device__ constexpr uint32_t shape_cand_joint(uint32_t s) { return (s >> 2) & 1u; }
__host__ __device__ constexpr uint32_t shape_roll_lg(uint32_t s) { return (s >> 3) & 3u; }
__host__ __device__ constexpr uint32_t shape_upd_lg(uint32_t s) { return (s >> 5) & 7u; }
// The most items: one joint of one candidate tile, one rollout tile and four
// refit outputs (one per wave) per item.  Queues are sized for this shape.
constexpr uint32_t kShapeFinest = make_shape(0, 1, 0, 2);
// The shape of loaded launches unless a schedule says otherwise: a candidate
// tile with all its joints, one rollout tile, 64 refit outputs per item.
constexpr uint32_t kShapeCoarseDefault = make_shape(0, 0, 0, 6);

struct BatchItem {
  uint32_t inst, phase, k, tile;   // phase: the stage in the low 16 bits, the item shape above
};
constexpr uint32_t kItemShapeShift = 16, kItemPhaseMask = 0xFFFFu;

// Items of one phase of an instance with B candidates (P tensor paths, horizon
// T, n joints) under item shape `shape`; the same function on host and device.
__host__ __device__ inline uint32_t phase_items(int B, int P, int T, int n, uint32_t phase, bool quad, bool pair,
                                                bool wor, uint32_t shape) {
  switch (phase) {
    case kPhShift: return 1u;
    case kPhPaths: return (P > 0 && wor) ? static_cast<uint32_t>((P + kCandThreads - 1) / kCandThreads) : 1u;
    case kPhCand: {
      const uint32_t tiles = static_cast<uint32_t>((B + kCandThreads - 1) / kCandThreads);
      const uint32_t per = 1u << shape_cand_lg(shape);
      return ((tiles + per - 1u) / per) * (shape_cand_joint(shape) ? static_cast<uint32_t>(n) : 1u);
    }
    case kPhRoll: {
      const int cands = quad ? kBatchThreads / 4 : (pair ? kBatchThreads / 2 : kBatchThreads);
      const uint32_t tiles = static_cast<uint32_t>((B + cands - 1) / cands);
      const uint32_t per = 1u << shape_roll_lg(shape);
      return (tiles + per - 1u) / per;
    }
    case kPhTopk: return 1u;
    default: {
      const uint32_t per = 1u << shape_upd_lg(shape);
      return (static_cast<uint32_t>(T * n) + per - 1u) / per;
    }
  }
}

struct BatchCtl {
  uint32_t head;       // next queue position to take
  uint32_t tail;       // next queue position to publish
  uint32_t total;      // items this launch will run
  uint32_t epoch;      // ready-flag value of this launch
  uint32_t finished;   // instances that completed their iterations
  uint32_t error;      // bit 0: a wait timed out, bit 1: queue overflow
  uint32_t capacity;   // queue length
  uint32_t pad;
};

struct InstCtl {
  uint32_t done;       // tiles of the current phase completed
  uint32_t k_begin;    // first CEM iteration this launch runs
  uint32_t k_end;      // one past the last
  uint32_t r;          // Philox replan index
  int32_t shift;       // warm-start shift applied when k_begin == 0
  int32_t x0_off;      // offset of this instance's x0 in the packed input (-1: keep)
  int32_t act_off;     // offset of its action in the packed output
  uint32_t shape;      // item shape of this launch (make_shape)
};

struct BatchLaunch {
  const PlanDesc* descs;
  InstCtl* ictl;
  BatchCtl* ctl;
  BatchItem* queue;
  uint32_t* ready;
  const int32_t* order;
  int32_t n_active;
  uint32_t total;
  const float* x0_packed;
  uint64_t wait_ticks;
};

hipError_t launch_batch_prepare(const BatchLaunch& L, hipStream_t st);
hipError_t launch_batch_persistent(const BatchLaunch& L, int grid, hipStream_t st);
hipError_t launch_batch_pack(const BatchLaunch& L, float* out, int32_t n_inst, int32_t status_off, hipStream_t st);
int batch_max_blocks_per_cu();
// Schedule values the persistent kernel supports (the ranges in mtp.h).
bool schedule_valid(const mtp_batch_schedule& s);

}  // namespace mtp

struct mtp_batch;

namespace mtp {

// Internal batch API used by the server.
// Batches whose instances come and go (the server): fixed slots, each with a
// place of kSlotX0 floats in the packed start states and kSlotAct in the packed
// actions; resident and transient memory is the caller's.
constexpr int kSlotX0 = 64, kSlotAct = 32;
size_t batch_dynamic_bytes(int32_t max_inst, uint32_t capacity);
mtp_status batch_create_dynamic(int32_t max_inst, uint32_t capacity, void* d_workspace, size_t ws_bytes,
                                void* hip_stream, mtp_batch** out);
// Place instance `cfg` in slot i with its resident buffers at `resident`
// (compute_layout(cfg).resident bytes, 256-aligned) and upload its tables;
// synchronises the batch's stream.
mtp_status batch_attach(mtp_batch* b, int32_t i, const mtp_config& cfg, uint8_t* resident);
void batch_detach(mtp_batch* b, int32_t i);
size_t batch_resident_bytes_of(const mtp_config& c);
// Copy slot i's warm-start mean and std (device to device) and synchronise.
mtp_status batch_copy_state(mtp_batch* b, int32_t i, float* d_mu, float* d_sigma);
void batch_set_transient(mtp_batch* b, int i, uint8_t* base);
mtp_status batch_enqueue_readback(mtp_batch* b, float* h_dst, hipEvent_t done);
int batch_act_total(const mtp_batch* b);
const char* batch_error(const mtp_batch* b);
hipStream_t batch_stream(const mtp_batch* b);

}  // namespace mtp
