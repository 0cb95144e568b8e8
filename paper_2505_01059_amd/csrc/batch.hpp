// Persistent batched launch: queue items, control blocks and host launchers.
#pragma once

#include <string>

#include "../../include/mtp.h"
#include "mtp_device.hpp"

namespace mtp {

constexpr int kBatchThreads = 256;       // workgroup of the persistent kernel
constexpr int kUpdOutputsPerTile = 64;   // refit outputs per queue item
constexpr int kUpdOutputsPerTileSplit = kBatchThreads / 64;   // ... with split items: one per wave

enum : uint32_t { kPhShift = 0, kPhPaths = 1, kPhCand = 2, kPhRoll = 3, kPhTopk = 4, kPhUpd = 5 };

struct BatchItem {
  uint32_t inst, phase, k, tile;   // phase: the stage in the low bits, the candidate split above
};
constexpr uint32_t kItemSplitShift = 16, kItemPhaseMask = 0xFFFFu;

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
  uint32_t cand_split; // 1: small items (candidates per (tile, joint), refit per 4 outputs), 0: large
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

// host mirror of the per-phase tile counts
inline uint32_t host_phase_tiles(int B, int P, int T, int n, uint32_t phase, bool quad, bool pair, bool wor,
                                 bool cand_split = false) {
  switch (phase) {
    case kPhShift: return 1u;
    case kPhPaths: return (P > 0 && wor) ? static_cast<uint32_t>((P + kCandThreads - 1) / kCandThreads) : 1u;
    case kPhCand:
      return static_cast<uint32_t>((B + kCandThreads - 1) / kCandThreads) * (cand_split ? static_cast<uint32_t>(n) : 1u);
    case kPhRoll: {
      const int per = quad ? kBatchThreads / 4 : (pair ? kBatchThreads / 2 : kBatchThreads);
      return static_cast<uint32_t>((B + per - 1) / per);
    }
    case kPhTopk: return 1u;
    default: {
      const int per = cand_split ? kUpdOutputsPerTileSplit : kUpdOutputsPerTile;
      return static_cast<uint32_t>((T * n + per - 1) / per);
    }
  }
}

}  // namespace mtp
