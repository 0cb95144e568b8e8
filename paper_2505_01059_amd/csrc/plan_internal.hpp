// Internal host-side helpers shared by the plan, batch and server objects.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/mtp.h"
#include "mtp_device.hpp"

namespace mtp {

// Byte offsets of every buffer of one plan (256-aligned).  The resident part
// (control block, start state, warm start, tables) lives as long as the plan;
// the transient part (graph, paths, candidates, costs, elites) is only needed
// while a replan runs, so a server can lend it from a shared pool.  Resident
// offsets are relative to the resident base, transient ones to the transient
// base; a single plan places the transient part right after the resident one.
struct Layout {
  size_t ldU;
  size_t ctrl, x0, mu, sigma, tmp, action, basis, span, task, sparams, entropy, seg_ctl, seg_done;   // resident
  size_t Z, I, U, cost, eidx, ecost, w, X, seg_state, U2;                                   // transient
  bool segmented;   // the rollout is time-sliced (see uses_segmented_rollout)
  bool overlap;     // second U buffer: next tensor paths drawn during the rollout (see uses_gen_overlap)
  size_t resident, transient;
  size_t total;   // resident + transient
};

bool validate_config(const mtp_config* c, std::string* why, mtp_status* code);
// plan: the layout of a single plan (which may add the second U buffer); the
// batched kernel and the server's transient slabs use the plain one.
Layout compute_layout(const mtp_config& c, bool plan = false);
void build_tables(const mtp_config& c, std::vector<float>* basis, std::vector<int32_t>* span);
mtp_status upload_plan_tables(const mtp_config& c, const PlanDesc& P, const float* task, const float* sparams,
                              hipStream_t st, std::string* err);
struct SideLane;
hipError_t enqueue_iterations(const PlanDesc& P, int k_begin, int k_end, hipStream_t st,
                              const SideLane* side = nullptr);
PlanDesc make_desc(const mtp_config& c, const Layout& L, uint8_t* resident, uint8_t* transient);
// Point a descriptor's transient buffers at a new base.
void set_transient(PlanDesc* P, const mtp_config& c, const Layout& L, uint8_t* transient);
// Whether a plan's rollout runs time-sliced: even chains of >= 10 links (two lanes
// per candidate) without randomised replicas whose launch has more waves than
// the chip has SIMDs.
bool uses_segmented_rollout(const mtp_config& c);
// Whether a single plan draws the next iteration's tensor-path controls during
// each rollout: more than one iteration, with-replacement tensor paths, and
// either a time-sliced rollout (the paths are then drawn by a kernel of their
// own beside it) or a rollout that leaves at least 32 of the 256 compute units
// free (drawn by workgroups the rollout launch adds).
bool uses_gen_overlap(const mtp_config& c);
// Segments of the time-sliced rollout for a given number of resident waves.
int segment_count(int groups, int resident_waves);
// Rounds of the without-replacement path permutation: 2 L ceil(log2 W).
int perm_rounds(int L, int W);
// Time steps per candidate workgroup of the single-plan candidate kernel.
int cand_time_chunk(int B, int T, int n);

}  // namespace mtp
