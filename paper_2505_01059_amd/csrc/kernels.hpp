// Host-callable launchers of the single-plan stage kernels (kernels.hip).
#pragma once

#include "mtp_device.hpp"

namespace mtp {

bool rollout_supported(int dyn, int n_links);
int supported_chain_links(int* out, int cap);

hipError_t launch_set_ctrl(const PlanDesc& P, uint32_t r, int shift, const float* x0_src, hipStream_t st);
hipError_t launch_shift(const PlanDesc& P, hipStream_t st);
// stage: 0 candidates, 1 rollout, 2 top-E, 3 refit (the replan index is read from P.ctrl[0])
hipError_t launch_stage(const PlanDesc& P, int stage, int k, hipStream_t st);
// A second stream that a launch sequence forks work onto and joins back from
// (fork / join events recorded on the streams; usable under graph capture).
struct SideLane {
  hipStream_t st;
  hipEvent_t fork, join;
};
// Stage of iteration k in a run of iterations [k0, k1) (next iteration's tensor
// paths drawn during the rollout when the plan has a second U buffer).  A
// time-sliced rollout fills every SIMD, so there the next tensor paths are drawn
// by a kernel of their own on `side`, beside the rollout (on `st` after it when
// side is null).
hipError_t launch_iteration_stage(const PlanDesc& P, int stage, int k, int k0, int k1, hipStream_t st,
                                  const SideLane* side = nullptr);
// Quad-lane chain rollout (rollout_quad.hip); one: the launch holds one
// workgroup per compute unit.
hipError_t launch_rollout_quad(const PlanDesc& P, dim3 grid, size_t lds, hipStream_t st, bool one);
// Time-sliced pair-lane rollout (rollout_seg.hip): epoch bump, then the
// persistent launch of P.seg_grid workgroups.
hipError_t launch_rollout_seg(const PlanDesc& P, hipStream_t st);
// Workgroups of the (not time-sliced) rollout kernel of a plan.
int rollout_blocks(const PlanDesc& P);
// Grid and segment count of the time-sliced pair-lane rollout for the current
// device (no-op for plans that do not use it).
hipError_t seg_configure(PlanDesc* P);
// Compute units of the current device: the workgroups of a rollout launch that
// also draws the next tensor paths, and the bound below which rollout launches
// keep one workgroup per unit.
hipError_t gen_configure(PlanDesc* P);
// defined in plan.cpp
int segment_count(int groups, int resident_waves);

}  // namespace mtp
