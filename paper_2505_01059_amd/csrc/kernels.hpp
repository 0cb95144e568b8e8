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
// Grid and segment count of the time-sliced pair-lane rollout for the current
// device (no-op for plans that do not use it).
hipError_t seg_configure(PlanDesc* P);
// defined in plan.cpp
int segment_count(int groups, int resident_waves);

}  // namespace mtp
