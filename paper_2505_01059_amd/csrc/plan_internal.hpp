// Internal host-side helpers shared by the plan, batch and server objects.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/mtp.h"
#include "mtp_device.hpp"

namespace mtp {

// Byte offsets of every buffer of one plan inside its workspace (256-aligned).
struct Layout {
  size_t ldU;
  size_t ctrl, x0, mu, sigma, tmp, action, basis, span, task, sparams, Z, I, U, cost, eidx, ecost, w, X;
  size_t total;
};

bool validate_config(const mtp_config* c, std::string* why, mtp_status* code);
Layout compute_layout(const mtp_config& c);
void build_tables(const mtp_config& c, std::vector<float>* basis, std::vector<int32_t>* span);
mtp_status upload_plan_tables(const mtp_config& c, const PlanDesc& P, const float* task, const float* sparams,
                              hipStream_t st, std::string* err);
hipError_t enqueue_iterations(const PlanDesc& P, int k_begin, int k_end, hipStream_t st);

}  // namespace mtp
