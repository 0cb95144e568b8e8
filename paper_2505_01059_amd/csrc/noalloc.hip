// One replan with no device allocation and no caller workspace, for callers
// that cannot allocate device memory (code under capture, tight serving loops,
// harnesses that forbid it).  Everything a replan needs besides its inputs and
// outputs (control block, start state, tables, graph, paths, candidates,
// costs, elites, time-slicing state) lives in a file-scope device array of
// kScratchBytes, laid out exactly as a plan's workspace.  Each device holds its
// own copy of the array for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress gives for that device.  Calls that
// overlap on one device share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/mtp.h"
#include "kernels.hpp"
#include "plan_internal.hpp"

namespace mtp {

constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device, looked up once per
// device with that device current.
hipError_t scratch_on_current_device(uint8_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace mtp

using namespace mtp;

extern "C" {

size_t mtp_noalloc_scratch_bytes(void) { return kScratchBytes; }

mtp_status mtp_replan_noalloc(const mtp_config* cfg, const float* d_x0, float* d_mu, float* d_sigma,
                              int32_t shift_steps, uint32_t replan_idx, float* d_action, void* hip_stream) {
  std::string why;
  mtp_status code = MTP_OK;
  if (!validate_config(cfg, &why, &code)) return code;
  if (d_x0 == nullptr || d_mu == nullptr || d_sigma == nullptr || d_action == nullptr || shift_steps < 0)
    return MTP_ERR_INVALID_ARG;
  // the plain launch sequence (no second candidate buffer): the same bits as a plan
  const Layout lay = compute_layout(*cfg, false);
  if (lay.total > kScratchBytes) return MTP_ERR_WORKSPACE;
  uint8_t* base = nullptr;
  if (scratch_on_current_device(&base) != hipSuccess) return MTP_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  PlanDesc P = make_desc(*cfg, lay, base, base + lay.resident);
  // tables, and everything that must start at zero (control block, time-slicing
  // counters and flags): the previous call's contents are not relied upon
  if (upload_plan_tables(*cfg, P, cfg->task_params, cfg->sample_params, st, &why) != MTP_OK) return MTP_ERR_DEVICE;
  if (seg_configure(&P) != hipSuccess || gen_configure(&P) != hipSuccess) return MTP_ERR_DEVICE;
  const size_t tn = sizeof(float) * static_cast<size_t>(cfg->horizon) * cfg->ctrl_dim;
  hipError_t e = hipMemcpyAsync(P.mu, d_mu, tn, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(P.sigma, d_sigma, tn, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = launch_set_ctrl(P, replan_idx, shift_steps, d_x0, st);
  if (e == hipSuccess) e = launch_shift(P, st);
  if (e == hipSuccess) e = enqueue_iterations(P, 0, cfg->n_iters, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_mu, P.mu, tn, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_sigma, P.sigma, tn, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_action, P.action, sizeof(float) * cfg->ctrl_dim, hipMemcpyDeviceToDevice, st);
  return e == hipSuccess ? MTP_OK : MTP_ERR_DEVICE;
}

}  // extern "C"
