// Time-sliced pair-lane rollout kernels (long chains whose pair-lane waves
// outnumber the SIMDs) and their launcher.  A unit of its own: these kernels
// run one wave per SIMD with long dependent chains in every lane, and LLVM's
// iterative ILP machine scheduler hides more of their latency than the default
// (24-link contact chain: 3756 -> 3640 us per launch).
#include "kernels.hpp"
#include "rollout_grid.hpp"

namespace mtp {

// Every wave of the grid is a worker.
constexpr uint64_t kSegWaitTicks = 1000000000ull;   // 10 s of the 100 MHz wall clock

// EQ: every link has the same length (P.eq_len), held once instead of per link.
template <int N, bool CONTACT, bool EQ>
__global__ __launch_bounds__(kRollThreads) MTP_ROLL_WAVES(N >= 20) void k_rollout_pair_seg(PlanDesc P) {
  rollout_pair_segmented<N, CONTACT, EQ>(P, P.seg_ctl, P.seg_done, P.seg_state, P.seg_S, P.seg_len, kSegWaitTicks);
  if (threadIdx.x == 0 && __hip_atomic_load(&P.seg_ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
    atomicOr(&P.ctrl[2], 4u);
}

// New launch of the time-sliced rollout: next epoch, unit counter and error cleared.
__global__ __launch_bounds__(64) void k_seg_init(SegCtl* ctl) {
  if (threadIdx.x == 0) {
    ctl->head = 0u;
    ctl->error = 0u;
    ctl->epoch = ctl->epoch + 1u;
  }
}

hipError_t launch_rollout_seg(const PlanDesc& P, hipStream_t st) {
  k_seg_init<<<1, 64, 0, st>>>(P.seg_ctl);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (P.dyn == kChain) {
    switch (P.n_links) {
#define X(N)                                                                                         \
  case N:                                                                                            \
    if constexpr (pair_chain_links<N>()) {                                                           \
      if (P.eq_len) k_rollout_pair_seg<N, false, true><<<P.seg_grid, kRollThreads, 0, st>>>(P);      \
      else k_rollout_pair_seg<N, false, false><<<P.seg_grid, kRollThreads, 0, st>>>(P);              \
      return hipGetLastError();                                                                      \
    }                                                                                                \
    break;
      MTP_CHAIN_LINKS(X)
#undef X
      default: break;
    }
    return hipErrorInvalidValue;
  }
  switch (P.n_links) {
#define X(N)                                                                                         \
  case N:                                                                                            \
    if constexpr (pair_chain_links<N>()) {                                                           \
      if (P.eq_len) k_rollout_pair_seg<N, true, true><<<P.seg_grid, kRollThreads, 0, st>>>(P);       \
      else k_rollout_pair_seg<N, true, false><<<P.seg_grid, kRollThreads, 0, st>>>(P);               \
      return hipGetLastError();                                                                      \
    }                                                                                                \
    break;
    MTP_CONTACT_LINKS(X)
#undef X
    default: break;
  }
  return hipErrorInvalidValue;
}

template <typename F>
static hipError_t seg_grid_for(F kernel, const PlanDesc& P, int* grid) {
  int dev = 0, cus = 0, occ = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, kRollThreads, 0);
  if (e != hipSuccess) return e;
  *grid = (occ > 0 ? occ : 1) * (cus > 0 ? cus : 1);
  (void)P;
  return hipSuccess;
}

hipError_t seg_configure(PlanDesc* P) {
  if (P->seg_ctl == nullptr) return hipSuccess;
  int grid = 0;
  hipError_t e = hipErrorInvalidValue;
  const bool contact = P->dyn == kChainContact;
  switch (P->n_links) {
#define X(N)                                                                                              \
  case N:                                                                                                 \
    if constexpr (pair_chain_links<N>()) {                                                                \
      if (P->eq_len)                                                                                      \
        e = contact ? seg_grid_for(k_rollout_pair_seg<N, true, true>, *P, &grid)                          \
                    : seg_grid_for(k_rollout_pair_seg<N, false, true>, *P, &grid);                        \
      else                                                                                                \
        e = contact ? seg_grid_for(k_rollout_pair_seg<N, true, false>, *P, &grid)                         \
                    : seg_grid_for(k_rollout_pair_seg<N, false, false>, *P, &grid);                       \
    }                                                                                                     \
    break;
    MTP_CHAIN_LINKS(X)
#undef X
    default: break;
  }
  if (e != hipSuccess) return e;
  const int groups = (P->B + 31) / 32;
  P->seg_S = segment_count(groups, grid * (kRollThreads / 64));
  P->seg_len = (P->T + P->seg_S - 1) / P->seg_S;
  P->seg_S = (P->T + P->seg_len - 1) / P->seg_len;   // no empty trailing segment
  P->seg_grid = grid;
  return hipSuccess;
}

}  // namespace mtp
