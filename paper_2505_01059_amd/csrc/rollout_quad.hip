// Quad-lane chain rollout kernels (5..8 links) and their launcher.  A unit of
// its own so that it can be compiled with its own scheduling options.
#include "kernels.hpp"
#include "rollout_grid.hpp"

namespace mtp {

template <int N, bool ONE>
__global__ __launch_bounds__(kRollThreads) MTP_ROLL_WAVES(ONE) void k_rollout_chain_quad(PlanDesc P) {
  if (static_cast<int>(blockIdx.x) >= P.roll_blocks) { gen_tensor_tiles(P); return; }
  const int g = xcd_contiguous_block(blockIdx.x, P.roll_blocks) * kRollThreads + threadIdx.x;
  const int b = g >> 2;
  if (b < P.B) rollout_chain_quad<N>(P, b, g & 3);
}

hipError_t launch_rollout_quad(const PlanDesc& P, dim3 grid, size_t lds, hipStream_t st, bool one) {
  switch (P.n_links) {
#define X(N)                                                                       \
  case N:                                                                          \
    if constexpr (quad_chain_links<N>()) {                                         \
      if (one) k_rollout_chain_quad<N, true><<<grid, kRollThreads, lds, st>>>(P);  \
      else k_rollout_chain_quad<N, false><<<grid, kRollThreads, lds, st>>>(P);     \
      return hipGetLastError();                                                    \
    }                                                                              \
    break;
    MTP_CHAIN_LINKS(X)
#undef X
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace mtp
