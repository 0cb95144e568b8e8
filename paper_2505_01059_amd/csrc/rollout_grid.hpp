// Device pieces shared by the single-plan rollout kernels (kernels.hip and
// rollout_quad.hip): the block remap, the tensor-path generator run by the
// workgroups a rollout launch adds, and the occupancy target of the two builds.
#pragma once

#include "mtp_device.hpp"

namespace mtp {

// The dispatcher hands workgroup g to XCD g mod 8, and each XCD has its own L2.
// Giving each XCD one contiguous run of workgroup indices keeps the U rows of
// neighbouring candidates, and the lines they share, in one L2.  A bijection of
// [0, G) for any G.
__device__ __forceinline__ int xcd_contiguous_block(int g, int G) {
  constexpr int kXcds = 8;
  const int x = g % kXcds, i = g / kXcds;
  const int per = G / kXcds, rem = G % kXcds;
  return x * per + min(x, rem) + i;
}

// Workgroups of a rollout launch beyond P.roll_blocks, each alone on its
// compute unit (the launch asks for enough LDS to keep one workgroup per unit),
// draw the tensor-path controls of iteration P.gen_k into P.U2 on the units the
// rollout leaves idle: items (tensor tile, joint) over the whole horizon.
__device__ __forceinline__ void gen_tensor_tiles(const PlanDesc& P) {
  extern __shared__ float gen_lds[];
  const CandView v = cand_view_dyn(gen_lds, P.L, P.W, P.T < kTChunk ? P.T : kTChunk);
  PlanDesc Q = P;
  Q.U = P.U2;
  const int first = (P.G - 1) / kCandThreads;                  // tile of the first tensor path
  const int last = (P.G - 1 + P.P - 1) / kCandThreads;         // tile of the last one
  const int items = (last - first + 1) * P.n;
  const int gens = static_cast<int>(gridDim.x) - P.roll_blocks;
  // drawing for the next replan: its index and iteration 0, leaving Z and I
  const uint32_t r = P.ctrl[0] + (P.gen_spec ? 1u : 0u);
  const int mode = P.gen_spec ? kCandTensorAhead : kCandTensor;
  for (int it = static_cast<int>(blockIdx.x) - P.roll_blocks; it < items; it += gens) {
    const int tile = first + it / P.n, j = it - (it / P.n) * P.n;
    cand_tile(Q, r, P.gen_k, j, tile * kCandThreads, 0, P.T, v, mode);
  }
}

// Rollout kernels come in two builds.  ONE: the launch puts at most one
// workgroup (one wave per SIMD) on a compute unit, so the compiler is told to
// schedule for a single resident wave (more registers, more independent work
// in flight); otherwise the usual occupancy target.
#define MTP_ROLL_WAVES(one) __attribute__((amdgpu_waves_per_eu(1, (one) ? 1 : 8)))

}  // namespace mtp
