// Single-plan kernels of one MTP replan for gfx950 and their host launchers.
// Each kernel is a thin grid over the stage tiles of mtp_device.hpp.
#include <algorithm>

#include "kernels.hpp"
#include "rollout_grid.hpp"

namespace mtp {

__global__ __launch_bounds__(64) void k_set_ctrl(PlanDesc P, uint32_t r, int shift, const float* x0_src) {
  set_ctrl_block(P, r, shift, x0_src);
}

// One workgroup (the shift is in place through a scratch copy and a barrier);
// 1024 threads keep four times as many loads in flight as 256.
__global__ __launch_bounds__(1024) void k_shift(PlanDesc P) {
  shift_block<1024>(P, static_cast<int>(P.ctrl[1]));
}

__global__ __launch_bounds__(kCandThreads) void k_paths(PlanDesc P, int k) {
  __shared__ PathSmem sm;
  path_tile(P, P.ctrl[0], k, blockIdx.x, gridDim.x, sm);
}

static int cand_chunk(const PlanDesc& P) { return P.tc < kTChunk ? P.tc : kTChunk; }

// grid (candidate tiles, joints, horizon chunks of P.tc steps); LDS sized for
// the plan so that several workgroups fit on a compute unit
__global__ __launch_bounds__(kCandThreads) void k_candidates(PlanDesc P, int k) {
  extern __shared__ float cand_lds[];
  // tensor paths already drawn by the previous replan: only the local samples
  // and the nominal are written, and tiles of tensor paths alone return
  const bool ahead = P.cand_skip && P.ctrl[4] != 0u;
  const int b0 = static_cast<int>(blockIdx.x) * kCandThreads;
  if (ahead && b0 >= P.G - 1 && b0 + kCandThreads <= P.B - 1) return;
  const CandView v = cand_view_dyn(cand_lds, P.L, P.W, P.tc < kTChunk ? P.tc : kTChunk);
  const int t_begin = blockIdx.z * P.tc;
  cand_tile(P, P.ctrl[0], k, blockIdx.y, b0, t_begin, min(P.T, t_begin + P.tc), v, ahead ? kCandLocal : kCandAll);
}

__global__ __launch_bounds__(kTopkThreads) void k_entropy(PlanDesc P, int k) {
  __shared__ EntropySmem sm;
  entropy_block<kTopkThreads>(P, k, sm);
}

// Rollout workgroups are four waves: the waves of one workgroup go to the four
// SIMDs of a compute unit, while single-wave workgroups sharing a unit were seen
// to stack two waves on one SIMD now and then, doubling the time of a launch
// with fewer waves than SIMDs.
template <bool ONE>
__global__ __launch_bounds__(kRollThreads) MTP_ROLL_WAVES(ONE) void k_rollout_point_mass(PlanDesc P) {
  if (static_cast<int>(blockIdx.x) >= P.roll_blocks) { gen_tensor_tiles(P); return; }
  __shared__ PointMassSmem sm;
  stage_obstacles(P, sm);
  __syncthreads();
  // eight lanes per candidate, each with an eighth of the obstacle table
  const int g = xcd_contiguous_block(blockIdx.x, P.roll_blocks) * kRollThreads + threadIdx.x;
  const int b = g / kPmLanes;
  if (b < P.B) rollout_point_mass_any<kPmLanes>(P, b, g % kPmLanes, sm);
}

template <int N, bool CONTACT, bool ONE>
__global__ __launch_bounds__(kRollThreads) MTP_ROLL_WAVES(ONE) void k_rollout_chain(PlanDesc P) {
  if (static_cast<int>(blockIdx.x) >= P.roll_blocks) { gen_tensor_tiles(P); return; }
  const int b = xcd_contiguous_block(blockIdx.x, P.roll_blocks) * kRollThreads + threadIdx.x;
  if (b < P.B) rollout_chain<N, CONTACT>(P, b);
}

template <int N, bool CONTACT, bool ONE>
__global__ __launch_bounds__(kRollThreads) MTP_ROLL_WAVES(ONE || N >= 20) void k_rollout_chain_pair(PlanDesc P) {
  if (static_cast<int>(blockIdx.x) >= P.roll_blocks) { gen_tensor_tiles(P); return; }
  const int g = xcd_contiguous_block(blockIdx.x, P.roll_blocks) * kRollThreads + threadIdx.x;
  const int b = g >> 1;
  if (b < P.B) rollout_chain_pair<N, CONTACT>(P, b, (g & 1) != 0);
}

// Tensor-path controls of iteration P.gen_k into P.U2 (P.roll_blocks = 0: every
// workgroup draws), run beside a time-sliced rollout that holds one wave per
// SIMD.  The launch asks for LDS that admits one of these workgroups per
// compute unit (one wave of 72 VGPRs per SIMD), so the rollout's workgroup
// (up to 440 registers per lane; 408 for 24 links with contact) finds its
// registers free on every unit whichever kernel is dispatched first.
__global__ __launch_bounds__(kCandThreads) void k_gen_tensor(PlanDesc P) { gen_tensor_tiles(P); }

__global__ __launch_bounds__(kTopkThreads) void k_topk(PlanDesc P) {
  __shared__ TopkSmem sm;
  topk_block<kTopkThreads>(P, sm);
}

__global__ __launch_bounds__(kUpdThreads) void k_update(PlanDesc P) {
  const int o = blockIdx.x * (kUpdThreads / 64) + (threadIdx.x >> 6);
  // the last refit of a replan that drew the next replan's first tensor paths
  // (its launch follows the generator's): record the replan they are for
  if (P.gen_spec && blockIdx.x == 0 && threadIdx.x == 0) {
    P.ctrl[3] = P.ctrl[0] + 1u;
    P.ctrl[5] = 1u;
  }
  if (o < P.T * P.n) update_output(P, o);
}

// Refit of iteration k at the four steps t = 4 tq + c of joint j (one wave per
// step), and from each refitted (t, j) iteration k_next's local samples and
// nominal mean at (t, j) into P.U2 (its tensor paths were drawn during
// iteration k's rollout).  The four steps of a local sample come from one
// Philox block; every thread draws its first samples' normals while the waves
// refit.
__global__ __launch_bounds__(kUpdThreads) void k_update_next(PlanDesc P, int k_next) {
  __shared__ float mom[4][2];
  const int tq = static_cast<int>(blockIdx.x) / P.n, j = static_cast<int>(blockIdx.x) - tq * P.n;
  const int c = static_cast<int>(threadIdx.x) >> 6;
  const int t = 4 * tq + c;
  const uint32_t r = P.ctrl[0];
  float z[kLocalKeep][4];
  local_normals<kUpdThreads>(P, tq, j, k_next, r, z);
  if (t < P.T) {
    float mn, sn;
    update_output(P, t * P.n + j, &mn, &sn);
    if ((threadIdx.x & 63) == 0) { mom[c][0] = mn; mom[c][1] = sn; }
  }
  __syncthreads();
  local_store<kUpdThreads>(P, P.U2, tq, j, k_next, r, z, mom);
}

// The refit of iteration k from its elites' controls drawn again
// (regen_elites) rather than gathered from U, one workgroup per four steps of
// a joint; with NEXT also iteration k_next's local samples and nominal (as
// k_update_next), without it the last iteration's refit (as k_update, which
// also records the replan whose tensor paths were drawn when P.gen_spec).
template <bool NEXT>
__global__ __launch_bounds__(kUpdThreads) void k_refit_regen(PlanDesc P, int k, int k_next) {
  __shared__ RegenSmem sm;
  __shared__ float mom[4][2];
  const int tq = static_cast<int>(blockIdx.x) / P.n, j = static_cast<int>(blockIdx.x) - tq * P.n;
  const int c = static_cast<int>(threadIdx.x) >> 6;
  const int t = 4 * tq + c;
  const uint32_t r = P.ctrl[0];
  float z[kLocalKeep][4];
  if constexpr (NEXT) local_normals<kUpdThreads>(P, tq, j, k_next, r, z);
  if (!NEXT && P.gen_spec && blockIdx.x == 0 && threadIdx.x == 0) {
    P.ctrl[3] = P.ctrl[0] + 1u;
    P.ctrl[5] = 1u;
  }
  regen_elites(P, k, tq, j, sm);
  if (t < P.T) {
    float mn, sn;
    update_output_from(P, t * P.n + j, [&](int e) { return sm.vals[c][e]; }, &mn, &sn);
    if ((threadIdx.x & 63) == 0) { mom[c][0] = mn; mom[c][1] = sn; }
  }
  if constexpr (NEXT) {
    __syncthreads();
    local_store<kUpdThreads>(P, P.U2, tq, j, k_next, r, z, mom);
  }
}

// ---------------------------------------------------------------- dispatch

static const int kChainLinks[] = {
#define X(N) N,
    MTP_CHAIN_LINKS(X)
#undef X
};
static const int kContactLinks[] = {
#define X(N) N,
    MTP_CONTACT_LINKS(X)
#undef X
};

bool rollout_supported(int dyn, int n_links) {
  if (dyn == kPointMass) return true;
  const int* tab = dyn == kChain ? kChainLinks : kContactLinks;
  const int cnt = dyn == kChain ? int(sizeof(kChainLinks) / sizeof(int)) : int(sizeof(kContactLinks) / sizeof(int));
  for (int i = 0; i < cnt; ++i)
    if (tab[i] == n_links) return true;
  return false;
}

int supported_chain_links(int* out, int cap) {
  const int cnt = int(sizeof(kChainLinks) / sizeof(int));
  for (int i = 0; i < cnt && i < cap; ++i) out[i] = kChainLinks[i];
  return cnt;
}

// Workgroups of the rollout kernel proper (one to four lanes per candidate).
int rollout_blocks(const PlanDesc& P) {
  const long long lanes_per = P.dyn == kPointMass             ? kPmLanes
                              : is_quad_chain(P.dyn, P.n_links) ? 4
                              : is_pair_chain(P.dyn, P.n_links) ? 2
                                                                : 1;
  return static_cast<int>((lanes_per * P.B + kRollThreads - 1) / kRollThreads);
}

// LDS that leaves room for only one workgroup per compute unit (160 KB each).
// A rollout launch with fewer workgroups than units asks for it so that no two
// of its workgroups, or a rollout and a generator workgroup, share a unit and
// its SIMDs (the dispatcher was seen to pair workgroups on a unit now and
// then, which doubles those waves' time).
constexpr size_t kOnePerUnitLds = 96 * 1024;

// LDS of a rollout launch that also draws tensor-path controls: the candidate
// tile's arrays over the whole horizon, at least kOnePerUnitLds.
static size_t gen_lds_bytes(const PlanDesc& P) {
  const size_t tile = sizeof(float) * static_cast<size_t>(cand_dyn_floats(P.L, P.W, P.T < kTChunk ? P.T : kTChunk));
  return tile > kOnePerUnitLds ? tile : kOnePerUnitLds;
}

template <bool ONE>
static hipError_t launch_rollout_kernel(const PlanDesc& P, dim3 grid, size_t lds, hipStream_t st);

// The rollout of P.U; with gen_k >= 0 the launch adds workgroups up to
// P.gen_grid that draw iteration gen_k's tensor-path controls into P.U2.
static hipError_t launch_rollout(const PlanDesc& P0, hipStream_t st, int gen_k) {
  PlanDesc P = P0;
  if (is_pair_chain(P.dyn, P.n_links) && P.seg_ctl != nullptr && P.seg_grid > 0) return launch_rollout_seg(P, st);
  P.roll_blocks = rollout_blocks(P);
  P.gen_k = gen_k;
  int blocks = P.roll_blocks;
  size_t lds = 0;
  if (gen_k >= 0 && P.U2 != nullptr && P.gen_grid > P.roll_blocks) {
    blocks = P.gen_grid;
    lds = gen_lds_bytes(P);
  } else if (P.roll_blocks < P.gen_grid) {
    lds = kOnePerUnitLds;
  }
  const dim3 grid(blocks);
  // a launch with LDS reserved holds one workgroup per unit
  return lds != 0 ? launch_rollout_kernel<true>(P, grid, lds, st) : launch_rollout_kernel<false>(P, grid, lds, st);
}

template <bool ONE>
static hipError_t launch_rollout_kernel(const PlanDesc& P, dim3 grid, size_t lds, hipStream_t st) {
  if (P.dyn == kPointMass) {
    k_rollout_point_mass<ONE><<<grid, kRollThreads, lds, st>>>(P);
    return hipGetLastError();
  }
  if (is_quad_chain(P.dyn, P.n_links)) return launch_rollout_quad(P, grid, lds, st, ONE);
  if (is_pair_chain(P.dyn, P.n_links)) {
    if (P.dyn == kChain) {
      switch (P.n_links) {
#define X(N) case N: if constexpr (pair_chain_links<N>()) { k_rollout_chain_pair<N, false, ONE><<<grid, kRollThreads, lds, st>>>(P); return hipGetLastError(); } break;
        MTP_CHAIN_LINKS(X)
#undef X
        default: break;
      }
    } else {
      switch (P.n_links) {
#define X(N) case N: if constexpr (pair_chain_links<N>()) { k_rollout_chain_pair<N, true, ONE><<<grid, kRollThreads, lds, st>>>(P); return hipGetLastError(); } break;
        MTP_CONTACT_LINKS(X)
#undef X
        default: break;
      }
    }
    return hipErrorInvalidValue;
  }
  if (P.dyn == kChain) {
    switch (P.n_links) {
#define X(N) case N: if constexpr (!pair_chain_links<N>() && !quad_chain_links<N>()) { k_rollout_chain<N, false, ONE><<<grid, kRollThreads, lds, st>>>(P); return hipGetLastError(); } break;
      MTP_CHAIN_LINKS(X)
#undef X
      default: break;
    }
    return hipErrorInvalidValue;
  }
  switch (P.n_links) {
#define X(N) case N: if constexpr (!pair_chain_links<N>()) { k_rollout_chain<N, true, ONE><<<grid, kRollThreads, lds, st>>>(P); return hipGetLastError(); } break;
    MTP_CONTACT_LINKS(X)
#undef X
    default: break;
  }
  return hipErrorInvalidValue;
}

static hipError_t launch_candidates(const PlanDesc& P, int k, hipStream_t st) {
  if (P.P > 0 && P.wor) {
    k_paths<<<(P.P + kCandThreads - 1) / kCandThreads, kCandThreads, 0, st>>>(P, k);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const dim3 grid((P.B + kCandThreads - 1) / kCandThreads, P.n, (P.T + P.tc - 1) / P.tc);
  const size_t lds = sizeof(float) * static_cast<size_t>(cand_dyn_floats(P.L, P.W, cand_chunk(P)));
  k_candidates<<<grid, kCandThreads, lds, st>>>(P, k);
  return hipGetLastError();
}

hipError_t launch_set_ctrl(const PlanDesc& P, uint32_t r, int shift, const float* x0_src, hipStream_t st) {
  k_set_ctrl<<<1, 64, 0, st>>>(P, r, shift, x0_src);
  return hipGetLastError();
}

hipError_t launch_shift(const PlanDesc& P, hipStream_t st) {
  k_shift<<<1, 1024, 0, st>>>(P);
  return hipGetLastError();
}

hipError_t launch_stage(const PlanDesc& P, int stage, int k, hipStream_t st) {
  switch (stage) {
    case 0:
      return launch_candidates(P, k, st);
    case 1:
      return launch_rollout(P, st, -1);
    case 2:
      k_topk<<<1, kTopkThreads, 0, st>>>(P);
      if (P.diag & 1) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_entropy<<<1, kTopkThreads, 0, st>>>(P, k);
      }
      return hipGetLastError();
    case 3: {
      const int outs = P.T * P.n;
      const int per = kUpdThreads / 64;
      k_update<<<(outs + per - 1) / per, kUpdThreads, 0, st>>>(P);
      return hipGetLastError();
    }
    default:
      return hipErrorInvalidValue;
  }
}

// Stage `stage` of iteration k within a run of iterations [k0, k1).  With the
// overlap (P.U2 set) iteration k works on U (k1 - 1 - k even, so the last
// iteration always ends in U) or U2 (odd); its rollout also draws iteration
// k+1's tensor-path controls into the other buffer on the compute units the
// rollout leaves idle, and its refit writes iteration k+1's local samples and
// nominal mean there from each refitted (t, j), so iteration k+1 launches no
// candidate kernel.  The values are those of the plain sequence: the tensor
// paths do not depend on the sampling distribution.
hipError_t launch_iteration_stage(const PlanDesc& P, int stage, int k, int k0, int k1, hipStream_t st,
                                  const SideLane* side) {
  // the plan's layout assumed a 256-unit chip; a device without a free unit
  // beyond the rollout's workgroups runs the plain sequence
  const bool sliced = is_pair_chain(P.dyn, P.n_links) && P.seg_ctl != nullptr && P.seg_grid > 0;
  const bool overlap = P.U2 != nullptr && (sliced || P.gen_grid > rollout_blocks(P));
  if (!overlap) return launch_stage(P, stage, k, st);
  PlanDesc Pk = P;
  if ((k1 - 1 - k) & 1) { Pk.U = P.U2; Pk.U2 = P.U; }
  // a whole replan of a plan that draws across replans: iteration 0 may take
  // the tensor paths the previous replan drew, and the last iteration draws
  // the next replan's into the buffer iteration 0 reads (the other one, K even)
  const bool across = P.spec && k0 == 0 && k1 == P.K;
  const bool last = k + 1 >= k1;
  switch (stage) {
    case 0:
      if (k > k0) return hipSuccess;
      Pk.cand_skip = across ? 1 : 0;
      return launch_candidates(Pk, k, st);
    case 1: {
      if (last && !across) return launch_rollout(Pk, st, -1);
      hipError_t e = hipSuccess;
      if (!sliced) {
        Pk.gen_spec = last ? 1 : 0;
        return launch_rollout(Pk, st, last ? 0 : k + 1);
      }
      PlanDesc G = Pk;
      G.roll_blocks = 0;
      G.gen_k = last ? 0 : k + 1;
      G.gen_spec = last ? 1 : 0;
      const size_t tile = sizeof(float) * static_cast<size_t>(cand_dyn_floats(P.L, P.W, P.T < kTChunk ? P.T : kTChunk));
      const size_t lds = std::max(tile, kOnePerUnitLds);
      const hipStream_t gs = side != nullptr ? side->st : st;
      if (side != nullptr) {
        e = hipEventRecord(side->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(side->st, side->fork, 0);
        if (e != hipSuccess) return e;
        k_gen_tensor<<<G.gen_grid, kCandThreads, lds, gs>>>(G);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
      e = launch_rollout(Pk, st, -1);
      if (e != hipSuccess) return e;
      if (side == nullptr) {
        k_gen_tensor<<<G.gen_grid, kCandThreads, lds, gs>>>(G);
        return hipGetLastError();
      }
      e = hipEventRecord(side->join, side->st);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, side->join, 0);
      return e;
    }
    case 3: {
      const bool regen = refit_regenerates(Pk.interp, Pk.p, Pk.wor, Pk.E, Pk.B);
      const int tiles = ((Pk.T + 3) / 4) * Pk.n;
      if (last) {
        // the last refit also records the replan whose tensor paths were drawn
        Pk.gen_spec = across ? 1 : 0;
        if (!regen) return launch_stage(Pk, stage, k, st);
        k_refit_regen<false><<<tiles, kUpdThreads, 0, st>>>(Pk, k, -1);
        return hipGetLastError();
      }
      if (regen) k_refit_regen<true><<<tiles, kUpdThreads, 0, st>>>(Pk, k, k + 1);
      else k_update_next<<<tiles, kUpdThreads, 0, st>>>(Pk, k + 1);
      return hipGetLastError();
    }
    default: return launch_stage(Pk, stage, k, st);
  }
}

hipError_t gen_configure(PlanDesc* P) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  P->gen_grid = cus;
  return hipSuccess;
}

}  // namespace mtp
