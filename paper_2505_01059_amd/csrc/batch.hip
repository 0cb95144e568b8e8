// Persistent batched execution of many MTP instances in one launch.
//
// Work is cut into items (instance, phase, iteration, tile).  A fixed grid of
// workgroups loops: take the next queue position with an atomic counter, wait
// until that position has been published, run the tile, and count it done for
// its instance.  The workgroup that finishes the last tile of an instance's
// phase publishes the tiles of that instance's next phase at the queue's tail.
// Positions are taken in order and every item is published by a tile that sat
// at a lower position, so the lowest unfinished position never waits on work
// behind it: the loop drains without any co-residency assumption.  Every wait
// is bounded by a wall-clock limit; a timeout raises an error flag that makes
// all workgroups leave, so the grid always terminates.
//
// Per-instance stages run the same tile functions as the single-plan kernels,
// and every reduction has an order fixed by the instance alone, so a result
// does not depend on which workgroup ran which tile or on the other instances.
#include "batch.hpp"

namespace mtp {

__device__ __forceinline__ uint32_t phase_tiles(const PlanDesc& P, uint32_t phase, uint32_t shape) {
  return phase_items(P.B, P.P, P.T, P.n, phase, is_quad_chain(P.dyn, P.n_links), is_pair_chain(P.dyn, P.n_links),
                     P.wor != 0, shape);
}

union BatchSmem {
  PathSmem path;
  CandSmem cand;
  TopkSmem topk;
  EntropySmem ent;
  PointMassSmem pm;
};

struct BatchShared {
  BatchItem item;
  uint32_t pos;
  uint32_t pub_pos, pub_count, pub_phase, pub_k;
  int32_t publish;
  int32_t abort;
};

__device__ __forceinline__ void run_rollout_tile(const PlanDesc& P, uint32_t tile, BatchSmem& sm) {
  const int b = static_cast<int>(tile) * kBatchThreads + static_cast<int>(threadIdx.x);
  if (P.dyn == kPointMass) {
    stage_obstacles(P, sm.pm);
    __syncthreads();
    if (b < P.B) rollout_point_mass_any<1>(P, b, 0, sm.pm);
    return;
  }
  if (is_quad_chain(P.dyn, P.n_links)) {
    const int bq = static_cast<int>(tile) * (kBatchThreads / 4) + static_cast<int>(threadIdx.x >> 2);
    if (bq >= P.B) return;
    switch (P.n_links) {
#define X(N) case N: if constexpr (quad_chain_links<N>()) rollout_chain_quad<N>(P, bq, threadIdx.x & 3); return;
      MTP_CHAIN_LINKS(X)
#undef X
      default: return;
    }
  }
  if (is_pair_chain(P.dyn, P.n_links)) {
    const int bp = static_cast<int>(tile) * (kBatchThreads / 2) + static_cast<int>(threadIdx.x >> 1);
    if (bp >= P.B) return;
    const bool lane_b = (threadIdx.x & 1) != 0;
    if (P.dyn == kChain) {
      switch (P.n_links) {
#define X(N) case N: if constexpr (pair_chain_links<N>()) rollout_chain_pair<N, false>(P, bp, lane_b); return;
        MTP_CHAIN_LINKS(X)
#undef X
        default: return;
      }
    }
    switch (P.n_links) {
#define X(N) case N: if constexpr (pair_chain_links<N>()) rollout_chain_pair<N, true>(P, bp, lane_b); return;
      MTP_CONTACT_LINKS(X)
#undef X
      default: return;
    }
  }
  if (b >= P.B) return;
  if (P.dyn == kChain) {
    switch (P.n_links) {
#define X(N) case N: if constexpr (!pair_chain_links<N>() && !quad_chain_links<N>()) rollout_chain<N, false>(P, b); return;
      MTP_CHAIN_LINKS(X)
#undef X
      default: return;
    }
  }
  switch (P.n_links) {
#define X(N) case N: if constexpr (!pair_chain_links<N>()) rollout_chain<N, true>(P, b); return;
    MTP_CONTACT_LINKS(X)
#undef X
    default: return;
  }
}

#ifndef MTP_BATCH_MIN_WG_PER_CU
#define MTP_BATCH_MIN_WG_PER_CU 1
#endif

__global__ __launch_bounds__(kBatchThreads, MTP_BATCH_MIN_WG_PER_CU) void k_batch_persistent(const PlanDesc* __restrict__ descs,
                                                                    InstCtl* __restrict__ ictl, BatchCtl* ctl,
                                                                    BatchItem* __restrict__ queue,
                                                                    uint32_t* __restrict__ ready,
                                                                    uint64_t wait_ticks) {
  __shared__ BatchSmem sm;
  __shared__ BatchShared sh;
  const int tid = threadIdx.x;
  const uint32_t epoch = ctl->epoch;
  const uint32_t total = ctl->total;
  // rollout items of several tiles run one tile per pass of this loop: `sub`
  // is the tile of the current item to run next (0: take a new item)
  uint32_t sub = 0;
  for (;;) {
    if (sub == 0u) {
      if (tid == 0) {
        sh.pos = atomicAdd(&ctl->head, 1u);
        sh.abort = 0;
      }
      __syncthreads();
      const uint32_t pos = sh.pos;
      if (pos >= total) break;
      if (tid == 0) {
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(&ready[pos], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
          if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
              wall_clock64() - t0 > wait_ticks) {
            atomicOr(&ctl->error, 1u);
            sh.abort = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (!sh.abort) sh.item = queue[pos];
      }
      __syncthreads();
      if (sh.abort) break;
      // acquire: the item's inputs were released by the workgroups that made
      // them (only an invalidation here, no write-back)
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const uint32_t inst = __builtin_amdgcn_readfirstlane(sh.item.inst);
    const uint32_t phase_word = __builtin_amdgcn_readfirstlane(sh.item.phase);
    const uint32_t phase = phase_word & kItemPhaseMask;
    const uint32_t shape = phase_word >> kItemShapeShift;   // the instance's item shape, carried by its items
    const uint32_t k = __builtin_amdgcn_readfirstlane(sh.item.k);
    const uint32_t tile = __builtin_amdgcn_readfirstlane(sh.item.tile);
    const PlanDesc P = descs[inst];

    switch (phase) {
      case kPhShift:
        shift_block<kBatchThreads>(P, static_cast<int>(P.ctrl[1]));
        break;
      case kPhPaths:
        path_tile(P, P.ctrl[0], static_cast<int>(k), static_cast<int>(tile), static_cast<int>(phase_tiles(P, kPhPaths, shape)),
                  sm.path);
        break;
      case kPhCand: {
        // an item is 2^cand_lg consecutive candidate tiles with all their
        // joints, or one joint of them
        const uint32_t r = P.ctrl[0];
        const CandView v = cand_view(sm.cand);
        const bool one_joint = shape_cand_joint(shape) != 0u;
        const int group = one_joint ? static_cast<int>(tile) / P.n : static_cast<int>(tile);
        const int j0 = one_joint ? static_cast<int>(tile) - group * P.n : 0;
        const int j1 = one_joint ? j0 + 1 : P.n;
        const int per = 1 << shape_cand_lg(shape);
        const int n_tiles = (P.B + kCandThreads - 1) / kCandThreads;
        const int ct1 = min(group * per + per, n_tiles);
        for (int ct = group * per; ct < ct1; ++ct)
          for (int j = j0; j < j1; ++j) {
            cand_tile(P, r, static_cast<int>(k), j, ct * kCandThreads, 0, P.T, v);
            __syncthreads();
          }
        break;
      }
      case kPhRoll:
        // an item is 2^roll_lg consecutive rollout tiles, one per pass
        run_rollout_tile(P, (tile << shape_roll_lg(shape)) + sub, sm);
        break;
      case kPhTopk:
        topk_block<kBatchThreads>(P, sm.topk);
        if (P.diag & 1) {
          __syncthreads();
          entropy_block<kBatchThreads>(P, static_cast<int>(k), sm.ent);
        }
        break;
      default: {
        const int wave = tid >> 6;
        const int per = 1 << shape_upd_lg(shape);
        const int base = static_cast<int>(tile) * per;
        for (int m = wave; m < per; m += kBatchThreads / 64) {
          const int o = base + m;
          if (o < P.T * P.n) update_output(P, o);
        }
        break;
      }
    }
    // release the item's results: after the barrier (every wave's stores have
    // reached the L2) one wave writes the L2 back for the other XCDs, instead
    // of every wave doing it
    __syncthreads();
    if (phase == kPhRoll) {
      const uint32_t lg = shape_roll_lg(shape);
      const uint32_t next = (tile << lg) + sub + 1u;
      if (sub + 1u < (1u << lg) && next < phase_tiles(P, kPhRoll, 0u)) {
        ++sub;   // the same item's next tile (the barrier above ordered its LDS reuse)
        continue;
      }
      sub = 0;
    }

    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      sh.publish = 0;
      const uint32_t nt = phase_tiles(P, phase, shape);
      const uint32_t done = atomicAdd(&ictl[inst].done, 1u) + 1u;
      if (done == nt) {
        // acquire the other tiles' results (released before their counts)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        atomicExch(&ictl[inst].done, 0u);
        uint32_t nph, nk;
        if (phase == kPhShift) {
          nph = kPhPaths; nk = ictl[inst].k_begin;
        } else if (phase == kPhUpd) {
          nph = kPhPaths; nk = k + 1u;
        } else {
          nph = phase + 1u; nk = k;
        }
        if (phase == kPhUpd && nk >= ictl[inst].k_end) {
          atomicAdd(&ctl->finished, 1u);
        } else {
          const uint32_t m = phase_tiles(P, nph, shape);
          sh.pub_pos = atomicAdd(&ctl->tail, m);
          sh.pub_count = m;
          sh.pub_phase = nph;
          sh.pub_k = nk;
          sh.publish = 1;
        }
      }
    }
    __syncthreads();
    if (sh.publish) {
      const uint32_t p0 = sh.pub_pos, m = sh.pub_count;
      if (p0 + m <= ctl->capacity) {
        for (uint32_t t = tid; t < m; t += kBatchThreads) {
          BatchItem it;
          it.inst = inst; it.phase = sh.pub_phase | (shape << kItemShapeShift); it.k = sh.pub_k; it.tile = t;
          queue[p0 + t] = it;
        }
        // one release (one L2 write-back) in wave 0, which then sets the ready
        // flags: the barrier orders every wave's queue entries before it
        __syncthreads();
        if (tid < 64) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          for (uint32_t t = tid; t < m; t += 64)
            __hip_atomic_store(&ready[p0 + t], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      } else if (tid == 0) {
        atomicOr(&ctl->error, 2u);   // queue overflow: items are never published, waiters time out
      }
    }
    __syncthreads();
  }
}

// Prepare one launch: per active instance record the replan index and shift,
// stage x0 and reset its tile counter; block 0 resets the queue and publishes
// one warm-start shift item per active instance in the given order.
__global__ __launch_bounds__(64) void k_batch_init(const PlanDesc* __restrict__ descs, InstCtl* __restrict__ ictl,
                                                   BatchCtl* ctl, BatchItem* __restrict__ queue,
                                                   uint32_t* __restrict__ ready, const int32_t* __restrict__ order,
                                                   int32_t n_active, uint32_t total, const float* __restrict__ x0_packed) {
  const int tid = threadIdx.x;
  const int slot = blockIdx.x;
  if (slot >= n_active) return;
  const int i = order[slot];
  const PlanDesc P = descs[i];
  const InstCtl ic = ictl[i];
  if (tid == 0) {
    P.ctrl[0] = ic.r;
    P.ctrl[1] = static_cast<uint32_t>(ic.k_begin == 0u ? ic.shift : 0);
    if (ic.k_begin == 0u) P.ctrl[2] = 0u;
    ictl[i].done = 0u;
  }
  if (x0_packed != nullptr && ic.x0_off >= 0)
    for (int e = tid; e < P.d; e += 64) P.x0[e] = x0_packed[ic.x0_off + e];
  if (tid == 0) {
    const uint32_t epoch = ctl->epoch + 1u;   // ctl is rewritten by the host-side reset below
    BatchItem it;
    it.inst = static_cast<uint32_t>(i);
    it.phase = kPhShift | (ic.shape << kItemShapeShift);
    it.k = ic.k_begin;
    it.tile = 0u;
    queue[slot] = it;
    ready[slot] = epoch;
  }
  (void)total;
}

__global__ void k_batch_reset(BatchCtl* ctl, int32_t n_active, uint32_t total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->head = 0u;
    ctl->tail = static_cast<uint32_t>(n_active);
    ctl->total = total;
    ctl->finished = 0u;
    ctl->error = 0u;
    ctl->epoch = ctl->epoch + 1u;
  }
}

// Gather every active instance's action into one packed array and append the
// launch status (error flags, finished count).
__global__ __launch_bounds__(64) void k_batch_pack(const PlanDesc* __restrict__ descs, const InstCtl* __restrict__ ictl,
                                                   const BatchCtl* ctl, float* __restrict__ out, int32_t n_inst,
                                                   int32_t status_off) {
  const int i = blockIdx.x;
  if (i < n_inst) {
    const PlanDesc P = descs[i];
    const int off = ictl[i].act_off;
    for (int j = threadIdx.x; j < P.n; j += 64) out[off + j] = P.action[j];
  }
  if (i == 0 && threadIdx.x == 0) {
    uint32_t* st = reinterpret_cast<uint32_t*>(out + status_off);
    st[0] = ctl->error;
    st[1] = ctl->finished;
    st[2] = ctl->head;
  }
}

hipError_t launch_batch_prepare(const BatchLaunch& L, hipStream_t st) {
  k_batch_init<<<L.n_active, 64, 0, st>>>(L.descs, L.ictl, L.ctl, L.queue, L.ready, L.order, L.n_active, L.total,
                                          L.x0_packed);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_batch_reset<<<1, 64, 0, st>>>(L.ctl, L.n_active, L.total);
  return hipGetLastError();
}

hipError_t launch_batch_persistent(const BatchLaunch& L, int grid, hipStream_t st) {
  k_batch_persistent<<<grid, kBatchThreads, 0, st>>>(L.descs, L.ictl, L.ctl, L.queue, L.ready, L.wait_ticks);
  return hipGetLastError();
}

hipError_t launch_batch_pack(const BatchLaunch& L, float* out, int32_t n_inst, int32_t status_off, hipStream_t st) {
  k_batch_pack<<<n_inst, 64, 0, st>>>(L.descs, L.ictl, L.ctl, out, n_inst, status_off);
  return hipGetLastError();
}

int batch_max_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_persistent, kBatchThreads, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

}  // namespace mtp
