// Device-side pieces of one MTP replan for gfx950: the plan descriptor shared
// by host and kernels, Philox4x32-10, and one __device__ function per stage
// tile.  The single-plan kernels and the persistent batched kernel both call
// these tile functions, so there is one implementation of every stage.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mtp {

constexpr int kMaxLayers = 16;
constexpr int kMaxWidth = 256;
constexpr int kMaxElites = 4096;
constexpr int kBasisStride = 8;     // spline table row: up to degree 5 (6 weights) or 4 Hermite weights
constexpr int kCandThreads = 256;   // candidate tile: 256 samples of one joint
constexpr int kRollThreads = 256;   // rollout workgroup: four waves, one per SIMD of a compute unit
constexpr int kTopkThreads = 1024;  // top-E: one workgroup per plan
constexpr int kUpdThreads = 256;    // refit tile: 4 waves, one (t, j) output per wave

enum Dyn : int32_t { kPointMass = 0, kChain = 1, kChainContact = 2 };

// Chain lengths the rollout is instantiated for (compile-time link count keeps
// the per-link state in registers).
#define MTP_CHAIN_LINKS(X) X(2) X(3) X(4) X(7) X(12) X(24)
#define MTP_CONTACT_LINKS(X) X(4) X(7) X(24)
enum Interp : int32_t { kBspline = 0, kAkima = 1, kLinear = 2 };

// Everything a stage needs, by value in kernel arguments (or in a device table
// for the batched kernel).  Pointers address the caller's workspace.
struct PlanDesc {
  int32_t dyn, interp, n_links, d, n, T, L, W, P, G, B, E, K, p, n_dbg, n_task;
  int32_t ldU;
  int32_t R;             // randomised models per candidate (contact chain), cost averaged
  int32_t wor;           // tensor paths drawn without replacement (keyed permutation of the W^L paths)
  int32_t sw_rounds;     // rounds of that permutation
  int32_t diag;          // bit 0: cost entropy of every CEM iteration into entropy[k]
  int32_t tc;            // time steps per candidate workgroup (a multiple of 4)
  float lam, alpha, sigma_min, sigma_init, u_min, u_max, dt;
  uint32_t key0, key1;
  uint32_t* ctrl;        // [0] replan index r, [1] shift, [2] flags (bit 0: all elites +inf, bit 1: selection fault)
  float* x0;             // [d]
  const float* x0_src;   // staging source for the prologue (may be null)
  float* mu;             // [T][n]
  float* sigma;          // [T][n]
  float* tmp;            // [2][T][n] scratch for the warm-start shift
  float* action;         // [n]
  const float* basis;    // [T][kBasisStride]
  const int32_t* span;   // [T] first control point (B-spline) or interval (Akima)
  const float* task;     // task parameters (see mtp.h)
  const float* sparams;  // [B][n+1] per-sample masses and friction, or null
  float* Z;              // [L][W][n]
  uint8_t* I;            // [L][P]
  float* U;              // [T][n][ldU]
  float* cost;           // [B]
  int32_t* eidx;         // [E]
  float* ecost;          // [E]
  float* w;              // [E]
  float* X;              // [R][T][d][n_dbg] or null (states of every randomised model)
  float* entropy;        // [K] cost entropy of each iteration of the last replan
  // time-sliced pair-lane rollout (long chains, launches of more waves than SIMDs); null when unused
  struct SegCtl* seg_ctl;
  uint32_t* seg_done;    // [groups] segments completed, tagged with the launch epoch
  float* seg_state;      // [(3n/2 + 1)][groups][64] angles, rates, cost and turns between segments
  int32_t seg_S, seg_len, seg_grid;
  // rollout launches that also draw the next iteration's tensor-path controls
  // (see gen_tensor_tiles): the first roll_blocks workgroups roll out, the rest
  // write the tensor-path controls of iteration gen_k into U2
  float* U2;             // second [T][n][ldU] buffer, or null
  int32_t roll_blocks, gen_k;
  int32_t eq_len;        // chains: every link has the same length (bit for bit)
  // Drawing across replans (single plans with an even number of iterations):
  // the last iteration's generator also draws the next replan's iteration-0
  // tensor paths; ctrl[3] holds the replan index they were drawn for and
  // ctrl[5] is set while they are unused, ctrl[4] tells iteration 0 of the
  // current replan whether it may take them.
  int32_t spec;          // the plan draws across replans
  int32_t gen_spec;      // this generator launch draws for replan ctrl[0] + 1, iteration 0, leaving Z and I
  int32_t cand_skip;     // this candidate launch leaves the tensor paths when ctrl[4] is set
  int32_t gen_grid;      // compute units: workgroups of such a launch (one per unit)
};

// ------------------------------------------------------------------ Philox
// Philox4x32-10 from Salmon et al., SC'11: ten rounds of two 32x32->64-bit
// multiplies with xor/permute, key bumped by the Weyl constants between rounds.
struct Words4 { uint32_t w[4]; };

// Word i (0..3) of a Philox block by selects: a runtime index into the array
// would place it in scratch memory.
__device__ __forceinline__ uint32_t word_at(const Words4& q, uint32_t i) {
  const uint32_t a = (i & 1u) ? q.w[1] : q.w[0];
  const uint32_t b = (i & 1u) ? q.w[3] : q.w[2];
  return (i & 2u) ? b : a;
}

__device__ __forceinline__ Words4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1) {
  // each 32x32 -> 64-bit product is one v_mad_u64_u32 (both halves at once)
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t p0 = static_cast<uint64_t>(c0) * 0xD2511F53u;
    const uint64_t p1 = static_cast<uint64_t>(c2) * 0xCD9E8D57u;
    const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    c0 = n0; c1 = static_cast<uint32_t>(p1); c2 = n2; c3 = static_cast<uint32_t>(p0);
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  Words4 r; r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
  return r;
}

// A device buffer pointer typed in the global address space.  Accesses through
// it compile to global memory instructions even where the pointer was read from
// memory (the persistent kernel's descriptor table) and would otherwise be a
// flat access; flat accesses also count against the LDS wait counter, so every
// LDS wait that follows one waits for it to reach memory as well.
// Fourth word of a raw (untyped, unswizzled) buffer descriptor on gfx9-family
// chips such as gfx950.
constexpr int kBufferWord3 = 0x00020000;

template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)(p);
}

constexpr uint32_t kTagZ = 1, kTagI = 2, kTagEps = 3, kTagPerm = 4;

__device__ __forceinline__ uint32_t stream_c3(uint32_t tag, int k) {
  return (tag << 16) | (static_cast<uint32_t>(k) & 0xFFFFu);
}

// top 24 bits scaled to [0, 1): exact in float32
__device__ __forceinline__ float u01(uint32_t w) { return static_cast<float>(w >> 8) * 0x1p-24f; }

// (0, 1] variant for the Box-Muller radius
__device__ __forceinline__ float u01_open0(uint32_t w) { return static_cast<float>((w >> 8) + 1u) * 0x1p-24f; }

// Box-Muller on the hardware transcendental unit: v_log gives log2 (times ln 2
// for the natural log), v_sqrt the radius (its argument is 0 or a normal
// number), and v_sin / v_cos take their argument in revolutions, so the angle
// 2*pi*u2 is exactly u2 revolutions.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
  const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u01_open0(a)));   // -2 ln u1
  const float u2 = u01(b);
  z0 = rad * __builtin_amdgcn_cosf(u2);
  z1 = rad * __builtin_amdgcn_sinf(u2);
}

__device__ __forceinline__ float clampf(float v, float lo, float hi) { return fminf(fmaxf(v, lo), hi); }

// sin and cos of an angle given in revolutions, with no reduction: for the
// rollouts that keep their angles reduced, whose arguments stay within a few
// revolutions of [0, 1), well inside the instructions' input domain.
__device__ __forceinline__ void rev_sincos(float rev, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(rev);
  *c = __builtin_amdgcn_cosf(rev);
}

// The same with the pair brought back to unit length.  The pair from v_sin /
// v_cos is a little short on average: over 2^22 arguments in [0, 1),
// s^2 + c^2 - 1 has mean -6.5e-8 and standard deviation 5.7e-8, and the error
// varies slowly with the argument.  Every link direction is built from such a
// pair, so in a long chain whose links turn slowly each link keeps the same
// small length deficit step after step and the trajectory drifts linearly from
// the exact one (24 links, 128 RK4 steps: 7.9e-5 of the state scale against
// 1.4e-5 with correctly rounded sin / cos).  One Newton step towards unit
// length, (s, c) *= 1 + (1 - s^2 - c^2) / 2, removes the bias (1.9e-5 after
// 128 steps) for five more instructions per pair.  The long-chain (pair-lane)
// rollouts use it; in the 7-link chain the bias is swamped by the rest of the
// rounding (2.6e-5 against 2.1e-5 after 128 steps) and the shorter chains keep
// the plain pair.
__device__ __forceinline__ void rev_sincos_unit(float rev, float* s, float* c, float* h_out = nullptr) {
  const float sv = __builtin_amdgcn_sinf(rev);
  const float cv = __builtin_amdgcn_cosf(rev);
  const float h = fmaf(-sv, sv, fmaf(-cv, cv, 1.0f)) * 0.5f;
  *s = fmaf(sv, h, sv);
  *c = fmaf(cv, h, cv);
  if (h_out != nullptr) *h_out = h;
}

// The same with a Newton factor h taken from a nearby argument: the RK4 stage
// angles of a step lie within a few thousandths of a turn of the step's start
// angle, where the length deficit is nearly the same (it follows the argument
// slowly), so the stages reuse the start angle's factor: two instructions per
// pair instead of five.  For a link that turns slowly (the case in which the
// deficit would pile up) the factor is the stage angle's own to within the
// deficit's local variation.
__device__ __forceinline__ void rev_sincos_scaled(float rev, float h, float* s, float* c) {
  const float sv = __builtin_amdgcn_sinf(rev);
  const float cv = __builtin_amdgcn_cosf(rev);
  *s = fmaf(sv, h, sv);
  *c = fmaf(cv, h, cv);
}

constexpr float kTwoPi = 6.283185307179586f;
constexpr float kInvTwoPi = 0.15915494309189535f;
constexpr float kTwoPiSq = 39.47841760435743f;

// ------------------------------------------------------------------ candidates
// Tile = joint j, candidates [b0, b0 + kCandThreads).  Writes U[t][j][b] for
// every candidate of the tile: local Gaussian samples (noise stream tag 3),
// tensor paths (graph tag 1, indices tag 2, spline) and the nominal mean.
// The tile regenerates column j of the graph Z in LDS from Philox; the tile
// holding the first tensor path also stores it to Z, and tiles of joint 0
// store the path indices I.
constexpr int kTChunk = 128;   // horizon steps whose tables are staged in LDS at a time

struct CandSmem {
  float z[kMaxLayers * kMaxWidth];                // Z[l][w] for this joint
  float ctrl[kMaxLayers][kCandThreads];          // per-thread control points
  float slope[kMaxLayers][kCandThreads];         // per-thread Akima slopes (unit spacing)
  float tb[kTChunk * kBasisStride];              // spline weights of the staged steps
  int32_t ts[kTChunk];                           // their span / interval index
  float tmu[kTChunk], tsg[kTChunk];              // mean and std of joint j at those steps
};

// The candidate tile's LDS arrays, either the fixed-size struct above or a
// block sized for one plan (L*W graph column, L control points and slopes per
// thread, `chunk` staged steps).
struct CandView {
  float* z;        // [L*W]
  float* ctrl;     // [L][kCandThreads]
  float* slope;    // [L][kCandThreads]
  float* tb;       // [chunk][kBasisStride]
  int32_t* ts;     // [chunk]
  float* tmu;      // [chunk]
  float* tsg;      // [chunk]
  int chunk;
};

__device__ __forceinline__ CandView cand_view(CandSmem& sm) {
  CandView v;
  v.z = sm.z; v.ctrl = &sm.ctrl[0][0]; v.slope = &sm.slope[0][0]; v.tb = sm.tb; v.ts = sm.ts;
  v.tmu = sm.tmu; v.tsg = sm.tsg; v.chunk = kTChunk;
  return v;
}

__host__ __device__ constexpr int cand_dyn_floats(int L, int W, int chunk) {
  return L * W + 2 * L * kCandThreads + chunk * (kBasisStride + 3);
}

__device__ __forceinline__ CandView cand_view_dyn(float* base, int L, int W, int chunk) {
  CandView v;
  v.z = base;
  v.ctrl = v.z + L * W;
  v.slope = v.ctrl + L * kCandThreads;
  v.tb = v.slope + L * kCandThreads;
  v.ts = reinterpret_cast<int32_t*>(v.tb + chunk * kBasisStride);
  v.tmu = reinterpret_cast<float*>(v.ts + chunk);
  v.tsg = v.tmu + chunk;
  v.chunk = chunk;
  return v;
}

__device__ __forceinline__ void akima_slopes_thread(int L, int tid, const CandView& sm) {
  // unit-spacing secants m_i = z_{i+1} - z_i; slope rules of the Akima spline
  // with the paper's end conditions; both weights zero -> mean of the secants.
  for (int i = 0; i < L; ++i) {
    float s;
    if (i == 0) {
      s = sm.ctrl[1 * kCandThreads + tid] - sm.ctrl[0 * kCandThreads + tid];
    } else if (i == L - 1) {
      s = sm.ctrl[(L - 1) * kCandThreads + tid] - sm.ctrl[(L - 2) * kCandThreads + tid];
    } else if (i == 1) {
      s = 0.5f * (sm.ctrl[2 * kCandThreads + tid] - sm.ctrl[0 * kCandThreads + tid]);
    } else if (i == L - 2) {
      s = 0.5f * (sm.ctrl[(L - 1) * kCandThreads + tid] - sm.ctrl[(L - 3) * kCandThreads + tid]);
    } else {
      const float m2 = sm.ctrl[(i - 1) * kCandThreads + tid] - sm.ctrl[(i - 2) * kCandThreads + tid];
      const float m1 = sm.ctrl[i * kCandThreads + tid] - sm.ctrl[(i - 1) * kCandThreads + tid];
      const float m0 = sm.ctrl[(i + 1) * kCandThreads + tid] - sm.ctrl[i * kCandThreads + tid];
      const float mp = sm.ctrl[(i + 2) * kCandThreads + tid] - sm.ctrl[(i + 1) * kCandThreads + tid];
      const float wa = fabsf(mp - m0);
      const float wb = fabsf(m1 - m2);
      const float den = wa + wb;
      s = (den == 0.0f) ? 0.5f * (m1 + m0) : (wa * m1 + wb * m0) / den;
    }
    sm.slope[i * kCandThreads + tid] = s;
  }
}

// ------------------------------------------------------------------ path indices
// Tensor path p takes layer indices I[l][p].  With replacement (Alg. 1) every
// index is an independent uniform draw from Philox stream tag 2.  Without
// replacement, path p is the image of p under a keyed permutation of the W^L
// paths (swap-or-not shuffle, Hoang, Morris and Rogaway, CRYPTO 2012): path
// numbers are L base-W digits (layer l is digit l, least significant first);
// round i maps x to K_i - x mod W^L when a pseudo-random bit of max(x, K_i - x)
// is set.  Each round pairs x with K_i - x, so every round and their
// composition are bijections: distinct p give distinct paths.  Round keys K_i
// (digits) and the bit function's Philox key come from stream tag 4.

constexpr int kMaxPermRounds = 2 * kMaxLayers * 8;   // 2 L ceil(log2 W) with W <= 256

struct PathSmem {
  uint8_t kd[kMaxPermRounds][kMaxLayers];   // round key digits
  uint32_t fk[kMaxPermRounds][2];           // bit-function key per round
};

__device__ __forceinline__ void perm_round_keys(const PlanDesc& P, uint32_t r, int k, PathSmem& sm) {
  const int groups = (P.L + 3) >> 2;
  for (int e = threadIdx.x; e < P.sw_rounds * (groups + 1); e += blockDim.x) {
    const int i = e / (groups + 1), g = e - i * (groups + 1);
    const Words4 q = philox(static_cast<uint32_t>(i), static_cast<uint32_t>(g), r, stream_c3(kTagPerm, k), P.key0,
                            P.key1);
    if (g < groups) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int l = 4 * g + c;
        if (l < P.L) sm.kd[i][l] = static_cast<uint8_t>(__umulhi(q.w[c], static_cast<uint32_t>(P.W)));
      }
    } else {
      sm.fk[i][0] = q.w[0];
      sm.fk[i][1] = q.w[1];
    }
  }
}

// Graph waypoints (Def. 1): Z[l][w][j] = lo + (hi - lo) u with u from stream
// tag 1, item l, element w*n + j.  Tile `tile` of `n_tiles` takes every
// n_tiles-th Philox block.
__device__ __forceinline__ void graph_tile(const PlanDesc& P, uint32_t r, int k, int tile, int n_tiles) {
  const int Wn = P.W * P.n;
  const int nb = (Wn + 3) >> 2;
  const float lo = P.u_min, span = P.u_max - P.u_min;
  for (int c = tile * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x); c < P.L * nb;
       c += n_tiles * static_cast<int>(blockDim.x)) {
    const int l = c / nb, blk = c - l * nb;
    const Words4 q = philox(static_cast<uint32_t>(blk), static_cast<uint32_t>(l), r, stream_c3(kTagZ, k), P.key0,
                            P.key1);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = 4 * blk + e;
      if (idx < Wn) P.Z[static_cast<size_t>(l) * Wn + idx] = fmaf(span, u01(q.w[e]), lo);
    }
  }
}

// Without replacement: draws the graph (its share) and writes I[.][p] for the
// tensor paths p of the tile.  Every thread of the workgroup must call this (it
// synchronises the workgroup).
__device__ __forceinline__ void path_tile(const PlanDesc& P, uint32_t r, int k, int tile, int n_tiles,
                                          PathSmem& sm) {
  if (!P.wor) return;   // with replacement the candidate tiles draw the graph and the indices
  if (P.P > 0) graph_tile(P, r, k, tile, n_tiles);
  const int pp = tile * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x);
  if (!P.wor) {
    if (pp >= P.P) return;
    for (int l4 = 0; l4 < P.L; l4 += 4) {
      const Words4 q = philox(static_cast<uint32_t>(l4 >> 2), static_cast<uint32_t>(pp), r, stream_c3(kTagI, k),
                              P.key0, P.key1);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int l = l4 + c;
        if (l < P.L)
          P.I[static_cast<size_t>(l) * P.P + pp] = static_cast<uint8_t>(__umulhi(q.w[c], static_cast<uint32_t>(P.W)));
      }
    }
    return;
  }
  perm_round_keys(P, r, k, sm);
  __syncthreads();
  if (pp >= P.P) return;
  const uint32_t W = static_cast<uint32_t>(P.W);
  const int L = P.L;
  uint32_t x[kMaxLayers];
  {
    uint32_t v = static_cast<uint32_t>(pp);
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) {
      x[l] = (l < L) ? v % W : 0u;
      v = (l < L) ? v / W : v;
    }
  }
  for (int i = 0; i < P.sw_rounds; ++i) {
    // x' = K_i - x mod W^L, digit by digit with a borrow
    uint32_t xs[kMaxLayers];
    uint32_t borrow = 0u;
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) {
      const int32_t dgt = static_cast<int32_t>(sm.kd[i][l < L ? l : 0]) - static_cast<int32_t>(x[l]) -
                          static_cast<int32_t>(borrow);
      xs[l] = (l < L) ? static_cast<uint32_t>(dgt < 0 ? dgt + static_cast<int32_t>(W) : dgt) : 0u;
      borrow = (l < L && dgt < 0) ? 1u : 0u;
    }
    // the larger of x and x' (most significant digit first) names the pair
    int cmp = 0;
#pragma unroll
    for (int l = kMaxLayers - 1; l >= 0; --l)
      if (cmp == 0 && l < L) cmp = (xs[l] > x[l]) ? 1 : ((xs[l] < x[l]) ? -1 : 0);
    uint32_t wd[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int l = 0; l < kMaxLayers; ++l) wd[l >> 2] |= (cmp > 0 ? xs[l] : x[l]) << (8 * (l & 3));
    const Words4 f = philox(wd[0], wd[1], wd[2], wd[3], sm.fk[i][0], sm.fk[i][1]);
    if (f.w[0] & 1u) {
#pragma unroll
      for (int l = 0; l < kMaxLayers; ++l) x[l] = xs[l];
    }
  }
#pragma unroll
  for (int l = 0; l < kMaxLayers; ++l)
    if (l < L) P.I[static_cast<size_t>(l) * P.P + pp] = static_cast<uint8_t>(x[l]);
}

// Which candidates a tile writes: all, or only the tensor paths (they do not
// depend on the sampling distribution, so they can be drawn an iteration ahead).
// kCandTensorAhead: tensor paths only, for a later replan: Z and I of the
// current one are left as they are.  kCandLocal: local samples and nominal only.
constexpr int kCandAll = 0, kCandTensor = 1, kCandTensorAhead = 2, kCandLocal = 3;

// Candidates [b0, b0 + kCandThreads) of joint j over steps [t_begin, t_end)
// (t_begin a multiple of 4).  Tensor paths read their layer indices from I.
// Every thread of the tile must call this (it synchronises the workgroup).
__device__ __forceinline__ void cand_tile(const PlanDesc& P, uint32_t r, int k, int j, int b0, int t_begin,
                                          int t_end, const CandView& sm, int mode = kCandAll) {
  const auto Ug = gptr(P.U);
  const auto Zg = gptr(P.Z);
  const auto Ig = gptr(P.I);
  const int tid = threadIdx.x;
  const int b = b0 + tid;
  const int G1 = P.G - 1;                       // local samples [0, G1)
  const int tens_lo = G1, tens_hi = G1 + P.P;   // tensor paths [G1, G1+P)
  const bool tensor_only = mode == kCandTensor || mode == kCandTensorAhead;
  const bool tile_has_tensor = mode != kCandLocal && (b0 < tens_hi) && (b0 + kCandThreads > tens_lo);
  const float lo = P.u_min, hi = P.u_max;
  const size_t ld = static_cast<size_t>(P.ldU);
  const bool live = b < P.B;
  const bool is_local = !tensor_only && live && b < G1;
  const bool is_tensor = mode != kCandLocal && live && b >= tens_lo && b < tens_hi;
  const bool is_nominal = !tensor_only && live && b >= tens_hi;

  if (tile_has_tensor) {
    if (P.wor) {
      // graph column of joint j, drawn by the path tiles
      for (int e = tid; e < P.L * P.W; e += kCandThreads) sm.z[e] = Zg[static_cast<size_t>(e) * P.n + j];
    } else {
      // draw the graph column of joint j here; the tile holding the first tensor
      // path stores it to Z
      const bool z_writer = mode != kCandTensorAhead && (b0 <= tens_lo) && t_begin == 0;
      const float span = hi - lo;
      for (int e = tid; e < P.L * P.W; e += kCandThreads) {
        const int l = e / P.W, w = e - l * P.W;
        const uint32_t idx = static_cast<uint32_t>(w * P.n + j);
        const Words4 q = philox(idx >> 2, static_cast<uint32_t>(l), r, stream_c3(kTagZ, k), P.key0, P.key1);
        const float z = fmaf(span, u01(word_at(q, idx & 3u)), lo);
        sm.z[e] = z;
        if (z_writer) Zg[static_cast<size_t>(e) * P.n + j] = z;
      }
    }
  }
  __syncthreads();
  if (is_tensor) {
    const int pp = b - G1;
    if (P.wor) {
      for (int l = 0; l < P.L; ++l) sm.ctrl[l * kCandThreads + tid] = sm.z[l * P.W + Ig[static_cast<size_t>(l) * P.P + pp]];
    } else {
      // Alg. 1 indices drawn here; the tiles of joint 0 and the first horizon chunk store I
      const bool i_writer = mode != kCandTensorAhead && j == 0 && t_begin == 0;
      for (int l4 = 0; l4 < P.L; l4 += 4) {
        const Words4 q = philox(static_cast<uint32_t>(l4 >> 2), static_cast<uint32_t>(pp), r, stream_c3(kTagI, k),
                                P.key0, P.key1);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int l = l4 + c;
          if (l < P.L) {
            const uint32_t wi = __umulhi(q.w[c], static_cast<uint32_t>(P.W));
            sm.ctrl[l * kCandThreads + tid] = sm.z[l * P.W + wi];
            if (i_writer) Ig[static_cast<size_t>(l) * P.P + pp] = static_cast<uint8_t>(wi);
          }
        }
      }
    }
    if (P.interp == kAkima) akima_slopes_thread(P.L, tid, sm);
  }
  const int Tq = (P.T + 3) >> 2;
  for (int t0 = t_begin; t0 < t_end; t0 += sm.chunk) {
    const int tn = min(sm.chunk, t_end - t0);
    for (int i = tid; i < tn; i += kCandThreads) {
      const int o = (t0 + i) * P.n + j;
      sm.ts[i] = gptr(P.span)[t0 + i];
      sm.tmu[i] = gptr(P.mu)[o];
      sm.tsg[i] = gptr(P.sigma)[o];
    }
    for (int i = tid; i < tn * kBasisStride; i += kCandThreads) sm.tb[i] = gptr(P.basis)[t0 * kBasisStride + i];
    __syncthreads();
    if (is_local) {
      // local sample g = b: u = clip(mu + sigma * eps), four steps per Philox block
#pragma unroll 2
      for (int tq = t0 >> 2; tq < ((t0 + tn + 3) >> 2); ++tq) {
        const Words4 q = philox(static_cast<uint32_t>(j * Tq + tq), static_cast<uint32_t>(b), r,
                                stream_c3(kTagEps, k), P.key0, P.key1);
        float z[4];
        box_muller(q.w[0], q.w[1], z[0], z[1]);
        box_muller(q.w[2], q.w[3], z[2], z[3]);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int t = 4 * tq + c;
          if (t < t0 + tn) {
            const int i = t - t0;
            __builtin_nontemporal_store(clampf(fmaf(sm.tsg[i], z[c], sm.tmu[i]), lo, hi), &Ug[(t * P.n + j) * ld + b]);
          }
        }
      }
    } else if (is_tensor) {
      if (P.interp == kBspline && P.p == 3) {
#pragma unroll 4
        for (int i = 0; i < tn; ++i) {
          const int s0 = sm.ts[i];
          const float* bw = sm.tb + i * kBasisStride;
          float v = bw[0] * sm.ctrl[s0 * kCandThreads + tid];
          v = fmaf(bw[1], sm.ctrl[(s0 + 1) * kCandThreads + tid], v);
          v = fmaf(bw[2], sm.ctrl[(s0 + 2) * kCandThreads + tid], v);
          v = fmaf(bw[3], sm.ctrl[(s0 + 3) * kCandThreads + tid], v);
          __builtin_nontemporal_store(clampf(v, lo, hi), &Ug[((t0 + i) * P.n + j) * ld + b]);
        }
      } else if (P.interp != kAkima) {
        const int np1 = P.interp == kLinear ? 2 : P.p + 1;
#pragma unroll 2
        for (int i = 0; i < tn; ++i) {
          const int s0 = sm.ts[i];
          const float* bw = sm.tb + i * kBasisStride;
          float v = 0.0f;
          for (int q = 0; q < np1; ++q) v = fmaf(bw[q], sm.ctrl[(s0 + q) * kCandThreads + tid], v);
          __builtin_nontemporal_store(clampf(v, lo, hi), &Ug[((t0 + i) * P.n + j) * ld + b]);
        }
      } else {
#pragma unroll 4
        for (int i = 0; i < tn; ++i) {
          const int iv = sm.ts[i];
          const float* h = sm.tb + i * kBasisStride;
          float v = h[0] * sm.ctrl[iv * kCandThreads + tid];
          v = fmaf(h[1], sm.slope[iv * kCandThreads + tid], v);
          v = fmaf(h[2], sm.ctrl[(iv + 1) * kCandThreads + tid], v);
          v = fmaf(h[3], sm.slope[(iv + 1) * kCandThreads + tid], v);
          __builtin_nontemporal_store(clampf(v, lo, hi), &Ug[((t0 + i) * P.n + j) * ld + b]);
        }
      }
    } else if (is_nominal) {
      // nominal mean
#pragma unroll 4
      for (int i = 0; i < tn; ++i) __builtin_nontemporal_store(clampf(sm.tmu[i], lo, hi), &Ug[((t0 + i) * P.n + j) * ld + b]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ rollout
// One lane per candidate; the state lives in registers for the whole horizon.

__device__ __forceinline__ float finite_or_inf(float c) { return (c == c && fabsf(c) <= 3.402823466e38f) ? c : INFINITY; }

constexpr int kMaxObstacles = 256;
struct PointMassSmem {
  float obs[3 * kMaxObstacles];   // centre x, centre y, squared radius
};

// The obstacle table is staged in LDS by the calling tile (all lanes read the
// same entry at once, so every read is a broadcast).
__device__ __forceinline__ void stage_obstacles(const PlanDesc& P, PointMassSmem& sm) {
  const float* tk = P.task;
  const int n_obs = static_cast<int>(tk[5]);
  for (int i = threadIdx.x; i < n_obs; i += blockDim.x) {
    const float r = tk[6 + 3 * i + 2];
    sm.obs[3 * i] = tk[6 + 3 * i];
    sm.obs[3 * i + 1] = tk[6 + 3 * i + 1];
    sm.obs[3 * i + 2] = r * r;
  }
}

// Quad-permute DPP: moves values among the four lanes of a quad.
constexpr int qperm_ctrl(int a, int b, int c, int d) { return a | (b << 2) | (c << 4) | (d << 6); }
constexpr int kQNext1 = qperm_ctrl(1, 2, 3, 3);
constexpr int kQPrev1 = qperm_ctrl(0, 0, 1, 2);
constexpr int kQNext2 = qperm_ctrl(2, 3, 2, 3);
constexpr int kQPrev2 = qperm_ctrl(0, 1, 0, 1);
constexpr int kQXor1 = qperm_ctrl(1, 0, 3, 2);
constexpr int kQXor2 = qperm_ctrl(2, 3, 0, 1);

template <int CTRL>
__device__ __forceinline__ float qperm(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float quad_sum(float v) {
  v += qperm<kQXor1>(v);
  return v + qperm<kQXor2>(v);
}

// Obstacle tests: the uniform obstacle table either lives in registers (up to
// NOBS obstacles, padded with radius^2 = -1 so the padding never hits) or, for
// longer tables, is read from LDS.  Register tables avoid one LDS round trip per
// obstacle and step, which dominates a rollout of a few hundred candidates.
//
// The obstacle penalties of a step are summed in eight groups, obstacle o in
// group o mod 8, each in increasing o, and the groups as
// ((g0 + g1) + (g2 + g3)) + ((g4 + g5) + (g6 + g7)).  LANES = 1: one lane per
// candidate holds every group.  LANES = 8: lane q of the candidate's eight
// holds group q (an eighth of the table); two quad permutes add the groups of
// each quad and a half-row mirror adds the two quads, in the same order, so
// every lane ends the step with the same bits as the one-lane form; the state
// update, goal and control terms run on all eight lanes alike.  A step is
// issue-bound on one wave per SIMD, and the eight-lane form issues about a
// quarter of the one-lane instructions per lane.
constexpr int kPmLanes = 8;
constexpr int kDppHalfMirror = 0x141;   // lane i of each eight reads lane 7 - i

__device__ __forceinline__ float half_mirror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppHalfMirror, 0xF, 0xF, true));
}

template <int NOBS, int LANES = 1>
__device__ __forceinline__ void rollout_point_mass(const PlanDesc& P, int b, int q, const PointMassSmem& sm) {
  static_assert(LANES == 1 || LANES == kPmLanes, "one lane or eight per candidate");
  static_assert(NOBS % 8 == 0, "register tables hold whole groups");
  // task: goal_x, goal_y, goal_w, obstacle_penalty, ctrl_w, n_obs, (cx, cy, r)*
  const float* tk = P.task;
  const float gx = tk[0], gy = tk[1], wg = tk[2], pen = tk[3], wu = tk[4];
  const int n_obs = static_cast<int>(tk[5]);
  constexpr int NL = NOBS > 0 ? NOBS / LANES : 1;   // register obstacles per lane
  float ocx[NL], ocy[NL], orr[NL];
  if constexpr (NOBS > 0) {
    // read from the LDS copy so that the table lands in vector registers (as
    // uniform scalars it would not fit the scalar register file)
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int o = LANES == 1 ? i : q + kPmLanes * i;
      const bool on = o < n_obs;
      ocx[i] = on ? sm.obs[3 * o] : 0.0f;
      ocy[i] = on ? sm.obs[3 * o + 1] : 0.0f;
      orr[i] = on ? sm.obs[3 * o + 2] : -1.0f;
    }
  }
  const float* obs = sm.obs;
  const float dt = P.dt;
  float px = P.x0[0], py = P.x0[1], vx = P.x0[2], vy = P.x0[3];
  const size_t ld = static_cast<size_t>(P.ldU);
  const float* u0 = P.U + b;
  float cost = 0.0f;
  // penalty of obstacle o (table entry i of this lane) at the new position
  auto hit = [&](float ox, float oy, float rr) { return (fmaf(ox, ox, oy * oy) < rr) ? pen : 0.0f; };
  // One step: semi-implicit Euler, then the cost of the new position and the
  // control.  Recording the states is a separate instantiation, chosen once
  // per wave, so the step loop of the other waves carries no branch.
  auto step = [&](float ux, float uy, int t, auto rec) {
    vx = fmaf(dt, ux, vx);
    vy = fmaf(dt, uy, vy);
    px = fmaf(dt, vx, px);
    py = fmaf(dt, vy, py);
    const float dx = px - gx, dy = py - gy;
    float obst;
    if constexpr (LANES == 1) {
      float pc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
      if constexpr (NOBS > 0) {
#pragma unroll
        for (int o = 0; o < NOBS; ++o) pc[o & 7] += hit(px - ocx[o], py - ocy[o], orr[o]);
      } else {
        for (int o = 0; o < n_obs; ++o) pc[o & 7] += hit(px - obs[3 * o], py - obs[3 * o + 1], obs[3 * o + 2]);
      }
      obst = ((pc[0] + pc[1]) + (pc[2] + pc[3])) + ((pc[4] + pc[5]) + (pc[6] + pc[7]));
    } else {
      float g = 0.0f;
      if constexpr (NOBS > 0) {
#pragma unroll
        for (int i = 0; i < NL; ++i) g += hit(px - ocx[i], py - ocy[i], orr[i]);
      } else {
        for (int o = q; o < n_obs; o += kPmLanes) g += hit(px - obs[3 * o], py - obs[3 * o + 1], obs[3 * o + 2]);
      }
      g = quad_sum(g);
      obst = g + half_mirror(g);
    }
    float c = fmaf(wg, fmaf(dx, dx, dy * dy), obst);
    c = fmaf(wu, fmaf(ux, ux, uy * uy), c);
    cost += c;
    if constexpr (decltype(rec)::value) {
      if (b < P.n_dbg && q == 0) {
        float* X = P.X + b;
        const size_t ldx = static_cast<size_t>(P.n_dbg);
        X[(t * 4 + 0) * ldx] = px; X[(t * 4 + 1) * ldx] = py;
        X[(t * 4 + 2) * ldx] = vx; X[(t * 4 + 3) * ldx] = vy;
      }
    }
  };
  // controls arrive in blocks of kPmBlock steps, the next block loading while
  // the current one is integrated: one step is too short to hide a load; whole
  // blocks run without a bound test, the last partial block step by step
  constexpr int kPmBlock = 8;
  auto run = [&](auto rec) {
    const int full = P.T / kPmBlock * kPmBlock;
    float cux[kPmBlock], cuy[kPmBlock];
#pragma unroll
    for (int i = 0; i < kPmBlock; ++i) {
      const int tt = i < P.T ? i : 0;
      cux[i] = u0[(2 * tt) * ld];
      cuy[i] = u0[(2 * tt + 1) * ld];
    }
    for (int t0 = 0; t0 < full; t0 += kPmBlock) {
      float nux[kPmBlock], nuy[kPmBlock];
#pragma unroll
      for (int i = 0; i < kPmBlock; ++i) {
        const int tn = t0 + kPmBlock + i < P.T ? t0 + kPmBlock + i : 0;
        nux[i] = u0[(2 * tn) * ld];
        nuy[i] = u0[(2 * tn + 1) * ld];
      }
#pragma unroll
      for (int i = 0; i < kPmBlock; ++i) step(cux[i], cuy[i], t0 + i, rec);
#pragma unroll
      for (int i = 0; i < kPmBlock; ++i) { cux[i] = nux[i]; cuy[i] = nuy[i]; }
    }
    for (int t = full; t < P.T; ++t) {
      const int i = t - full;
      float ux = cux[0], uy = cuy[0];
#pragma unroll
      for (int k = 1; k < kPmBlock; ++k)
        if (k == i) { ux = cux[k]; uy = cuy[k]; }
      step(ux, uy, t, rec);
    }
  };
  if (__builtin_amdgcn_ballot_w64(b < P.n_dbg) != 0) run(std::true_type{});
  else run(std::false_type{});
  if (q == 0) P.cost[b] = finite_or_inf(cost);
}

// Obstacle-table size class of a point-mass plan: 8, 16, 24, 32 in registers, 0 in LDS.
__device__ __host__ __forceinline__ int point_mass_obs_class(int n_obs) {
  return n_obs <= 8 ? 8 : (n_obs <= 16 ? 16 : (n_obs <= 24 ? 24 : (n_obs <= 32 ? 32 : 0)));
}

template <int LANES = 1>
__device__ __forceinline__ void rollout_point_mass_any(const PlanDesc& P, int b, int q, const PointMassSmem& sm) {
  switch (point_mass_obs_class(static_cast<int>(P.task[5]))) {
    case 8: rollout_point_mass<8, LANES>(P, b, q, sm); return;
    case 16: rollout_point_mass<16, LANES>(P, b, q, sm); return;
    case 24: rollout_point_mass<24, LANES>(P, b, q, sm); return;
    case 32: rollout_point_mass<32, LANES>(P, b, q, sm); return;
    default: rollout_point_mass<0, LANES>(P, b, q, sm); return;
  }
}

// Planar chain of point masses on massless links, absolute angles from the
// downward vertical.  Instead of assembling the dense mass matrix, the link
// tensions solve a symmetric tridiagonal system (each link is a rigid rod whose
// length constraint couples its two end masses), solved by forward elimination
// and back substitution; the angular accelerations then follow link by link.
// O(n) work, no n x n matrix, same equations of motion as the Lagrangian form.
template <int N>
struct ChainConsts {
  float l[N], invl[N];
  float im[N];                      // inverse masses (per sample with contact)
  float g, wg, wu, tx, ty;
  float yg, kc, dc, inv_vs, muf;   // contact only
};

// Long chains recompute per-link products instead of keeping them, to stay
// within the register file.
template <int N>
struct ChainLean {
  static constexpr bool value = N > 12;
};

// tanh from the hardware base-2 exponential: 1 - 2 / (1 + e^{2x}); saturates
// to +-1 without overflow trouble.
__device__ __forceinline__ float fast_tanh(float x) {
  const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * x);   // e^{2x}
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
}

// (u_k - u_{k+1}) / l_k: torque difference across link k over its length
template <int N>
__device__ __forceinline__ float chain_q(const float (&u)[N], const ChainConsts<N>& K, int k) {
  return (u[k] - ((k + 1 < N) ? u[k + 1] : 0.0f)) * K.invl[k];
}

template <int N, bool CONTACT>
__device__ __forceinline__ void chain_accel(const float (&s)[N], const float (&c)[N], const float (&om)[N],
                                            const float (&u)[N], const ChainConsts<N>& K, float (&acc)[N]) {
  constexpr bool lean = ChainLean<N>::value;
  float cp[N], dp[N];
  float ndf[CONTACT ? N : 1];
  float qs[lean ? 1 : N], Cs[lean ? 1 : N], Ss[lean ? 1 : N];
  float im_prev = 0.0f, Cn_prev = 0.0f, Sn_prev = 0.0f, cp_prev = 0.0f, dp_prev = 0.0f;
  float fx_prev = 0.0f, fy_prev = 0.0f;
  float px = 0.0f, py = 0.0f, vx = 0.0f, vy = 0.0f;
  float q_prev = 0.0f;
  float qk = chain_q<N>(u, K, 0);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    float Cnk = 0.0f, Snk = 0.0f, qn = 0.0f;
    if (k + 1 < N) {
      Cnk = fmaf(c[k], c[k + 1], s[k] * s[k + 1]);   // cos(phi_k - phi_{k+1})
      Snk = fmaf(s[k], c[k + 1], -c[k] * s[k + 1]);  // sin(phi_k - phi_{k+1})
      qn = chain_q<N>(u, K, k + 1);
    }
    if constexpr (!lean) {
      Cs[k] = Cnk;
      Ss[k] = Snk;
      qs[k] = qk;
    }
    const float imk = K.im[k];
    float dfx, dfy;   // change of the non-constraint acceleration from mass k-1 to mass k
    if constexpr (CONTACT) {
      px = fmaf(K.l[k], s[k], px);
      py = fmaf(-K.l[k], c[k], py);
      const float lw = K.l[k] * om[k];
      vx = fmaf(lw, c[k], vx);
      vy = fmaf(lw, s[k], vy);
      const float pen = K.yg - py;
      float fx = 0.0f, fy = 0.0f;
      if (pen > 0.0f) {
        const float fn = fmaxf(fmaf(K.kc, pen, -K.dc * vy), 0.0f);
        const float ft = -K.muf * fn * fast_tanh(vx * K.inv_vs);
        fx = ft * imk;
        fy = fn * imk;
      }
      dfx = fx - fx_prev;
      dfy = fy - fy_prev;
      fx_prev = fx;
      fy_prev = fy;
      if (k == 0) dfy -= K.g;
      ndf[k] = fmaf(c[k], dfx, s[k] * dfy);
    } else {
      dfx = 0.0f;
      dfy = (k == 0) ? -K.g : 0.0f;
    }
    const float D = imk + im_prev;
    const float Up = -imk * Cnk;
    const float Lo = -im_prev * Cn_prev;
    float rhs = K.l[k] * om[k] * om[k];
    rhs = fmaf(s[k], dfx, rhs);
    rhs = fmaf(-c[k], dfy, rhs);
    rhs = fmaf(-imk * qn, Snk, rhs);
    rhs = fmaf(im_prev * q_prev, Sn_prev, rhs);
    const float inv = __builtin_amdgcn_rcpf(fmaf(-Lo, cp_prev, D));
    cp_prev = Up * inv;
    dp_prev = fmaf(-Lo, dp_prev, rhs) * inv;
    cp[k] = cp_prev;
    dp[k] = dp_prev;
    im_prev = imk;
    Cn_prev = Cnk;
    Sn_prev = Snk;
    q_prev = qk;
    qk = qn;
  }
  // back substitution: dp[k] becomes the tension of link k
#pragma unroll
  for (int k = N - 2; k >= 0; --k) dp[k] = fmaf(-cp[k], dp[k + 1], dp[k]);
  // link accelerations
  float Cp = 0.0f, Sp = 0.0f, qp = 0.0f;
  float qc = lean ? chain_q<N>(u, K, 0) : qs[0];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    float Cn = 0.0f, Sn = 0.0f, qn = 0.0f;
    if (k + 1 < N) {
      if constexpr (lean) {
        Cn = fmaf(c[k], c[k + 1], s[k] * s[k + 1]);
        Sn = fmaf(s[k], c[k + 1], -c[k] * s[k + 1]);
        qn = chain_q<N>(u, K, k + 1);
      } else {
        Cn = Cs[k];
        Sn = Ss[k];
        qn = qs[k + 1];
      }
    }
    const float Tn = (k + 1 < N) ? dp[k + 1] : 0.0f;
    const float Tp = (k > 0) ? dp[k - 1] : 0.0f;
    const float imp = (k > 0) ? K.im[k - 1] : 0.0f;
    float a = (K.im[k] + imp) * qc;
    a = fmaf(-K.im[k], fmaf(Tn, Sn, qn * Cn), a);
    a = fmaf(-imp, fmaf(-Tp, Sp, qp * Cp), a);
    if constexpr (CONTACT) {
      a += ndf[k];
    } else {
      if (k == 0) a = fmaf(-K.g, s[0], a);
    }
    acc[k] = a * K.invl[k];
    Cp = Cn;
    Sp = Sn;
    qp = qc;
    qc = qn;
  }
}

template <int N, bool CONTACT>
__device__ __forceinline__ void rollout_chain(const PlanDesc& P, int b) {
  // task: gravity, goal_w, ctrl_w, target_x, target_y, masses[N], lengths[N], (contact: yg, kc, dc, v_slip)
  const float* tk = P.task;
  ChainConsts<N> K;
  K.g = tk[0]; K.wg = tk[1]; K.wu = tk[2]; K.tx = tk[3]; K.ty = tk[4];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    K.l[k] = tk[5 + N + k];
    K.invl[k] = 1.0f / K.l[k];
  }
  if constexpr (CONTACT) {
    K.yg = tk[5 + 2 * N]; K.kc = tk[6 + 2 * N]; K.dc = tk[7 + 2 * N]; K.inv_vs = 1.0f / tk[8 + 2 * N];
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) K.im[k] = 1.0f / tk[5 + k];
    K.muf = 0.0f; K.yg = 0.0f; K.kc = 0.0f; K.dc = 0.0f; K.inv_vs = 0.0f;
  }
  const float dt = P.dt, hdt = 0.5f * P.dt, dt6 = P.dt * (1.0f / 6.0f);
  const float dtr = kInvTwoPi * dt, hdtr = kInvTwoPi * hdt, dt6r = kInvTwoPi * dt6;
  // randomised models: the candidate's cost is the mean over R rollouts
  const int R = CONTACT ? P.R : 1;
  float total = 0.0f;
#pragma unroll 1
  for (int rep = 0; rep < R; ++rep) {
  if constexpr (CONTACT) {
    const float* sp = P.sparams + (static_cast<size_t>(rep) * P.B + b) * (N + 1);
#pragma unroll
    for (int k = 0; k < N; ++k) K.im[k] = 1.0f / sp[k];
    K.muf = sp[N];
  }
  // Angles are carried in revolutions, reduced to [0, 1) after every step, so a
  // stage angle goes to v_sin / v_cos as it is; rates stay in rad/s and the
  // stage offsets h / 2pi are uniform.  The whole turns taken off are kept up
  // to date only for recorded candidates (the state output gives radians).
  float ph[N], om[N], turn[N], s[N], c[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const float r = kInvTwoPi * P.x0[k];
    turn[k] = floorf(r);
    ph[k] = r - turn[k];
    om[k] = P.x0[N + k];
    rev_sincos(ph[k], &s[k], &c[k]);
  }
  const size_t ld = static_cast<size_t>(P.ldU);
  const float* ub = P.U + b;
  float u[N];
#pragma unroll
  for (int k = 0; k < N; ++k) u[k] = ub[k * ld];
  float cost = 0.0f;
  for (int t = 0; t < P.T; ++t) {
    // next step's controls, loaded a whole step ahead; the last step re-reads
    // its own row (no select on the loaded values, which would make the wave
    // wait for the loads at once)
    float un[N];
    const int tn = (t + 1 < P.T) ? t + 1 : t;
#pragma unroll
    for (int k = 0; k < N; ++k) un[k] = ub[(tn * N + k) * ld];

    // classical RK4 with the control held: stage s evaluates at
    // phi_s = phi + c_s dt omega_{s-1},  omega_s = omega + c_s dt k_{s-1}
    float kk[N], oms[N], aph[N], aom[N];
    chain_accel<N, CONTACT>(s, c, om, u, K, kk);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      aph[k] = om[k];
      aom[k] = kk[k];
      oms[k] = om[k];
    }
#pragma unroll 1
    for (int stage = 1; stage < 4; ++stage) {
      const float h = (stage == 3) ? dt : hdt;
      const float hr = (stage == 3) ? dtr : hdtr;
      float s2[N], c2[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        rev_sincos(fmaf(hr, oms[k], ph[k]), &s2[k], &c2[k]);
        oms[k] = fmaf(h, kk[k], om[k]);
      }
      chain_accel<N, CONTACT>(s2, c2, oms, u, K, kk);
      const float wgt = (stage == 3) ? 1.0f : 2.0f;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        aph[k] = fmaf(wgt, oms[k], aph[k]);
        aom[k] = fmaf(wgt, kk[k], aom[k]);
      }
    }
    float pu[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      pu[k] = fmaf(dt6r, aph[k], ph[k]);
      ph[k] = __builtin_amdgcn_fractf(pu[k]);
      om[k] = fmaf(dt6, aom[k], om[k]);
    }
    // cost of the new state (its sin/cos also start the next step)
    float ex = 0.0f, ey = 0.0f, uu = 0.0f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      rev_sincos(ph[k], &s[k], &c[k]);
      ex = fmaf(K.l[k], s[k], ex);
      ey = fmaf(-K.l[k], c[k], ey);
      uu = fmaf(u[k], u[k], uu);
    }
    const float dx = ex - K.tx, dy = ey - K.ty;
    cost += fmaf(K.wg, fmaf(dx, dx, dy * dy), K.wu * uu);
    if (b < P.n_dbg) {
      float* X = P.X + static_cast<size_t>(rep) * P.T * P.d * P.n_dbg + b;
      const size_t ldx = static_cast<size_t>(P.n_dbg);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        turn[k] += floorf(pu[k]);
        X[(t * 2 * N + k) * ldx] = kTwoPi * (turn[k] + ph[k]);
        X[(t * 2 * N + N + k) * ldx] = om[k];
      }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) u[k] = un[k];
  }
  total += cost;
  }
  P.cost[b] = finite_or_inf(R == 1 ? total : total / static_cast<float>(R));
}

// ------------------------------------------------------------------ quad-lane chain
// Chains of 5..8 links: four lanes share one candidate, each owning two
// consecutive links (rows 2s and 2s+1 of the tension system; rows past the
// chain end are identity rows).  The tridiagonal solve is one level of cyclic
// reduction inside the lane (eliminating the even rows), a two-level parallel
// cyclic reduction of the four odd rows across the quad, and back-substitution
// of the even rows.  Cross-lane values move with quad-permute DPP, which never
// leaves the four lanes of a candidate.  Four times as many lanes as the
// one-lane form for the same candidates, at about 60% of its instructions per lane.

template <int N>
constexpr bool quad_chain_links() { return N >= 5 && N <= 8; }

__host__ __device__ constexpr bool is_quad_chain(int dyn, int n) { return dyn == kChain && n >= 5 && n <= 8; }

// Per-lane constants.  Rows past the chain end and couplings to links that do
// not exist are handled by zero coefficients instead of branches: every inverse
// mass that multiplies a missing coupling is stored as 0 here, and the diagonal
// of a padded row is 1, so the padded rows solve to zero tension and zero
// acceleration with the same instructions as real rows.
struct QuadChain {
  float l0, l1, invl0, invl1;   // own links r0 = 2s, r1 = 2s+1 (padded: 1)
  float cw0, cw1;               // (2 pi)^2 l: centripetal weight of a rate in rev/s
  float ra0, ra1;               // 1 / (2 pi l): accelerations out in rev/s^2
  float De, Do;                 // diagonals of rows r0, r1 (padded: 1)
  float imD0, imD1;             // im[r0] + im[r0-1], im[r1] + im[r0] (padded: 0)
  float imU0;                   // im[r0]: coupling r0 - r1 (0 unless r1 exists)
  float imU1;                   // im[r1]: coupling r1 - r1+1 (0 unless r1+1 exists)
  float impV;                   // im[r0-1]: coupling r0-1 - r0 (0 on lane 0 or padded r0)
  float g0;                     // gravity on lane 0, 0 elsewhere
  float v0f, v1f, nxt1f;        // 1 where row r0 / r1 / link r1+1 exists
};

template <int CTRL>
__device__ __forceinline__ float qmul(float a, float b) { return qperm<CTRL>(a) * b; }

// Accelerations of the lane's two links from the stage angles' sin/cos, the
// stage angular velocities and the per-step torque terms
// q0, q1 (own links), qp (link r0-1), qn (link r1+1).  Rates come in and
// accelerations go out in revolutions (per second, per second squared).
__device__ __forceinline__ void quad_accel(float s0, float c0, float s1, float c1, float w0, float w1, float q0,
                                           float q1, float qp, float qn, const QuadChain& K, float& a0, float& a1) {
  const float sN = qperm<kQNext1>(s0), cN = qperm<kQNext1>(c0);
  const float Cn0 = fmaf(c0, c1, s0 * s1);           // links r0, r1
  const float Sn0 = fmaf(s0, c1, -c0 * s1);
  const float Cn1 = fmaf(c1, cN, s1 * sN);           // links r1, r1+1
  const float Sn1 = fmaf(s1, cN, -c1 * sN);
  const float Cp = qperm<kQPrev1>(Cn1), Sp = qperm<kQPrev1>(Sn1);   // links r0-1, r0
  // tension rows r0 (even) and r1 (odd): Lo x_{r-1} + D x_r + Up x_{r+1} = R
  const float Ue = -K.imU0 * Cn0, Le = -K.impV * Cp;
  const float Re = fmaf(K.cw0 * w0, w0, fmaf(-K.imU0 * q1, Sn0, fmaf(K.impV * qp, Sp, K.g0 * c0)));
  const float Uo = -K.imU1 * Cn1, Lo = Ue;
  const float Ro = fmaf(K.cw1 * w1, w1, fmaf(-K.imU1 * qn, Sn1, K.imU0 * q0 * Sn0));
  // eliminate the even unknowns from the odd rows
  const float iDe = __builtin_amdgcn_rcpf(K.De);
  const float al = Lo * iDe;
  const float ga = qmul<kQNext1>(iDe, Uo);
  float A = -al * Le;
  float Bv = fmaf(-ga, qperm<kQNext1>(Le), fmaf(-al, Ue, K.Do));
  float C = -ga * qperm<kQNext1>(Ue);
  float R = fmaf(-ga, qperm<kQNext1>(Re), fmaf(-al, Re, Ro));
  // parallel cyclic reduction of the four odd rows, distance 1 (A = 0 on lane
  // 0 and C = 0 on lane 3 already, so the wrapped neighbours contribute 0)
  {
    const float iB = __builtin_amdgcn_rcpf(Bv);
    const float x1 = -A * qperm<kQPrev1>(iB);
    const float y1 = -C * qperm<kQNext1>(iB);
    const float Ap = qperm<kQPrev1>(A), Cp1 = qperm<kQPrev1>(C), Rp = qperm<kQPrev1>(R);
    const float An = qperm<kQNext1>(A), Cn = qperm<kQNext1>(C), Rn = qperm<kQNext1>(R);
    Bv = fmaf(y1, An, fmaf(x1, Cp1, Bv));
    R = fmaf(y1, Rn, fmaf(x1, Rp, R));
    A = x1 * Ap;
    C = y1 * Cn;
  }
  // distance 2
  {
    const float iB = __builtin_amdgcn_rcpf(Bv);
    const float x2 = -A * qperm<kQPrev2>(iB);
    const float y2 = -C * qperm<kQNext2>(iB);
    Bv = fmaf(y2, qperm<kQNext2>(A), fmaf(x2, qperm<kQPrev2>(C), Bv));
    R = fmaf(y2, qperm<kQNext2>(R), fmaf(x2, qperm<kQPrev2>(R), R));
  }
  const float xo = R * __builtin_amdgcn_rcpf(Bv);              // tension of link r1
  const float xo_prev = qperm<kQPrev1>(xo);                     // tension of link r0-1
  const float xe = fmaf(-Le, xo_prev, fmaf(-Ue, xo, Re)) * iDe; // tension of link r0
  const float xe_next = qperm<kQNext1>(xe);                     // tension of link r1+1
  float A0 = fmaf(K.imD0, q0, -K.g0 * s0);
  A0 = fmaf(-K.imU0, fmaf(xo, Sn0, q1 * Cn0), A0);
  A0 = fmaf(-K.impV, fmaf(-xo_prev, Sp, qp * Cp), A0);
  float A1 = K.imD1 * q1;
  A1 = fmaf(-K.imU1, fmaf(xe_next, Sn1, qn * Cn1), A1);
  A1 = fmaf(-K.imU0, fmaf(-xe, Sn0, q0 * Cn0), A1);
  a0 = A0 * K.ra0;
  a1 = A1 * K.ra1;
}

// One candidate b per quad; s is the lane within the quad.  All four lanes of a
// quad must run this together.
template <int N>
__device__ __forceinline__ void rollout_chain_quad(const PlanDesc& P, int b, int s) {
  static_assert(N >= 5 && N <= 8, "quad-lane chain covers 5..8 links");
  const float* tk = P.task;
  QuadChain K;
  const int r0 = 2 * s, r1 = 2 * s + 1;
  const bool v0 = r0 < N, v1 = r1 < N, nxt1 = r1 + 1 < N;
  const float g = tk[0];
  const float wg = tk[1], wu = tk[2], tx = tk[3], ty = tk[4];
  const float im0 = v0 ? 1.0f / tk[5 + r0] : 0.0f;
  const float im1 = v1 ? 1.0f / tk[5 + r1] : 0.0f;
  const float imp = (r0 > 0 && r0 - 1 < N) ? 1.0f / tk[5 + r0 - 1] : 0.0f;
  K.l0 = v0 ? tk[5 + N + r0] : 1.0f;
  K.l1 = v1 ? tk[5 + N + r1] : 1.0f;
  K.invl0 = 1.0f / K.l0;
  K.invl1 = 1.0f / K.l1;
  K.cw0 = kTwoPiSq * K.l0;
  K.cw1 = kTwoPiSq * K.l1;
  K.ra0 = kInvTwoPi * K.invl0;
  K.ra1 = kInvTwoPi * K.invl1;
  K.De = v0 ? im0 + imp : 1.0f;
  K.Do = v1 ? im1 + im0 : 1.0f;
  K.imD0 = v0 ? im0 + imp : 0.0f;
  K.imD1 = v1 ? im1 + im0 : 0.0f;
  K.imU0 = v1 ? im0 : 0.0f;
  K.imU1 = nxt1 ? im1 : 0.0f;
  K.impV = v0 ? imp : 0.0f;
  K.g0 = (s == 0) ? g : 0.0f;
  K.v0f = v0 ? 1.0f : 0.0f;
  K.v1f = v1 ? 1.0f : 0.0f;
  K.nxt1f = nxt1 ? 1.0f : 0.0f;
  const float dt = P.dt, hdt = 0.5f * P.dt, dt6 = P.dt * (1.0f / 6.0f);
  // Angles and rates are carried in revolutions (per second): v_sin / v_cos
  // take revolutions, so a stage angle goes to them as it is.  The own angles
  // are kept reduced to [0, 1) (once per step), which holds every stage
  // argument within a step's motion of that range; the whole turns taken off
  // are only tracked for the state output.
  float ph0 = v0 ? kInvTwoPi * P.x0[r0] : 0.0f, ph1 = v1 ? kInvTwoPi * P.x0[r1] : 0.0f;
  float om0 = v0 ? kInvTwoPi * P.x0[N + r0] : 0.0f, om1 = v1 ? kInvTwoPi * P.x0[N + r1] : 0.0f;
  float turn0 = floorf(ph0), turn1 = floorf(ph1);
  ph0 -= turn0;
  ph1 -= turn1;
  float s0, c0, s1, c1;
  rev_sincos(ph0, &s0, &c0);
  rev_sincos(ph1, &s1, &c1);
  // controls of padded rows are read from the last real row and zeroed by v0f/v1f
  const size_t ld = static_cast<size_t>(P.ldU);
  const float* p0 = P.U + b + static_cast<size_t>(v0 ? r0 : N - 1) * ld;
  const float* p1 = P.U + b + static_cast<size_t>(v1 ? r1 : N - 1) * ld;
  const size_t row = static_cast<size_t>(N) * ld;
  float u0 = K.v0f * *p0, u1 = K.v1f * *p1;
  float cost = 0.0f;   // goal term; the control term is summed per lane (uacc) and joined once
  float uacc = 0.0f;
  // recording the states is a separate instantiation, chosen once per wave, so
  // the step loop of the other waves carries no branch
  auto run = [&](auto rec) {
  for (int t = 0; t < P.T; ++t) {
    // next step's controls (the last step re-reads its own row)
    const size_t adv = (t + 1 < P.T) ? row : 0;
    p0 += adv;
    p1 += adv;
    const float un0 = K.v0f * *p0;
    const float un1 = K.v1f * *p1;
    // torque terms of this step
    const float q0 = (u0 - u1) * K.invl0;
    const float q1 = fmaf(-K.nxt1f, qperm<kQNext1>(u0), u1) * K.invl1;
    const float qp = qperm<kQPrev1>(q1), qn = qperm<kQNext1>(q0);

    float k0, k1;
    quad_accel(s0, c0, s1, c1, om0, om1, q0, q1, qp, qn, K, k0, k1);
    float aph0 = om0, aph1 = om1, aom0 = k0, aom1 = k1, oms0 = om0, oms1 = om1;
    // one RK4 stage at offset h with weight wgt; the two half-step stages share
    // a loop body and the full step follows with its constants in place
    auto stage = [&](float h, float wgt) {
      float ss0, cc0, ss1, cc1;
      rev_sincos(fmaf(h, oms0, ph0), &ss0, &cc0);
      rev_sincos(fmaf(h, oms1, ph1), &ss1, &cc1);
      oms0 = fmaf(h, k0, om0);
      oms1 = fmaf(h, k1, om1);
      quad_accel(ss0, cc0, ss1, cc1, oms0, oms1, q0, q1, qp, qn, K, k0, k1);
      aph0 = fmaf(wgt, oms0, aph0);
      aph1 = fmaf(wgt, oms1, aph1);
      aom0 = fmaf(wgt, k0, aom0);
      aom1 = fmaf(wgt, k1, aom1);
    };
#pragma unroll 1
    for (int half = 0; half < 2; ++half) stage(hdt, 2.0f);
    stage(dt, 1.0f);
    // padded rows have zero velocity and acceleration, so their angle stays 0
    const float pu0 = fmaf(dt6, aph0, ph0), pu1 = fmaf(dt6, aph1, ph1);
    ph0 = __builtin_amdgcn_fractf(pu0);
    ph1 = __builtin_amdgcn_fractf(pu1);
    om0 = fmaf(dt6, aom0, om0);
    om1 = fmaf(dt6, aom1, om1);
    rev_sincos(ph0, &s0, &c0);
    rev_sincos(ph1, &s1, &c1);
    const float l0v = K.v0f * K.l0, l1v = K.v1f * K.l1;
    float ex = fmaf(l0v, s0, l1v * s1);
    float ey = -fmaf(l0v, c0, l1v * c1);
    uacc = fmaf(u0, u0, fmaf(u1, u1, uacc));
    ex = quad_sum(ex);
    ey = quad_sum(ey);
    const float dx = ex - tx, dy = ey - ty;
    cost = fmaf(wg, fmaf(dx, dx, dy * dy), cost);
    if (decltype(rec)::value && b < P.n_dbg) {
      float* X = P.X + b;
      const size_t ldx = static_cast<size_t>(P.n_dbg);
      turn0 += floorf(pu0);
      turn1 += floorf(pu1);
      if (v0) { X[(t * 2 * N + r0) * ldx] = kTwoPi * (turn0 + ph0); X[(t * 2 * N + N + r0) * ldx] = kTwoPi * om0; }
      if (v1) { X[(t * 2 * N + r1) * ldx] = kTwoPi * (turn1 + ph1); X[(t * 2 * N + N + r1) * ldx] = kTwoPi * om1; }
    }
    u0 = un0;
    u1 = un1;
  }
  };
  if (__builtin_amdgcn_ballot_w64(b < P.n_dbg) != 0) run(std::true_type{});
  else run(std::false_type{});
  cost = fmaf(wu, quad_sum(uacc), cost);
  if (s == 0) P.cost[b] = finite_or_inf(cost);
}

// ------------------------------------------------------------------ pair-lane chain
// Even chains of 10 or more links: two lanes share one candidate.  Lane A owns
// links 0..M-1 in order, lane B links N-1..M in reverse (M = N/2), so local row
// i of both lanes runs the same instructions: the tension system is eliminated
// from both ends towards the middle (a twisted factorisation), the two middle
// unknowns come from a 2x2 solve with one value swapped across the pair, and
// back-substitution runs outwards.  Neighbour terms are picked with per-lane
// selects on compile-time indices, so nothing is indexed dynamically.  Half the
// registers of the one-lane form and twice the lanes.

__host__ __device__ constexpr bool is_pair_chain(int dyn, int n) {
  return (dyn == kChain || dyn == kChainContact) && n >= 10 && (n % 2) == 0;
}

template <int N>
constexpr bool pair_chain_links() { return N >= 10 && (N % 2) == 0; }

__device__ __forceinline__ float pswap(float v) { return qperm<kQXor1>(v); }

// Both lanes work in their own local order: local link i of lane B is global
// link N-1-i, so walking i upwards moves from the lane's outer end towards the
// middle.  Lane B also takes its link directions reversed (sin and cos of
// phi + pi), i.e. pointing from local node i to local node i+1 as in lane A.  In
// that frame the tension system, the contact terms and the accelerations have
// the same form in both lanes: with node i between local links i-1 and i,
//   row i:  -imP_i P_{i-1} T_{i-1} + (imP_i + imN_i) T_i - imN_i P_i T_{i+1} = rhs_i
// (imP, imN: inverse masses of the nodes before and after the link), and the
// relative acceleration of a link's two nodes is F[i+1] - F[i].  Lane A's node 0
// is the pinned base (inverse mass 0, relative acceleration +g against free fall);
// lane B's node 0 is the free tip.  Only the torque difference q, the start of
// the node positions (the tip, for lane B) and the sign of the end-effector sum
// depend on the lane, once per step.

// EQ: every link of the chain has the same length, held once (the per-link
// arrays would sit in AGPRs of the long-chain kernels and cost a move per use).
template <int N, bool EQ = false>
struct PairConsts {
  static constexpr int M = N / 2;
  float l[EQ ? 1 : M], invl[EQ ? 1 : M];   // own links in local order
  __device__ __forceinline__ float len(int i) const { return l[EQ ? 0 : i]; }
  __device__ __forceinline__ float ilen(int i) const { return invl[EQ ? 0 : i]; }
  float im[M + 1];       // inverse masses of local nodes 0..M (node M is the middle one)
  float half;            // revolution offset of the local frame: 0 (lane A) or 1/2 (lane B)
  float bf;              // 1 for lane B, 0 for lane A
  float g0;              // base node's relative acceleration against free fall: g (lane A), 0 (lane B)
  float sgn;             // +1 (lane A), -1 (lane B)
  float yg, kc, dc, inv_vs, muf;   // contact only
  float ks;              // contact only: 2 log2(e) / v_slip, the slip-velocity scale of the tanh by exp2
  bool B;                // lane owns the tip half
};

// Torque products of one RK4 step (the controls are held over its four
// stages), per local link i with q_i = (u_i - u_distal) / l_i and q_n the next
// link's term (the other lane's at the middle):
//   qa_i = -im_{i+1} q_n,  qb_i = im_i q_{i-1} (i > 0),  qc_i = (im_i + im_{i+1}) q_i.
template <int N>
struct PairTorque {
  float qa[N / 2], qb[N / 2], qc[N / 2];
};

template <int N>
__device__ __forceinline__ int pair_link(bool B, int i) { return B ? N - 1 - i : i; }

// mass index (0-based link whose distal end carries it) of local node i
template <int N>
__device__ __forceinline__ int pair_node_mass(bool B, int i) { return B ? (i < N / 2 ? N - 1 - i : N / 2 - 1) : i - 1; }

template <int N, bool EQ>
__device__ __forceinline__ void pair_load_masses(const float* m, PairConsts<N, EQ>& K) {
  constexpr int M = N / 2;
#pragma unroll
  for (int i = 0; i <= M; ++i) K.im[i] = (i == 0 && !K.B) ? 0.0f : 1.0f / m[pair_node_mass<N>(K.B, i)];
}



// Local-frame accelerations of the lane's M links from the local sin/cos, the
// angular velocities and the per-step torque terms q (q_o: the other lane's
// link next to the middle).
// Tension solve and link accelerations of pair_accel from the node relative
// accelerations F[0..M] (contact and, at the base node, gravity).  FORCES =
// false: no node touches the ground, so F is zero but for the base node's g0,
// and the terms that would multiply zeros are left out (same values).
template <int N, bool FORCES, bool EQ>
__device__ __forceinline__ void pair_solve(const float (&s)[N / 2], const float (&c)[N / 2], const float (&w)[N / 2],
                                           const PairTorque<N>& Q, const PairConsts<N, EQ>& K, float so, float co,
                                           const float (&Fx)[N / 2 + 1], const float (&Fy)[N / 2 + 1],
                                           float (&acc)[N / 2]) {
  constexpr int M = N / 2;
  // forward elimination from the lane's outer end towards the middle
  float cp[M], dp[M];
  float cp_prev = 0.0f, dp_prev = 0.0f;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const float sn = (i + 1 < M) ? s[i + 1] : so, cn = (i + 1 < M) ? c[i + 1] : co;
    const float Pn = fmaf(c[i], cn, s[i] * sn);            // cos(phi_i - phi_{i+1})
    const float Qn = fmaf(s[i], cn, -c[i] * sn);           // sin(phi_i - phi_{i+1})
    float rhs = K.len(i) * w[i] * w[i];
    if constexpr (FORCES) {
      rhs = fmaf(s[i], Fx[i + 1] - Fx[i], rhs);
      rhs = fmaf(-c[i], Fy[i + 1] - Fy[i], rhs);
    } else if (i == 0) {
      rhs = fmaf(-c[0], -K.g0, rhs);
    }
    rhs = fmaf(Q.qa[i], Qn, rhs);
    float Dg = K.im[i] + K.im[i + 1];
    if (i > 0) {
      const float Pp = fmaf(c[i - 1], c[i], s[i - 1] * s[i]);
      const float Qp = fmaf(s[i - 1], c[i], -c[i - 1] * s[i]);
      rhs = fmaf(Q.qb[i], Qp, rhs);
      const float Lp = -K.im[i] * Pp;
      const float inv = __builtin_amdgcn_rcpf(fmaf(-Lp, cp_prev, Dg));
      cp_prev = -K.im[i + 1] * Pn * inv;
      dp_prev = fmaf(-Lp, dp_prev, rhs) * inv;
    } else {
      const float inv = __builtin_amdgcn_rcpf(Dg);
      cp_prev = -K.im[i + 1] * Pn * inv;
      dp_prev = rhs * inv;
    }
    cp[i] = cp_prev;
    dp[i] = dp_prev;
  }
  // the two middle unknowns, then back-substitution outwards (dp becomes the tension)
  {
    const float cpo = pswap(cp[M - 1]), dpo = pswap(dp[M - 1]);
    dp[M - 1] = fmaf(-cp[M - 1], dpo, dp[M - 1]) * __builtin_amdgcn_rcpf(fmaf(-cp[M - 1], cpo, 1.0f));
  }
#pragma unroll
  for (int i = M - 2; i >= 0; --i) dp[i] = fmaf(-cp[i], dp[i + 1], dp[i]);
  const float xo = pswap(dp[M - 1]);
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const float sn = (i + 1 < M) ? s[i + 1] : so, cn = (i + 1 < M) ? c[i + 1] : co;
    const float Pn = fmaf(c[i], cn, s[i] * sn);
    const float Qn = fmaf(s[i], cn, -c[i] * sn);
    const float Tn = (i + 1 < M) ? dp[i + 1] : xo;
    float a = fmaf(Q.qa[i], Pn, Q.qc[i]);
    a = fmaf(-K.im[i + 1] * Tn, Qn, a);
    if (i > 0) {
      const float Pp = fmaf(c[i - 1], c[i], s[i - 1] * s[i]);
      const float Qp = fmaf(s[i - 1], c[i], -c[i - 1] * s[i]);
      a = fmaf(-Q.qb[i], Pp, a);
      a = fmaf(K.im[i] * dp[i - 1], Qp, a);
    }
    if constexpr (FORCES) {
      a = fmaf(c[i], Fx[i + 1] - Fx[i], fmaf(s[i], Fy[i + 1] - Fy[i], a));
    } else if (i == 0) {
      a = fmaf(s[0], -K.g0, a);
    }
    acc[i] = a * K.ilen(i);
  }
}


template <int N, bool CONTACT, bool EQ>
__device__ __forceinline__ void pair_accel(const float (&s)[N / 2], const float (&c)[N / 2], const float (&w)[N / 2],
                                           const PairTorque<N>& Q, const PairConsts<N, EQ>& K, float (&acc)[N / 2]) {
  constexpr int M = N / 2;
  // the other lane's middle link in this lane's frame (its frame is reversed)
  const float so = -pswap(s[M - 1]), co = -pswap(c[M - 1]);
  // node relative accelerations F[0..M]
  float Fx[M + 1], Fy[M + 1];
  if constexpr (CONTACT) {
    // node heights y_{i+1} = y_i - l_i c_i; lane B starts at the tip: the sum
    // of lane A's links minus its own (reversed) ones
    float py[M + 1];
    py[0] = 0.0f;
#pragma unroll
    for (int i = 0; i < M; ++i) py[i + 1] = fmaf(-K.len(i), c[i], py[i]);
    const float y0 = K.bf * (pswap(py[M]) - py[M]);
    // One branch for the wave: the contact terms of all nodes are formed when
    // some node of some lane is below the ground (the lowest height decides, as
    // rounding of the offset is monotone), otherwise every node is free.  In
    // the branch the normal force is selected (zero above the ground) and the
    // friction factor is formed for every node, so the thirteen transcendental
    // chains interleave; a select on the friction term itself would be turned
    // back into a branch per node by the compiler.
    float lowest = py[0];
#pragma unroll
    for (int i = 1; i <= M; ++i) lowest = fminf(lowest, py[i]);
    if (__builtin_amdgcn_ballot_w64(lowest + y0 < K.yg) != 0) {
      // node velocities v_{i+1} = v_i + l_i w_i (c_i, s_i), lane B's from the tip
      float vx[M + 1], vy[M + 1];
      vx[0] = 0.0f; vy[0] = 0.0f;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const float lw = K.len(i) * w[i];
        vx[i + 1] = fmaf(lw, c[i], vx[i]);
        vy[i + 1] = fmaf(lw, s[i], vy[i]);
      }
      const float u0 = K.bf * (pswap(vx[M]) - vx[M]), v0 = K.bf * (pswap(vy[M]) - vy[M]);
      // the tip offsets of lane B folded into per-evaluation constants:
      // penetration (yg - y0) - y_i, damping dc (v_i + v0), slip ks (u_i + u0)
      const float ygl = K.yg - y0, dv0 = -K.dc * v0, ku0 = K.ks * u0;
      // friction -muf tanh(v / v_slip) = -muf (1 - 2 r) = 2 muf r - muf, r = 1 / (1 + e^{2 v / v_slip})
      const float mu2 = 2.0f * K.muf, nmu = -K.muf;
#pragma unroll
      for (int i = 0; i <= M; ++i) {
        const float pen = ygl - py[i];
        const float fn = pen > 0.0f ? fmaxf(fmaf(K.kc, pen, fmaf(-K.dc, vy[i], dv0)), 0.0f) : 0.0f;
        const float fr = fmaf(mu2, __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(fmaf(K.ks, vx[i], ku0))), nmu);
        Fy[i] = fn * K.im[i];
        Fx[i] = Fy[i] * fr;
      }
      Fy[0] += K.g0;
      pair_solve<N, true>(s, c, w, Q, K, so, co, Fx, Fy, acc);
      return;
    }
  }
  pair_solve<N, false>(s, c, w, Q, K, so, co, Fx, Fy, acc);
}

template <int N, bool CONTACT, bool EQ>
__device__ __forceinline__ void pair_setup(const PlanDesc& P, bool B, PairConsts<N, EQ>& K) {
  constexpr int M = N / 2;
  const float* tk = P.task;
  K.B = B;
  K.half = B ? 0.5f : 0.0f;
  K.bf = B ? 1.0f : 0.0f;
  K.g0 = B ? 0.0f : tk[0];
  K.sgn = B ? -1.0f : 1.0f;
#pragma unroll
  for (int i = 0; i < (EQ ? 1 : M); ++i) {
    K.l[i] = tk[5 + N + pair_link<N>(B, i)];
    K.invl[i] = 1.0f / K.l[i];
  }
  if constexpr (CONTACT) {
    K.yg = tk[5 + 2 * N]; K.kc = tk[6 + 2 * N]; K.dc = tk[7 + 2 * N]; K.inv_vs = 1.0f / tk[8 + 2 * N];
    K.ks = 2.8853900817779268f * K.inv_vs;
  } else {
    pair_load_masses<N>(tk + 5, K);
    K.ks = 0.0f;
    K.muf = 0.0f; K.yg = 0.0f; K.kc = 0.0f; K.dc = 0.0f; K.inv_vs = 0.0f;
  }
}

// Steps [t0, t1) of candidate b from the lane's link angles ph and rates om
// (updated in place), adding each step's cost to `cost`.  Angles are carried
// in revolutions of the lane's local frame (lane B's are offset by half a
// turn) and reduced to [0, 1) after every step, so a stage angle goes to
// v_sin / v_cos as it is; rates stay in rad/s, and the stage offsets h / 2pi
// are uniform.  `turn` holds the whole turns taken off, kept up to date only
// for recorded candidates (the state output gives physical radians).
template <int N, bool CONTACT, bool EQ>
__device__ __forceinline__ void pair_steps(const PlanDesc& P, const PairConsts<N, EQ>& K, int b, float (&ph)[N / 2],
                                           float (&om)[N / 2], float (&turn)[N / 2], float& cost, int t0, int t1,
                                           bool record, int rep = 0) {
  constexpr int M = N / 2;
  const bool B = K.B;
  const float* tk = P.task;
  const float wg = tk[1], wu = tk[2], tgx = tk[3], tgy = tk[4];
  const float dt = P.dt, hdt = 0.5f * P.dt, dt6 = P.dt * (1.0f / 6.0f);
  const float dtr = kInvTwoPi * dt, hdtr = kInvTwoPi * hdt, dt6r = kInvTwoPi * dt6;
  float s[M], c[M], hu[M];
#pragma unroll
  for (int i = 0; i < M; ++i) rev_sincos_unit(ph[i], &s[i], &c[i], &hu[i]);
  // Controls through a buffer descriptor based at step t's block of U rows:
  // the lane's byte offset (its link's row and its candidate) is the same at
  // every step and below 2^31 for every valid plan (N <= 24, ldU <= 2^24 + 64),
  // so a load takes no address arithmetic.
  const uint32_t ldu = static_cast<uint32_t>(P.ldU);
  uint32_t uoff[M];
#pragma unroll
  for (int i = 0; i < M; ++i) uoff[i] = (static_cast<uint32_t>(pair_link<N>(B, i)) * ldu + static_cast<uint32_t>(b)) * 4u;
  const int step_bytes = static_cast<int>(static_cast<uint32_t>(N) * ldu * 4u);
  auto step_rows = [&](int t) {
    return __builtin_amdgcn_make_buffer_rsrc(P.U + static_cast<size_t>(t) * N * ldu, static_cast<short>(0), step_bytes,
                                             kBufferWord3);
  };
  float u[M];
  {
    const auto rs = step_rows(t0);
#pragma unroll
    for (int i = 0; i < M; ++i) u[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, uoff[i], 0, 0));
  }
  for (int t = t0; t < t1; ++t) {
    // next step's controls, loaded a whole step ahead; the last step re-reads
    // its own row (no select on the loaded values, which would make the wave
    // wait for the loads at once)
    float un[M];
    const int tn = (t + 1 < t1) ? t + 1 : t;
    const auto rs = step_rows(tn);
#pragma unroll
    for (int i = 0; i < M; ++i) un[i] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, uoff[i], 0, 0));
    // torque terms (u_k - u_{k+1}) / l_k: the distal neighbour is local i+1 in lane A
    // (the other lane's link at the middle) and local i-1 in lane B (none at the tip)
    float q[M];
    const float u_other = pswap(u[M - 1]);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const float u_tip = B ? (i > 0 ? u[i - 1] : 0.0f) : (i + 1 < M ? u[i + 1] : u_other);
      q[i] = (u[i] - u_tip) * K.ilen(i);
    }
    const float q_o = pswap(q[M - 1]);
    PairTorque<N> Q;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      Q.qa[i] = -K.im[i + 1] * ((i + 1 < M) ? q[i + 1] : q_o);
      Q.qb[i] = (i > 0) ? K.im[i] * q[i - 1] : 0.0f;
      Q.qc[i] = (K.im[i] + K.im[i + 1]) * q[i];
    }

    float kk[M], oms[M], aph[M], aom[M];
    pair_accel<N, CONTACT>(s, c, om, Q, K, kk);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      aph[i] = om[i];
      aom[i] = kk[i];
      oms[i] = om[i];
    }
#pragma unroll 1
    for (int stage = 1; stage < 4; ++stage) {
      const float h = (stage == 3) ? dt : hdt;
      const float hr = (stage == 3) ? dtr : hdtr;
      float s2[M], c2[M];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        rev_sincos_scaled(fmaf(hr, oms[i], ph[i]), hu[i], &s2[i], &c2[i]);
        oms[i] = fmaf(h, kk[i], om[i]);
      }
      pair_accel<N, CONTACT>(s2, c2, oms, Q, K, kk);
      const float wgt = (stage == 3) ? 1.0f : 2.0f;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        aph[i] = fmaf(wgt, oms[i], aph[i]);
        aom[i] = fmaf(wgt, kk[i], aom[i]);
      }
    }
    float ex = 0.0f, ey = 0.0f, uu = 0.0f;
    float pu[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      pu[i] = fmaf(dt6r, aph[i], ph[i]);
      ph[i] = __builtin_amdgcn_fractf(pu[i]);
      om[i] = fmaf(dt6, aom[i], om[i]);
      rev_sincos_unit(ph[i], &s[i], &c[i], &hu[i]);
      ex = fmaf(K.len(i), s[i], ex);
      ey = fmaf(-K.len(i), c[i], ey);
      uu = fmaf(u[i], u[i], uu);
    }
    // end effector: the lanes' link sums, lane B's taken back to the physical frame
    ex *= K.sgn;
    ey *= K.sgn;
    ex += pswap(ex);
    ey += pswap(ey);
    uu += pswap(uu);
    const float dx = ex - tgx, dy = ey - tgy;
    cost += fmaf(wg, fmaf(dx, dx, dy * dy), wu * uu);
    if (record && b < P.n_dbg) {
      float* X = P.X + static_cast<size_t>(rep) * P.T * P.d * P.n_dbg + b;
      const size_t ldx = static_cast<size_t>(P.n_dbg);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const int k = pair_link<N>(B, i);
        turn[i] += floorf(pu[i]);
        X[(t * 2 * N + k) * ldx] = kTwoPi * ((turn[i] + ph[i]) - K.half);
        X[(t * 2 * N + N + k) * ldx] = om[i];
      }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) u[i] = un[i];
  }
}

// Start state of the lane's links: angles in revolutions of the local frame,
// reduced to [0, 1), with the whole turns taken off; rates in rad/s.
template <int N, bool EQ>
__device__ __forceinline__ void pair_start(const PlanDesc& P, const PairConsts<N, EQ>& K, float (&ph)[N / 2],
                                           float (&om)[N / 2], float (&turn)[N / 2]) {
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const int k = pair_link<N>(K.B, i);
    const float r = fmaf(P.x0[k], kInvTwoPi, K.half);
    turn[i] = floorf(r);
    ph[i] = r - turn[i];
    om[i] = P.x0[N + k];
  }
}

// One candidate b per lane pair; B is the tip-half lane.  Both lanes of a pair
// must run this together.
template <int N, bool CONTACT>
__device__ __forceinline__ void rollout_chain_pair(const PlanDesc& P, int b, bool B) {
  static_assert(N >= 10 && N % 2 == 0, "pair-lane chain needs an even link count >= 10");
  constexpr int M = N / 2;
  PairConsts<N> K;
  pair_setup<N, CONTACT>(P, B, K);
  // randomised models: the candidate's cost is the mean over R rollouts
  const int R = CONTACT ? P.R : 1;
  float total = 0.0f;
#pragma unroll 1
  for (int rep = 0; rep < R; ++rep) {
    if constexpr (CONTACT) {
      const float* sp = P.sparams + (static_cast<size_t>(rep) * P.B + b) * (N + 1);
      pair_load_masses<N>(sp, K);
      K.muf = sp[N];
    }
    float ph[M], om[M], turn[M];
    pair_start<N>(P, K, ph, om, turn);
    float cost = 0.0f;
    pair_steps<N, CONTACT>(P, K, b, ph, om, turn, cost, 0, P.T, true, rep);
    total += cost;
  }
  if (!B) P.cost[b] = finite_or_inf(R == 1 ? total : total / static_cast<float>(R));
}

// ------------------------------------------------------------------ time-sliced pair rollout
// A launch of G pair-lane waves on fewer SIMDs runs in ceil(G / SIMDs) rounds
// of whole horizons; when G is slightly above a multiple, the last round leaves
// most SIMDs idle (24 links, 69632 candidates: 2176 waves, 3 rounds for 2.125
// rounds of work).  Here the horizon is cut into S segments and resident waves
// take (wave group, segment) units from a counter in segment-major order, saving
// the group's state (angles, rates, cost so far) between segments; a unit waits
// for its group's previous segment, taken at least one full round earlier.  The
// arithmetic per candidate is exactly that of the plain rollout.

struct SegCtl {
  uint32_t head;     // next unit
  uint32_t epoch;    // launch counter: done flags hold epoch * 256 + segments completed
  uint32_t error;    // bit 0: a wait timed out
  uint32_t pad;
};

__device__ __forceinline__ uint32_t seg_tag(uint32_t epoch, int done) { return (epoch << 8) | static_cast<uint32_t>(done); }

// One wave: lanes 2c, 2c+1 hold candidate g*32 + c.  `state` holds 3M + 1
// floats per lane per group, laid out [k][group][lane]: angles, rates, cost so
// far, and the whole turns of recorded candidates.
template <int N, bool CONTACT, bool EQ = false>
__device__ __forceinline__ void rollout_pair_segmented(const PlanDesc& P, SegCtl* ctl, uint32_t* done, float* state,
                                                       int S, int seg_len, uint64_t wait_ticks) {
  constexpr int M = N / 2;
  const int lane = threadIdx.x & 63;
  const bool B = (lane & 1) != 0;
  const int groups = (P.B + 31) / 32;
  const uint32_t total = static_cast<uint32_t>(groups) * static_cast<uint32_t>(S);
  const uint32_t epoch = __hip_atomic_load(&ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  PairConsts<N, EQ> K;
  pair_setup<N, CONTACT>(P, B, K);
  for (;;) {
    uint32_t u = 0u;
    if (lane == 0) u = atomicAdd(&ctl->head, 1u);
    u = __builtin_amdgcn_readfirstlane(u);
    if (u >= total) break;
    const int seg = static_cast<int>(u / static_cast<uint32_t>(groups));
    const int g = static_cast<int>(u - static_cast<uint32_t>(seg) * static_cast<uint32_t>(groups));
    if (seg > 0) {
      int ok = 1;
      if (lane == 0) {
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(&done[g], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != seg_tag(epoch, seg)) {
          if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
              wall_clock64() - t0 > wait_ticks) {
            atomicOr(&ctl->error, 1u);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      ok = __builtin_amdgcn_readfirstlane(ok);
      if (!ok) break;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const int bb = g * 32 + (lane >> 1);
    const bool live = bb < P.B;
    const int b = live ? bb : P.B - 1;   // idle pairs shadow the last candidate and store nothing
    if constexpr (CONTACT) {
      const float* sp = P.sparams + static_cast<size_t>(b) * (N + 1);
      pair_load_masses<N>(sp, K);
      K.muf = sp[N];
    }
    float ph[M], om[M], turn[M], cost;
    const size_t gl = static_cast<size_t>(g) * 64 + static_cast<size_t>(lane);
    const size_t kstride = static_cast<size_t>(groups) * 64;
    // the whole turns travel between segments only where states are recorded
    const bool rec = live && b < P.n_dbg;
    if (seg == 0) {
      pair_start<N>(P, K, ph, om, turn);
      cost = 0.0f;
    } else {
#pragma unroll
      for (int i = 0; i < M; ++i) {
        ph[i] = state[i * kstride + gl];
        om[i] = state[(M + i) * kstride + gl];
        turn[i] = rec ? state[(2 * M + 1 + i) * kstride + gl] : 0.0f;
      }
      cost = state[2 * M * kstride + gl];
    }
    const int t0 = seg * seg_len;
    const int t1 = min(P.T, t0 + seg_len);
    pair_steps<N, CONTACT>(P, K, b, ph, om, turn, cost, t0, t1, live);
    if (seg + 1 < S) {
#pragma unroll
      for (int i = 0; i < M; ++i) {
        state[i * kstride + gl] = ph[i];
        state[(M + i) * kstride + gl] = om[i];
        if (rec) state[(2 * M + 1 + i) * kstride + gl] = turn[i];
      }
      state[2 * M * kstride + gl] = cost;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      if (lane == 0) __hip_atomic_store(&done[g], seg_tag(epoch, seg + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (live && !B) {
      P.cost[b] = finite_or_inf(cost);
    }
  }
}

// ------------------------------------------------------------------ reductions
// One DPP step of a wave reduction: lanes without a source (and rows outside
// ROWS) contribute +0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xF, false));
}

// Sum over the wave in a fixed order with DPP row shifts and row broadcasts
// (no LDS round trips): in-row steps of 1, 2, 4 and 8 lanes, row 0's total into
// row 1 and row 2's into row 3, then lane 31 into rows 2 and 3; lane 63 holds
// the sum, which every lane reads.
__device__ __forceinline__ float wave_sum64(float v) {
  v += dpp_f32<0x111, 0xF>(v);
  v += dpp_f32<0x112, 0xF>(v);
  v += dpp_f32<0x114, 0xF>(v);
  v += dpp_f32<0x118, 0xF>(v);
  v += dpp_f32<0x142, 0xA>(v);
  v += dpp_f32<0x143, 0xC>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// ------------------------------------------------------------------ top-E
// 64-bit keys (order-preserving image of the float cost) << 32 | index are all
// distinct, so an 8-pass byte-wise radix select finds the E-th smallest key
// exactly; the E keys at or below it are then sorted by a bitonic network in
// LDS.  NaN sorts as +inf and -0 as +0.

__device__ __forceinline__ uint32_t cost_order(float c) {
  if (c != c) c = INFINITY;
  uint32_t u = __float_as_uint(c);
  if (u == 0x80000000u) u = 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Inverse of cost_order on its images: the cost itself, except that NaN comes
// back as +inf and -0 as +0 (callers read those two cases from memory).
__device__ __forceinline__ float order_cost(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

// Wave-wide minimum, maximum and inclusive sum with DPP row shifts and row
// broadcasts (no LDS round trips): in-row steps of 1, 2, 4 and 8 lanes, then
// row 0's last lane into row 1 and row 2's into row 3, then lane 31 into rows
// 2 and 3.  Lanes without a source keep their own value (min, max) or add 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(static_cast<int>(old), static_cast<int>(v), CTRL, ROWS, 0xF, false));
}
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, dpp_u32<kDppRowShr1, 0xF>(v, v));
  v = min(v, dpp_u32<kDppRowShr2, 0xF>(v, v));
  v = min(v, dpp_u32<kDppRowShr4, 0xF>(v, v));
  v = min(v, dpp_u32<kDppRowShr8, 0xF>(v, v));
  v = min(v, dpp_u32<kDppRowBcast15, 0xA>(v, v));
  v = min(v, dpp_u32<kDppRowBcast31, 0xC>(v, v));
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, dpp_u32<kDppRowShr1, 0xF>(v, v));
  v = max(v, dpp_u32<kDppRowShr2, 0xF>(v, v));
  v = max(v, dpp_u32<kDppRowShr4, 0xF>(v, v));
  v = max(v, dpp_u32<kDppRowShr8, 0xF>(v, v));
  v = max(v, dpp_u32<kDppRowBcast15, 0xA>(v, v));
  v = max(v, dpp_u32<kDppRowBcast31, 0xC>(v, v));
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
}

__device__ __forceinline__ uint32_t wave_inclusive_sum_u32(uint32_t v) {
  v += dpp_u32<kDppRowShr1, 0xF>(0u, v);
  v += dpp_u32<kDppRowShr2, 0xF>(0u, v);
  v += dpp_u32<kDppRowShr4, 0xF>(0u, v);
  v += dpp_u32<kDppRowShr8, 0xF>(0u, v);
  v += dpp_u32<kDppRowBcast15, 0xA>(0u, v);
  v += dpp_u32<kDppRowBcast31, 0xC>(0u, v);
  return v;
}

constexpr int kTopkBins = 2048;      // radix digits of up to 11 bits
constexpr int kTopkCache = 16384;    // batches up to this size keep their cost images in LDS
constexpr int kTopkRankSort = 1024;  // elite sets up to this size are ordered by counting ranks
constexpr int kTopkBoundary = 256;   // a boundary bin this small is ordered by counting ranks

struct TopkSmem {
  uint32_t cache[kTopkCache];                 // cost images of the batch (when it fits)
  unsigned long long keys[kMaxElites];        // selected keys, unordered
  unsigned long long sorted[kTopkRankSort];   // selected keys by rank; the boundary bin before that
  uint32_t hist[kTopkBins];
  unsigned long long prefix;
  uint32_t rank;
  uint32_t count, count2;
  uint32_t sel_count;
  float red[kTopkThreads / 64];
  uint32_t wlo[kTopkThreads / 64], whi[kTopkThreads / 64];
};

// All BS threads find the digit whose bin holds the rank-th key (1-based) of
// hist[0..nbins): each thread owns a run of consecutive bins, a wave scan and
// the wave totals give every run's offset, and the one thread whose run holds
// the rank writes the digit (into the prefix at `shift`), the rank left inside
// that bin and the bin's size to shared memory.  The caller synchronises.
template <int BS>
__device__ __forceinline__ void topk_find_bin(TopkSmem& sm, int nbins, uint32_t rank, unsigned long long prefix,
                                              int shift) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (nbins + BS - 1) / BS;
  const int first = tid * per;
  uint32_t tot = 0;
  for (int i = 0; i < per; ++i)
    if (first + i < nbins) tot += sm.hist[first + i];
  uint32_t inc = wave_inclusive_sum_u32(tot);
  if (lane == 63) sm.wlo[wave] = inc;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < BS / 64 - 1; ++w)
    if (w < wave) inc += sm.wlo[w];
  const uint32_t exc = inc - tot;
  if (exc < rank && rank <= inc) {
    uint32_t rr = rank - exc;
    int d = first;
    for (int i = 0; i < per; ++i) {
      const uint32_t h = sm.hist[first + i];
      if (rr <= h) { d = first + i; sm.sel_count = h; break; }
      rr -= h;
    }
    sm.prefix = prefix | (static_cast<unsigned long long>(d) << shift);
    sm.rank = rr;
  }
}

// Counting ranks of n distinct keys src[0..n) among themselves: tpk threads
// share each key's comparisons (as many as the block allows, at most a wave),
// then the first of them sums their counts (DPP suffix sums within a row of 16
// lanes, LDS permutes across rows).  sink(key, rank) runs once per key.
template <int BS, class Sink>
__device__ __forceinline__ void topk_rank(const unsigned long long* src, int n, Sink sink) {
  int tpk = 1;
  while (tpk < 64 && tpk * 2 * n <= BS) tpk <<= 1;
  const int tid = threadIdx.x, sub = tid & (tpk - 1), per_pass = BS / tpk;
  for (int i0 = 0; i0 < n; i0 += per_pass) {
    const int i = i0 + tid / tpk;
    const unsigned long long k = i < n ? src[i] : 0ull;
    int r = 0;
    if (i < n) {
      int q = sub;
      for (; q + 7 * tpk < n; q += 8 * tpk) {   // eight loads in flight
        unsigned long long c[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) c[u] = src[q + u * tpk];
#pragma unroll
        for (int u = 0; u < 8; ++u) r += c[u] < k ? 1 : 0;
      }
      for (; q < n; q += tpk) r += src[q] < k ? 1 : 0;
    }
    auto shl = [](int x, auto c) {
      return __builtin_amdgcn_update_dpp(0, x, decltype(c)::value, 0xF, 0xF, false);
    };
    if (tpk > 1) r += shl(r, std::integral_constant<int, 0x101>{});
    if (tpk > 2) r += shl(r, std::integral_constant<int, 0x102>{});
    if (tpk > 4) r += shl(r, std::integral_constant<int, 0x104>{});
    if (tpk > 8) r += shl(r, std::integral_constant<int, 0x108>{});
    for (int o = 16; o < tpk; o <<= 1) r += __shfl_xor(r, o, 64);
    if (i < n && sub == 0) sink(k, r);
  }
}

// Appends key to dst, at slots counted by *counter (one bump per wave), on the
// lanes where t holds.  Every lane of the wave must call it.
__device__ __forceinline__ void wave_append(bool t, unsigned long long key, uint32_t* counter,
                                            unsigned long long* dst, uint32_t cap) {
  const unsigned long long m = __ballot(t);
  if (m == 0ull) return;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int leader = __ffsll(static_cast<long long>(m)) - 1;
  uint32_t slot0 = 0u;
  if (lane == leader) slot0 = atomicAdd(counter, static_cast<uint32_t>(__popcll(m)));
  slot0 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(slot0), leader));
  const uint32_t slot = slot0 + static_cast<uint32_t>(__popcll(m & ((1ull << lane) - 1ull)));
  if (t && slot < cap) dst[slot] = key;
}

// Appends every key (image << 32 | index) <= limit to dst.
template <int BS, class Image>
__device__ __forceinline__ void topk_gather(int B, Image image, unsigned long long limit, uint32_t* counter,
                                            unsigned long long* dst, uint32_t cap) {
  for (int base = 0; base < B; base += BS) {
    const int b = base + static_cast<int>(threadIdx.x);
    const unsigned long long key =
        b < B ? (static_cast<unsigned long long>(image(b)) << 32) | static_cast<uint32_t>(b) : ~0ull;
    wave_append(b < B && key <= limit, key, counter, dst, cap);
  }
}

// One sweep, two lists: the keys whose digits above `shift` (of v = image - lo)
// are below the boundary bin's, and the keys of the boundary bin itself.
template <int BS, class Image>
__device__ __forceinline__ void topk_gather_split(int B, uint32_t lo, Image image, int shift,
                                                  unsigned long long pd, uint32_t* c_lo, unsigned long long* d_lo,
                                                  uint32_t cap_lo, uint32_t* c_b, unsigned long long* d_b,
                                                  uint32_t cap_b) {
  if constexpr (BS >= 1024) {
    // one row at a time, one counter bump per wave and list (measured faster
    // than the grouped form below in the 1024-thread single-plan kernel)
    for (int base = 0; base < B; base += BS) {
      const int b = base + static_cast<int>(threadIdx.x);
      unsigned long long key = 0ull, hv = 0ull;
      if (b < B) {
        const uint32_t im = image(b);
        key = (static_cast<unsigned long long>(im) << 32) | static_cast<uint32_t>(b);
        hv = static_cast<unsigned long long>(im - lo) >> shift;
      }
      wave_append(b < B && hv < pd, key, c_lo, d_lo, cap_lo);
      wave_append(b < B && hv == pd, key, c_b, d_b, cap_b);
    }
    return;
  }
  // groups of kGroup rows per wave: the wave ballots every row of the group,
  // reserves the group's slots of each list with one counter bump, then writes
  // (kGroup times fewer round trips to the counters than one bump per row;
  // measured faster in the 256-thread blocks of the batched kernel)
  constexpr int kGroup = 8;
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int base = 0; base < B; base += kGroup * BS) {
    unsigned long long key[kGroup], ml[kGroup], mb[kGroup];
    uint32_t nl = 0u, nbd = 0u;
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int b = base + u * BS + static_cast<int>(threadIdx.x);
      unsigned long long hv = 0ull;
      key[u] = 0ull;
      if (b < B) {
        const uint32_t im = image(b);
        key[u] = (static_cast<unsigned long long>(im) << 32) | static_cast<uint32_t>(b);
        hv = static_cast<unsigned long long>(im - lo) >> shift;
      }
      ml[u] = __ballot(b < B && hv < pd);
      mb[u] = __ballot(b < B && hv == pd);
      nl += static_cast<uint32_t>(__popcll(ml[u]));
      nbd += static_cast<uint32_t>(__popcll(mb[u]));
    }
    uint32_t sl = 0u, sb = 0u;
    if (lane == 0) {
      if (nl) sl = atomicAdd(c_lo, nl);
      if (nbd) sb = atomicAdd(c_b, nbd);
    }
    sl = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(sl), 0));
    sb = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(sb), 0));
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      if ((ml[u] >> lane) & 1ull) {
        const uint32_t slot = sl + static_cast<uint32_t>(__popcll(ml[u] & below));
        if (slot < cap_lo) d_lo[slot] = key[u];
      }
      if ((mb[u] >> lane) & 1ull) {
        const uint32_t slot = sb + static_cast<uint32_t>(__popcll(mb[u] & below));
        if (slot < cap_b) d_b[slot] = key[u];
      }
      sl += static_cast<uint32_t>(__popcll(ml[u]));
      sb += static_cast<uint32_t>(__popcll(mb[u]));
    }
  }
}

// Top-E by a radix select over the order-preserving 32-bit cost image, taken
// relative to the batch minimum so that the first digit spreads the keys over
// the bins instead of piling them on the few that share an exponent.  Once the
// bin that holds the E-th key has at most kTopkBoundary keys (after the first
// digit, for spread-out costs) the select stops: the keys of lower bins are
// elites, and the rank-th smallest keys (image << 32 | index, all distinct) of
// the boundary bin complete the set.  A bin that stays larger down to the last
// digit holds equal images only; a radix over the index bits then orders those
// ties.  The E keys are finally ordered by counting ranks, or by a bitonic
// network for very large E.
template <int BS>
__device__ __forceinline__ const unsigned long long* topk_select(const PlanDesc& P, TopkSmem& sm) {
  const auto cost = gptr(P.cost);
  const int tid = threadIdx.x;
  const int B = P.B, E = P.E;
  const bool cached = B <= kTopkCache;
  auto image = [&](int b) -> uint32_t { return cached ? sm.cache[b] : cost_order(cost[b]); };

  // images, their minimum and maximum (up to eight loads in flight per thread)
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
  constexpr int kLoads = 8;
  for (int b0 = tid; b0 < B; b0 += kLoads * BS) {
    float c[kLoads];
#pragma unroll
    for (int u = 0; u < kLoads; ++u) c[u] = b0 + u * BS < B ? cost[b0 + u * BS] : 0.0f;
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int b = b0 + u * BS;
      if (b < B) {
        const uint32_t o = cost_order(c[u]);
        if (cached) sm.cache[b] = o;
        lo = min(lo, o);
        hi = max(hi, o);
      }
    }
  }
  lo = wave_min_u32(lo);
  hi = wave_max_u32(hi);
  if ((tid & 63) == 0) { sm.wlo[tid >> 6] = lo; sm.whi[tid >> 6] = hi; }
  if (tid == 0) { sm.count = 0u; sm.count2 = 0u; }
  // the first radix pass's histogram is cleared before the same barrier
  for (int i = tid; i < kTopkBins; i += BS) sm.hist[i] = 0u;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < BS / 64; ++w) { lo = min(lo, sm.wlo[w]); hi = max(hi, sm.whi[w]); }
  const uint32_t range = hi - lo;
  const int bits = range == 0u ? 0 : 32 - __clz(static_cast<int>(range));

  // radix select over v = image - lo, digits of up to 11 bits from the top,
  // until the boundary bin is small enough to rank
  unsigned long long prefix = 0ull, mask = 0ull;
  uint32_t rank = static_cast<uint32_t>(E), sel = static_cast<uint32_t>(B);
  int shift = bits;
  bool cleared = true;
  while (shift > 0 && sel > static_cast<uint32_t>(kTopkBoundary)) {
    const int width = shift < 11 ? shift : 11;
    shift -= width;
    const int nb = 1 << width;
    if (!cleared) {
      for (int i = tid; i < nb; i += BS) sm.hist[i] = 0u;
      __syncthreads();
    }
    cleared = false;
#pragma unroll 4
    for (int b = tid; b < B; b += BS) {
      const uint32_t v = image(b) - lo;
      if ((static_cast<unsigned long long>(v) & mask) == prefix) atomicAdd(&sm.hist[(v >> shift) & (nb - 1)], 1u);
    }
    __syncthreads();
    topk_find_bin<BS>(sm, nb, rank, prefix, shift);
    __syncthreads();
    prefix = sm.prefix;
    rank = sm.rank;
    sel = sm.sel_count;
    mask |= static_cast<unsigned long long>(nb - 1) << shift;
    __syncthreads();
  }

  if (sel <= static_cast<uint32_t>(kTopkBoundary)) {
    // lower bins: elites; boundary bin (top digits equal to the prefix): ranked.
    // With no pass taken (B small) shift = bits, which may be 32: 64-bit shifts.
    const unsigned long long pd = prefix >> shift;
    const uint32_t below = static_cast<uint32_t>(E) - rank;
    topk_gather_split<BS>(B, lo, image, shift, pd, &sm.count, sm.keys, static_cast<uint32_t>(kMaxElites), &sm.count2,
                          sm.sorted, static_cast<uint32_t>(kTopkBoundary));
    __syncthreads();
    topk_rank<BS>(sm.sorted, static_cast<int>(sel), [&](unsigned long long k, int r) {
      if (static_cast<uint32_t>(r) < rank) sm.keys[below + static_cast<uint32_t>(r)] = k;
    });
  } else {
    // the boundary bin holds one image c* only
    const uint32_t cstar = lo + static_cast<uint32_t>(prefix);
    unsigned long long limit;   // elites are the keys <= limit
    if (rank == sel) {
      limit = (static_cast<unsigned long long>(cstar) << 32) | 0xFFFFFFFFull;
    } else {
      // ties at the boundary: radix over the index bits of the keys with image c*
      unsigned long long kp = 0ull, km = 0ull;
      for (int pass = 0; pass < 3; ++pass) {
        const int sh = pass == 0 ? 21 : (pass == 1 ? 10 : 0), nb = pass == 2 ? 1024 : 2048;
        for (int i = tid; i < nb; i += BS) sm.hist[i] = 0u;
        __syncthreads();
        for (int b = tid; b < B; b += BS) {
          const unsigned long long ib = static_cast<uint32_t>(b);
          if (image(b) == cstar && (ib & km) == kp) atomicAdd(&sm.hist[(ib >> sh) & static_cast<unsigned long long>(nb - 1)], 1u);
        }
        __syncthreads();
        topk_find_bin<BS>(sm, nb, rank, kp, sh);
        __syncthreads();
        kp = sm.prefix;
        rank = sm.rank;
        km |= static_cast<unsigned long long>(nb - 1) << sh;
        __syncthreads();
      }
      limit = (static_cast<unsigned long long>(cstar) << 32) | kp;
    }
    topk_gather<BS>(B, image, limit, &sm.count, sm.keys, static_cast<uint32_t>(kMaxElites));
  }
  __syncthreads();
  const unsigned long long* ord;
  if (E <= kTopkRankSort) {
    topk_rank<BS>(sm.keys, E, [&](unsigned long long k, int r) { sm.sorted[r] = k; });
    ord = sm.sorted;
  } else {
    int M = 1;
    while (M < E) M <<= 1;
    for (int i = E + tid; i < M; i += BS) sm.keys[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= M; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = tid; i < M; i += BS) {
          const int jx = i ^ stride;
          if (jx > i) {
            const bool up = ((i & size) == 0);
            const unsigned long long a = sm.keys[i], c = sm.keys[jx];
            if ((a > c) == up) { sm.keys[i] = c; sm.keys[jx] = a; }
          }
        }
        __syncthreads();
      }
    }
    ord = sm.keys;
  }
  return ord;
}

// Batches of at most one key per thread: every key counts the keys below it
// (broadcast LDS reads), and that count is its place in the order; the keys
// are distinct, so this is the same exact order as the radix path's.
template <int BS>
__device__ __forceinline__ const unsigned long long* topk_select_small(const PlanDesc& P, TopkSmem& sm) {
  const auto cost = gptr(P.cost);
  const int tid = threadIdx.x;
  const int B = P.B, E = P.E;
  unsigned long long* all = reinterpret_cast<unsigned long long*>(sm.cache);
  const unsigned long long key =
      tid < B ? (static_cast<unsigned long long>(cost_order(cost[tid])) << 32) | static_cast<uint32_t>(tid) : ~0ull;
  if (tid < B) all[tid] = key;
  __syncthreads();
  if (tid < B) {
    int rank = 0;
#pragma unroll 8
    for (int j = 0; j < B; ++j) rank += all[j] < key ? 1 : 0;
    if (rank < E) sm.sorted[rank] = key;
  }
  return sm.sorted;
}

template <int BS>
__device__ __forceinline__ void topk_block(const PlanDesc& P, TopkSmem& sm) {
  const auto cost = gptr(P.cost);
  const int tid = threadIdx.x;
  const int B = P.B, E = P.E;
  const unsigned long long* ord = B <= BS ? topk_select_small<BS>(P, sm) : topk_select<BS>(P, sm);
  __syncthreads();
  // elites, costs and softmax weights w_e = exp(-(s_e - s_0)/lambda) / sum;
  // the unnormalised weights wait in LDS (the image cache is free by now)
  float* wbuf = reinterpret_cast<float*>(sm.cache);
  // elite costs come back from their keys' images; +inf (also NaN) and zero
  // (also -0) are read from memory to keep the cost as it was
  auto elite_cost = [&](unsigned long long key, int idx) -> float {
    const float v = order_cost(static_cast<uint32_t>(key >> 32));
    return (v == 0.0f || v == INFINITY) ? cost[idx] : v;
  };
  const uint32_t i0 = static_cast<uint32_t>(ord[0]);
  const float s0 = elite_cost(ord[0], static_cast<int>(i0 < static_cast<uint32_t>(B) ? i0 : 0u));
  const bool uniform = !(P.lam < INFINITY) || !(s0 < INFINITY);
  for (int e = tid; e < E; e += BS) {
    uint32_t uidx = static_cast<uint32_t>(ord[e]);
    if (uidx >= static_cast<uint32_t>(B)) { uidx = 0u; atomicOr(&P.ctrl[2], 2u); }   // never expected
    const int idx = static_cast<int>(uidx);
    const float ce = elite_cost(ord[e], idx);
    gptr(P.eidx)[e] = idx;
    gptr(P.ecost)[e] = ce;
    wbuf[e] = uniform ? 1.0f : expf(-(ce - s0) / P.lam);
  }
  // normalisation sum in an order fixed by E alone (independent of the block
  // size): lane l of wave 0 adds e = l, l+64, ... in turn, then wave_sum64.
  __syncthreads();
  if (tid < 64) {
    float acc = 0.0f;
    for (int e = tid; e < E; e += 64) acc += wbuf[e];
    acc = wave_sum64(acc);
    if (tid == 0) sm.red[0] = acc;
  }
  __syncthreads();
  const float inv = 1.0f / sm.red[0];
  for (int e = tid; e < E; e += BS) gptr(P.w)[e] = wbuf[e] * inv;
  if (tid == 0 && !(s0 < INFINITY)) atomicOr(&P.ctrl[2], 1u);
}

// Iteration k_next's candidates that depend on the refitted distribution, at
// output o = (t, j): the local samples b < G-1 (the same Philox words and
// arithmetic as cand_tile: block (j, t / 4) of sample b, word pair by t mod 4)
// and the nominal mean (candidate B-1), from the mean and std just refitted.
// The normals do not depend on the refit: local_normals draws a thread's share
// (samples tid, tid + BS, ...; the first kLocalKeep kept in registers) while
// the refit runs, local_store writes them once the moments are known.
constexpr int kLocalKeep = 4;

// Iteration k_next's local-sample normals at the four steps t = 4 tq + c
// (c = 0..3) of joint j for candidates b = threadIdx.x + i BS, i < kLocalKeep:
// the one Philox block of (j, tq, b) gives all four, two Box-Muller pairs,
// exactly as the candidate tile draws them.
__device__ __forceinline__ void local_normals4(const PlanDesc& P, int tq, int j, int b, int k_next, uint32_t r,
                                               float (&z)[4]) {
  const int Tq = (P.T + 3) >> 2;
  const Words4 q = philox(static_cast<uint32_t>(j * Tq + tq), static_cast<uint32_t>(b), r,
                          stream_c3(kTagEps, k_next), P.key0, P.key1);
  box_muller(q.w[0], q.w[1], z[0], z[1]);
  box_muller(q.w[2], q.w[3], z[2], z[3]);
}

template <int BS>
__device__ __forceinline__ void local_normals(const PlanDesc& P, int tq, int j, int k_next, uint32_t r,
                                              float (&z)[kLocalKeep][4]) {
  const int G1 = P.G - 1;
#pragma unroll
  for (int i = 0; i < kLocalKeep; ++i) {
    const int b = static_cast<int>(threadIdx.x) + i * BS;
    if (b < G1) {
      local_normals4(P, tq, j, b, k_next, r, z[i]);
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) z[i][c] = 0.0f;
    }
  }
}

// Local samples clip(mu_t + sg_t z) and the nominal clip(mu_t) of iteration
// k_next at the steps t = 4 tq + c < T of joint j, from the refitted moments
// mom[c] = (mu_t, sg_t).
template <int BS>
__device__ __forceinline__ void local_store(const PlanDesc& P, float* U, int tq, int j, int k_next, uint32_t r,
                                            const float (&z)[kLocalKeep][4], const float (&mom)[4][2]) {
  const auto Ug = gptr(U);
  const size_t ld = static_cast<size_t>(P.ldU);
  const float lo = P.u_min, hi = P.u_max;
  const int G1 = P.G - 1;
  const int nc = min(4, P.T - 4 * tq);
  size_t row[4];
  float mu_t[4], sg_t[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    row[c] = static_cast<size_t>((4 * tq + c) * P.n + j) * ld;
    mu_t[c] = mom[c][0];
    sg_t[c] = mom[c][1];
  }
#pragma unroll
  for (int i = 0; i < kLocalKeep; ++i) {
    const int b = static_cast<int>(threadIdx.x) + i * BS;
    if (b < G1) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < nc) __builtin_nontemporal_store(clampf(fmaf(sg_t[c], z[i][c], mu_t[c]), lo, hi), &Ug[row[c] + b]);
    }
  }
  for (int b = static_cast<int>(threadIdx.x) + kLocalKeep * BS; b < G1; b += BS) {
    float zz[4];
    local_normals4(P, tq, j, b, k_next, r, zz);
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < nc) __builtin_nontemporal_store(clampf(fmaf(sg_t[c], zz[c], mu_t[c]), lo, hi), &Ug[row[c] + b]);
  }
  if (static_cast<int>(threadIdx.x) < nc) {
    const int c = static_cast<int>(threadIdx.x);
    __builtin_nontemporal_store(clampf(mom[c][0], lo, hi), &Ug[row[c] + (P.B - 1)]);
  }
}

// ------------------------------------------------------------------ cost entropy
// H = -sum_j P_j log P_j with P_j = exp(J_j) / sum_l exp(J_l) over the finite
// rollout costs J of one iteration (the exploration diagnostic of Section 5.1),
// as H = log S0 - S1 / S0 with S0 = sum e^{J - m}, S1 = sum e^{J - m} (J - m),
// m = max J.  1024 virtual lanes each fold the costs b = v, v + 1024, ... in
// turn with a running maximum, then a fixed binary tree combines the lanes,
// so the value depends neither on the block size nor on scheduling.

constexpr int kEntLanes = 1024;

struct EntropySmem {
  float m[kEntLanes], s0[kEntLanes], s1[kEntLanes];
};

__device__ __forceinline__ void ent_fold(float& m, float& s0, float& s1, float m2, float a0, float a1) {
  if (!(a0 > 0.0f)) return;
  if (!(s0 > 0.0f)) { m = m2; s0 = a0; s1 = a1; return; }
  const float mm = fmaxf(m, m2);
  const float fa = __expf(m - mm), fb = __expf(m2 - mm);
  s1 = fa * fmaf(m - mm, s0, s1) + fb * fmaf(m2 - mm, a0, a1);
  s0 = fa * s0 + fb * a0;
  m = mm;
}

template <int BS>
__device__ __forceinline__ void entropy_block(const PlanDesc& P, int k, EntropySmem& sm) {
  for (int v = threadIdx.x; v < kEntLanes; v += BS) {
    float m = 0.0f, s0 = 0.0f, s1 = 0.0f;
    for (int b = v; b < P.B; b += kEntLanes) {
      const float J = P.cost[b];
      if (!(fabsf(J) <= 3.402823466e38f)) continue;
      ent_fold(m, s0, s1, J, 1.0f, 0.0f);
    }
    sm.m[v] = m; sm.s0[v] = s0; sm.s1[v] = s1;
  }
  __syncthreads();
  for (int h = kEntLanes / 2; h > 0; h >>= 1) {
    for (int v = threadIdx.x; v < h; v += BS) {
      float m = sm.m[v], s0 = sm.s0[v], s1 = sm.s1[v];
      ent_fold(m, s0, s1, sm.m[v + h], sm.s0[v + h], sm.s1[v + h]);
      sm.m[v] = m; sm.s0[v] = s0; sm.s1[v] = s1;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) P.entropy[k] = (sm.s0[0] > 0.0f) ? __logf(sm.s0[0]) - sm.s1[0] / sm.s0[0] : 0.0f;
}

// ------------------------------------------------------------------ refit
// One wave per output (t, j): lanes stride over the elites, a fixed-order
// wave sum, then the sigma floor and exponential smoothing.

// The elite values of a row are gathered once: up to kUpdKeep per lane stay in
// registers for the variance pass (each gather touches its own cache line, so
// the second pass would double the line traffic); larger elite sets re-read.
constexpr int kUpdKeep = 16;

// Refits output o = (t, j); every lane returns the new mean and std, lane 0 stores them.
// The refit of output o from the elites' controls val(e) (e < E), in a fixed
// order: weighted mean, weighted variance about it, sigma floor, smoothing.
template <class Val>
__device__ __forceinline__ void update_output_from(const PlanDesc& P, int o, Val val, float* mu_new, float* sg_new) {
  const int lane = threadIdx.x & 63;
  const auto w = gptr(P.w);
  // the old moments do not depend on the elite values: their loads go out first
  const auto mu = gptr(P.mu), sigma = gptr(P.sigma);
  const float mu_old = mu[o], sg_old = sigma[o];
  float keep[kUpdKeep];
  float m = 0.0f;
  if (P.E <= 64 * kUpdKeep) {
#pragma unroll
    for (int q = 0; q < kUpdKeep; ++q) {
      const int e = lane + 64 * q;
      keep[q] = e < P.E ? val(e) : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kUpdKeep; ++q) {
      const int e = lane + 64 * q;
      if (e < P.E) m = fmaf(w[e], keep[q], m);
    }
  } else {
    for (int e = lane; e < P.E; e += 64) m = fmaf(w[e], val(e), m);
  }
  m = wave_sum64(m);
  float v = 0.0f;
  if (P.E <= 64 * kUpdKeep) {
#pragma unroll
    for (int q = 0; q < kUpdKeep; ++q) {
      const int e = lane + 64 * q;
      if (e < P.E) {
        const float dv = keep[q] - m;
        v = fmaf(w[e], dv * dv, v);
      }
    }
  } else {
    for (int e = lane; e < P.E; e += 64) {
      const float dv = val(e) - m;
      v = fmaf(w[e], dv * dv, v);
    }
  }
  v = wave_sum64(v);
  const float sd = fmaxf(sqrtf(v), P.sigma_min);
  const float mn = fmaf(P.alpha, mu_old - m, m);
  const float sn = fmaf(P.alpha, sg_old - sd, sd);
  if (mu_new) *mu_new = mn;
  if (sg_new) *sg_new = sn;
  if (lane == 0) {
    mu[o] = mn;
    sigma[o] = sn;
    // first control of the best candidate (lane 0 holds elite 0 already)
    if (o < P.n) gptr(P.action)[o] = P.E <= 64 * kUpdKeep ? keep[0] : val(0);
  }
}

// The refit of output o from the elites' rows of U (one gathered value each).
__device__ __forceinline__ void update_output(const PlanDesc& P, int o, float* mu_new = nullptr,
                                              float* sg_new = nullptr) {
  const auto row = gptr(P.U) + static_cast<size_t>(o) * static_cast<size_t>(P.ldU);
  const auto eidx = gptr(P.eidx);
  update_output_from(P, o, [&](int e) { return row[eidx[e]]; }, mu_new, sg_new);
}

// Elite controls drawn again instead of gathered.  The gather reads one value
// per elite from a 4-byte slot of its own cache line, 360 MB of lines per
// 24-link refit for 12.6 MB of values; the values are functions of the seed,
// the replan and iteration index and the moments the iteration sampled from,
// so the refit tile of steps 4 tq..4 tq+3 of joint j recomputes them with the
// arithmetic that drew them (cand_tile): the graph column of joint j (Def. 1),
// each tensor elite's layer indices at the spans it needs (Alg. 1) and the
// cubic B-spline, each local elite's normals (one Philox block) and the
// nominal mean.  For plans drawing paths with replacement and cubic B-splines,
// up to kRegenMaxElites elites; the values are the same bits as the gathered
// ones.  Small batches keep the gather: their rows span a few lines that the
// elites share, and the redraw's latency would cost more (C0: 6.8 -> 7.7 us
// per refit, against 59.5 -> 33 us at the 24-link size).
constexpr int kRegenMaxElites = 1024;
constexpr int kRegenMinCandidates = 16384;

struct RegenSmem {
  float zc[kMaxLayers * kMaxWidth];          // graph column of joint j
  uint8_t wi[kMaxLayers][kUpdThreads];       // each thread's current elite's layer indices
  float vals[4][kRegenMaxElites];            // elite controls at the tile's four steps
  float old[4][2];                           // the sampled moments at those steps
};

__host__ __device__ __forceinline__ bool refit_regenerates(int interp, int degree, int wor, int E, int B) {
  return interp == kBspline && degree == 3 && !wor && E <= kRegenMaxElites && B >= kRegenMinCandidates;
}

__device__ __forceinline__ void regen_elites(const PlanDesc& P, int k, int tq, int j, RegenSmem& sm) {
  const int tid = threadIdx.x;
  const uint32_t r = P.ctrl[0];
  const float lo = P.u_min, hi = P.u_max, span = hi - lo;
  const int G1 = P.G - 1;
  const int t0 = 4 * tq, nc = min(4, P.T - t0);
  if (tid < nc) {
    const int o = (t0 + tid) * P.n + j;
    sm.old[tid][0] = gptr(P.mu)[o];
    sm.old[tid][1] = gptr(P.sigma)[o];
  }
  for (int e = tid; e < P.L * P.W; e += kUpdThreads) {
    const int l = e / P.W, w = e - l * P.W;
    const uint32_t idx = static_cast<uint32_t>(w * P.n + j);
    const Words4 q = philox(idx >> 2, static_cast<uint32_t>(l), r, stream_c3(kTagZ, k), P.key0, P.key1);
    sm.zc[e] = fmaf(span, u01(word_at(q, idx & 3u)), lo);
  }
  __syncthreads();
  const auto eidx = gptr(P.eidx);
  const auto spn = gptr(P.span);
  const auto basis = gptr(P.basis);
  const int s_lo = spn[t0], s_hi = min(spn[t0 + nc - 1] + 3, P.L - 1);
  for (int e = tid; e < P.E; e += kUpdThreads) {
    const int b = eidx[e];
    if (b < G1) {
      float z[4];
      local_normals4(P, tq, j, b, k, r, z);
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < nc) sm.vals[c][e] = clampf(fmaf(sm.old[c][1], z[c], sm.old[c][0]), lo, hi);
    } else if (b < G1 + P.P) {
      const int pp = b - G1;
      for (int l4 = s_lo >> 2; l4 <= (s_hi >> 2); ++l4) {
        const Words4 q = philox(static_cast<uint32_t>(l4), static_cast<uint32_t>(pp), r, stream_c3(kTagI, k),
                                P.key0, P.key1);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int l = 4 * l4 + c;
          if (l >= s_lo && l <= s_hi) sm.wi[l][tid] = static_cast<uint8_t>(__umulhi(q.w[c], static_cast<uint32_t>(P.W)));
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c < nc) {
          const int t = t0 + c, s0 = spn[t];
          const auto bw = basis + t * kBasisStride;
          float v = bw[0] * sm.zc[s0 * P.W + sm.wi[s0][tid]];
          v = fmaf(bw[1], sm.zc[(s0 + 1) * P.W + sm.wi[s0 + 1][tid]], v);
          v = fmaf(bw[2], sm.zc[(s0 + 2) * P.W + sm.wi[s0 + 2][tid]], v);
          v = fmaf(bw[3], sm.zc[(s0 + 3) * P.W + sm.wi[s0 + 3][tid]], v);
          sm.vals[c][e] = clampf(v, lo, hi);
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < nc) sm.vals[c][e] = clampf(sm.old[c][0], lo, hi);
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ prologue
// Replan prologue.  set_ctrl runs outside any captured graph (its arguments
// change every replan): it records the replan index and the shift and stages
// x0.  shift_block runs inside the graph and shifts the warm start by the
// recorded amount; a single workgroup stages through the tmp buffer so the
// in-place shift has no read-after-write hazard.
__device__ __forceinline__ void set_ctrl_block(const PlanDesc& P, uint32_t r, int shift, const float* x0_src) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    // tensor paths drawn ahead by the previous replan are for this one only if
    // it is the replan they were drawn for; either way they are used up now
    P.ctrl[4] = (P.spec && P.ctrl[5] != 0u && P.ctrl[3] == r) ? 1u : 0u;
    P.ctrl[5] = 0u;
    P.ctrl[0] = r; P.ctrl[1] = static_cast<uint32_t>(shift > 0 ? shift : 0); P.ctrl[2] = 0u;
  }
  if (x0_src != nullptr)
    for (int i = tid; i < P.d; i += blockDim.x) P.x0[i] = x0_src[i];
}

template <int BS>
__device__ __forceinline__ void shift_block(const PlanDesc& P, int shift) {
  const int tid = threadIdx.x;
  if (shift <= 0) return;
  const int Tn = P.T * P.n;
  const int s = shift < P.T ? shift : P.T;
  // the value that lands at flat index e: step t + s of the warm start, or
  // the last step's mean with the initial spread past the end
  auto src_mu = [&](int e) {
    const int t = e / P.n;
    return P.mu[t < P.T - s ? e + s * P.n : (P.T - 1) * P.n + (e - t * P.n)];
  };
  auto src_sg = [&](int e) { return e / P.n < P.T - s ? P.sigma[e + s * P.n] : P.sigma_init; };
  constexpr int R = 8;
  if (Tn <= BS * R) {
    // every value held in registers across the barrier: all loads in flight
    // at once and no staging copy
    float m[R], g[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int e = tid + i * BS < Tn ? tid + i * BS : 0;
      m[i] = src_mu(e);
      g[i] = src_sg(e);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (tid + i * BS < Tn) {
        P.mu[tid + i * BS] = m[i];
        P.sigma[tid + i * BS] = g[i];
      }
    return;
  }
  float* tmu = P.tmp;
  float* tsg = P.tmp + Tn;
  for (int e = tid; e < Tn; e += BS) {
    tmu[e] = src_mu(e);
    tsg[e] = src_sg(e);
  }
  __syncthreads();
  for (int e = tid; e < Tn; e += BS) {
    P.mu[e] = tmu[e];
    P.sigma[e] = tsg[e];
  }
}

}  // namespace mtp
