// Host runtime of a single MTP plan: config validation, workspace layout,
// host-side interpolation tables, launch sequencing, hipGraph capture, and
// the C ABI declared in include/mtp.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mtp.h"
#include "kernels.hpp"
#include "plan_internal.hpp"

namespace mtp {

// ------------------------------------------------------------------ validation

static size_t expected_task_params(const mtp_config& c) {
  switch (c.dynamics) {
    case MTP_DYN_POINT_MASS:
      return 0;  // variable: 6 + 3 * n_obs, checked separately
    case MTP_DYN_CHAIN:
      return 5 + 2 * static_cast<size_t>(c.n_links);
    case MTP_DYN_CHAIN_CONTACT:
      return 9 + 2 * static_cast<size_t>(c.n_links);
    default:
      return 0;
  }
}

bool validate_config(const mtp_config* c, std::string* why, mtp_status* code) {
  auto fail = [&](mtp_status s, const char* msg) {
    if (why) *why = msg;
    if (code) *code = s;
    return false;
  };
  if (c == nullptr) return fail(MTP_ERR_INVALID_ARG, "config is NULL");
  if (c->abi_version != MTP_ABI_VERSION) return fail(MTP_ERR_INVALID_ARG, "abi_version mismatch");
  if (c->dynamics < 0 || c->dynamics > 2) return fail(MTP_ERR_INVALID_ARG, "unknown dynamics");
  if (c->interp < 0 || c->interp > 2) return fail(MTP_ERR_INVALID_ARG, "unknown interpolation");
  if (c->dynamics == MTP_DYN_POINT_MASS) {
    if (c->state_dim != 4 || c->ctrl_dim != 2) return fail(MTP_ERR_INVALID_ARG, "point mass needs state_dim 4, ctrl_dim 2");
  } else {
    if (c->n_links < 1) return fail(MTP_ERR_INVALID_ARG, "chain needs n_links >= 1");
    if (c->ctrl_dim != c->n_links || c->state_dim != 2 * c->n_links)
      return fail(MTP_ERR_INVALID_ARG, "chain needs ctrl_dim = n_links and state_dim = 2 n_links");
  }
  if (c->horizon < 1 || c->horizon > 4096) return fail(MTP_ERR_INVALID_ARG, "horizon must be in 1..4096");
  if (c->n_width < 1 || c->n_width > kMaxWidth) return fail(MTP_ERR_INVALID_ARG, "n_width must be in 1..256");
  if (c->n_layers > kMaxLayers) return fail(MTP_ERR_INVALID_ARG, "n_layers must be <= 16");
  if (c->interp == MTP_INTERP_BSPLINE) {
    if (c->bspline_degree < 1 || c->bspline_degree > 5) return fail(MTP_ERR_INVALID_ARG, "bspline_degree must be in 1..5");
    if (c->n_layers < c->bspline_degree + 1) return fail(MTP_ERR_INVALID_ARG, "B-spline needs n_layers >= degree + 1");
  } else if (c->n_layers < 2) {
    return fail(MTP_ERR_INVALID_ARG, "Akima and linear paths need n_layers >= 2");
  }
  if (c->n_tensor < 0) return fail(MTP_ERR_INVALID_ARG, "n_tensor must be >= 0");
  if (c->n_gauss < 1) return fail(MTP_ERR_INVALID_ARG, "n_gauss must be >= 1 (it holds the nominal mean)");
  const long long B = static_cast<long long>(c->n_tensor) + c->n_gauss;
  if (B > (1ll << 24)) return fail(MTP_ERR_INVALID_ARG, "n_tensor + n_gauss must be <= 2^24");
  if (c->n_elites < 1 || c->n_elites > B) return fail(MTP_ERR_INVALID_ARG, "n_elites must be in 1..n_tensor+n_gauss");
  if (c->n_elites > kMaxElites) return fail(MTP_ERR_UNSUPPORTED, "n_elites above 4096 is not supported");
  if (c->n_iters < 1 || c->n_iters > 65535) return fail(MTP_ERR_INVALID_ARG, "n_iters must be in 1..65535");
  if (!(c->temperature > 0.0f)) return fail(MTP_ERR_INVALID_ARG, "temperature must be > 0 (inf allowed)");
  if (!(c->smoothing >= 0.0f && c->smoothing < 1.0f)) return fail(MTP_ERR_INVALID_ARG, "smoothing must be in [0, 1)");
  if (!(c->sigma_min >= 0.0f) || !std::isfinite(c->sigma_min)) return fail(MTP_ERR_INVALID_ARG, "sigma_min must be finite and >= 0");
  if (!(c->sigma_init >= 0.0f) || !std::isfinite(c->sigma_init)) return fail(MTP_ERR_INVALID_ARG, "sigma_init must be finite and >= 0");
  if (!std::isfinite(c->u_min) || !std::isfinite(c->u_max) || !(c->u_min < c->u_max))
    return fail(MTP_ERR_INVALID_ARG, "need finite u_min < u_max");
  if (!(c->dt > 0.0f) || !std::isfinite(c->dt)) return fail(MTP_ERR_INVALID_ARG, "dt must be finite and > 0");
  if (c->n_debug_states < 0 || c->n_debug_states > B) return fail(MTP_ERR_INVALID_ARG, "n_debug_states must be in 0..B");
  if (c->n_replicas < 0 || c->n_replicas > 64) return fail(MTP_ERR_INVALID_ARG, "n_replicas must be in 0..64");
  if (c->sample_wor != 0 && c->sample_wor != 1) return fail(MTP_ERR_INVALID_ARG, "sample_wor must be 0 or 1");
  if (c->diagnostics < 0 || c->diagnostics > 1) return fail(MTP_ERR_INVALID_ARG, "diagnostics must be 0 or 1");
  if (c->sample_wor == 1) {
    // P distinct paths need P <= W^L
    long double paths = 1.0L;
    for (int l = 0; l < c->n_layers && paths < static_cast<long double>(c->n_tensor); ++l) paths *= c->n_width;
    if (paths < static_cast<long double>(c->n_tensor))
      return fail(MTP_ERR_INVALID_ARG, "sampling without replacement needs n_tensor <= n_width^n_layers");
  }
  if (c->n_task_params < 0 || (c->n_task_params > 0 && c->task_params == nullptr))
    return fail(MTP_ERR_INVALID_ARG, "task_params missing");
  if (c->dynamics == MTP_DYN_POINT_MASS) {
    if (c->n_replicas > 1) return fail(MTP_ERR_INVALID_ARG, "randomised replicas need the contact chain");
    if (c->n_task_params < 6) return fail(MTP_ERR_INVALID_ARG, "point mass task needs >= 6 parameters");
    const float nobs = c->task_params[5];
    if (!(nobs >= 0.0f) || nobs != std::floor(nobs) || nobs > static_cast<float>(kMaxObstacles) ||
        c->n_task_params != 6 + 3 * static_cast<int>(nobs))
      return fail(MTP_ERR_INVALID_ARG, "point mass task: n_task_params must be 6 + 3 n_obs, n_obs <= 256");
  } else {
    if (static_cast<size_t>(c->n_task_params) != expected_task_params(*c))
      return fail(MTP_ERR_INVALID_ARG, "chain task parameter count does not match n_links");
    for (int k = 0; k < c->n_links; ++k) {
      if (!(c->task_params[5 + c->n_links + k] > 0.0f)) return fail(MTP_ERR_INVALID_ARG, "link lengths must be > 0");
      if (c->dynamics == MTP_DYN_CHAIN && !(c->task_params[5 + k] > 0.0f))
        return fail(MTP_ERR_INVALID_ARG, "link masses must be > 0");
    }
    if (c->dynamics == MTP_DYN_CHAIN_CONTACT) {
      if (c->sample_params == nullptr) return fail(MTP_ERR_INVALID_ARG, "contact chain needs sample_params");
      if (!(c->task_params[8 + 2 * c->n_links] > 0.0f)) return fail(MTP_ERR_INVALID_ARG, "v_slip must be > 0");
      const size_t rows = static_cast<size_t>(B) * static_cast<size_t>(c->n_replicas > 1 ? c->n_replicas : 1);
      for (size_t b = 0; b < rows; ++b)
        for (int k = 0; k < c->n_links; ++k)
          if (!(c->sample_params[b * (c->n_links + 1) + k] > 0.0f))
            return fail(MTP_ERR_INVALID_ARG, "sample masses must be > 0");
    }
    if (c->dynamics == MTP_DYN_CHAIN && c->n_replicas > 1)
      return fail(MTP_ERR_INVALID_ARG, "randomised replicas need the contact chain's per-sample table");
    if (!rollout_supported(c->dynamics, c->n_links))
      return fail(MTP_ERR_UNSUPPORTED, "chain length not instantiated in this build");
  }
  return true;
}

// ------------------------------------------------------------------ layout

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

Layout compute_layout(const mtp_config& c, bool plan) {
  Layout L{};
  const size_t T = c.horizon, n = c.ctrl_dim, d = c.state_dim;
  const size_t B = static_cast<size_t>(c.n_tensor) + c.n_gauss;
  L.ldU = align256(B * sizeof(float)) / sizeof(float);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
  L.ctrl = take(64);
  L.x0 = take(d * 4);
  L.mu = take(T * n * 4);
  L.sigma = take(T * n * 4);
  L.tmp = take(2 * T * n * 4);
  L.action = take(n * 4);
  L.basis = take(T * kBasisStride * 4);
  L.span = take(T * 4);
  L.task = take(static_cast<size_t>(c.n_task_params) * 4);
  const size_t R = c.n_replicas > 1 ? static_cast<size_t>(c.n_replicas) : 1;
  L.sparams = c.dynamics == MTP_DYN_CHAIN_CONTACT ? take(R * B * (n + 1) * 4) : 0;
  L.entropy = take(static_cast<size_t>(c.n_iters) * 4);
  L.segmented = uses_segmented_rollout(c);
  const size_t groups = (B + 31) / 32;
  L.seg_ctl = L.segmented ? take(64) : 0;
  L.seg_done = L.segmented ? take(groups * 4) : 0;
  L.resident = off;
  off = 0;
  L.Z = take(static_cast<size_t>(c.n_layers) * c.n_width * n * 4);
  L.I = take(static_cast<size_t>(c.n_layers) * (c.n_tensor > 0 ? c.n_tensor : 1));
  L.U = take(T * n * L.ldU * 4);
  L.cost = take(B * 4);
  L.eidx = take(static_cast<size_t>(c.n_elites) * 4);
  L.ecost = take(static_cast<size_t>(c.n_elites) * 4);
  L.w = take(static_cast<size_t>(c.n_elites) * 4);
  L.X = c.n_debug_states > 0 ? take(static_cast<size_t>(R) * T * d * static_cast<size_t>(c.n_debug_states) * 4) : 0;
  L.seg_state = L.segmented ? take((n + n / 2 + 1) * groups * 64 * 4) : 0;
  L.overlap = plan && uses_gen_overlap(c);
  L.U2 = L.overlap ? take(T * n * L.ldU * 4) : 0;
  L.transient = off;
  L.total = L.resident + L.transient;
  return L;
}

// ------------------------------------------------------------------ tables

// Non-zero uniform B-spline basis functions on the span containing tau, by the
// triangular (de Boor) scheme on the local knot window; knots at the integers.
static void bspline_span_basis(int p, int span, double tau, double* N) {
  double left[8], right[8];
  N[0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    left[j] = tau - static_cast<double>(span + 1 - j);
    right[j] = static_cast<double>(span + j) - tau;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      const double tmp = N[r] / (right[r + 1] + left[j - r]);
      N[r] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    N[j] = saved;
  }
}

void build_tables(const mtp_config& c, std::vector<float>* basis, std::vector<int32_t>* span) {
  const int T = c.horizon, L = c.n_layers;
  basis->assign(static_cast<size_t>(T) * kBasisStride, 0.0f);
  span->assign(T, 0);
  for (int j = 0; j < T; ++j) {
    float* row = basis->data() + static_cast<size_t>(j) * kBasisStride;
    if (c.interp == MTP_INTERP_BSPLINE) {
      const int p = c.bspline_degree;
      // horizon mapped onto the valid span [knot_p, knot_L): tau = p + (L-p) j / T
      const long long num = static_cast<long long>(L - p) * j;
      const int s = p + static_cast<int>(num / T);
      const double tau = p + static_cast<double>(num) / T;
      double N[8];
      bspline_span_basis(p, s, tau, N);
      for (int q = 0; q <= p; ++q) row[q] = static_cast<float>(N[q]);
      (*span)[j] = s - p;
    } else if (c.interp == MTP_INTERP_LINEAR) {
      // knots i/(L-1) over [0, 1], sample at j/T: weights 1-xi, xi in interval i
      const long long num = static_cast<long long>(L - 1) * j;
      const int i = static_cast<int>(num / T);
      const double xi = static_cast<double>(num - static_cast<long long>(i) * T) / T;
      row[0] = static_cast<float>(1.0 - xi);
      row[1] = static_cast<float>(xi);
      (*span)[j] = i;
    } else {
      // Akima knots at i/L, sample at j/T; cubic Hermite weights in xi = L j / T - i
      const long long num = static_cast<long long>(L) * j;
      int i = static_cast<int>(num / T);
      if (i > L - 2) i = L - 2;
      const double xi = static_cast<double>(num - static_cast<long long>(i) * T) / T;
      const double x2 = xi * xi, x3 = x2 * xi;
      row[0] = static_cast<float>(2 * x3 - 3 * x2 + 1);
      row[1] = static_cast<float>(x3 - 2 * x2 + xi);
      row[2] = static_cast<float>(-2 * x3 + 3 * x2);
      row[3] = static_cast<float>(x3 - x2);
      (*span)[j] = i;
    }
  }
}

}  // namespace mtp

using namespace mtp;

// ------------------------------------------------------------------ plan object

struct mtp_plan {
  mtp_config cfg;
  std::vector<float> task, sparams;
  Layout lay;
  PlanDesc P;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  SideLane side{nullptr, nullptr, nullptr};   // second stream of plans that draw beside a time-sliced rollout
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  bool use_graph = true;
  bool timing = false;
  std::vector<hipEvent_t> ev_free;
  struct Pending { int stage; hipEvent_t a, b; };
  std::vector<Pending> pending;
  double stage_ms[4] = {0, 0, 0, 0};
  uint64_t stage_count[4] = {0, 0, 0, 0};
  uint32_t next_r = 0;
  bool sticky = false;
  std::string err;
};

static mtp_status set_err(mtp_plan* p, mtp_status s, const std::string& msg) {
  if (p) p->err = msg;
  return s;
}

static mtp_status device_err(mtp_plan* p, hipError_t e, const char* where) {
  if (p) {
    p->sticky = true;
    p->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return MTP_ERR_DEVICE;
}

#define HIPCHK(p, expr, where)                      \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return device_err(p, e_, where); \
  } while (0)

void mtp::set_transient(PlanDesc* P, const mtp_config& c, const Layout& L, uint8_t* tb) {
  P->Z = reinterpret_cast<float*>(tb + L.Z);
  P->I = tb + L.I;
  P->U = reinterpret_cast<float*>(tb + L.U);
  P->cost = reinterpret_cast<float*>(tb + L.cost);
  P->eidx = reinterpret_cast<int32_t*>(tb + L.eidx);
  P->ecost = reinterpret_cast<float*>(tb + L.ecost);
  P->w = reinterpret_cast<float*>(tb + L.w);
  P->X = c.n_debug_states > 0 ? reinterpret_cast<float*>(tb + L.X) : nullptr;
  P->seg_state = L.segmented ? reinterpret_cast<float*>(tb + L.seg_state) : nullptr;
  P->U2 = L.overlap ? reinterpret_cast<float*>(tb + L.U2) : nullptr;
}

bool mtp::uses_gen_overlap(const mtp_config& c) {
  constexpr long long kUnits = 256;     // compute units
  constexpr long long kMinFree = 32;    // units left for drawing the next tensor paths
  if (c.n_iters < 2 || c.sample_wor || c.n_tensor < 1) return false;
  if (uses_segmented_rollout(c)) return true;
  const long long B = static_cast<long long>(c.n_tensor) + c.n_gauss;
  const bool chain = c.dynamics == MTP_DYN_CHAIN || c.dynamics == MTP_DYN_CHAIN_CONTACT;
  const bool quad = c.dynamics == MTP_DYN_CHAIN && c.n_links >= 5 && c.n_links <= 8;
  const bool pair = chain && c.n_links >= 10 && (c.n_links % 2) == 0;
  const bool pm = c.dynamics == MTP_DYN_POINT_MASS;
  const long long lanes = (pm ? kPmLanes : quad ? 4 : pair ? 2 : 1) * B;
  return (lanes + kRollThreads - 1) / kRollThreads <= kUnits - kMinFree;
}

bool mtp::uses_segmented_rollout(const mtp_config& c) {
  constexpr long long kSimds = 1024;   // 256 compute units x 4 SIMDs
  const long long B = static_cast<long long>(c.n_tensor) + c.n_gauss;
  const bool pair = (c.dynamics == MTP_DYN_CHAIN || c.dynamics == MTP_DYN_CHAIN_CONTACT) && c.n_links >= 10 &&
                    (c.n_links % 2) == 0;
  const int R = c.n_replicas > 1 ? c.n_replicas : 1;
  return pair && R == 1 && (B + 31) / 32 > kSimds && c.horizon >= 16;
}

// The S in 4..16 whose unit count groups*S is closest above to a whole number
// of rounds of the resident waves (ties to the smaller S).
int mtp::segment_count(int groups, int resident_waves) {
  int best = 4;
  double best_eff = 0.0;
  for (int S = 4; S <= 16; ++S) {
    const long long units = static_cast<long long>(groups) * S;
    const long long rounds = (units + resident_waves - 1) / resident_waves;
    const double eff = static_cast<double>(units) / static_cast<double>(rounds * resident_waves);
    if (eff > best_eff + 1e-9) { best_eff = eff; best = S; }
  }
  return best;
}

int mtp::perm_rounds(int L, int W) {
  int bits = 0;
  while ((1 << bits) < W) ++bits;
  return 2 * L * (bits > 0 ? bits : 1);
}

// Enough workgroups to give every SIMD of the chip a few waves: short horizons
// and small batches split the horizon into chunks of a multiple of 4 steps.
int mtp::cand_time_chunk(int B, int T, int n) {
  constexpr long long kTargetWaves = 4096;
  const long long waves = static_cast<long long>((B + kCandThreads - 1) / kCandThreads) * n * (kCandThreads / 64);
  long long chunks = waves >= kTargetWaves ? 1 : (kTargetWaves + waves - 1) / waves;
  chunks = std::min<long long>(chunks, std::max(1, T / 4));
  int tc = static_cast<int>((T + chunks - 1) / chunks);
  tc = (tc + 3) & ~3;
  // long horizons: chunks of at most 64 steps even when the grid is large
  // (a few per cent faster on the 256-step, 24-link workload than whole horizons)
  constexpr int kMaxChunk = 64;
  tc = std::min(tc, kMaxChunk);
  return std::max(tc, 4);
}

PlanDesc mtp::make_desc(const mtp_config& c, const Layout& L, uint8_t* base, uint8_t* tb) {
  PlanDesc P{};
  P.dyn = c.dynamics; P.interp = c.interp; P.n_links = c.n_links; P.d = c.state_dim; P.n = c.ctrl_dim;
  P.T = c.horizon; P.L = c.n_layers; P.W = c.n_width; P.P = c.n_tensor; P.G = c.n_gauss;
  P.B = c.n_tensor + c.n_gauss; P.E = c.n_elites; P.K = c.n_iters; P.p = c.bspline_degree;
  P.n_dbg = c.n_debug_states; P.n_task = c.n_task_params; P.ldU = static_cast<int32_t>(L.ldU);
  P.R = c.n_replicas > 1 ? c.n_replicas : 1;
  P.wor = c.sample_wor;
  P.sw_rounds = c.sample_wor ? perm_rounds(c.n_layers, c.n_width) : 0;
  P.diag = c.diagnostics;
  // task of a chain: gravity, goal weight, control weight, target (2), masses[N], lengths[N], ...
  P.eq_len = 0;
  if ((c.dynamics == MTP_DYN_CHAIN || c.dynamics == MTP_DYN_CHAIN_CONTACT) && c.task_params != nullptr &&
      c.n_task_params >= 5 + 2 * c.n_links) {
    P.eq_len = 1;
    for (int k = 1; k < c.n_links; ++k)
      if (std::memcmp(&c.task_params[5 + c.n_links + k], &c.task_params[5 + c.n_links], sizeof(float)) != 0) P.eq_len = 0;
  }
  P.tc = cand_time_chunk(P.B, P.T, P.n);
  P.lam = c.temperature; P.alpha = c.smoothing; P.sigma_min = c.sigma_min; P.sigma_init = c.sigma_init;
  P.u_min = c.u_min; P.u_max = c.u_max; P.dt = c.dt;
  P.key0 = static_cast<uint32_t>(c.seed & 0xFFFFFFFFull);
  P.key1 = static_cast<uint32_t>(c.seed >> 32);
  P.ctrl = reinterpret_cast<uint32_t*>(base + L.ctrl);
  P.x0 = reinterpret_cast<float*>(base + L.x0);
  P.x0_src = nullptr;
  P.mu = reinterpret_cast<float*>(base + L.mu);
  P.sigma = reinterpret_cast<float*>(base + L.sigma);
  P.tmp = reinterpret_cast<float*>(base + L.tmp);
  P.action = reinterpret_cast<float*>(base + L.action);
  P.basis = reinterpret_cast<const float*>(base + L.basis);
  P.span = reinterpret_cast<const int32_t*>(base + L.span);
  P.task = reinterpret_cast<const float*>(base + L.task);
  P.sparams = c.dynamics == MTP_DYN_CHAIN_CONTACT ? reinterpret_cast<const float*>(base + L.sparams) : nullptr;
  P.entropy = reinterpret_cast<float*>(base + L.entropy);
  P.seg_ctl = L.segmented ? reinterpret_cast<SegCtl*>(base + L.seg_ctl) : nullptr;
  P.seg_done = L.segmented ? reinterpret_cast<uint32_t*>(base + L.seg_done) : nullptr;
  P.seg_S = 0; P.seg_len = 0; P.seg_grid = 0;   // set by the launcher's device query (seg_configure)
  P.roll_blocks = 0; P.gen_k = -1; P.gen_grid = 0;   // gen_grid: device query (gen_configure)
  if (tb != nullptr) set_transient(&P, c, L, tb);
  return P;
}

// Upload a plan's tables and initial state into its workspace (synchronous).
mtp_status mtp::upload_plan_tables(const mtp_config& c, const PlanDesc& P, const float* task, const float* sparams,
                                   hipStream_t st, std::string* err) {
  std::vector<float> basis;
  std::vector<int32_t> span;
  build_tables(c, &basis, &span);
  const size_t Tn = static_cast<size_t>(c.horizon) * c.ctrl_dim;
  std::vector<float> mu(Tn, 0.5f * (c.u_min + c.u_max)), sg(Tn, c.sigma_init);
  const uint32_t ctrl[6] = {0u, 0u, 0u, 0u, 0u, 0u};
  const size_t B = static_cast<size_t>(c.n_tensor) + c.n_gauss;
  hipError_t e = hipSuccess;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes > 0) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  cp(const_cast<float*>(P.basis), basis.data(), basis.size() * 4);
  cp(const_cast<int32_t*>(P.span), span.data(), span.size() * 4);
  cp(const_cast<float*>(P.task), task, static_cast<size_t>(c.n_task_params) * 4);
  const size_t R = c.n_replicas > 1 ? static_cast<size_t>(c.n_replicas) : 1;
  if (P.sparams) cp(const_cast<float*>(P.sparams), sparams, R * B * (c.ctrl_dim + 1) * 4);
  cp(P.mu, mu.data(), Tn * 4);
  cp(P.sigma, sg.data(), Tn * 4);
  cp(P.ctrl, ctrl, sizeof(ctrl));
  const std::vector<uint32_t> seg_zero(P.seg_ctl != nullptr ? 4 + (B + 31) / 32 : 0, 0u);   // lives past the sync
  if (P.seg_ctl != nullptr) {
    cp(P.seg_ctl, seg_zero.data(), 16);
    cp(P.seg_done, seg_zero.data() + 4, ((B + 31) / 32) * 4);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    if (err) *err = std::string("upload: ") + hipGetErrorString(e);
    return MTP_ERR_DEVICE;
  }
  return MTP_OK;
}

hipError_t mtp::enqueue_iterations(const PlanDesc& P, int k_begin, int k_end, hipStream_t st, const SideLane* side) {
  for (int k = k_begin; k < k_end; ++k)
    for (int stage = 0; stage < 4; ++stage) {
      const hipError_t e = launch_iteration_stage(P, stage, k, k_begin, k_end, st, side);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

static hipError_t take_event(mtp_plan* p, hipEvent_t* ev) {
  if (!p->ev_free.empty()) {
    *ev = p->ev_free.back();
    p->ev_free.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(ev);
}

static hipError_t drain_events(mtp_plan* p) {
  for (auto& q : p->pending) {
    hipError_t e = hipEventSynchronize(q.b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, q.a, q.b);
    if (e != hipSuccess) return e;
    p->stage_ms[q.stage] += ms;
    p->stage_count[q.stage] += 1;
    p->ev_free.push_back(q.a);
    p->ev_free.push_back(q.b);
  }
  p->pending.clear();
  return hipSuccess;
}

// Launch iterations [k0, k1) one kernel at a time, with event pairs around each
// stage when timing is on.
// The plan's second stream and its fork / join events, created on first use by
// plans that draw the next tensor paths beside a time-sliced rollout; null for
// the others.
static hipError_t side_lane(mtp_plan* p, const SideLane** out) {
  *out = nullptr;
  if (!(p->lay.overlap && p->lay.segmented)) return hipSuccess;
  if (p->side.st == nullptr) {
    hipError_t e = hipStreamCreateWithFlags(&p->side.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->side.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->side.join, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  *out = &p->side;
  return hipSuccess;
}

static hipError_t enqueue_iterations_plan(mtp_plan* p, int k0, int k1) {
  const SideLane* side = nullptr;
  hipError_t es = side_lane(p, &side);
  if (es != hipSuccess) return es;
  if (!p->timing) return enqueue_iterations(p->P, k0, k1, p->stream, side);
  for (int k = k0; k < k1; ++k)
    for (int stage = 0; stage < 4; ++stage) {
      hipEvent_t a, b;
      hipError_t e = take_event(p, &a);
      if (e == hipSuccess) e = take_event(p, &b);
      if (e == hipSuccess) e = hipEventRecord(a, p->stream);
      if (e == hipSuccess) e = launch_iteration_stage(p->P, stage, k, k0, k1, p->stream, side);
      if (e == hipSuccess) e = hipEventRecord(b, p->stream);
      if (e != hipSuccess) return e;
      p->pending.push_back({stage, a, b});
      if (p->pending.size() >= 4096) {
        e = drain_events(p);
        if (e != hipSuccess) return e;
      }
    }
  return hipSuccess;
}

extern "C" {

size_t mtp_workspace_bytes(const mtp_config* cfg) {
  if (!validate_config(cfg, nullptr, nullptr)) return 0;
  return compute_layout(*cfg, true).total;
}

size_t mtp_transient_bytes(const mtp_config* cfg) {
  if (!validate_config(cfg, nullptr, nullptr)) return 0;
  return compute_layout(*cfg).transient;
}

size_t mtp_resident_bytes(const mtp_config* cfg) {
  if (!validate_config(cfg, nullptr, nullptr)) return 0;
  return compute_layout(*cfg).resident;
}

mtp_status mtp_validate_config(const mtp_config* cfg, char* why, size_t why_len) {
  std::string msg;
  mtp_status code = MTP_OK;
  const bool ok = validate_config(cfg, &msg, &code);
  if (why != nullptr && why_len > 0) {
    const size_t n = msg.size() < why_len - 1 ? msg.size() : why_len - 1;
    std::memcpy(why, msg.data(), n);
    why[n] = '\0';
  }
  return ok ? MTP_OK : code;
}

mtp_status mtp_plan_create(const mtp_config* cfg, void* d_workspace, size_t ws_bytes, void* hip_stream,
                           mtp_plan** out) {
  if (out == nullptr) return MTP_ERR_INVALID_ARG;
  *out = nullptr;
  std::string why;
  mtp_status code = MTP_OK;
  if (!validate_config(cfg, &why, &code)) return code;
  const Layout lay = compute_layout(*cfg, true);
  if (d_workspace == nullptr || ws_bytes < lay.total || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) != 0)
    return MTP_ERR_WORKSPACE;
  mtp_plan* p = new (std::nothrow) mtp_plan();
  if (p == nullptr) return MTP_ERR_INVALID_ARG;
  p->cfg = *cfg;
  p->task.assign(cfg->task_params, cfg->task_params + cfg->n_task_params);
  const size_t B = static_cast<size_t>(cfg->n_tensor) + cfg->n_gauss;
  const size_t R = cfg->n_replicas > 1 ? static_cast<size_t>(cfg->n_replicas) : 1;
  if (cfg->dynamics == MTP_DYN_CHAIN_CONTACT)
    p->sparams.assign(cfg->sample_params, cfg->sample_params + R * B * (cfg->ctrl_dim + 1));
  p->cfg.task_params = p->task.data();
  p->cfg.sample_params = p->sparams.empty() ? nullptr : p->sparams.data();
  p->lay = lay;
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->P = make_desc(p->cfg, lay, static_cast<uint8_t*>(d_workspace),
                   static_cast<uint8_t*>(d_workspace) + lay.resident);
  const mtp_status s = upload_plan_tables(p->cfg, p->P, p->task.data(), p->cfg.sample_params, p->stream, &p->err);
  if (s != MTP_OK) {
    delete p;
    return s;
  }
  if (seg_configure(&p->P) != hipSuccess || gen_configure(&p->P) != hipSuccess) {
    delete p;
    return MTP_ERR_DEVICE;
  }
  // with an even iteration count the last iteration's generator writes the
  // buffer that the next replan's iteration 0 reads
  p->P.spec = (mtp_plan_draws_ahead(p) && cfg->n_iters % 2 == 0) ? 1 : 0;
  *out = p;
  return MTP_OK;
}

static mtp_status ensure_graph(mtp_plan* p) {
  if (p->exec) return MTP_OK;
  if (!p->cap_stream) HIPCHK(p, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "stream create");
  const SideLane* side = nullptr;
  HIPCHK(p, side_lane(p, &side), "side stream create");
  HIPCHK(p, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  hipError_t e = launch_shift(p->P, p->cap_stream);
  if (e == hipSuccess) e = enqueue_iterations(p->P, 0, p->cfg.n_iters, p->cap_stream, side);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(p->cap_stream, &g);
  if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return device_err(p, e, "capture launch"); }
  if (e2 != hipSuccess) return device_err(p, e2, "end capture");
  p->graph = g;
  HIPCHK(p, hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0), "graph instantiate");
  return MTP_OK;
}

mtp_status mtp_replan_at(mtp_plan* p, const float* d_x0, int32_t shift_steps, uint32_t replan_idx) {
  if (p == nullptr) return MTP_ERR_INVALID_ARG;
  if (p->sticky) return MTP_ERR_DEVICE;
  if (d_x0 == nullptr) return set_err(p, MTP_ERR_INVALID_ARG, "d_x0 is NULL");
  if (shift_steps < 0) return set_err(p, MTP_ERR_INVALID_ARG, "shift_steps must be >= 0");
  const bool graph = p->use_graph && !p->timing;
  if (graph) {
    const mtp_status s = ensure_graph(p);
    if (s != MTP_OK) return s;
  }
  HIPCHK(p, launch_set_ctrl(p->P, replan_idx, shift_steps, d_x0, p->stream), "set ctrl");
  if (graph) {
    HIPCHK(p, hipGraphLaunch(p->exec, p->stream), "graph launch");
  } else {
    HIPCHK(p, launch_shift(p->P, p->stream), "shift");
    HIPCHK(p, enqueue_iterations_plan(p, 0, p->cfg.n_iters), "iterations");
  }
  p->next_r = replan_idx + 1;
  return MTP_OK;
}

mtp_status mtp_replan(mtp_plan* p, const float* d_x0, int32_t shift_steps) {
  if (p == nullptr) return MTP_ERR_INVALID_ARG;
  return mtp_replan_at(p, d_x0, shift_steps, p->next_r);
}

mtp_status mtp_get_action(mtp_plan* p, float* h_u) {
  if (p == nullptr || h_u == nullptr) return MTP_ERR_INVALID_ARG;
  if (p->sticky) return MTP_ERR_DEVICE;
  HIPCHK(p, hipMemcpyAsync(h_u, p->P.action, p->cfg.ctrl_dim * sizeof(float), hipMemcpyDeviceToHost, p->stream), "action copy");
  HIPCHK(p, hipStreamSynchronize(p->stream), "sync");
  return MTP_OK;
}

mtp_status mtp_get_state(const mtp_plan* pc, float* d_mu, float* d_sigma, uint32_t* replan_idx) {
  mtp_plan* p = const_cast<mtp_plan*>(pc);
  if (p == nullptr) return MTP_ERR_INVALID_ARG;
  if (p->sticky) return MTP_ERR_DEVICE;
  const size_t bytes = static_cast<size_t>(p->cfg.horizon) * p->cfg.ctrl_dim * sizeof(float);
  if (d_mu) HIPCHK(p, hipMemcpyAsync(d_mu, p->P.mu, bytes, hipMemcpyDeviceToDevice, p->stream), "mu copy");
  if (d_sigma) HIPCHK(p, hipMemcpyAsync(d_sigma, p->P.sigma, bytes, hipMemcpyDeviceToDevice, p->stream), "sigma copy");
  if (replan_idx) *replan_idx = p->next_r;
  HIPCHK(p, hipStreamSynchronize(p->stream), "sync");
  return MTP_OK;
}

mtp_status mtp_set_state(mtp_plan* p, const float* d_mu, const float* d_sigma, uint32_t replan_idx) {
  if (p == nullptr || d_mu == nullptr || d_sigma == nullptr) return MTP_ERR_INVALID_ARG;
  if (p->sticky) return MTP_ERR_DEVICE;
  const size_t bytes = static_cast<size_t>(p->cfg.horizon) * p->cfg.ctrl_dim * sizeof(float);
  HIPCHK(p, hipMemcpyAsync(p->P.mu, d_mu, bytes, hipMemcpyDeviceToDevice, p->stream), "mu copy");
  HIPCHK(p, hipMemcpyAsync(p->P.sigma, d_sigma, bytes, hipMemcpyDeviceToDevice, p->stream), "sigma copy");
  p->next_r = replan_idx;
  return MTP_OK;
}

mtp_status mtp_set_x0(mtp_plan* p, const float* d_x0) {
  if (p == nullptr || d_x0 == nullptr) return MTP_ERR_INVALID_ARG;
  if (p->sticky) return MTP_ERR_DEVICE;
  HIPCHK(p, hipMemcpyAsync(p->P.x0, d_x0, p->cfg.state_dim * sizeof(float), hipMemcpyDeviceToDevice, p->stream), "x0 copy");
  return MTP_OK;
}

mtp_status mtp_run_stage(mtp_plan* p, int32_t stage, uint32_t replan_idx, int32_t k) {
  if (p == nullptr) return MTP_ERR_INVALID_ARG;
  if (p->sticky) return MTP_ERR_DEVICE;
  if (stage < 0 || stage > MTP_STAGE_ALL) return set_err(p, MTP_ERR_INVALID_ARG, "unknown stage");
  if (k < 0 || k > 65535) return set_err(p, MTP_ERR_INVALID_ARG, "iteration index out of range");
  HIPCHK(p, launch_set_ctrl(p->P, replan_idx, 0, nullptr, p->stream), "set ctrl");
  if (stage == MTP_STAGE_ALL) {
    HIPCHK(p, enqueue_iterations_plan(p, k, k + 1), "iteration");
  } else {
    HIPCHK(p, launch_stage(p->P, stage, k, p->stream), "stage");
  }
  return MTP_OK;
}

int32_t mtp_plan_draws_ahead(const mtp_plan* p) {
  return (p != nullptr && p->lay.overlap && (p->lay.segmented || p->P.gen_grid > rollout_blocks(p->P))) ? 1 : 0;
}

mtp_status mtp_set_graph_mode(mtp_plan* p, int32_t use_graph) {
  if (p == nullptr) return MTP_ERR_INVALID_ARG;
  p->use_graph = use_graph != 0;
  return MTP_OK;
}

mtp_status mtp_set_stage_timing(mtp_plan* p, int32_t enable) {
  if (p == nullptr) return MTP_ERR_INVALID_ARG;
  if (p->sticky) return MTP_ERR_DEVICE;
  HIPCHK(p, drain_events(p), "timing drain");
  p->timing = enable != 0;
  for (int i = 0; i < 4; ++i) { p->stage_ms[i] = 0.0; p->stage_count[i] = 0; }
  return MTP_OK;
}

mtp_status mtp_get_stage_times(mtp_plan* p, double* h_ms4, uint64_t* h_count4) {
  if (p == nullptr || h_ms4 == nullptr || h_count4 == nullptr) return MTP_ERR_INVALID_ARG;
  if (p->sticky) return MTP_ERR_DEVICE;
  HIPCHK(p, drain_events(p), "timing drain");
  for (int i = 0; i < 4; ++i) { h_ms4[i] = p->stage_ms[i]; h_count4[i] = p->stage_count[i]; }
  return MTP_OK;
}

mtp_status mtp_get_buffers(const mtp_plan* p, mtp_buffers* out) {
  if (p == nullptr || out == nullptr) return MTP_ERR_INVALID_ARG;
  const PlanDesc& P = p->P;
  out->Z = P.Z; out->I = P.I; out->U = P.U; out->cost = P.cost; out->elite_idx = P.eidx;
  out->elite_cost = P.ecost; out->weights = P.w; out->mu = P.mu; out->sigma = P.sigma; out->x0 = P.x0;
  out->action = P.action; out->X_dbg = P.X; out->entropy = P.entropy; out->ld_U = static_cast<size_t>(P.ldU);
  return MTP_OK;
}

mtp_status mtp_get_flags(mtp_plan* p, uint32_t* h_flags) {
  if (p == nullptr || h_flags == nullptr) return MTP_ERR_INVALID_ARG;
  if (p->sticky) return MTP_ERR_DEVICE;
  HIPCHK(p, hipMemcpyAsync(h_flags, p->P.ctrl + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, p->stream), "flags copy");
  HIPCHK(p, hipStreamSynchronize(p->stream), "sync");
  return MTP_OK;
}

mtp_status mtp_plan_destroy(mtp_plan* p) {
  if (p == nullptr) return MTP_ERR_INVALID_ARG;
  (void)drain_events(p);
  for (auto ev : p->ev_free) (void)hipEventDestroy(ev);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->side.fork) (void)hipEventDestroy(p->side.fork);
  if (p->side.join) (void)hipEventDestroy(p->side.join);
  if (p->side.st) (void)hipStreamDestroy(p->side.st);
  delete p;
  return MTP_OK;
}

const char* mtp_status_str(mtp_status s) {
  switch (s) {
    case MTP_OK: return "ok";
    case MTP_ERR_INVALID_ARG: return "invalid argument";
    case MTP_ERR_UNSUPPORTED: return "unsupported configuration";
    case MTP_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case MTP_ERR_DEVICE: return "device error";
    case MTP_ERR_BUSY: return "busy";
    case MTP_ERR_NOT_READY: return "not ready";
  }
  return "unknown status";
}

const char* mtp_last_error(const mtp_plan* p) { return p ? p->err.c_str() : "no plan"; }

mtp_status mtp_interp_table(const mtp_config* cfg, float* h_basis, int32_t* h_span) {
  mtp_status code = MTP_OK;
  if (!validate_config(cfg, nullptr, &code)) return code;
  if (h_basis == nullptr || h_span == nullptr) return MTP_ERR_INVALID_ARG;
  std::vector<float> basis;
  std::vector<int32_t> span;
  build_tables(*cfg, &basis, &span);
  std::memcpy(h_basis, basis.data(), basis.size() * sizeof(float));
  std::memcpy(h_span, span.data(), span.size() * sizeof(int32_t));
  return MTP_OK;
}

int32_t mtp_supported_chain_links(int32_t* out, int32_t cap) {
  if (out == nullptr || cap < 0) return supported_chain_links(nullptr, 0);
  return supported_chain_links(out, cap);
}

}  // extern "C"
