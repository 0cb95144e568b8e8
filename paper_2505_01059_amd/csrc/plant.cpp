// Host-side float64 plant of the serving loop: one step x_{t+1} = f(x_t, u_t)
// of a robot's model, so that a load generator can close the receding-horizon
// loop of Alg. 2 (execute the returned control, replan from the new state).
//
// The models are those the rollout kernels integrate: the planar point mass
// (semi-implicit Euler) and the chain of point masses on massless links with
// torques between neighbouring links and optional penalty ground contact
// (RK4).  The chain's link accelerations come from the link tensions, which
// solve a symmetric tridiagonal system: the length constraint of link k
// couples the accelerations of its two end masses.  The contact chain's plant
// uses the first row of the config's per-sample parameters (masses, friction).
#include <cmath>
#include <vector>

#include "../../include/mtp.h"
#include "plan_internal.hpp"

namespace {

struct ChainModel {
  int n;
  double g, yg, kc, dc, vslip, muf;
  bool contact;
  std::vector<double> l, im;   // link lengths, inverse masses of the masses at their distal ends
};

// d(phi, omega)/dt of the chain at (phi, om) with torques u held.
void chain_rates(const ChainModel& M, const double* phi, const double* om, const float* u, double* dphi,
                 double* dom) {
  const int n = M.n;
  std::vector<double> s(n), c(n), q(n), fx(n, 0.0), fy(n, 0.0), C(n, 0.0), S(n, 0.0);
  for (int k = 0; k < n; ++k) {
    s[k] = std::sin(phi[k]);
    c[k] = std::cos(phi[k]);
    q[k] = (static_cast<double>(u[k]) - (k + 1 < n ? static_cast<double>(u[k + 1]) : 0.0)) / M.l[k];
  }
  for (int k = 0; k + 1 < n; ++k) {
    C[k] = std::cos(phi[k] - phi[k + 1]);
    S[k] = std::sin(phi[k] - phi[k + 1]);
  }
  if (M.contact) {
    double y = 0.0, vx = 0.0, vy = 0.0;
    for (int k = 0; k < n; ++k) {
      y -= M.l[k] * c[k];
      vx += M.l[k] * om[k] * c[k];
      vy += M.l[k] * om[k] * s[k];
      const double pen = M.yg - y;
      if (pen > 0.0) {
        const double fn = std::fmax(M.kc * pen - M.dc * vy, 0.0);
        fx[k] = -M.muf * fn * std::tanh(vx / M.vslip) * M.im[k];   // accelerations of mass k
        fy[k] = fn * M.im[k];
      }
    }
  }
  // a_k - a_{k-1} of the external (gravity, contact) accelerations; the base is fixed
  std::vector<double> dfx(n), dfy(n);
  for (int k = 0; k < n; ++k) {
    dfx[k] = fx[k] - (k > 0 ? fx[k - 1] : 0.0);
    dfy[k] = fy[k] - (k > 0 ? fy[k - 1] : 0.0) - (k == 0 ? M.g : 0.0);
  }
  // tensions: row k couples T_{k-1}, T_k, T_{k+1}
  std::vector<double> cp(n), dp(n);
  for (int k = 0; k < n; ++k) {
    const double imp = k > 0 ? M.im[k - 1] : 0.0;
    const double diag = M.im[k] + imp;
    const double up = -M.im[k] * C[k];
    const double lo = k > 0 ? -imp * C[k - 1] : 0.0;
    double rhs = M.l[k] * om[k] * om[k] + s[k] * dfx[k] - c[k] * dfy[k];
    if (k + 1 < n) rhs -= M.im[k] * q[k + 1] * S[k];
    if (k > 0) rhs += imp * q[k - 1] * S[k - 1];
    const double piv = diag - (k > 0 ? lo * cp[k - 1] : 0.0);
    cp[k] = up / piv;
    dp[k] = (rhs - (k > 0 ? lo * dp[k - 1] : 0.0)) / piv;
  }
  for (int k = n - 2; k >= 0; --k) dp[k] -= cp[k] * dp[k + 1];
  for (int k = 0; k < n; ++k) {
    const double imp = k > 0 ? M.im[k - 1] : 0.0;
    double a = (M.im[k] + imp) * q[k];
    if (k + 1 < n) a -= M.im[k] * (dp[k + 1] * S[k] + q[k + 1] * C[k]);
    if (k > 0) a -= imp * (-dp[k - 1] * S[k - 1] + q[k - 1] * C[k - 1]);
    a += c[k] * dfx[k] + s[k] * dfy[k];
    dphi[k] = om[k];
    dom[k] = a / M.l[k];
  }
}

}  // namespace

extern "C" mtp_status mtp_plant_step(const mtp_config* cfg, const double* h_x, const float* h_u, double* h_x_next) {
  if (!mtp::validate_config(cfg, nullptr, nullptr) || h_x == nullptr || h_u == nullptr || h_x_next == nullptr)
    return MTP_ERR_INVALID_ARG;
  const double dt = cfg->dt;
  const float* tk = cfg->task_params;
  if (cfg->dynamics == MTP_DYN_POINT_MASS) {
    const double vx = h_x[2] + dt * h_u[0], vy = h_x[3] + dt * h_u[1];
    h_x_next[0] = h_x[0] + dt * vx;
    h_x_next[1] = h_x[1] + dt * vy;
    h_x_next[2] = vx;
    h_x_next[3] = vy;
    return MTP_OK;
  }
  const int n = cfg->n_links;
  ChainModel M;
  M.n = n;
  M.g = tk[0];
  M.contact = cfg->dynamics == MTP_DYN_CHAIN_CONTACT;
  M.l.resize(n);
  M.im.resize(n);
  for (int k = 0; k < n; ++k) {
    M.l[k] = tk[5 + n + k];
    M.im[k] = 1.0 / (M.contact ? cfg->sample_params[k] : tk[5 + k]);
  }
  M.yg = M.kc = M.dc = M.muf = 0.0;
  M.vslip = 1.0;
  if (M.contact) {
    M.yg = tk[5 + 2 * n];
    M.kc = tk[6 + 2 * n];
    M.dc = tk[7 + 2 * n];
    M.vslip = tk[8 + 2 * n];
    M.muf = cfg->sample_params[n];
  }
  // classical RK4 on (phi, omega), control held
  const int d = 2 * n;
  std::vector<double> x(h_x, h_x + d), k1(d), k2(d), k3(d), k4(d), y(d);
  auto rates = [&](const std::vector<double>& z, std::vector<double>& out) {
    chain_rates(M, z.data(), z.data() + n, h_u, out.data(), out.data() + n);
  };
  rates(x, k1);
  for (int i = 0; i < d; ++i) y[i] = x[i] + 0.5 * dt * k1[i];
  rates(y, k2);
  for (int i = 0; i < d; ++i) y[i] = x[i] + 0.5 * dt * k2[i];
  rates(y, k3);
  for (int i = 0; i < d; ++i) y[i] = x[i] + dt * k3[i];
  rates(y, k4);
  for (int i = 0; i < d; ++i) h_x_next[i] = x[i] + (dt / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  return MTP_OK;
}
