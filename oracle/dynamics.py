"""Analytic dynamics x_{t+1} = f(x_t, u_t) and per-step costs (oracle side).

Section 2.1 fixes the rollout x_{t+1} = f(x_t, u_t) and the cumulative cost
J = sum_t c(x_t, u_t) + c_T(x_T) (Eq. 1); Alg. 2 evaluates a cost matrix
S in R^{B x T}.  Here S[b, t] = c_state(x_{t+1}) + c_ctrl(u_t): this equals
Eq. 1 with c_T = c_state up to the candidate-independent term c_state(x_0),
so rankings and softmax weights are the same.

Models (the paper's MuJoCo tasks are not available; these are stand-ins):

point mass -- planar double integrator, state (p, v), control = acceleration,
  semi-implicit Euler: v' = v + dt u, p' = p + dt v'.
  cost = w_g |p' - goal|^2 + penalty * #{k : |p' - c_k|^2 < r_k^2} + w_u |u|^2.

n-link chain -- planar chain of point masses m_i at the distal ends of
  massless links of length l_i, base pinned at the origin, absolute link
  angles phi_i measured from the downward vertical, state (phi, dphi).  The
  torque tau_i acts between link i-1 (or the base) and link i, so the
  generalised force on phi_i is tau_i - tau_{i+1}.  Equations of motion from
  the Lagrangian, written densely:
      M(phi) ddphi = Q - h(phi, dphi) - g(phi)
      M_ij = l_i l_j cos(phi_i - phi_j) mu_max(i,j),  mu_k = sum_{q >= k} m_q
      h_i  = sum_j l_i l_j mu_max(i,j) sin(phi_i - phi_j) dphi_j^2
      g_i  = grav l_i mu_i sin(phi_i)
  integrated with classical RK4 (control held over the step).
  cost = w_g |p_end(x') - target|^2 + w_u |tau|^2.

contact -- each mass below the ground y_g feels a penalty spring-damper
  normal force F_n = max(0, k (y_g - y) - d vy) and smoothed Coulomb friction
  F_t = -mu_f F_n tanh(vx / v_slip); the generalised force on phi_i is
  sum_{k >= i} l_i (F_kx cos phi_i + F_ky sin phi_i).
"""
import numpy as np

import mtp_workloads as W


# ------------------------------------------------------------- point mass

def point_mass_step(x, u, dt):
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    v = x[..., 2:4] + dt * u
    p = x[..., 0:2] + dt * v
    return np.concatenate([p, v], axis=-1)


def point_mass_cost(task, x_next, u):
    p = x_next[..., 0:2]
    goal = np.asarray(task.goal, dtype=np.float64)
    c = float(task.goal_weight) * np.sum((p - goal) ** 2, axis=-1)
    obs = np.asarray(task.obstacles, dtype=np.float64)
    for cx, cy, r in obs:
        d2 = (p[..., 0] - cx) ** 2 + (p[..., 1] - cy) ** 2
        c = c + float(task.obstacle_penalty) * (d2 < r * r)
    return c + float(task.ctrl_weight) * np.sum(np.asarray(u, np.float64) ** 2, axis=-1)


def point_mass_obstacle_margin(task, x_next):
    """min_k | |p - c_k|^2 - r_k^2 |: how close a state is to an indicator switch."""
    p = x_next[..., 0:2]
    out = np.full(p.shape[:-1], np.inf)
    for cx, cy, r in np.asarray(task.obstacles, dtype=np.float64):
        d2 = (p[..., 0] - cx) ** 2 + (p[..., 1] - cy) ** 2
        out = np.minimum(out, np.abs(d2 - r * r))
    return out


# ------------------------------------------------------------- chain

def chain_positions(phi, lengths):
    """Mass positions p_k = sum_{i<=k} l_i (sin phi_i, -cos phi_i); shape (..., n, 2)."""
    ex = lengths * np.sin(phi)
    ey = -lengths * np.cos(phi)
    return np.stack([np.cumsum(ex, axis=-1), np.cumsum(ey, axis=-1)], axis=-1)


def chain_velocities(phi, dphi, lengths):
    vx = lengths * np.cos(phi) * dphi
    vy = lengths * np.sin(phi) * dphi
    return np.stack([np.cumsum(vx, axis=-1), np.cumsum(vy, axis=-1)], axis=-1)


def chain_tail_masses(masses):
    """mu_k = sum_{q >= k} m_q."""
    return np.flip(np.cumsum(np.flip(masses, axis=-1), axis=-1), axis=-1)


def chain_mass_matrix(phi, masses, lengths):
    n = phi.shape[-1]
    mu = chain_tail_masses(masses)                              # (..., n)
    idx = np.maximum.outer(np.arange(n), np.arange(n))          # max(i, j)
    mu_ij = mu[..., idx]                                        # (..., n, n)
    dphi_ij = phi[..., :, None] - phi[..., None, :]
    return lengths[..., :, None] * lengths[..., None, :] * np.cos(dphi_ij) * mu_ij


def chain_bias(phi, dphi, masses, lengths, gravity):
    """h + g of the equations of motion."""
    n = phi.shape[-1]
    mu = chain_tail_masses(masses)
    idx = np.maximum.outer(np.arange(n), np.arange(n))
    mu_ij = mu[..., idx]
    s_ij = np.sin(phi[..., :, None] - phi[..., None, :])
    h = np.sum(lengths[..., :, None] * lengths[..., None, :] * mu_ij * s_ij
               * (dphi ** 2)[..., None, :], axis=-1)
    g = gravity * lengths * mu * np.sin(phi)
    return h + g


def contact_forces(phi, dphi, lengths, mu_f, task):
    """Penalty-spring ground forces on each mass; shape (..., n, 2)."""
    p = chain_positions(phi, lengths)
    v = chain_velocities(phi, dphi, lengths)
    y, vx, vy = p[..., 1], v[..., 0], v[..., 1]
    below = y < float(task.ground_y)
    fn = float(task.k_contact) * (float(task.ground_y) - y) - float(task.d_contact) * vy
    fn = np.where(below, np.maximum(fn, 0.0), 0.0)
    ft = -np.asarray(mu_f)[..., None] * fn * np.tanh(vx / float(task.v_slip))
    return np.stack([ft, fn], axis=-1)


def chain_accel(x, tau, task, masses, mu_f=None, contact=False, dtype=np.float64):
    """State derivative (dphi, ddphi).  `dtype` is float64 for the oracle; the
    float32 setting exists only to measure how fast float32 rounding drifts
    from the float64 trajectory (same formulas, other precision)."""
    x = np.asarray(x, dtype=dtype)
    n = x.shape[-1] // 2
    phi, dphi = x[..., :n], x[..., n:]
    lengths = np.asarray(task.lengths, dtype=dtype)
    tau = np.asarray(tau, dtype=dtype)
    Q = tau - np.concatenate([tau[..., 1:], np.zeros_like(tau[..., :1])], axis=-1)
    if contact:
        F = contact_forces(phi, dphi, lengths, mu_f, task)      # (..., n, 2)
        Fx = np.flip(np.cumsum(np.flip(F[..., 0], -1), -1), -1)  # sum_{k >= i}
        Fy = np.flip(np.cumsum(np.flip(F[..., 1], -1), -1), -1)
        Q = Q + lengths * (Fx * np.cos(phi) + Fy * np.sin(phi))
    M = chain_mass_matrix(phi, masses, lengths)
    rhs = Q - chain_bias(phi, dphi, masses, lengths, float(task.gravity))
    ddphi = np.linalg.solve(M, rhs[..., None])[..., 0]
    return np.concatenate([dphi, ddphi], axis=-1)


def rk4_step(f, x, u, dt):
    """Classical fourth-order Runge-Kutta step with u held constant."""
    k1 = f(x, u)
    k2 = f(x + 0.5 * dt * k1, u)
    k3 = f(x + 0.5 * dt * k2, u)
    k4 = f(x + dt * k3, u)
    return x + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def chain_end_effector(x, task):
    n = x.shape[-1] // 2
    return chain_positions(x[..., :n], np.asarray(task.lengths, np.float64))[..., -1, :]


def chain_cost(task, x_next, u):
    pe = chain_end_effector(x_next, task)
    tgt = np.asarray(task.target, dtype=np.float64)
    c = float(task.goal_weight) * np.sum((pe - tgt) ** 2, axis=-1)
    return c + float(task.ctrl_weight) * np.sum(np.asarray(u, np.float64) ** 2, axis=-1)


def chain_energy(x, task, masses):
    """Kinetic + potential energy of the chain (no contact), for invariant tests."""
    n = x.shape[-1] // 2
    phi, dphi = x[..., :n], x[..., n:]
    lengths = np.asarray(task.lengths, np.float64)
    v = chain_velocities(phi, dphi, lengths)
    p = chain_positions(phi, lengths)
    ke = 0.5 * np.sum(masses * np.sum(v ** 2, axis=-1), axis=-1)
    pe = float(task.gravity) * np.sum(masses * p[..., 1], axis=-1)
    return ke + pe


# ------------------------------------------------------------- model dispatch

class Model:
    """f(x, u) and c(x', u) for one configuration, vectorised over samples.

    `sample_index` selects rows of the per-sample domain-randomisation table
    (link masses, friction) for the contact chain."""

    def __init__(self, cfg, sample_index=None, dtype=np.float64):
        self.cfg = cfg
        self.dtype = dtype
        self.dt = float(cfg.dt)
        self.task = cfg.task
        if cfg.dynamics == W.POINT_MASS:
            return
        self.contact = cfg.dynamics == W.CHAIN_CONTACT
        n = cfg.n_links
        if self.contact:
            sp = np.asarray(cfg.sample_params, dtype=dtype)
            if sample_index is not None:
                sp = sp[np.asarray(sample_index)]
            self.masses = sp[:, :n]
            self.mu_f = sp[:, n]
        else:
            self.masses = np.asarray(cfg.task.masses, dtype=dtype)
            self.mu_f = None

    def step(self, x, u):
        if self.cfg.dynamics == W.POINT_MASS:
            return point_mass_step(x, u, self.dt)
        f = lambda xx, uu: chain_accel(xx, uu, self.task, self.masses, self.mu_f, self.contact, self.dtype)
        return rk4_step(f, x, u, self.dtype(self.cfg.dt))

    def cost(self, x_next, u):
        if self.cfg.dynamics == W.POINT_MASS:
            return point_mass_cost(self.task, x_next, u)
        return chain_cost(self.task, x_next, u)
