"""Parity rules for the contact chain (float32 HIP rollout vs the float64 oracle).

The penalty contact (reading A22: F_n = max(0, k (y_g - y) - d vy) for a mass
below the ground, F_t = -mu_f F_n tanh(vx / v_slip)) makes the rollout of the
chain sensitive in two ways that a plain "every state within 1e-4" rule cannot
survive, and the rules below treat them separately instead of loosening the
tolerance:

* Onset switch.  At the ground crossing of a mass moving down the normal force
  jumps from 0 to -d vy.  When an RK4 stage state of a step puts a mass within
  ONSET_MARGIN of the ground, float32 and float64 may take opposite sides of
  the switch and the step differs by the jump.  Such steps are flagged,
  counted and bounded.
* Stiffness after contact.  With k = 1e4 and v_slip = 0.01 the friction slope
  mu_f F_n / v_slip reaches 1e5..1e6 N s/m, so the step map amplifies float32
  rounding of the stage states, and free-running float32 and float64
  trajectories part after contact (the float32 drift test on the CPU shows it
  with the oracle's own formulas in both precisions).

The rules:

1. Cost bookkeeping: the GPU cost equals the float64 sum of the per-step costs
   of the GPU's own recorded states (mean over the R randomised models) within
   COST_SUM_TOL.
2. Before contact: free-running states within 1e-4 max(1, |x|_inf) and the
   cost of the steps so far within 1e-4, for every step before the candidate's
   first contact (a stage of the float64 trajectory within CONTACT_MARGIN of
   the ground) and before the horizon cut of the workload.
3. A candidate that never comes near the ground within the horizon is
   unflagged: its whole cost within 1e-4.
4. After contact: one step from the GPU's own state against the float64 step
   from the same state, within max(STEP_FLOOR, 2 n * spread) of the state's
   scale, where spread is the largest deviation of float64 steps whose stage
   states and stage derivatives are perturbed at float32 resolution (2 n: a
   float32 evaluation rounds along recurrences over the n links, the spread
   perturbs once).  Steps on the onset switch are excluded and counted.
"""
import numpy as np

from oracle import dynamics as OD, planner as OP

S_TOL = 1e-4                 # spec cost / state tolerance
COST_SUM_TOL = 1e-5          # GPU cost vs float64 sum over its own states
CONTACT_MARGIN = 1e-3        # metres above the ground that count as contact for rule 2
ONSET_MARGIN = 1e-5          # metres: a stage this close to the ground sits on the onset switch
STEP_FLOOR = 1e-5            # smallest one-step tolerance, relative to max(1, |x|_inf)
FREE_RUN_CUT = 128           # steps of free-running state parity from a contact-free start (drift test)
SPREAD_SAMPLES = 6
F32_EPS = 2.0 ** -24


def _lengths(cfg):
    return np.asarray(cfg.task.lengths, np.float64)


def node_heights(cfg, X):
    """y of every mass; X (..., 2n) -> (..., n)."""
    n = cfg.n_links
    return OD.chain_positions(np.asarray(X, np.float64)[..., :n], _lengths(cfg))[..., 1]


def _accel(model, u):
    return lambda xx: OD.chain_accel(xx, u, model.task, model.masses, model.mu_f, True)


def stage_states(model, x, u):
    """The four RK4 stage states of the float64 step from x (Alg. 2 rollout, RK4 as in the oracle)."""
    f = _accel(model, u)
    dt = float(model.cfg.dt)
    k1 = f(x)
    x2 = x + 0.5 * dt * k1
    k2 = f(x2)
    x3 = x + 0.5 * dt * k2
    k3 = f(x3)
    x4 = x + dt * k3
    return (x, x2, x3, x4)


def ground_gap(model, x, u):
    """min over masses and RK4 stages of y - y_g (negative: below the ground); (B,)."""
    cfg = model.cfg
    yg = float(cfg.task.ground_y)
    g = np.full(x.shape[0], np.inf)
    for s in stage_states(model, x, u):
        g = np.minimum(g, np.min(node_heights(cfg, s) - yg, axis=-1))
    return g


def onset_distance(model, x, u):
    """min over masses and RK4 stages of |y - y_g|; (B,)."""
    cfg = model.cfg
    yg = float(cfg.task.ground_y)
    g = np.full(x.shape[0], np.inf)
    for s in stage_states(model, x, u):
        g = np.minimum(g, np.min(np.abs(node_heights(cfg, s) - yg), axis=-1))
    return g


def perturbed_step(model, x, u, rng):
    """A float64 RK4 step whose stage states and stage derivatives carry random
    relative perturbations of float32 size."""
    f = _accel(model, u)
    dt = float(model.cfg.dt)

    def r(a):
        return a * (1.0 + F32_EPS * rng.uniform(-1.0, 1.0, size=a.shape))

    x = r(x)
    k1 = r(f(x))
    k2 = r(f(r(x + 0.5 * dt * k1)))
    k3 = r(f(r(x + 0.5 * dt * k2)))
    k4 = r(f(r(x + dt * k3)))
    return x + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def scale_of(x):
    return np.maximum(1.0, np.max(np.abs(x), axis=-1))


def reference_trajectories(cfg, x0, U, idx):
    """float64 free-running states of every randomised model: (R, B, T, d), and costs (B,)."""
    R = int(getattr(cfg, "n_replicas", 1))
    B = cfg.n_samples
    Xs = []
    s = np.zeros(len(idx))
    for r in range(R):
        sr, X = OP.rollout(cfg.replace(n_replicas=1), x0, U, r * B + np.asarray(idx), keep_states=True)
        Xs.append(X)
        s = s + sr
    s = s / R
    return np.where(np.isfinite(s), s, np.inf), np.stack(Xs)


def first_contact(cfg, x0, U, idx, X_ref):
    """First step t whose float64 step (any stage, any randomised model) comes
    within CONTACT_MARGIN of the ground; T if none.  (B,) int."""
    R, Bn, T, _ = X_ref.shape
    B = cfg.n_samples
    out = np.full(Bn, T)
    for r in range(R):
        model = OD.Model(cfg, r * B + np.asarray(idx))
        xprev = np.broadcast_to(np.asarray(x0, np.float64), (Bn, len(x0))).copy()
        for t in range(T):
            hit = (ground_gap(model, xprev, U[:, t]) < CONTACT_MARGIN) & (out > t)
            out[hit] = t
            xprev = X_ref[r, :, t]
    return out


def _reference_chunk(args):
    cfg, x0, U, idx = args
    s, X = reference_trajectories(cfg, x0, U, idx)
    return s, X, first_contact(cfg, x0, U, idx, X)


def reference_and_contact(cfg, x0, U, idx, workers=1):
    """reference_trajectories and first_contact of candidates idx, split over
    `workers` CPU processes (spawned, so they never touch the GPU)."""
    idx = np.asarray(idx)
    if workers <= 1 or len(idx) < 2 * workers:
        return _reference_chunk((cfg, x0, U, idx))
    import concurrent.futures as cf
    import multiprocessing as mp
    parts = np.array_split(np.arange(len(idx)), workers)
    jobs = [(cfg, x0, U[p], idx[p]) for p in parts]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        outs = list(ex.map(_reference_chunk, jobs))
    return (np.concatenate([o[0] for o in outs]), np.concatenate([o[1] for o in outs], axis=1),
            np.concatenate([o[2] for o in outs]))


def cost_from_states(cfg, X, U):
    """float64 cost sums of recorded states (R, B, T, d) with controls U (B, T, n): per-step (B, T)."""
    R = X.shape[0]
    S = np.zeros(X.shape[1:3])
    for r in range(R):
        for t in range(X.shape[2]):
            S[:, t] += OD.chain_cost(cfg.task, X[r, :, t], U[:, t])
    return S / R


def one_step_check(cfg, x0, U, X_gpu, idx, t_from, rng):
    """Rule 4 over the recorded candidates: for every step t >= t_from[b] the
    float64 step from the GPU's state x_t (x0 at t = 0) against the GPU's
    x_{t+1}.  Returns (errors, tolerances, onset mask, checked mask), each (R, B, T)."""
    R, Bn, T, _ = X_gpu.shape
    B = cfg.n_samples
    K = 2.0 * cfg.n_links
    err = np.zeros((R, Bn, T))
    tol = np.zeros((R, Bn, T))
    onset = np.zeros((R, Bn, T), bool)
    checked = np.zeros((R, Bn, T), bool)
    for r in range(R):
        for t in range(T):
            live = t >= t_from
            if not live.any():
                continue
            xprev = (np.broadcast_to(np.asarray(x0, np.float64), (Bn, len(x0))) if t == 0
                     else X_gpu[r, :, t - 1])
            sub = OD.Model(cfg, r * B + np.asarray(idx)[live])
            xs, us = xprev[live], U[live, t]
            x1 = sub.step(xs, us)
            sc = scale_of(x1)
            spread = np.zeros(len(xs))
            for _ in range(SPREAD_SAMPLES):
                spread = np.maximum(spread, np.max(np.abs(perturbed_step(sub, xs, us, rng) - x1), axis=-1) / sc)
            err[r, live, t] = np.max(np.abs(X_gpu[r, live, t] - x1), axis=-1) / sc
            tol[r, live, t] = np.maximum(STEP_FLOOR, K * spread)
            onset[r, live, t] = onset_distance(sub, xs, us) < ONSET_MARGIN
            checked[r, live, t] = True
    return err, tol, onset, checked
