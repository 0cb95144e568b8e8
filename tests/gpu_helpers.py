"""Shared helpers of the GPU parity tests: layout conversion and the parity rules.

Parity rules (float32 GPU vs float64 oracle on identical inputs):
  * Z, I, elite index sets: bit-exact (elites: exact whenever the oracle's gap
    at the elite boundary exceeds the float32 cost error, and always exact when
    the oracle's selection is applied to the GPU's own costs);
  * controls U: |a - b| <= 1e-4 * max(|b|, u_max);
  * costs s: |a - b| <= 1e-4 * |b| except candidates the oracle flags as sitting
    on a switching surface (obstacle boundary, ill-conditioned Akima weights,
    at most 1% of the tensor paths), which are counted and reported; contact
    chains that reach the ground follow chain_contact_parity (tests/contact_parity.py);
  * elite sets against the float64 costs: equal once the flagged candidates
    and those within twice the largest observed cost error of either elite
    boundary are left out;
  * mean / std refit from identical candidates and costs: 1e-4 relative to
    max(|b|, 1e-3 * (u_max - u_min)).
"""
import numpy as np
import torch

from oracle import planner as OP, interp as OI, dynamics as OD
from tests import contact_parity as CP

U_TOL = 1e-4
S_TOL = 1e-4


def to_oracle_U(U_dev):
    """device view (T, n, B) -> (B, T, n) float64."""
    return U_dev.detach().cpu().numpy().transpose(2, 0, 1).astype(np.float64)


def write_U(bufs, U_bt_n):
    U32 = np.ascontiguousarray(np.asarray(U_bt_n, np.float32).transpose(1, 2, 0))
    bufs["U"].copy_(torch.from_numpy(U32).to(bufs["U"].device))


def u_close(a, b, u_max):
    return np.abs(a - b) <= U_TOL * np.maximum(np.abs(b), float(u_max))


def akima_ill_conditioned(cfg, I, Z):
    """Tensor paths whose Akima slope weights nearly vanish (float32 cannot resolve
    the weighted mean there).  Returns a bool mask over tensor paths."""
    if cfg.interp != 1 or cfg.n_tensor == 0 or cfg.n_layers < 5:
        return np.zeros(cfg.n_tensor, bool)
    C = Z[np.arange(cfg.n_layers)[None, :], I, :].astype(np.float64)      # (P, L, n)
    m = np.diff(C, axis=1)
    L = cfg.n_layers
    scale = np.max(np.abs(m), axis=1, keepdims=True) + 1e-30
    bad = np.zeros(C.shape[0], bool)
    for i in range(2, L - 2):
        den = np.abs(m[:, i + 1] - m[:, i]) + np.abs(m[:, i - 1] - m[:, i - 2])
        bad |= np.any(den < 1e-4 * scale[:, 0], axis=-1)
    return bad


def switching_flags(cfg, x0, U, margin=1e-5):
    """Candidates whose float64 rollout sits on a switching surface the cost
    tolerance cannot cover: a point-mass trajectory within `margin` of an
    obstacle boundary (the penalty indicator), or a contact-chain trajectory
    that comes near the ground at all within the horizon (contact is checked
    by chain_contact_parity instead)."""
    B = U.shape[0]
    if cfg.dynamics == 0:
        s, X = OP.rollout(cfg, x0, U, keep_states=True)
        m = OD.point_mass_obstacle_margin(cfg.task, X)                    # (B, T)
        return np.min(m, axis=1) < margin
    if cfg.dynamics == 2:
        idx = np.arange(B)
        _, X = CP.reference_trajectories(cfg, x0, U, idx)
        return CP.first_contact(cfg, x0, U, idx, X) < cfg.horizon
    return np.zeros(B, bool)


def cost_check(s_gpu, s_ref, flagged):
    s_gpu = np.asarray(s_gpu, np.float64)
    ok = np.abs(s_gpu - s_ref) <= S_TOL * np.abs(s_ref) + 1e-6
    both_inf = np.isinf(s_gpu) & np.isinf(s_ref)
    ok |= both_inf
    bad = ~ok & ~flagged
    return bad


def assert_costs(cfg, s_gpu, s_ref, flagged):
    """Cost parity: every unflagged candidate within S_TOL, whatever the model."""
    bad = cost_check(s_gpu, s_ref, flagged)
    assert not bad.any(), f"{bad.sum()} costs out of tolerance at {np.flatnonzero(bad)[:10]}"


def akima_excluded(cfg, ill):
    """Akima paths left out of the control check; at most 1% of the tensor paths (and 2)."""
    cap = max(2, cfg.n_tensor // 100)
    assert ill.sum() <= cap, f"{ill.sum()} ill-conditioned Akima paths excluded (cap {cap})"
    return ill


def chain_contact_parity(cfg, x0, U, s_gpu, X_gpu, label, rows=None, one_step_rows=None, seed=0, workers=1):
    """The contact-chain rules (tests/contact_parity.py) on the candidates `rows`
    (default 0..nb-1).

    U (nb, T, n) float64 of the GPU's float32 controls of those candidates,
    s_gpu (nb,) their GPU costs, X_gpu (R, nb, T, d) their recorded states;
    one_step_rows picks positions (into rows) for the one-step rule.  Returns
    the mask of candidates whose whole cost is not compared free-running
    (contact within the horizon, or a horizon beyond the free-running cut)."""
    nb, T = U.shape[0], U.shape[1]
    idx = np.arange(nb) if rows is None else np.asarray(rows)
    s_gpu = np.asarray(s_gpu, np.float64)
    s_ref, X_ref, t_c = CP.reference_and_contact(cfg, x0, U, idx, workers)
    cut = np.minimum(t_c, min(T, CP.FREE_RUN_CUT))
    # rule 1: the GPU's cost is the sum of its own states' step costs
    S_g = CP.cost_from_states(cfg, X_gpu, U)
    e1 = np.abs(S_g.sum(axis=1) - s_gpu) / np.maximum(np.abs(s_gpu), 1e-6)
    assert np.all(e1 <= CP.COST_SUM_TOL), f"[{label}] GPU cost != sum over its states ({e1.max():.2e})"
    # rule 2: free-running states and cost prefix before contact and the horizon cut
    S_r = CP.cost_from_states(cfg, X_ref, U)
    err_t = np.zeros((nb, T))
    for r in range(X_gpu.shape[0]):
        e = np.max(np.abs(X_gpu[r] - X_ref[r]), axis=-1) / CP.scale_of(X_ref[r])
        err_t = np.maximum(err_t, e)
    before = np.arange(T)[None, :] < cut[:, None]
    worst = np.max(np.where(before, err_t, 0.0))
    assert worst <= CP.S_TOL, f"[{label}] state error {worst:.2e} before contact / horizon cut"
    Pg = np.where(before, S_g, 0.0).sum(axis=1)
    Pr = np.where(before, S_r, 0.0).sum(axis=1)
    ep = np.abs(Pg - Pr) / np.maximum(np.abs(Pr), 1e-6)
    assert np.all(ep <= CP.S_TOL), f"[{label}] cost before contact off by {ep.max():.2e}"
    # rule 3: candidates that stay clear of the ground within a horizon below the cut
    free = cut >= T
    cost_rel = np.abs(s_gpu - s_ref) / np.maximum(np.abs(s_ref), 1e-12)
    assert np.all(cost_rel[free] <= CP.S_TOL), f"[{label}] contact-free cost off by {cost_rel[free].max():.2e}"
    # rule 4: one step from the GPU's own state once free running stops
    pos = np.arange(nb) if one_step_rows is None else np.asarray(one_step_rows)
    pos = pos[cut[pos] < T]
    n_onset = n_steps = 0
    ratio = 0.0
    if len(pos):
        err, tol, onset, checked = CP.one_step_check(cfg, x0, U[pos], X_gpu[:, pos], idx[pos], cut[pos],
                                                     np.random.default_rng(seed))
        bad = checked & ~onset & (err > tol)
        n_onset, n_steps = int(onset.sum()), int(checked.sum())
        ratio = float(np.max(np.where(checked & ~onset, err / tol, 0.0)))
        assert not bad.any(), (f"[{label}] {bad.sum()} steps from the GPU's own states break the one-step "
                               f"rule (worst error / tolerance {ratio:.1f})")
        assert n_onset <= max(2, 0.02 * n_steps), f"[{label}] {n_onset} of {n_steps} steps on the onset switch"
    # report: free-running error against t (it is not asserted past the cut)
    marks = sorted(set(np.linspace(0, T - 1, 9).astype(int)))
    print(f"[{label}] contact chain: {int((t_c < T).sum())}/{nb} candidates reach the ground "
          f"(first at step {int(t_c.min())}); state error before the cut {worst:.2e}; "
          f"cost from own states {e1.max():.2e}; one-step rule {n_steps} steps, {n_onset} onset, "
          f"worst error/tolerance {ratio:.2f}", flush=True)
    print(f"[{label}]   free-running state error vs t: " +
          " ".join(f"t{t}:{err_t[:, t].max():.1e}" for t in marks) +
          f"; whole-cost error max {cost_rel.max():.1e}, >1e-4: {int((cost_rel > CP.S_TOL).sum())}", flush=True)
    return ~free


def elite_sets_agree(iE_gpu, s_gpu, s_ref, flagged, E):
    """Alg. 2 top-E against the oracle's float64 costs.  With delta the largest
    cost difference over the unflagged candidates (each already within 1e-4),
    an unflagged candidate whose oracle cost lies more than 2 delta below (or
    above) both elite boundaries, the GPU's and the oracle's, is an elite (or
    not) on both sides.  So: leave out the flagged candidates and those inside
    that band, and the two elite sets must be equal.  Returns the number of
    distinct oracle costs among the unflagged candidates left out by the band."""
    s_gpu = np.asarray(s_gpu, np.float64)
    s_ref = np.where(np.isnan(s_ref), np.inf, s_ref)
    flagged = np.asarray(flagged, bool)
    iE_ref = OP.top_elites(s_ref, E)
    if E >= len(s_ref):
        assert set(iE_gpu) == set(iE_ref)
        return 0
    unf = ~flagged & np.isfinite(s_ref) & np.isfinite(s_gpu)
    delta = float(np.max(np.abs(s_gpu - s_ref)[unf])) if unf.any() else 0.0
    thr = [float(s_ref[iE_ref[-1]]), float(s_gpu[iE_gpu[-1]])]
    lo, hi = min(thr), max(thr)
    band = (s_ref >= lo - 2 * delta) & (s_ref <= hi + 2 * delta)
    drop = flagged | band
    a = {int(b) for b in iE_gpu if not drop[b]}
    b_ = {int(b) for b in iE_ref if not drop[b]}
    assert a == b_, f"elite sets differ outside the boundary band: {sorted(a ^ b_)[:10]}"
    # exact ties (identical candidates, e.g. duplicated paths) count once
    return int(np.unique(s_ref[band & ~flagged]).size)


def refit_close(a, b, cfg):
    scale = np.maximum(np.abs(b), 1e-3 * float(cfg.u_max - cfg.u_min))
    return np.abs(a - b) <= 1e-4 * scale


def check_iteration(cfg, b, x0, mu, sg, r, k, label, X_all=None):
    """One CEM iteration (Alg. 2 loop body) that ran on the GPU, against the
    oracle's same iteration from the same mean and std (teacher forcing):
    graph and path indices bit-exact, candidates within U_TOL, costs by the
    rules above (contact chains from the recorded states X_all, (R, B, T, d)),
    the oracle's top-E on the GPU's costs bit-exact and elite sets against the
    oracle's costs, the refit from the GPU's elites and the action.  `b` holds
    the iteration's buffers as numpy arrays or torch views.  Returns the number
    of distinct costs left out at the elite boundary."""
    def np_(v):
        return v.cpu().numpy() if hasattr(v, "cpu") else np.asarray(v)
    mu = np.asarray(mu, np.float64)
    sg = np.asarray(sg, np.float64)
    ref = OP.iterate(cfg, x0, mu, sg, r, k)
    if cfg.n_tensor > 0:
        assert np.array_equal(np_(b["Z"]), ref["Z"]), f"[{label}] graph waypoints"
        assert np.array_equal(np_(b["I"]).T.astype(np.int64), ref["I"]), f"[{label}] path indices"
    U = to_oracle_U(b["U"]) if hasattr(b["U"], "cpu") else np.asarray(b["U"], np.float64)
    ill = akima_excluded(cfg, akima_ill_conditioned(cfg, ref["I"], ref["Z"]))
    G1 = cfg.n_gauss - 1
    rows_bad = ~np.all(u_close(U, ref["U"], cfg.u_max), axis=(1, 2))
    rows_bad[G1:G1 + cfg.n_tensor] &= ~ill
    assert not rows_bad.any(), f"[{label}] {rows_bad.sum()} candidates differ"
    s = np_(b["cost"]).astype(np.float64)
    iE = np_(b["elite_idx"])
    if cfg.dynamics == 2:
        assert X_all is not None, "contact chains are checked from their recorded states"
        flagged = chain_contact_parity(cfg, x0, U, s, X_all, label)
    else:
        flagged = switching_flags(cfg, x0, ref["U"])
    flagged[G1:G1 + cfg.n_tensor] |= ill
    assert_costs(cfg, s, ref["s"], flagged)
    assert np.array_equal(iE, OP.top_elites(s, cfg.n_elites)), f"[{label}] elites on the GPU's costs"
    band = elite_sets_agree(iE, s, ref["s"], flagged, cfg.n_elites)
    assert band <= max(4, cfg.n_elites // 4), f"[{label}] {band} costs within the elite boundary band"
    mu2, sg2, _ = OP.refit(ref["U"], s, iE, mu, sg, cfg)
    assert refit_close(np_(b["mu"]), mu2, cfg).all(), f"[{label}] refit mean"
    assert refit_close(np_(b["sigma"]), sg2, cfg).all(), f"[{label}] refit std"
    np.testing.assert_array_equal(np_(b["action"]), U[iE[0], 0].astype(np.float32), err_msg=f"[{label}] action")
    print(f"[{label}] flagged {int(flagged.sum())}, elite boundary band {band}", flush=True)
    return band
