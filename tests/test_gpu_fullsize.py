"""Parity at the benchmark sizes, in the launch configuration the benchmark
times (graph replay of whole replans), on outputs the oracle can compute one
by one: the full graph and path indices of the last iteration, a sample of
candidate trajectories and rollouts (the contact chain: 1024 candidates with
their states), the exact elite selection on the GPU's own costs, and the
refit and action from the GPU's candidates, all teacher-forced from the mean
and std the same graph path reaches one iteration earlier."""
import numpy as np
import pytest

import mtp_workloads as W
from oracle import planner as OP, sampling as OS, interp as OI
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

SAMPLE = 256              # candidate rows checked per smooth workload
CONTACT_LOCAL = 512       # contact chain: the first 512 local samples, 511 tensor paths and the nominal
ONE_STEP_ROWS = 64        # rows of the contact subset that also take the one-step rule
WORKERS = 8               # CPU processes for the oracle's contact-chain rollouts


def _log(msg):
    print(msg, flush=True)


def sampled_rows(cfg, rng):
    """Candidate indices to check: the nominal, some local samples, some tensor paths."""
    G1 = cfg.n_gauss - 1
    if cfg.dynamics == W.CHAIN_CONTACT:
        loc = np.arange(min(CONTACT_LOCAL, G1))
        ten = G1 + np.sort(rng.choice(cfg.n_tensor, size=min(1023 - len(loc), cfg.n_tensor), replace=False))
    else:
        loc = rng.choice(G1, size=min(SAMPLE // 8, G1), replace=False) if G1 > 0 else np.array([], int)
        ten = G1 + rng.choice(cfg.n_tensor, size=min(SAMPLE - len(loc) - 1, cfg.n_tensor), replace=False)
    return np.unique(np.concatenate([loc, ten, [cfg.n_samples - 1]])).astype(int)


def oracle_candidates_rows(cfg, mu, sg, r, k, rows, Z, I):
    """Oracle controls for selected candidate rows only."""
    G1 = cfg.n_gauss - 1
    out = np.zeros((len(rows), cfg.horizon, cfg.ctrl_dim))
    eps = None
    for n_, b in enumerate(rows):
        if b < G1:
            if eps is None:
                eps = OP.gaussian_noise(cfg, r, k)
            u = mu + sg * eps[b]
        elif b < G1 + cfg.n_tensor:
            C = OS.gather(Z, I[b - G1:b - G1 + 1]).astype(np.float64)
            if cfg.interp == W.BSPLINE:
                u = OI.bspline_interp(C, cfg.bspline_degree, cfg.horizon)[0]
            else:
                u = OI.akima_interp(C, cfg.horizon)[0]
        else:
            u = mu
        out[n_] = np.clip(u, float(cfg.u_min), float(cfg.u_max))
    return out


def rows_of(t, rows, dim):
    import torch
    return t.index_select(dim, torch.as_tensor(rows, device=t.device)).cpu().numpy()


def check_fullsize(cfg, label):
    """One whole replan from the captured graph (the benchmark's path), then a
    teacher-forced check of its last iteration: the oracle re-runs iteration
    K-1 from the mean and std that the same graph path leaves after K-1
    iterations (a plan of the same config with one iteration fewer)."""
    import torch
    import paper_2505_01059_amd as mtp
    rng = np.random.default_rng(0)
    x0 = W.initial_state(cfg)
    contact = cfg.dynamics == W.CHAIN_CONTACT
    K = cfg.n_iters
    _log(f"[{label}] B={cfg.n_samples} T={cfg.horizon} n={cfg.ctrl_dim} K={K}")
    if K > 1:
        prev = mtp.Plan(cfg.replace(n_iters=K - 1), device="cuda:0")
        prev.replan(x0, shift=1, replan_idx=0)
        torch.cuda.synchronize()
        pb = prev.buffers()
        mu_in, sg_in = pb["mu"].cpu().numpy().astype(np.float64), pb["sigma"].cpu().numpy().astype(np.float64)
        prev.close()
        del prev, pb
    else:
        mu_in, sg_in = OP.shift_distribution(*OP.initial_distribution(cfg), 1, cfg.sigma_init)
    plan = mtp.Plan(cfg, device="cuda:0", n_debug_states=cfg.n_samples if contact else 0)
    plan.replan(x0, shift=1, replan_idx=0)
    torch.cuda.synchronize()
    assert plan.flags() & 6 == 0, "selection fault or segment wait time-out"
    b = plan.buffers()
    r, k = 0, K - 1
    Z_ref = OS.waypoints(cfg.seed, r, k, cfg.n_layers, cfg.n_width, cfg.ctrl_dim, cfg.u_min, cfg.u_max)
    I_ref = OS.path_indices(cfg.seed, r, k, cfg.n_tensor, cfg.n_layers, cfg.n_width)
    assert np.array_equal(b["Z"].cpu().numpy(), Z_ref)
    assert np.array_equal(b["I"].cpu().numpy().T.astype(np.int64), I_ref)
    rows = sampled_rows(cfg, rng)
    U_rows = rows_of(b["U"], rows, 2).transpose(2, 0, 1).astype(np.float64)
    U_ref = oracle_candidates_rows(cfg, mu_in, sg_in, r, k, rows, Z_ref, I_ref)
    ill = H.akima_excluded(cfg, H.akima_ill_conditioned(cfg, I_ref, Z_ref))
    G1 = cfg.n_gauss - 1
    skip = np.array([G1 <= x < G1 + cfg.n_tensor and ill[x - G1] for x in rows])
    ok = H.u_close(U_rows, U_ref, cfg.u_max).all(axis=(1, 2)) | skip
    assert ok.all(), f"candidate rows differ: {rows[~ok]}"
    # rollout of the sampled candidates from the GPU's own controls
    s = b["cost"].cpu().numpy()
    if contact:
        X_rows = rows_of(b["X_all"], rows, 3).transpose(0, 3, 1, 2).astype(np.float64)
        pos = np.sort(rng.choice(len(rows), ONE_STEP_ROWS, replace=False))
        H.chain_contact_parity(cfg, x0, U_rows, s[rows], X_rows, label, rows=rows, one_step_rows=pos,
                               workers=WORKERS)
    else:
        s_ref = OP.rollout(cfg, x0, U_rows)
        flagged = H.switching_flags(cfg, x0, U_rows) | skip
        rel = np.abs(s[rows] - s_ref) / np.maximum(np.abs(s_ref), 1e-12)
        _log(f"  sampled cost rel err max {rel[~flagged].max() if (~flagged).any() else 0:.2e}, "
             f"flagged {flagged.sum()}")
        H.assert_costs(cfg, s[rows], s_ref, flagged)
    # elite selection on the GPU's costs: bit-exact
    iE = b["elite_idx"].cpu().numpy()
    assert np.array_equal(iE, OP.top_elites(s.astype(np.float64), cfg.n_elites))
    # refit of the last iteration from the GPU's elite candidates and costs
    Ue = rows_of(b["U"], iE.astype(np.int64), 2).transpose(2, 0, 1).astype(np.float64)
    U_sparse = np.zeros((cfg.n_samples, cfg.horizon, cfg.ctrl_dim))
    U_sparse[iE] = Ue
    mu2, sg2, _ = OP.refit(U_sparse, s.astype(np.float64), iE, mu_in, sg_in, cfg)
    assert H.refit_close(b["mu"].cpu().numpy(), mu2, cfg).all()
    assert H.refit_close(b["sigma"].cpu().numpy(), sg2, cfg).all()
    # the action is the first control of the best candidate of the last iteration
    np.testing.assert_array_equal(plan.action(), Ue[0, 0].astype(np.float32))
    plan.close()


def test_chain7_akima_full():
    check_fullsize(W.c1(), "chain7 full")


def test_point_mass_full():
    check_fullsize(W.c0(), "point mass full")


def test_chain24_contact_full():
    check_fullsize(W.c4(), "chain24 contact full")


@pytest.mark.parametrize("contact", [False, True])
def test_time_sliced_rollout_equals_plain(contact):
    """Launches of more pair-lane waves than SIMDs run time-sliced (segments of
    the horizon taken from a counter, state saved between them); the batched
    kernel runs the same instance with plain whole-horizon tiles.  One replan of
    each must agree bit for bit, and no wait may time out."""
    import torch
    import paper_2505_01059_amd as mtp
    if contact:
        cfg = W.chain_contact_config(name="ts_contact", n_tensor=68000, n_gauss=2000, horizon=40,
                                     n_elites=64, n_iters=2, seed=3)
    else:
        cfg = W.chain_config(name="ts_chain24", n_links=24, interp=W.BSPLINE, n_tensor=68000, n_gauss=2000,
                             horizon=40, n_layers=12, n_width=64, n_elites=64, n_iters=2, seed=4)
    x0 = W.initial_state(cfg, seed=1)
    _log(f"[time-sliced] contact={contact} B={cfg.n_samples}")
    plan = mtp.Plan(cfg, device="cuda:0")
    plan.replan(x0, shift=1, replan_idx=0)
    torch.cuda.synchronize()
    assert plan.flags() & 4 == 0, "a segment wait timed out"
    b = plan.buffers()
    mu, sg, act = b["mu"].cpu().numpy().copy(), b["sigma"].cpu().numpy().copy(), plan.action()
    cost = b["cost"].cpu().numpy().copy()
    plan.close()
    bt = mtp.Batch([cfg], device="cuda:0")
    bt.replan(bt.pack_x0([x0]), shift=1)
    acts = bt.actions()
    bb = bt.buffers(0)
    assert np.array_equal(bb["cost"].cpu().numpy(), cost)
    assert np.array_equal(bb["mu"].cpu().numpy(), mu)
    assert np.array_equal(bb["sigma"].cpu().numpy(), sg)
    assert np.array_equal(acts[0], act)
    bt.close()
