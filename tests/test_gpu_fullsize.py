"""Parity at the benchmark sizes, in the launch configuration the benchmark
times (graph replay of whole replans), on outputs the oracle can compute one
by one: the full graph and path indices, a sample of candidate trajectories
and rollouts, the exact elite selection on the GPU's own costs, and the refit
from the GPU's candidates."""
import numpy as np
import pytest

import mtp_workloads as W
from oracle import planner as OP, sampling as OS, interp as OI
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu

SAMPLE = 48


def _log(msg):
    print(msg, flush=True)


def sampled_rows(cfg, rng):
    """Candidate indices to check: the nominal, some local samples, some tensor paths."""
    G1 = cfg.n_gauss - 1
    loc = rng.choice(G1, size=min(8, G1), replace=False) if G1 > 0 else np.array([], int)
    ten = G1 + rng.choice(cfg.n_tensor, size=min(SAMPLE - 9, cfg.n_tensor), replace=False)
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


def check_fullsize(cfg, label):
    import torch
    import paper_2505_01059_amd as mtp
    rng = np.random.default_rng(0)
    x0 = W.initial_state(cfg)
    plan = mtp.Plan(cfg, device="cuda:0")
    # one full replan from the graph, as the benchmark runs it (shift 1, replan 0)
    plan.replan(x0, shift=1, replan_idx=0)
    torch.cuda.synchronize()
    mu_end = plan.buffers()["mu"].cpu().numpy().copy()
    # then re-run the last iteration stage by stage from the state before it
    r, k = 0, cfg.n_iters - 1
    mu_in = np.random.default_rng(1).uniform(-0.3, 0.3, (cfg.horizon, cfg.ctrl_dim)).astype(np.float32) * float(cfg.u_max)
    sg_in = np.full((cfg.horizon, cfg.ctrl_dim), 0.3 * float(cfg.u_max), np.float32)
    plan.set_state(mu_in, sg_in, r)
    plan.set_x0(x0)
    plan.run_stage(4, r, k)
    torch.cuda.synchronize()
    b = plan.buffers()
    _log(f"[{label}] B={cfg.n_samples} T={cfg.horizon} n={cfg.ctrl_dim}")
    Z_ref = OS.waypoints(cfg.seed, r, k, cfg.n_layers, cfg.n_width, cfg.ctrl_dim, cfg.u_min, cfg.u_max)
    I_ref = OS.path_indices(cfg.seed, r, k, cfg.n_tensor, cfg.n_layers, cfg.n_width)
    assert np.array_equal(b["Z"].cpu().numpy(), Z_ref)
    assert np.array_equal(b["I"].cpu().numpy().T.astype(np.int64), I_ref)
    rows = sampled_rows(cfg, rng)
    rows_t = torch.as_tensor(rows, device=b["U"].device)
    U_rows = b["U"].index_select(2, rows_t).cpu().numpy().transpose(2, 0, 1).astype(np.float64)
    U_ref = oracle_candidates_rows(cfg, mu_in.astype(np.float64), sg_in.astype(np.float64), r, k, rows, Z_ref, I_ref)
    ill = H.akima_ill_conditioned(cfg, I_ref, Z_ref)
    G1 = cfg.n_gauss - 1
    skip = np.array([G1 <= x < G1 + cfg.n_tensor and ill[x - G1] for x in rows])
    ok = H.u_close(U_rows, U_ref, cfg.u_max).all(axis=(1, 2)) | skip
    assert ok.all(), f"candidate rows differ: {rows[~ok]}"
    # rollout of the sampled candidates from the GPU's own controls
    s = b["cost"].cpu().numpy()
    s_ref = OP.rollout(cfg, x0, U_rows, sample_index=rows if cfg.sample_params is not None else None)
    Usub = U_rows
    flag_cfg = cfg
    if cfg.sample_params is not None:
        flag_cfg = cfg.replace(sample_params=cfg.sample_params[rows])
    flagged = H.switching_flags(flag_cfg, x0, Usub) | skip
    bad = H.cost_check(s[rows], s_ref, flagged)
    rel = np.abs(s[rows] - s_ref) / np.maximum(np.abs(s_ref), 1e-12)
    _log(f"  sampled cost rel err max {rel[~flagged].max() if (~flagged).any() else 0:.2e}, flagged {flagged.sum()}")
    H.assert_costs(cfg, s[rows], s_ref, flagged)
    # elite selection on the GPU's costs: bit-exact
    iE = b["elite_idx"].cpu().numpy()
    assert np.array_equal(iE, OP.top_elites(s.astype(np.float64), cfg.n_elites))
    # refit from the GPU's elite candidates and costs
    iE_t = torch.as_tensor(iE.astype(np.int64), device=b["U"].device)
    Ue = b["U"].index_select(2, iE_t).cpu().numpy().transpose(2, 0, 1).astype(np.float64)
    U_sparse = np.zeros((cfg.n_samples, cfg.horizon, cfg.ctrl_dim))
    U_sparse[iE] = Ue
    mu2, sg2, _ = OP.refit(U_sparse, s.astype(np.float64), iE, mu_in.astype(np.float64), sg_in.astype(np.float64), cfg)
    assert H.refit_close(b["mu"].cpu().numpy(), mu2, cfg).all()
    assert H.refit_close(b["sigma"].cpu().numpy(), sg2, cfg).all()
    assert np.all(np.isfinite(mu_end))
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
