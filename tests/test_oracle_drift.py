"""Float32 drift of the contact chain against float64, on the CPU.

The parity protocol compares a float32 rollout with the float64 oracle; for
the chain with penalty ground contact (reading A22) that comparison only makes
sense where float32 rounding has not yet been amplified beyond the tolerance.
These tests measure the amplification with the oracle's own formulas run in
float32 and in float64 (nothing of the HIP path is involved) and fix the
horizon cuts used by the GPU parity checks:

* from the 24-link workload's canonical start (horizontal, at rest, ground
  4 m below the base) the chain falls freely for well over 128 steps, and over
  those steps float32 stays within a quarter of the 1e-4 state tolerance, so
  128 steps is the free-running horizon cut of that workload;
* once masses reach the ground the stiff friction (mu_f F_n / v_slip up to
  1e6 N s/m) amplifies rounding, and free-running float32 states part from
  float64 by more than the tolerance: past first contact only the one-step
  rule of tests/contact_parity.py is meaningful, and a float32 evaluation of
  the oracle's step satisfies that rule.
"""
import numpy as np
import pytest

import mtp_workloads as W
from oracle import dynamics as OD, interp as OI
from tests import contact_parity as CP

T_CUT_C4 = 128          # free-running horizon cut of the 24-link contact workload (steps)


def _controls(cfg, n, seed):
    """Half smooth tensor-path-like controls (cubic B-spline through random
    waypoints), half local-sample-like noise around zero at sigma_init, clipped."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(float(cfg.u_min), float(cfg.u_max), size=(n // 2, cfg.n_layers, cfg.ctrl_dim))
    smooth = OI.bspline_interp(C, 3, cfg.horizon)
    noise = rng.normal(0.0, float(cfg.sigma_init), size=(n - n // 2, cfg.horizon, cfg.ctrl_dim))
    U = np.concatenate([smooth, noise], axis=0)
    return np.clip(U, float(cfg.u_min), float(cfg.u_max)).astype(np.float32).astype(np.float64)


def _states(cfg, x0, U, idx, dtype):
    model = OD.Model(cfg, idx, dtype=dtype)
    x = np.broadcast_to(np.asarray(x0, dtype), (len(idx), len(x0))).copy()
    X = []
    for t in range(U.shape[1]):
        x = model.step(x, U[:, t].astype(dtype))
        assert x.dtype == dtype
        X.append(x.astype(np.float64))
    return np.stack(X, axis=1)


def _drift(X32, X64):
    """|x32 - x64|_inf / max(1, |x64|_inf) per candidate and step."""
    return np.max(np.abs(X32 - X64), axis=-1) / CP.scale_of(X64)


def _report(name, e, t_c):
    print(f"[drift] {name}: first contact steps {np.sort(t_c)}")
    for t in range(0, e.shape[1], max(1, e.shape[1] // 8)):
        print(f"[drift]   t={t:4d}  max {e[:, t].max():.2e}  median {np.median(e[:, t]):.2e}")


def test_float32_drift_24_link_canonical_start():
    cfg = W.c4()
    x0 = W.initial_state(cfg)
    idx = np.arange(16)
    U = _controls(cfg, len(idx), 1)
    X64 = _states(cfg, x0, U, idx, np.float64)
    X32 = _states(cfg, x0, U, idx, np.float32)
    e = _drift(X32, X64)
    t_c = CP.first_contact(cfg, x0, U, idx, X64[None])
    _report("24 links, canonical start", e, t_c)
    assert t_c.min() > T_CUT_C4, "the chain is expected to fall freely past the horizon cut"
    assert e[:, :T_CUT_C4].max() <= 0.25 * CP.S_TOL, "float32 drift before the horizon cut"
    # past first contact the free-running comparison stops being meaningful
    post = np.array([e[b, t_c[b]:].max() if t_c[b] < cfg.horizon else 0.0 for b in range(len(idx))])
    assert post.max() > CP.S_TOL, "contact no longer amplifies float32 rounding: revisit the horizon cut"


@pytest.mark.parametrize("n_links, ground, horizon", [(7, -0.5, 100), (24, -2.0, 110)])
def test_float32_drift_after_contact_and_one_step_rule(n_links, ground, horizon):
    """A chain that falls onto a raised ground: float32 tracks float64 until
    first contact and parts from it after; every float32 step of the oracle
    from its own state meets the one-step rule (its onset-switch steps aside)."""
    cfg = W.chain_contact_config(name="drop", n_links=n_links, n_tensor=16, n_gauss=8, horizon=horizon,
                                 n_layers=6, n_width=8, n_elites=4, n_iters=1, ground_y=ground)
    x0 = W.initial_state(cfg, seed=7)
    idx = np.arange(cfg.n_samples)
    U = _controls(cfg, len(idx), 2)
    X64 = _states(cfg, x0, U, idx, np.float64)
    X32 = _states(cfg, x0, U, idx, np.float32)
    e = _drift(X32, X64)
    t_c = CP.first_contact(cfg, x0, U, idx, X64[None])
    _report(f"{n_links} links onto ground {ground}", e, t_c)
    assert np.all(t_c > 10) and np.all(t_c < horizon - 20), "every candidate should reach the ground mid-horizon"
    pre = np.array([e[b, :t_c[b]].max() for b in range(len(idx))])
    assert pre.max() <= 0.25 * CP.S_TOL
    post = np.array([e[b, t_c[b]:].max() for b in range(len(idx))])
    assert post.max() > CP.S_TOL
    err, tol, onset, checked = CP.one_step_check(cfg, x0, U, X32[None], idx, np.zeros(len(idx), int),
                                                 np.random.default_rng(0))
    bad = checked & ~onset & (err > tol)
    ratio = np.max(np.where(checked & ~onset, err / tol, 0.0))
    print(f"[drift]   one-step rule: {checked.sum()} steps, {onset.sum()} on the onset switch, "
          f"largest error / tolerance {ratio:.2f}")
    assert not bad.any(), f"{bad.sum()} float32 steps break the one-step rule"
