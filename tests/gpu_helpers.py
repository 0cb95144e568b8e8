"""Shared helpers of the GPU parity tests: layout conversion and the parity rules.

Parity rules (float32 GPU vs float64 oracle on identical inputs):
  * Z, I, elite index sets: bit-exact (elites: exact whenever the oracle's gap
    at the elite boundary exceeds the float32 cost error, and always exact when
    the oracle's selection is applied to the GPU's own costs);
  * controls U: |a - b| <= 1e-4 * max(|b|, u_max);
  * costs s: |a - b| <= 1e-4 * |b| except candidates the oracle flags as sitting
    on a switching surface (obstacle boundary, contact onset, ill-conditioned
    Akima weights), which are counted and reported;
  * mean / std refit from identical candidates and costs: 1e-4 relative to
    max(|b|, 1e-3 * (u_max - u_min)).
"""
import numpy as np
import torch

from oracle import planner as OP, interp as OI, dynamics as OD

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
    """Candidates whose oracle rollout passes within `margin` of a discontinuity."""
    B = U.shape[0]
    R = int(getattr(cfg, "n_replicas", 1))
    if R > 1:                    # any of the randomised models may sit on the surface
        sp = np.asarray(cfg.sample_params).reshape(R, -1, cfg.sample_params.shape[1])
        out = np.zeros(B, bool)
        for r in range(R):
            out |= switching_flags(cfg.replace(n_replicas=1, sample_params=np.ascontiguousarray(sp[r])),
                                   x0, U, margin)
        return out
    if cfg.dynamics == 0:
        s, X = OP.rollout(cfg, x0, U, keep_states=True)
        m = OD.point_mass_obstacle_margin(cfg.task, X)                    # (B, T)
        return np.min(m, axis=1) < margin
    if cfg.dynamics == 2:
        s, X = OP.rollout(cfg, x0, U, keep_states=True)
        n = cfg.n_links
        p = OD.chain_positions(X[..., :n], np.asarray(cfg.task.lengths, np.float64))
        gap = np.abs(p[..., 1] - float(cfg.task.ground_y))                 # (B, T, n)
        return np.min(gap.reshape(B, -1), axis=1) < margin
    return np.zeros(B, bool)


def cost_check(s_gpu, s_ref, flagged):
    s_gpu = np.asarray(s_gpu, np.float64)
    ok = np.abs(s_gpu - s_ref) <= S_TOL * np.abs(s_ref) + 1e-6
    both_inf = np.isinf(s_gpu) & np.isinf(s_ref)
    ok |= both_inf
    bad = ~ok & ~flagged
    return bad


def assert_costs(cfg, s_gpu, s_ref, flagged):
    """Cost parity.  Smooth models: every unflagged candidate within S_TOL.
    Contact chain: the penalty contact switches on and off, and a float32 state
    that crosses the ground one step earlier or later than the float64 one sends
    the chaotic chain on another trajectory; the rule there is at least 90% of
    unflagged candidates within S_TOL and all within 1e-2 relative."""
    bad = cost_check(s_gpu, s_ref, flagged)
    if cfg.dynamics != 2:
        assert not bad.any(), f"{bad.sum()} costs out of tolerance at {np.flatnonzero(bad)[:10]}"
        return
    rel = np.abs(np.asarray(s_gpu, np.float64) - s_ref) / np.maximum(np.abs(s_ref), 1e-12)
    n = max(1, int((~flagged).sum()))
    assert bad.sum() <= 0.1 * n, f"{bad.sum()} of {n} contact-chain costs out of tolerance"
    assert np.all(rel[~flagged] < 1e-2), f"max contact-chain cost error {rel[~flagged].max():.2e}"


def elite_margin_safe(s_ref, E):
    srt = np.sort(s_ref)
    if E >= len(srt):
        return True
    return (srt[E] - srt[E - 1]) > 2 * S_TOL * max(abs(srt[E]), 1e-6)


def refit_close(a, b, cfg):
    scale = np.maximum(np.abs(b), 1e-3 * float(cfg.u_max - cfg.u_min))
    return np.abs(a - b) <= 1e-4 * scale
