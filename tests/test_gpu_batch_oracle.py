"""The persistent batched launch against the oracle directly.

One launch runs one CEM iteration (Alg. 2 loop body) of every instance of an
uneven mix from a mean and std set per instance; each instance's graph, paths,
candidates, costs, elites, refit and action are then compared with the
oracle's same iteration (teacher forcing, gpu_helpers.check_iteration).  The
mix covers every rollout form (point mass, one-, four- and two-lane chains,
contact chains that reach the ground, randomised models), every interpolation
and sampling without replacement.  Few candidate tiles make the launch split
candidate and refit items per joint and per four outputs; the large variant
adds a 66000-candidate instance so that the items stay whole."""
import numpy as np
import pytest

import mtp_workloads as W
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def oracle_mix():
    return [
        W.point_mass_config(name="q_pm", n_tensor=300, n_gauss=45, horizon=37, n_layers=5, n_width=7,
                            n_elites=20, n_iters=3, seed=1),
        W.point_mass_config(name="q_pm_ak", interp=W.AKIMA, n_tensor=260, n_gauss=33, horizon=50,
                            n_layers=6, n_width=9, n_elites=16, n_iters=2, seed=3),
        W.point_mass_config(name="q_pm_lin", interp=W.LINEAR, n_tensor=250, n_gauss=40, n_layers=6,
                            horizon=45, n_elites=16, n_iters=2, seed=11),
        W.chain_config(name="q_c2", n_links=2, n_tensor=200, n_gauss=57, horizon=30, n_layers=4, n_width=5,
                       n_elites=10, n_iters=3, seed=4),
        W.chain_config(name="q_c7", n_tensor=700, n_gauss=101, horizon=66, n_elites=40, n_iters=2, seed=2),
        W.chain_config(name="q_c12", n_links=12, interp=W.BSPLINE, n_tensor=250, n_gauss=70, horizon=32,
                       n_layers=9, n_width=40, n_elites=30, n_iters=2, seed=5),
        W.chain_config(name="q_c24", n_links=24, interp=W.AKIMA, n_tensor=130, n_gauss=70, horizon=24,
                       n_layers=12, n_width=64, n_elites=16, n_iters=2, seed=6),
        W.chain_contact_config(name="q_k4g", n_links=4, n_tensor=150, n_gauss=42, horizon=80, n_layers=6,
                               n_width=12, n_elites=12, n_iters=2, ground_y=-0.5, seed=12),
        W.chain_contact_config(name="q_k7g_r2", n_links=7, n_tensor=120, n_gauss=40, horizon=90, n_layers=6,
                               n_width=16, n_elites=12, n_iters=2, n_replicas=2, ground_y=-0.5, seed=13),
        W.chain_contact_config(name="q_k24g", n_tensor=100, n_gauss=28, horizon=100, n_elites=12, n_iters=2,
                               ground_y=-2.0, seed=14),
        W.chain_config(name="q_wor", n_tensor=500, n_gauss=60, horizon=40, n_elites=20, n_iters=3,
                       seed=8).replace(sample_wor=1),
        W.chain_config(name="q_c5p", interp=W.BSPLINE, bspline_degree=5, n_links=3, n_layers=9, n_tensor=300,
                       n_gauss=60, horizon=50, n_elites=20, n_iters=2, seed=15),
    ]


def random_state(cfg, seed):
    rng = np.random.default_rng(seed)
    um = float(cfg.u_max)
    mu = rng.uniform(-0.5 * um, 0.5 * um, size=(cfg.horizon, cfg.ctrl_dim)).astype(np.float32)
    sg = rng.uniform(0.1 * um, 0.6 * um, size=(cfg.horizon, cfg.ctrl_dim)).astype(np.float32)
    return mu, sg


@pytest.mark.parametrize("large", [False, True])
def test_batched_iteration_against_oracle(large):
    import torch
    import paper_2505_01059_amd as mtp
    cfgs = oracle_mix()
    if large:
        cfgs.append(W.point_mass_config(name="q_big", n_tensor=64000, n_gauss=2000, horizon=16, n_elites=64,
                                        n_iters=1, seed=16))
    nd = [c.n_samples if c.dynamics == W.CHAIN_CONTACT else 0 for c in cfgs]
    print(f"[batch vs oracle] {len(cfgs)} instances, {sum(c.n_samples for c in cfgs)} candidates", flush=True)
    bt = mtp.Batch(cfgs, device="cuda:0", n_debug_states=nd)
    x0s = [W.initial_state(c, seed=7) for c in cfgs]
    states = [random_state(c, 100 + i) for i, c in enumerate(cfgs)]
    for i, (mu, sg) in enumerate(states):
        bt.set_state(i, mu, sg)
    torch.cuda.synchronize()
    r = 9
    n = len(cfgs)
    order = list(range(n))[::-1]            # launch order is not config order
    bt.step(order, [0] * n, [1] * n, [0] * n, [r] * n, bt.pack_x0(x0s))
    bt.actions()                            # waits and checks the launch status
    for i, c in enumerate(cfgs):
        b = bt.buffers(i)
        X_all = b["X_all"].cpu().numpy().transpose(0, 3, 1, 2).astype(np.float64) if nd[i] else None
        H.check_iteration(c, b, x0s[i], states[i][0], states[i][1], r, 0, f"batch {c.name}", X_all)
    bt.close()
