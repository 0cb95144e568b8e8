"""Serving loop on the GPU: every served replan equals the same replan run alone."""
import numpy as np
import pytest

import mtp_workloads as W

pytestmark = pytest.mark.gpu


def fleet():
    return [
        W.point_mass_config(name="s_pm", n_tensor=300, n_gauss=45, horizon=37, n_layers=5, n_width=7,
                            n_elites=20, n_iters=3, seed=11),
        W.chain_config(name="s_c7", n_tensor=700, n_gauss=101, horizon=66, n_elites=40, n_iters=2, seed=12),
        W.point_mass_config(name="s_pm_ak", interp=W.AKIMA, n_tensor=260, n_gauss=33, horizon=50, n_layers=6,
                            n_width=9, n_elites=16, n_iters=4, seed=13),
        W.chain_config(name="s_c12", n_links=12, interp=W.BSPLINE, n_tensor=250, n_gauss=70, horizon=32,
                       n_layers=9, n_width=40, n_elites=30, n_iters=2, seed=14),
        W.chain_config(name="s_c2", n_links=2, n_tensor=200, n_gauss=57, horizon=30, n_layers=4, n_width=5,
                       n_elites=10, n_iters=3, seed=15),
    ]


def test_served_equals_alone():
    import torch
    import paper_2505_01059_amd as mtp
    from paper_2505_01059_amd import _native as N
    robots = fleet()
    rounds = 3
    x0 = {(i, k): W.initial_state(c, seed=100 * k + i) for i, c in enumerate(robots) for k in range(rounds)}
    slabs = [N.transient_bytes(c) for c in robots]
    srv = mtp.Server(robots, pool_bytes=int(1.05 * max(slabs)), iters_per_launch=1, max_inflight=2, device="cuda:0")
    got = []
    order = [(i, k) for k in range(rounds) for i in (3, 0, 4, 1, 2)]
    for n, (i, k) in enumerate(order):
        srv.submit(i, x0[(i, k)], shift=1)
        if n % 2 == 0:
            srv.pump()
        got += srv.poll()
    while len(got) < len(order):
        srv.pump(wait_us=500)
        got += srv.poll()
    st = srv.stats()
    assert st["completed"] == len(order) and st["pool_peak"] <= st["pool_bytes"]
    assert st["deferred_for_budget"] > 0            # the budget really limited admission
    srv.close()
    for i, c in enumerate(robots):
        mine = sorted([g for g in got if g["robot"] == i], key=lambda g: g["replan_idx"])
        assert [g["replan_idx"] for g in mine] == list(range(rounds))
        p = mtp.Plan(c, device="cuda:0")
        for k in range(rounds):
            p.replan(x0[(i, k)], shift=1, replan_idx=k)
            a = p.action()
            assert np.array_equal(a, mine[k]["u"]), (c.name, k)
        p.close()
