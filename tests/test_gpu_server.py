"""Serving loop on the GPU: served replans against the oracle, served == alone,
and robots added and removed while requests are on the device."""
import numpy as np
import pytest

import mtp_workloads as W
from tests import gpu_helpers as H

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


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


def budget_for(robots, slabs):
    from paper_2505_01059_amd import _native as N
    a = lambda x: (x + 255) // 256 * 256
    return sum(a(N.resident_bytes(c)) for c in robots) + int(slabs * max(N.transient_bytes(c) for c in robots))


def run_requests(srv, order, x0, shift=1):
    got = []
    for n, (i, k) in enumerate(order):
        srv.submit(i, x0[(i, k)], shift=shift)
        if n % 2 == 0:
            srv.pump()
        got += srv.poll()
    while len(got) < len(order):
        srv.pump(wait_us=500)
        got += srv.poll()
    return got


def alone_actions(cfg, x0s):
    import paper_2505_01059_amd as mtp
    p = mtp.Plan(cfg, device="cuda:0")
    out = []
    for k, x in enumerate(x0s):
        p.replan(x, shift=1, replan_idx=k)
        out.append(p.action())
    p.close()
    return out


def test_served_equals_alone():
    import paper_2505_01059_amd as mtp
    robots = fleet()
    rounds = 3
    x0 = {(i, k): W.initial_state(c, seed=100 * k + i) for i, c in enumerate(robots) for k in range(rounds)}
    srv = mtp.Server(budget_for(robots, 1.05), len(robots), iters_per_launch=1, max_inflight=2, device="cuda:0",
                     robots=robots)
    order = [(i, k) for k in range(rounds) for i in (3, 0, 4, 1, 2)]
    got = run_requests(srv, order, x0)
    st = srv.stats()
    assert st["completed"] == len(order) and st["pool_peak"] <= st["pool_bytes"]
    assert st["deferred_for_budget"] > 0            # the budget really limited admission
    srv.close()
    for i, c in enumerate(robots):
        mine = sorted([g for g in got if g["robot"] == i], key=lambda g: g["replan_idx"])
        assert [g["replan_idx"] for g in mine] == list(range(rounds))
        want = alone_actions(c, [x0[(i, k)] for k in range(rounds)])
        for k in range(rounds):
            assert np.array_equal(want[k], mine[k]["u"]), (c.name, k)


def oracle_fleet():
    """One CEM iteration per request, every candidate an elite and uniform
    weights: a served request's refitted mean and std then follow from the
    oracle's candidates alone (no ranking involved), and its action from the
    oracle's cheapest candidate."""
    inf = np.float32(np.inf)
    cfgs = [
        W.point_mass_config(name="o_pm", n_tensor=300, n_gauss=45, horizon=37, n_layers=5, n_width=7,
                            n_elites=345, n_iters=1, seed=21, temperature=inf),
        W.chain_config(name="o_c7", n_tensor=700, n_gauss=101, horizon=66, n_elites=801, n_iters=1, seed=22,
                       temperature=inf),
        W.chain_config(name="o_c24", n_links=24, interp=W.BSPLINE, n_tensor=200, n_gauss=56, horizon=32,
                       n_layers=12, n_width=64, n_elites=256, n_iters=1, seed=23, temperature=inf),
        W.chain_contact_config(name="o_k7", n_links=7, n_tensor=150, n_gauss=42, horizon=40, n_layers=6,
                               n_width=16, n_elites=192, n_iters=1, seed=24, temperature=inf),
        W.chain_config(name="o_c2", n_links=2, interp=W.LINEAR, n_tensor=200, n_gauss=57, horizon=30, n_layers=4,
                       n_width=5, n_elites=257, n_iters=1, seed=25, temperature=inf),
    ]
    for c in cfgs:
        assert c.n_elites == c.n_samples
    return cfgs


# The action compares candidates by cost: it is checked when the oracle's two
# cheapest candidates are further apart than ten times the largest relative
# float32 cost error the rollout parity tests observe on these models (1e-6).
BEST_GAP = 1e-5


def test_served_requests_against_oracle():
    """Each served request against the oracle's Alg. 2 iteration from the
    robot's warm start as the server held it before the request (read back
    through mtp_server_get_robot_state, shifted one step as the request asks):
    the refitted mean and std every time, the action whenever the oracle's
    cheapest candidate is clear of the float32 cost error."""
    import paper_2505_01059_amd as mtp
    from oracle import planner as OP
    robots = oracle_fleet()
    rounds = 3
    srv = mtp.Server(budget_for(robots, 2.5), len(robots), iters_per_launch=1, max_inflight=2, device="cuda:0",
                     robots=robots)
    unclear = checked = 0
    for k in range(rounds):
        before = {}
        for i in range(len(robots)):
            mu, sg, r = srv.robot_state(i)
            before[i] = (mu.cpu().numpy().astype(np.float64), sg.cpu().numpy().astype(np.float64), r)
        x0 = {(i, k): W.initial_state(c, seed=200 * k + i) for i, c in enumerate(robots)}
        got = run_requests(srv, [(i, k) for i in (2, 0, 4, 1, 3)], x0)
        for g in got:
            i = g["robot"]
            cfg = robots[i]
            mu_b, sg_b, r = before[i]
            assert g["replan_idx"] == r
            mu_s, sg_s = OP.shift_distribution(mu_b, sg_b, 1, np.float64(cfg.sigma_init))
            ref = OP.iterate(cfg, x0[(i, k)], mu_s, sg_s, r, 0)
            mu_a, sg_a, r_a = srv.robot_state(i)
            assert r_a == r + 1
            assert H.refit_close(mu_a.cpu().numpy(), ref["mu"], cfg).all(), (cfg.name, k, "mean")
            assert H.refit_close(sg_a.cpu().numpy(), ref["sigma"], cfg).all(), (cfg.name, k, "std")
            srt = np.sort(ref["s"])
            checked += 1
            if srt[1] - srt[0] > BEST_GAP * abs(srt[1]):
                assert H.u_close(g["u"], ref["action"], cfg.u_max).all(), (cfg.name, k, "action")
            else:
                unclear += 1
    _log(f"[served vs oracle] {checked} requests, {unclear} actions left unchecked (cheapest two within "
         f"{BEST_GAP:g})")
    assert unclear <= checked // 3
    srv.close()


def test_robots_added_and_removed_while_serving():
    """A robot removed while its request is on the device never delivers it; a
    robot added into the freed slot (and memory) plans as if alone, and so do
    the robots that stayed."""
    import paper_2505_01059_amd as mtp
    robots = fleet()
    newcomer = W.chain_config(name="s_new", n_tensor=400, n_gauss=80, horizon=40, n_elites=24, n_iters=3, seed=31)
    srv = mtp.Server(budget_for(robots + [newcomer], 3), len(robots), iters_per_launch=1, max_inflight=2,
                     device="cuda:0", robots=robots)
    x0 = {(i, k): W.initial_state(c, seed=300 * k + i) for i, c in enumerate(robots + [newcomer]) for k in range(2)}
    for i in range(len(robots)):
        srv.submit(i, x0[(i, 0)], shift=1)
    srv.pump()
    srv.remove_robot(1)                            # its request is admitted: the completion is dropped
    got = []
    while srv.stats()["in_flight"] > 0:
        srv.pump(wait_us=500)
        got += srv.poll()
    assert sorted(g["robot"] for g in got) == [0, 2, 3, 4]
    assert srv.stats()["dropped"] == 1
    assert srv.add_robot(newcomer) == 1
    for i in (1, 0, 2):
        srv.submit(i, x0[(len(robots), 1) if i == 1 else (i, 1)], shift=1)
    got2 = []
    while len(got2) < 3:
        srv.pump(wait_us=500)
        got2 += srv.poll()
    srv.close()
    by = {g["robot"]: g for g in got2}
    assert np.array_equal(by[1]["u"], alone_actions(newcomer, [x0[(len(robots), 1)]])[0])
    for i in (0, 2):
        want = alone_actions(robots[i], [x0[(i, 0)], x0[(i, 1)]])
        assert np.array_equal(by[i]["u"], want[1]), robots[i].name
        assert np.array_equal([g for g in got if g["robot"] == i][0]["u"], want[0]), robots[i].name


def test_fleet_sample_alone_vs_mix():
    """The 512-robot serving fleet (the uneven batching mix's instance types) with
    one request per robot in flight together; a sample of robots' actions equal
    the same replans run alone, bit for bit."""
    import paper_2505_01059_amd as mtp
    robots = W.robot_fleet(512)
    x0 = [W.initial_state(c, seed=i) for i, c in enumerate(robots)]
    srv = mtp.Server(32 << 30, len(robots), iters_per_launch=1, max_inflight=2, device="cuda:0", robots=robots)
    for i in range(len(robots)):
        srv.submit(i, x0[i], shift=1)
    got = []
    while len(got) < len(robots):
        srv.pump(wait_us=1000)
        got += srv.poll()
    srv.close()
    by = {g["robot"]: g for g in got}
    for i in (0, 3, 17, 100, 257, 400, 511):
        want = alone_actions(robots[i], [x0[i]])[0]
        assert np.array_equal(by[i]["u"], want), robots[i].name
    _log(f"[fleet] {len(got)} requests served together; 7 sampled robots equal their alone replans")
