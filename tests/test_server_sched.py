"""Scheduler of the serving loop on a host-only stand-in for the device (CPU).

Admission by the memory budget, one request in flight per robot, arrival order,
continuous batching at iteration boundaries, and argument checks."""
import time

import numpy as np
import pytest

import mtp_workloads as W
import paper_2505_01059_amd as mtp
from paper_2505_01059_amd import _native as N


def robots(n=4):
    return [W.point_mass_config(name=f"r{i}", n_tensor=200, n_gauss=56, horizon=40, n_layers=4, n_width=8,
                                n_elites=16, n_iters=3, seed=i) for i in range(n)]


def slab(cfg):
    # transient bytes of one robot's slab, as the library lays it out
    T, n, B, E = cfg.horizon, cfg.ctrl_dim, cfg.n_samples, cfg.n_elites
    a = lambda x: (x + 255) // 256 * 256
    ld = a(B * 4) // 4
    return (a(cfg.n_layers * cfg.n_width * n * 4) + a(cfg.n_layers * cfg.n_tensor) + a(T * n * ld * 4)
            + a(B * 4) + 3 * a(E * 4))


def drain(srv, want, timeout=10.0):
    got = []
    t0 = time.time()
    while len(got) < want and time.time() - t0 < timeout:
        srv.pump(wait_us=200)
        got += srv.poll()
    return got


def test_budget_limits_admission_and_everything_completes():
    rs = robots(5)
    srv = mtp.Server(rs, pool_bytes=2 * slab(rs[0]), iters_per_launch=1, max_inflight=2,
                     simulated=True, ns_per_sample_step=0.05)
    x0 = W.initial_state(rs[0])
    for r in range(5):
        srv.submit(r, x0)
    srv.pump()
    st = srv.stats()
    assert st["admitted"] == 2 and st["queued"] == 3 and st["deferred_for_budget"] >= 1
    assert st["pool_in_use"] <= st["pool_bytes"]
    got = drain(srv, 5)
    assert sorted(c["robot"] for c in got) == list(range(5))
    st = srv.stats()
    assert st["completed"] == 5 and st["pool_in_use"] == 0 and st["pool_peak"] <= st["pool_bytes"]
    srv.close()


def test_one_request_per_robot_in_order():
    rs = robots(2)
    srv = mtp.Server(rs, pool_bytes=8 * slab(rs[0]), iters_per_launch=2, simulated=True, ns_per_sample_step=0.01)
    x0 = W.initial_state(rs[0])
    tickets = [srv.submit(0, x0) for _ in range(4)] + [srv.submit(1, x0)]
    srv.pump()
    assert srv.stats()["in_flight"] == 2          # robot 0 has one request admitted, robot 1 one
    got = drain(srv, 5)
    r0 = [c for c in got if c["robot"] == 0]
    assert [c["ticket"] for c in r0] == tickets[:4]
    assert [c["replan_idx"] for c in r0] == [0, 1, 2, 3]
    srv.close()


def test_late_request_joins_at_iteration_boundary():
    """A request that arrives while another is mid-replan starts in the next launch,
    alongside the first one's remaining iterations, not after it finishes."""
    rs = robots(2)
    srv = mtp.Server(rs, pool_bytes=4 * slab(rs[0]), iters_per_launch=1, max_inflight=1,
                     simulated=True, ns_per_sample_step=1.0)
    x0 = W.initial_state(rs[0])
    srv.submit(0, x0)
    srv.pump()                                     # launch 1: robot 0, iteration 0
    srv.submit(1, x0)
    got = []
    while srv.stats()["launches"] < 2:
        srv.pump(wait_us=100)
        got += srv.poll()
    st = srv.stats()
    assert st["admitted"] == 2 and not got        # robot 1 admitted before robot 0 finished
    got += drain(srv, 2)
    done = {c["robot"]: c for c in got}
    assert done[1]["t_admit_ns"] < done[0]["t_done_ns"]
    # three iterations each, one per launch, overlapping: 4 launches, not 6
    assert srv.stats()["launches"] == 4
    srv.close()


def test_bad_arguments():
    rs = robots(2)
    srv = mtp.Server(rs, pool_bytes=slab(rs[0]), simulated=True)
    x0 = W.initial_state(rs[0])
    with pytest.raises(N.MtpError):
        srv.submit(5, x0)
    with pytest.raises(N.MtpError):
        srv.submit(0, x0, shift=-1)
    srv.close()
    with pytest.raises(N.MtpError):
        mtp.Server(rs, pool_bytes=slab(rs[0]) // 2, simulated=True).submit(0, x0)


def test_slab_size_matches_library_layout():
    lib = mtp.load()
    rs = robots(1)
    c, keep = N.config_struct(rs[0])
    import ctypes
    total = N.workspace_bytes(rs[0])
    assert total >= slab(rs[0])
