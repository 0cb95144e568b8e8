"""Scheduler of the serving loop on a host-only stand-in for the device (CPU).

Admission by the memory budget (robots' resident buffers and requests'
transient slabs share the pool), one request in flight per robot, arrival
order, continuous batching at iteration boundaries, adding and removing robots
(queued and in-flight requests of a removed robot are dropped), and argument
checks."""
import time

import numpy as np
import pytest

import mtp_workloads as W
import paper_2505_01059_amd as mtp
from paper_2505_01059_amd import _native as N


def robots(n=4):
    return [W.point_mass_config(name=f"r{i}", n_tensor=200, n_gauss=56, horizon=40, n_layers=4, n_width=8,
                                n_elites=16, n_iters=3, seed=i) for i in range(n)]


def a256(x):
    return (x + 255) // 256 * 256


def slab(cfg):
    # transient bytes of one robot's slab, as the library lays it out
    T, n, B, E = cfg.horizon, cfg.ctrl_dim, cfg.n_samples, cfg.n_elites
    ld = a256(B * 4) // 4
    return (a256(cfg.n_layers * cfg.n_width * n * 4) + a256(cfg.n_layers * cfg.n_tensor) + a256(T * n * ld * 4)
            + a256(B * 4) + 3 * a256(E * 4))


def resident(cfgs):
    return sum(a256(N.resident_bytes(c)) for c in cfgs)


def sim(rs, slabs, max_robots=None, **kw):
    """A simulated server holding `rs` with room for `slabs` transient slabs of rs[0]."""
    budget = resident(rs) + int(slabs * slab(rs[0]))
    return mtp.Server(budget, max_robots or len(rs), simulated=True, robots=rs, **kw)


def drain(srv, want, timeout=10.0):
    got = []
    t0 = time.time()
    while len(got) < want and time.time() - t0 < timeout:
        srv.pump(wait_us=200)
        got += srv.poll()
    return got


def test_budget_limits_admission_and_everything_completes():
    rs = robots(5)
    srv = sim(rs, 2, iters_per_launch=1, max_inflight=2, ns_per_sample_step=0.05)
    assert srv.stats()["robots"] == 5 and srv.stats()["resident_bytes"] == resident(rs)
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
    assert st["completed"] == 5 and st["pool_in_use"] == st["resident_bytes"]
    assert st["pool_peak"] <= st["pool_bytes"]
    srv.close()


def test_slab_size_matches_library_layout():
    rs = robots(1)
    assert N.transient_bytes(rs[0]) == slab(rs[0])


def test_one_request_per_robot_in_order():
    rs = robots(2)
    srv = sim(rs, 8, iters_per_launch=2, ns_per_sample_step=0.01)
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
    srv = sim(rs, 4, iters_per_launch=1, max_inflight=1, ns_per_sample_step=1.0)
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


def test_add_robots_until_slots_or_budget_run_out():
    rs = robots(3)
    srv = mtp.Server(resident(rs[:2]) + slab(rs[0]), 3, simulated=True, ns_per_sample_step=1.0)
    assert srv.add_robot(rs[0]) == 0 and srv.add_robot(rs[1]) == 1
    srv.submit(0, W.initial_state(rs[0]))
    srv.pump()                                     # the request's slab takes the rest of the pool
    with pytest.raises(N.MtpError) as e:          # so the third robot's resident buffers do not fit
        srv.add_robot(rs[2])
    assert e.value.status == 5
    drain(srv, 1)
    assert srv.add_robot(rs[2]) == 2               # they do once the slab is back
    srv.close()
    srv = mtp.Server(10 * (resident(rs) + slab(rs[0])), 2, simulated=True)
    srv.add_robot(rs[0])
    srv.add_robot(rs[1])
    with pytest.raises(N.MtpError) as e:          # every slot taken
        srv.add_robot(rs[2])
    assert e.value.status == 5
    srv.close()


def test_queue_capacity_limits_robots():
    rs = robots(3)
    srv = mtp.Server(10 * (resident(rs) + slab(rs[0])), 3, queue_items=60, simulated=True)
    srv.add_robot(rs[0])                          # one robot needs more than 20 items per launch
    with pytest.raises(N.MtpError) as e:
        for c in rs[1:]:
            srv.add_robot(c)
    assert e.value.status == 5
    srv.close()


def test_remove_robot_drops_queued_and_in_flight_requests():
    """Unregistering a robot drops its queued requests at once and the completion
    of its request on the device; its memory returns to the pool once that
    launch retires, and the id can be reused."""
    rs = robots(3)
    srv = sim(rs, 3, iters_per_launch=1, max_inflight=1, ns_per_sample_step=1.0)
    x0 = W.initial_state(rs[0])
    srv.submit(0, x0)
    srv.submit(1, x0)
    srv.submit(1, x0)
    srv.submit(1, x0)
    srv.pump()                                     # robots 0 and 1 admitted, two of robot 1 queued
    assert srv.stats()["in_flight"] == 2
    srv.remove_robot(1)
    st = srv.stats()
    assert st["dropped"] == 2 and st["queued"] == 0 and st["robots"] == 2
    with pytest.raises(N.MtpError):
        srv.submit(1, x0)                          # no such robot any more
    got = drain(srv, 1)
    time.sleep(0.05)
    for _ in range(50):
        srv.pump(wait_us=200)
        got += srv.poll()
    assert [c["robot"] for c in got] == [0]        # robot 1's in-flight completion was dropped
    st = srv.stats()
    assert st["dropped"] == 3 and st["in_flight"] == 0
    assert st["resident_bytes"] == resident([rs[0], rs[2]]) and st["pool_in_use"] == st["resident_bytes"]
    assert srv.add_robot(rs[1]) == 1               # the slot is free again
    srv.submit(1, x0)
    assert [c["robot"] for c in drain(srv, 1)] == [1]
    srv.close()


def test_remove_idle_robot_frees_memory_at_once():
    rs = robots(2)
    srv = sim(rs, 1)
    before = srv.stats()["pool_in_use"]
    srv.remove_robot(0)
    st = srv.stats()
    assert st["pool_in_use"] == before - a256(N.resident_bytes(rs[0])) and st["robots"] == 1
    with pytest.raises(N.MtpError):
        srv.remove_robot(0)
    srv.close()


def test_bad_arguments():
    rs = robots(2)
    srv = sim(rs, 1)
    x0 = W.initial_state(rs[0])
    with pytest.raises(N.MtpError):
        srv.submit(5, x0)
    with pytest.raises(N.MtpError):
        srv.submit(0, x0, shift=-1)
    srv.close()
    with pytest.raises(N.MtpError):                 # the slab alone exceeds the whole budget
        mtp.Server(resident(rs) + slab(rs[0]) // 2, 2, simulated=True, robots=rs[:1]).add_robot(rs[1])
    with pytest.raises(N.MtpError):
        mtp.Server(0, 2, simulated=True)
    with pytest.raises(N.MtpError):
        mtp.Server(1 << 20, 0, simulated=True)
