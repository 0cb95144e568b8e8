"""Persistent batched launch: every instance's result equals running it alone.

Per-instance reductions have an order fixed by the instance, so the batched
mean, std and action must match a standalone plan bit for bit, whatever the
other instances are and whichever workgroups ran the tiles."""
import sys

import numpy as np
import pytest

import mtp_workloads as W

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)


def small_mix():
    return [
        W.point_mass_config(name="b_pm", n_tensor=300, n_gauss=45, horizon=37, n_layers=5, n_width=7,
                            n_elites=20, n_iters=3, seed=1),
        W.chain_config(name="b_c7", n_tensor=700, n_gauss=101, horizon=66, n_elites=40, n_iters=2, seed=2),
        W.point_mass_config(name="b_pm_ak", interp=W.AKIMA, n_tensor=260, n_gauss=33, horizon=50,
                            n_layers=6, n_width=9, n_elites=16, n_iters=4, seed=3),
        W.chain_config(name="b_c2", n_links=2, n_tensor=200, n_gauss=57, horizon=30, n_layers=4, n_width=5,
                       n_elites=10, n_iters=3, seed=4),
        W.chain_config(name="b_c12", n_links=12, interp=W.BSPLINE, n_tensor=250, n_gauss=70, horizon=32,
                       n_layers=9, n_width=40, n_elites=30, n_iters=2, seed=5),
        W.chain_config(name="b_c24", n_links=24, interp=W.AKIMA, n_tensor=130, n_gauss=70, horizon=24,
                       n_layers=12, n_width=64, n_elites=16, n_iters=2, seed=6),
        W.chain_contact_config(name="b_k24", n_tensor=200, n_gauss=56, horizon=48, n_elites=16, n_iters=2,
                               seed=7),
        # paths without replacement and the cost-entropy diagnostic
        W.chain_config(name="b_wor", n_tensor=500, n_gauss=60, horizon=40, n_elites=20, n_iters=3,
                       seed=8).replace(sample_wor=1, diagnostics=1),
        W.point_mass_config(name="b_pmwor", n_tensor=200, n_gauss=40, horizon=30, n_layers=4, n_width=4,
                            n_elites=16, n_iters=2, seed=9).replace(sample_wor=1, diagnostics=1),
    ]


def overlap_mix():
    """Plans for which the single-plan path draws each next iteration's tensor
    paths during the rollout (at least 1024 tensor paths, a rollout that leaves
    compute units free, more than one iteration), with odd and even iteration
    counts (the last iteration in either U buffer), a tile shared by local and
    tensor candidates, every rollout form and every interpolation."""
    return [
        W.chain_config(name="o_c7", interp=W.AKIMA, n_tensor=1100, n_gauss=101, horizon=40, n_elites=40,
                       n_iters=3, seed=21),
        W.chain_config(name="o_c7b", interp=W.BSPLINE, n_tensor=2048, n_gauss=256, horizon=33, n_elites=64,
                       n_iters=4, seed=22),
        W.point_mass_config(name="o_pm", n_tensor=3000, n_gauss=77, horizon=45, n_elites=32, n_iters=5, seed=23),
        W.chain_config(name="o_c12", n_links=12, interp=W.BSPLINE, n_tensor=1500, n_gauss=100, horizon=32,
                       n_layers=6, n_width=20, n_elites=30, n_iters=2, seed=24),
        W.chain_contact_config(name="o_k4", n_links=4, n_tensor=1200, n_gauss=64, horizon=30, n_layers=6,
                               n_width=16, n_elites=16, n_iters=3, seed=25),
        W.chain_config(name="o_c3", n_links=3, interp=W.LINEAR, n_tensor=1024, n_gauss=1, horizon=20,
                       n_elites=8, n_iters=2, seed=26),
        # local samples end exactly on a tile boundary (G - 1 = 256)
        W.point_mass_config(name="o_pm257", interp=W.AKIMA, n_tensor=1500, n_gauss=257, horizon=36,
                            n_elites=24, n_iters=3, seed=27),
        # randomised replicas on the one-lane contact rollout
        W.chain_contact_config(name="o_k7r2", n_links=7, n_tensor=1100, n_gauss=90, horizon=28, n_layers=5,
                               n_width=12, n_elites=20, n_iters=2, seed=28, n_replicas=2),
        # time-sliced pair-lane rollouts (more pair-lane waves than SIMDs): the
        # next tensor paths are drawn by their own kernel beside the rollout
        W.chain_config(name="o_c12s", n_links=12, interp=W.BSPLINE, n_tensor=32000, n_gauss=1000, horizon=16,
                       n_layers=5, n_width=16, n_elites=64, n_iters=3, seed=29),
        W.chain_contact_config(name="o_k24s", n_links=24, n_tensor=32800, n_gauss=70, horizon=24, n_layers=6,
                               n_width=12, n_elites=48, n_iters=2, seed=30, ground_y=-0.02),
        # the same with links of different lengths (the time-sliced rollout's
        # per-link form; the ones above have equal links, held once)
        _uneven_links(W.chain_config(name="o_c12u", n_links=12, interp=W.BSPLINE, n_tensor=32000, n_gauss=1000,
                                     horizon=16, n_layers=5, n_width=16, n_elites=64, n_iters=2, seed=31)),
        _uneven_links(W.chain_contact_config(name="o_k24u", n_links=24, n_tensor=32800, n_gauss=70, horizon=24,
                                             n_layers=6, n_width=12, n_elites=48, n_iters=2, seed=32,
                                             ground_y=-0.02)),
    ]


def _uneven_links(cfg):
    """The config with link lengths drawn in [0.7, 1.3] (seeded by the config)."""
    import dataclasses
    rng = np.random.default_rng(cfg.seed + 1000)
    lengths = rng.uniform(0.7, 1.3, cfg.n_links).astype(np.float32)
    return cfg.replace(task=dataclasses.replace(cfg.task, lengths=lengths))


def standalone(cfg, x0, replans, shift=1):
    import torch
    import paper_2505_01059_amd as mtp
    p = mtp.Plan(cfg, device="cuda:0")
    for r in range(replans):
        p.replan(x0, shift=shift, replan_idx=r)
    torch.cuda.synchronize()
    b = p.buffers()
    out = (b["mu"].cpu().numpy().copy(), b["sigma"].cpu().numpy().copy(), p.action(),
           b["entropy"].cpu().numpy().copy())
    p.close()
    return out


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_equals_standalone(use_graph):
    import torch
    import paper_2505_01059_amd as mtp
    cfgs = small_mix()
    x0s = [W.initial_state(c, seed=i) for i, c in enumerate(cfgs)]
    _log(f"[batch] {len(cfgs)} instances, graph={use_graph}")
    bt = mtp.Batch(cfgs, device="cuda:0", use_graph=use_graph)
    xp = bt.pack_x0(x0s)
    for r in range(2):
        bt.replan(xp, shift=1)
    acts = bt.actions()
    for i, c in enumerate(cfgs):
        mu, sg, a, ent = standalone(c, x0s[i], 2)
        b = bt.buffers(i)
        assert np.array_equal(b["mu"].cpu().numpy(), mu), c.name
        assert np.array_equal(b["sigma"].cpu().numpy(), sg), c.name
        assert np.array_equal(acts[i], a), c.name
        if c.diagnostics:
            assert np.array_equal(b["entropy"].cpu().numpy(), ent), c.name
    bt.close()


def test_overlapped_tensor_paths_equal_the_plain_sequence():
    """Single plans that draw iteration k+1's tensor paths during iteration k's
    rollout (graph replay and the stage-timed launch sequence) give the bits of
    the batched kernel, which runs the stages one after the other."""
    import torch
    import paper_2505_01059_amd as mtp
    cfgs = overlap_mix()
    x0s = [W.initial_state(c, seed=i) for i, c in enumerate(cfgs)]
    _log(f"[overlap] {len(cfgs)} instances")
    bt = mtp.Batch(cfgs, device="cuda:0")
    xp = bt.pack_x0(x0s)
    for r in range(2):
        bt.replan(xp, shift=1)
    acts = bt.actions()
    for i, c in enumerate(cfgs):
        b = bt.buffers(i)
        for timed in (False, True):
            p = mtp.Plan(c, device="cuda:0")
            assert p.draws_ahead(), c.name
            p.set_stage_timing(timed)
            for r in range(2):
                p.replan(x0s[i], shift=1, replan_idx=r)
            torch.cuda.synchronize()
            pb = p.buffers()
            assert np.array_equal(pb["mu"].cpu().numpy(), b["mu"].cpu().numpy()), (c.name, timed)
            assert np.array_equal(pb["sigma"].cpu().numpy(), b["sigma"].cpu().numpy()), (c.name, timed)
            assert np.array_equal(p.action(), acts[i]), (c.name, timed)
            # the U buffer holds the last iteration's candidates in both
            B = c.n_samples
            assert np.array_equal(pb["U"][:, :, :B].cpu().numpy(), b["U"][:, :, :B].cpu().numpy()), (c.name, timed)
            p.close()
    bt.close()


@pytest.mark.parametrize("mode", ["graph", "eager", "timed"])
def test_draws_across_replans_follow_the_replan_index(mode):
    """Plans with an even iteration count draw the next replan's first tensor
    paths during their last rollout.  A replan takes them only when its index
    is the one they were drawn for: consecutive replans, a jump in the index, a
    single iteration run in between and a repeat of the same index all give the
    bits of the batched kernel, which draws every iteration's paths itself
    (replayed graph, eager launches and stage-timed launches alike)."""
    import torch
    import paper_2505_01059_amd as mtp
    mix = {c.name: c for c in overlap_mix()}
    cfgs = [mix["o_c7b"], mix["o_c12"], mix["o_k24s"], mix["o_k7r2"],
            W.point_mass_config(name="a_pm", n_tensor=2048, n_gauss=100, horizon=40, n_elites=32, n_iters=4,
                                seed=50)]
    x0s = [W.initial_state(c, seed=40 + i) for i, c in enumerate(cfgs)]
    ops = [("replan", 0), ("replan", 1), ("replan", 5), ("replan", 6), ("iter", 7), ("replan", 7),
           ("replan", 8), ("replan", 8)]
    n = len(cfgs)
    bt = mtp.Batch(cfgs, device="cuda:0")
    xp = bt.pack_x0(x0s)
    plans = []
    for i, c in enumerate(cfgs):
        p = mtp.Plan(c, device="cuda:0", use_graph=(mode == "graph"))
        p.set_stage_timing(mode == "timed")
        assert p.draws_ahead() and c.n_iters % 2 == 0, c.name
        plans.append(p)
    for op, r in ops:
        _log(f"[across] {mode} {op} {r}")
        if op == "replan":
            bt.step(list(range(n)), [0] * n, [c.n_iters for c in cfgs], [1] * n, [r] * n, xp)
            for i, p in enumerate(plans):
                p.replan(x0s[i], shift=1, replan_idx=r)
        else:
            bt.step(list(range(n)), [0] * n, [1] * n, [0] * n, [r] * n, xp)
            for p in plans:
                p.run_stage(mtp.STAGE_ALL, r, 0)
        torch.cuda.synchronize()
        for i, (c, p) in enumerate(zip(cfgs, plans)):
            b, pb = bt.buffers(i), p.buffers()
            assert np.array_equal(pb["mu"].cpu().numpy(), b["mu"].cpu().numpy()), (c.name, op, r)
            assert np.array_equal(pb["sigma"].cpu().numpy(), b["sigma"].cpu().numpy()), (c.name, op, r)
    for p in plans:
        p.close()
    bt.close()


@pytest.mark.parametrize("E", [1024, 1025])
def test_refit_from_redrawn_elites_equals_the_gather(E):
    """Large cubic B-spline plans refit from elite controls drawn again rather
    than gathered from U (up to 1024 elites; one more falls back to the
    gather): the same bits as the batched kernel, which gathers, with local
    and tensor candidates among the elites."""
    import torch
    import paper_2505_01059_amd as mtp
    c = W.chain_config(name=f"regen_e{E}", n_links=12, interp=W.BSPLINE, n_tensor=18000, n_gauss=2000, horizon=16,
                       n_layers=5, n_width=16, n_elites=E, n_iters=3, seed=60 + E)
    x0 = W.initial_state(c, seed=3)
    _log(f"[regen] E={E}")
    bt = mtp.Batch([c], device="cuda:0")
    xp = bt.pack_x0([x0])
    p = mtp.Plan(c, device="cuda:0")
    assert p.draws_ahead()
    for r in range(2):
        bt.replan(xp, shift=1)
        p.replan(x0, shift=1, replan_idx=r)
    torch.cuda.synchronize()
    b, pb = bt.buffers(0), p.buffers()
    assert np.array_equal(pb["mu"].cpu().numpy(), b["mu"].cpu().numpy())
    assert np.array_equal(pb["sigma"].cpu().numpy(), b["sigma"].cpu().numpy())
    assert np.array_equal(p.action(), bt.actions()[0])
    iE = pb["elite_idx"].cpu().numpy()
    G1 = c.n_gauss - 1
    assert (iE < G1).any() and (iE >= G1).any(), "elites of one kind only"
    p.close()
    bt.close()


def test_batch_step_split_iterations_and_subsets():
    """Running iterations [0, 1) and then [1, K) of a replan, in launches that
    include other instances or not, gives the same bits as one replan."""
    import torch
    import paper_2505_01059_amd as mtp
    cfgs = small_mix()[:4]
    x0s = [W.initial_state(c, seed=10 + i) for i, c in enumerate(cfgs)]
    bt = mtp.Batch(cfgs, device="cuda:0")
    xp = bt.pack_x0(x0s)
    # launch 1: instances 0 and 2 do their first iteration, 1 does the whole replan
    bt.step([0, 2, 1], [0, 0, 0], [1, 1, cfgs[1].n_iters], [1, 1, 1], [0, 0, 0], xp)
    # launch 2: 0 and 2 finish, 3 does everything
    bt.step([2, 3, 0], [1, 0, 1], [cfgs[2].n_iters, cfgs[3].n_iters, cfgs[0].n_iters], [0, 1, 0], [0, 0, 0], xp)
    acts = bt.actions()
    torch.cuda.synchronize()
    for i, c in enumerate(cfgs):
        mu, sg, a, _ = standalone(c, x0s[i], 1)
        b = bt.buffers(i)
        assert np.array_equal(b["mu"].cpu().numpy(), mu), c.name
        assert np.array_equal(b["sigma"].cpu().numpy(), sg), c.name
        if i in (0, 2, 3):
            assert np.array_equal(acts[i], a), c.name
    bt.close()


def test_batch_autotune_and_reset():
    import paper_2505_01059_amd as mtp
    cfgs = small_mix()[:3]
    x0s = [W.initial_state(c) for c in cfgs]
    bt = mtp.Batch(cfgs, device="cuda:0")
    wg, order, ms = bt.autotune(reps=1)
    _log(f"[autotune] wg/CU={wg} order={order} {ms:.3f} ms")
    assert wg >= 1 and order in (0, 1) and ms > 0
    xp = bt.pack_x0(x0s)
    bt.replan(xp, shift=1)                       # replan index 0 after the reset
    acts = bt.actions()
    for i, c in enumerate(cfgs):
        mu, sg, a, _ = standalone(c, x0s[i], 1)
        assert np.array_equal(acts[i], a)
    bt.close()


# Schedules far from the default: several candidate and rollout tiles per item,
# few refit outputs per item, the finest items always, and never.
SCHEDULES = [
    dict(cand_tiles=4, roll_tiles=2, refit_outputs=8, split_pct=0),
    dict(cand_tiles=2, roll_tiles=4, refit_outputs=16, split_pct=0, order=0),
    dict(cand_tiles=4, roll_tiles=4, refit_outputs=32, split_pct=1 << 30),
    dict(cand_tiles=1, roll_tiles=1, refit_outputs=4, split_pct=0, wg_per_cu=1),
]


def test_every_schedule_gives_the_standalone_bits():
    """Item shapes, split threshold, queue order and grid change which
    workgroup computes what, never a value: every instance under every
    schedule equals its standalone plan bit for bit."""
    import paper_2505_01059_amd as mtp
    cfgs = small_mix()
    x0s = [W.initial_state(c, seed=50 + i) for i, c in enumerate(cfgs)]
    ref = [standalone(c, x0s[i], 2) for i, c in enumerate(cfgs)]
    for sched in SCHEDULES:
        _log(f"[schedule] {sched}")
        bt = mtp.Batch(cfgs, device="cuda:0")
        bt.set_schedule(**sched)
        got = bt.schedule()
        assert all(got[k] == v for k, v in sched.items()), got
        xp = bt.pack_x0(x0s)
        for r in range(2):
            bt.replan(xp, shift=1)
        acts = bt.actions()
        for i, c in enumerate(cfgs):
            mu, sg, a, ent = ref[i]
            b = bt.buffers(i)
            assert np.array_equal(b["mu"].cpu().numpy(), mu), (c.name, sched)
            assert np.array_equal(b["sigma"].cpu().numpy(), sg), (c.name, sched)
            assert np.array_equal(acts[i], a), (c.name, sched)
            if c.diagnostics:
                assert np.array_equal(b["entropy"].cpu().numpy(), ent), (c.name, sched)
        bt.close()


def test_unsupported_schedules_are_refused():
    import paper_2505_01059_amd as mtp
    bt = mtp.Batch(small_mix()[:2], device="cuda:0")
    before = bt.schedule()
    for bad in (dict(cand_tiles=3), dict(roll_tiles=8), dict(refit_outputs=2), dict(order=2)):
        with pytest.raises(mtp.MtpError):
            bt.set_schedule(**bad)
        assert bt.schedule() == before
    bt.close()


def test_tuned_schedule_is_cached_and_reused(tmp_path):
    """The first tune searches and writes the cache; a new batch of the same
    mix on the same GPU takes the cached schedule without searching, and its
    replans equal the standalone plans bit for bit."""
    import json
    import torch
    import paper_2505_01059_amd as mtp
    cfgs = small_mix()[:5]
    x0s = [W.initial_state(c, seed=60 + i) for i, c in enumerate(cfgs)]
    path = str(tmp_path / "schedules.json")
    bt = mtp.Batch(cfgs, device="cuda:0")
    sched, ms, hit = bt.tune(reps=1, cache_path=path)
    _log(f"[tune] {sched} {ms:.3f} ms from_cache={hit}")
    assert not hit and ms > 0 and bt.schedule() == sched
    bt.close()
    (entry,) = json.load(open(path))["entries"]
    props = torch.cuda.get_device_properties(0)
    assert entry["cus"] == props.multi_processor_count
    assert entry["arch"].split(":")[0] == props.gcnArchName.split(":")[0]
    assert entry["mix"] == f"{mtp.mix_signature(cfgs):016x}"
    bt = mtp.Batch(cfgs, device="cuda:0")
    sched2, ms2, hit2 = bt.tune(reps=1, cache_path=path)
    assert hit2 and sched2 == sched and ms2 == pytest.approx(ms, rel=1e-5)
    assert bt.schedule() == sched
    xp = bt.pack_x0(x0s)
    bt.replan(xp, shift=1)
    acts = bt.actions()
    for i, c in enumerate(cfgs):
        mu, sg, a, _ = standalone(c, x0s[i], 1)
        b = bt.buffers(i)
        assert np.array_equal(b["mu"].cpu().numpy(), mu), c.name
        assert np.array_equal(b["sigma"].cpu().numpy(), sg), c.name
        assert np.array_equal(acts[i], a), c.name
    bt.close()
    # another mix misses and adds its own entry
    bt = mtp.Batch(cfgs[:3], device="cuda:0")
    _, _, hit3 = bt.tune(reps=1, cache_path=path)
    assert not hit3
    assert len(json.load(open(path))["entries"]) == 2
    bt.close()


def test_mix_of_256_sampled_against_standalone():
    """The full uneven mix in one launch; a sample of instances checked bit for bit."""
    import torch
    import paper_2505_01059_amd as mtp
    cfgs = W.mix(256)
    x0s = [W.initial_state(c, seed=i) for i, c in enumerate(cfgs)]
    _log(f"[mix] total candidates {sum(c.n_samples for c in cfgs)}")
    bt = mtp.Batch(cfgs, device="cuda:0")
    xp = bt.pack_x0(x0s)
    bt.replan(xp, shift=1)
    acts = bt.actions()
    for i in (0, 1, 5, 77, 128, 255):
        mu, sg, a, _ = standalone(cfgs[i], x0s[i], 1)
        b = bt.buffers(i)
        assert np.array_equal(b["mu"].cpu().numpy(), mu), cfgs[i].name
        assert np.array_equal(acts[i], a), cfgs[i].name
    bt.close()


def large_launch_mix():
    """Plans whose rollout launch fills the chip (at least one workgroup per
    compute unit), so the single plan uses the rollout build that targets the
    usual occupancy rather than the one-wave-per-SIMD build: quad-lane,
    one-lane, point-mass and pair-lane with replicas (not time-sliced)."""
    return [
        W.chain_config(name="L_c7", interp=W.AKIMA, n_tensor=19000, n_gauss=1001, horizon=12, n_elites=64,
                       n_iters=2, seed=31),
        W.chain_config(name="L_c2", n_links=2, n_tensor=68000, n_gauss=2000, horizon=8, n_layers=4, n_width=8,
                       n_elites=32, n_iters=2, seed=32),
        W.point_mass_config(name="L_pm", n_tensor=68000, n_gauss=2000, horizon=8, n_elites=32, n_iters=2,
                            seed=33),
        W.chain_contact_config(name="L_k24r2", n_tensor=34000, n_gauss=1000, horizon=6, n_elites=32, n_iters=2,
                               seed=34, n_replicas=2),
    ]


def test_large_launches_equal_the_batch():
    import torch
    import paper_2505_01059_amd as mtp
    cfgs = large_launch_mix()
    x0s = [W.initial_state(c, seed=40 + i) for i, c in enumerate(cfgs)]
    _log(f"[large launches] {[c.name for c in cfgs]}")
    bt = mtp.Batch(cfgs, device="cuda:0")
    bt.replan(bt.pack_x0(x0s), shift=1)
    acts = bt.actions()
    for i, c in enumerate(cfgs):
        p = mtp.Plan(c, device="cuda:0")
        p.replan(x0s[i], shift=1, replan_idx=0)
        torch.cuda.synchronize()
        b, bb = p.buffers(), bt.buffers(i)
        assert np.array_equal(bb["cost"].cpu().numpy(), b["cost"].cpu().numpy()), c.name
        assert np.array_equal(bb["mu"].cpu().numpy(), b["mu"].cpu().numpy()), c.name
        assert np.array_equal(bb["sigma"].cpu().numpy(), b["sigma"].cpu().numpy()), c.name
        assert np.array_equal(acts[i], p.action()), c.name
        p.close()
    bt.close()
