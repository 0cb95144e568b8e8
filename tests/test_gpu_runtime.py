"""Plan runtime on the GPU: graph replay against eager launches (with other
eager work between replays), determinism, checkpoint / resume, the warm-start
shift, the replan counter and non-finite start states."""
import numpy as np
import pytest

import mtp_workloads as W
from oracle import planner as OP

pytestmark = pytest.mark.gpu


def cfg_small(**kw):
    base = dict(n_tensor=300, n_gauss=45, horizon=37, n_layers=5, n_width=7, n_elites=20, n_iters=3)
    base.update(kw)
    return W.point_mass_config(**base)


def run(plan, x0, n, shift=1, between=None):
    import torch
    outs = []
    for r in range(n):
        plan.replan(x0, shift=shift)
        if between is not None:
            between()
        torch.cuda.synchronize()
        b = plan.buffers()
        outs.append((b["mu"].cpu().numpy().copy(), b["sigma"].cpu().numpy().copy(), plan.action()))
    return outs


@pytest.mark.parametrize("cfg", [cfg_small(), W.chain_config(n_tensor=500, n_gauss=76, horizon=40, n_elites=24,
                                                               n_iters=2)])
def test_graph_replays_equal_eager(cfg):
    import torch
    import paper_2505_01059_amd as mtp
    x0 = W.initial_state(cfg, seed=1)
    scratch = torch.zeros(1 << 20, device="cuda:0")

    def other_work():
        # unrelated eager work (fills, reductions over many blocks) between replays
        scratch.fill_(1.5)
        _ = scratch.sum().item()
        scratch.zero_()

    g = mtp.Plan(cfg, device="cuda:0", use_graph=True)
    e = mtp.Plan(cfg, device="cuda:0", use_graph=False)
    og = run(g, x0, 4, between=other_work)
    oe = run(e, x0, 4)
    for (m1, s1, a1), (m2, s2, a2) in zip(og, oe):
        assert np.array_equal(m1, m2) and np.array_equal(s1, s2) and np.array_equal(a1, a2)
    g.close()
    e.close()


def test_same_seed_same_bits_and_seed_matters():
    import paper_2505_01059_amd as mtp
    cfg = cfg_small()
    x0 = W.initial_state(cfg)
    a = run(mtp.Plan(cfg, device="cuda:0"), x0, 2)
    b = run(mtp.Plan(cfg, device="cuda:0"), x0, 2)
    c = run(mtp.Plan(cfg.replace(seed=12345), device="cuda:0"), x0, 2)
    assert all(np.array_equal(p[0], q[0]) for p, q in zip(a, b))
    assert not np.array_equal(a[-1][0], c[-1][0])


def test_checkpoint_resume_is_bit_identical():
    import paper_2505_01059_amd as mtp
    cfg = cfg_small()
    x0 = W.initial_state(cfg)
    full = mtp.Plan(cfg, device="cuda:0")
    ref = run(full, x0, 3)
    first = mtp.Plan(cfg, device="cuda:0")
    run(first, x0, 2)
    mu, sg, r = first.get_state()
    assert r == 2
    resumed = mtp.Plan(cfg, device="cuda:0")
    resumed.set_state(mu, sg, r)
    out = run(resumed, x0, 1)
    assert np.array_equal(out[0][0], ref[2][0]) and np.array_equal(out[0][2], ref[2][2])


@pytest.mark.parametrize("shift", [0, 1, 5, 100])
def test_warm_start_shift(shift):
    """With one iteration the nominal candidate is the shifted mean and the local
    samples are drawn around the shifted mean / std."""
    import torch
    import paper_2505_01059_amd as mtp
    cfg = cfg_small(n_iters=1)
    x0 = W.initial_state(cfg)
    rng = np.random.default_rng(shift)
    mu = rng.uniform(-0.5, 0.5, (cfg.horizon, 2)).astype(np.float32)
    sg = rng.uniform(0.1, 0.4, (cfg.horizon, 2)).astype(np.float32)
    p = mtp.Plan(cfg, device="cuda:0")
    p.set_state(mu, sg, 7)
    p.replan(x0, shift=shift)
    torch.cuda.synchronize()
    mu2, sg2 = OP.shift_distribution(mu.astype(np.float64), sg.astype(np.float64), shift, cfg.sigma_init)
    _, _, U_ref = OP.candidates(cfg, mu2, sg2, 7, 0)
    U = p.buffers()["U"].cpu().numpy().transpose(2, 0, 1)
    np.testing.assert_array_equal(U[-1], np.clip(mu2, -1, 1).astype(np.float32))
    G1 = cfg.n_gauss - 1
    assert np.max(np.abs(U[:G1] - U_ref[:G1])) < 1e-4
    assert p.get_state()[2] == 8


def test_non_finite_start_state_sets_flag():
    import torch
    import paper_2505_01059_amd as mtp
    cfg = cfg_small(n_iters=1)
    x0 = W.initial_state(cfg)
    x0[0] = np.nan
    p = mtp.Plan(cfg, device="cuda:0")
    p.replan(x0, shift=0)
    torch.cuda.synchronize()
    b = p.buffers()
    assert np.all(np.isinf(b["cost"].cpu().numpy()))
    assert p.flags() & 1
    np.testing.assert_allclose(b["weights"].cpu().numpy(), 1.0 / cfg.n_elites, rtol=1e-6)
    assert np.all(np.isfinite(b["mu"].cpu().numpy()))


def test_invalid_calls_raise_without_breaking_the_plan():
    import paper_2505_01059_amd as mtp
    from paper_2505_01059_amd import _native as N
    cfg = cfg_small()
    p = mtp.Plan(cfg, device="cuda:0")
    with pytest.raises(N.MtpError):
        p.run_stage(9, 0, 0)
    with pytest.raises(N.MtpError):
        p.replan(W.initial_state(cfg), shift=-1)
    p.replan(W.initial_state(cfg), shift=1)       # still usable
    assert np.all(np.isfinite(p.action()))
