"""The allocation-free replan (mtp_replan_noalloc, a static device scratch array)
against the ordinary plan entry point, through the C ABI: two calls in a row,
the second on a smaller problem, each bit-identical to a plan replanned from
the same warm start, start state, shift and replan index."""
import ctypes

import numpy as np
import pytest

import mtp_workloads as W

pytestmark = pytest.mark.gpu


def noalloc(lib, cfg, x0, mu, sg, shift, r):
    import torch
    from paper_2505_01059_amd import _native as N
    c, keep = N.config_struct(cfg)
    dev = torch.device("cuda:0")
    dx = torch.tensor(np.asarray(x0, np.float32), device=dev)
    dmu = torch.tensor(np.asarray(mu, np.float32), device=dev)
    dsg = torch.tensor(np.asarray(sg, np.float32), device=dev)
    act = torch.empty(cfg.ctrl_dim, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    st = lib.mtp_replan_noalloc(ctypes.byref(c), ctypes.c_void_p(dx.data_ptr()), ctypes.c_void_p(dmu.data_ptr()),
                                ctypes.c_void_p(dsg.data_ptr()), int(shift), int(r), ctypes.c_void_p(act.data_ptr()),
                                ctypes.c_void_p(stream.cuda_stream))
    assert st == 0, lib.mtp_status_str(st)
    torch.cuda.synchronize()
    return dmu.cpu().numpy(), dsg.cpu().numpy(), act.cpu().numpy()


def with_plan(cfg, x0, mu, sg, shift, r):
    import torch
    import paper_2505_01059_amd as mtp
    p = mtp.Plan(cfg, device="cuda:0")
    p.set_state(mu, sg, r)
    p.replan(x0, shift=shift, replan_idx=r)
    a = p.action()
    b = p.buffers()
    out = b["mu"].cpu().numpy().copy(), b["sigma"].cpu().numpy().copy(), a
    p.close()
    torch.cuda.synchronize()
    return out


def cases():
    big = W.chain_config(name="na_c7", n_tensor=3000, n_gauss=200, horizon=64, n_elites=64, n_iters=3, seed=41)
    small = W.point_mass_config(name="na_pm", n_tensor=300, n_gauss=45, horizon=37, n_layers=5, n_width=7,
                                n_elites=20, n_iters=2, seed=42)
    contact = W.chain_contact_config(name="na_k4", n_links=4, n_tensor=400, n_gauss=40, horizon=60, n_layers=6,
                                     n_width=12, n_elites=16, n_iters=2, ground_y=-0.5, seed=43)
    return big, small, contact


def test_noalloc_equals_plan_twice_in_a_row_second_smaller():
    import paper_2505_01059_amd as mtp
    lib = mtp.load()
    assert lib.mtp_noalloc_scratch_bytes() == 64 << 20
    rng = np.random.default_rng(5)
    for n, cfg in enumerate(cases()):
        um = float(cfg.u_max)
        mu = rng.uniform(-0.4 * um, 0.4 * um, (cfg.horizon, cfg.ctrl_dim)).astype(np.float32)
        sg = rng.uniform(0.1 * um, 0.5 * um, (cfg.horizon, cfg.ctrl_dim)).astype(np.float32)
        x0 = W.initial_state(cfg, seed=n)
        for shift, r in ((1, 3), (0, 4)):
            got = noalloc(lib, cfg, x0, mu, sg, shift, r)
            want = with_plan(cfg, x0, mu, sg, shift, r)
            for g, w, what in zip(got, want, ("mean", "std", "action")):
                assert np.array_equal(g, w), (cfg.name, shift, r, what)
        print(f"[noalloc] {cfg.name}: equal to the plan entry point", flush=True)
