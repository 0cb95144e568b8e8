#!/usr/bin/env python
"""Throughput of one MTP replan on one MI355X.

A step is one replan: n_iters CEM iterations of candidate generation (Philox
graph + paths + spline, Gaussian samples), fused rollout + cost, top-E and
softmax refit, replayed from a captured hipGraph with every input already in
HBM.  The default workload is the largest single-GPU configuration: the
24-link chain with ground contact and per-candidate domain randomisation
(69632 candidates = 65536 tensor + 4096 Gaussian, horizon 256, 12x64 graph,
512 elites, 6 iterations, cubic B-spline).  The 7-link chain (9216
candidates, horizon 128, Akima) is timed after it and reported under
"secondary".

Prints one JSON line:
  value        rollout steps/s = candidates x horizon x iterations per replan,
               times replans, over the wall time of the timed replans;
  roofline     the rollout kernel's algorithmic FP32 flops per launch over its
               mean launch time (HIP events around every rollout launch on the
               plan's stream, in a second timed pass launching kernels one by one);
  cpu_baseline the FP64 oracle on one CEM iteration of the workload (batches
               above 20000 candidates: a 1024-candidate subset), one thread;
               cpu_baseline_all_cores the same sample with its rollouts split
               over every host core.
"""
import argparse
import json
import os
import platform
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rollout steps/sec (samples x horizon) + replans/sec; p50/p99 replan latency"


def workloads():
    import mtp_workloads as W
    return {
        "chain7_akima": W.c1,
        "point_mass_bspline": W.c0,
        "chain24_contact_bspline": W.c4,
        "chain24_contact_share8": lambda: W.c4_share(8),
        "point_mass_paper": W.p0,
        "mix256": lambda: W.mix(256),
        "serve512": lambda: ("serve", W.robot_fleet(512)),
    }


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def kernel_sources_digest():
    """SHA-256 over the HIP sources of the library: a counter summary taken from
    other sources no longer describes the kernels that run."""
    import hashlib
    import glob
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_2505_01059_amd", "csrc", "*"))):
        if path.endswith((".hip", ".hpp", ".cpp")):
            with open(path, "rb") as f:
                h.update(os.path.basename(path).encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload):
    """HBM bytes per rollout launch from the committed PMC summary, if it was
    taken from the kernel sources that are built now (else None)."""
    path = os.path.join(ROOT, "profiles", f"rollout_{workload}_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha") != kernel_sources_digest():
        return None
    return rec.get("bytes_per_launch")


def baseline_sample(cfg):
    """The oracle's bounded sample: the whole batch, or for batches above 20000
    candidates the first 512 local samples, 511 tensor paths and the nominal
    (1024 candidates) at the same horizon and model."""
    import numpy as np
    if cfg.n_samples <= 20000:
        return cfg
    G = min(cfg.n_gauss, 513)
    sub = cfg.replace(n_tensor=1024 - G, n_gauss=G, n_elites=min(cfg.n_elites, 64))
    if cfg.sample_params is not None:
        B, R = cfg.n_samples, max(1, int(cfg.n_replicas))
        rows = [cfg.sample_params[r * B:r * B + sub.n_samples] for r in range(R)]
        sub = sub.replace(sample_params=np.concatenate(rows, axis=0))
    return sub


def cpu_baseline(cfg, x0, min_seconds=10.0, max_iters=100000):
    """Oracle (FP64 NumPy, as written) on CEM iterations of the same workload, one
    thread: whole iterations until at least min_seconds have passed."""
    from threadpoolctl import threadpool_limits
    from oracle import planner as OP
    mu, sg = OP.initial_distribution(cfg)
    sub = baseline_sample(cfg)
    iters = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while True:
            out = OP.iterate(sub, x0, mu, sg, 0, iters)
            mu, sg = out["mu"], out["sigma"]
            iters += 1
            dt = time.perf_counter() - t0
            if dt >= min_seconds or iters >= max_iters:
                break
    steps = sub.n_samples * sub.horizon * iters
    return {
        "value": steps / dt, "unit": "rollout steps/s", "cores": 1, "kind": "oracle",
        "sample": f"{iters} CEM iteration(s), {sub.n_samples} candidates x {sub.horizon} steps each "
                  f"(FP64 NumPy oracle, 1 thread, {dt:.1f} s; host {cpu_model()}, nproc {os.cpu_count()})",
    }


def _oracle_rollout_chunk(args):
    cfg, x0, U, idx = args
    from threadpoolctl import threadpool_limits
    from oracle import planner as OP
    with threadpool_limits(limits=1):
        return OP.rollout(cfg, x0, U, sample_index=idx)


def cpu_baseline_all_cores(cfg, x0):
    """The oracle's rollouts of one CEM iteration of the same sample, split over
    every host core (spawned worker processes, one thread each); candidates,
    top-E and refit stay in this process."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import planner as OP
    sub = baseline_sample(cfg)
    cores = os.cpu_count() or 1
    mu, sg = OP.initial_distribution(sub)
    parts = np.array_split(np.arange(sub.n_samples), cores)
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_oracle_rollout_chunk, [(sub, x0, np.zeros((1, 1, sub.ctrl_dim)), np.array([0]))] * cores))
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            _, _, U = OP.candidates(sub, mu, sg, 0, 0)
            s = np.concatenate(list(ex.map(_oracle_rollout_chunk, [(sub, x0, U[p], p) for p in parts])))
            iE = OP.top_elites(s, sub.n_elites)
            OP.refit(U, s, iE, mu, sg, sub)
            dt = time.perf_counter() - t0
    return {
        "value": sub.n_samples * sub.horizon / dt, "unit": "rollout steps/s", "cores": cores, "kind": "oracle",
        "sample": f"1 CEM iteration, {sub.n_samples} candidates x {sub.horizon} steps, rollouts split over "
                  f"{cores} processes ({dt:.1f} s; host {cpu_model()})",
    }


def copy_probe(mib, reps):
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings per dispatch
    give the factor that turns the counters into bytes."""
    import torch
    dev = torch.device("cuda:0")
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)                  # runtime copy (a blit kernel or a DMA engine)
        torch.neg(src, out=dst)         # elementwise kernel with a copy's traffic
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "reps": reps}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="chain24_contact_bspline", choices=sorted(workloads()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 7-link chain's extra keys")
    ap.add_argument("--tune-cache", default=None,
                    help="mix256: JSON schedule cache to read (and write after a search)")
    ap.add_argument("--rate", type=float, nargs="+", default=[2000.0],
                    help="serving: Poisson request rates (req/s) to run, one after another")
    ap.add_argument("--duration", type=float, default=20.0, help="serving: measured seconds per rate")
    ap.add_argument("--budget-gb", type=float, default=32.0, help="serving: device-memory budget of the pool")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run device-to-device copies of this many MiB (the reference kernel that "
                         "scales the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_probe_mib > 0:
        return copy_probe(args.copy_probe_mib, max(args.steps, 1))
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(instances shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import mtp_workloads as W

    cfg = workloads()[args.workload]()
    if isinstance(cfg, tuple):
        return bench_serve(args, cfg[1])
    if isinstance(cfg, list):
        return bench_mix(args, cfg)
    rec, plan_info = time_plan(cfg, args.workload, args.steps, args.warmup)
    out = {
        "metric": METRIC, "value": rec["rollout_steps_per_s"], "unit": "rollout steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["ms_per_replan"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": plan_info,
        "replans_per_s": rec["replans_per_s"],
        "latency_ms_p50": rec["latency_ms_p50"], "latency_ms_p99": rec["latency_ms_p99"],
        "stage_ms_per_launch": rec["stage_ms_per_launch"],
        "roofline": rec["roofline"],
    }
    if args.workload == "chain24_contact_bspline" and not args.no_secondary:
        # the 7-link chain of the other single-instance configuration, as extra keys
        sec, sec_info = time_plan(W.c1(), "chain7_akima", max(args.steps, 20), args.warmup)
        sec["config"] = sec_info
        out["secondary"] = {"chain7_akima": sec}
    if not args.no_cpu_baseline:
        x0 = W.initial_state(cfg)
        print("[bench] timing the oracle on the host (1 thread)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, x0)
        print("[bench] timing the oracle on the host (all cores)", file=sys.stderr, flush=True)
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(cfg, x0)
    print(json.dumps(out), flush=True)


def time_plan(cfg, name, steps, warmup):
    """Replans of one plan from its captured graph: wall-clock throughput, per-replan
    latency (replan + action read-back) and per-stage kernel times from HIP events."""
    import torch
    import mtp_workloads as W
    import paper_2505_01059_amd as mtp
    from paper_2505_01059_amd import roofline as RF
    x0 = W.initial_state(cfg)
    dev = torch.device("cuda:0")
    plan = mtp.Plan(cfg, device=dev)
    x0_dev = torch.tensor(x0, device=dev)
    B, T, K = cfg.n_samples, cfg.horizon, cfg.n_iters
    print(f"[bench] workload {name}: B={B} T={T} n={cfg.ctrl_dim} K={K}", file=sys.stderr, flush=True)

    for _ in range(warmup):
        plan.replan(x0_dev, shift=1)
    torch.cuda.synchronize()

    # timed region: back-to-back replans from the captured graph
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.replan(x0_dev, shift=1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / steps * 1e3
    print(f"[bench] {ms_per_step:.3f} ms/replan", file=sys.stderr, flush=True)

    # latency: submit a replan and wait for its action, per replan (one untimed
    # round first: the process's first read-back to host memory carries a
    # one-time set-up of tens of ms on a fresh box)
    plan.replan(x0_dev, shift=1)
    plan.action()
    # (enough samples that p99 is not simply the slowest one)
    lat = []
    for _ in range(max(steps, 200 if B * T < 10 ** 7 else 100)):
        t = time.perf_counter()
        plan.replan(x0_dev, shift=1)
        plan.action()
        lat.append((time.perf_counter() - t) * 1e3)
    lat.sort()
    p50 = statistics.median(lat)
    p99 = lat[min(len(lat) - 1, int(round(0.99 * (len(lat) - 1))))]

    # kernel timing pass: HIP events around every stage launch on the plan's stream
    plan.set_stage_timing(True)
    for _ in range(steps):
        plan.replan(x0_dev, shift=1)
    torch.cuda.synchronize()
    st = plan.stage_times()
    plan.set_stage_timing(False)
    roll_ms, roll_n = st["rollout"]
    roll_avg_ms = roll_ms / max(roll_n, 1)
    n_obs = len(cfg.task.obstacles) if cfg.dynamics == 0 else 0
    flops_step = RF.flops_per_sample_step(cfg.dynamics, cfg.n_links, n_obs)
    achieved = B * T * flops_step / (roll_avg_ms * 1e-3) / 1e12
    traffic = traffic_from_profiles(name)
    roofline = {
        "bound": "alu", "achieved": round(achieved, 3), "peak": RF.PEAK_FP32_VECTOR_TFLOPS,
        "unit": "TFLOP/s", "frac": round(achieved / RF.PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": traffic,
        "kernel": f"rollout ({'point mass' if cfg.dynamics == 0 else f'{cfg.n_links}-link chain'})",
        "flops_per_sample_step": flops_step, "launch_ms": round(roll_avg_ms, 4),
        "frac_of_unpacked_fp32": round(achieved / RF.PEAK_FP32_UNPACKED_TFLOPS, 4),
    }
    info = {"workload": name, "candidates": B, "tensor": cfg.n_tensor,
            "gaussian": cfg.n_gauss, "horizon": T, "ctrl_dim": cfg.ctrl_dim,
            "layers": cfg.n_layers, "width": cfg.n_width, "elites": cfg.n_elites,
            "iters": K, "interp": W.INTERP_NAMES[int(cfg.interp)],
            "overlap_tensor_paths": plan.draws_ahead()}
    rec = {"rollout_steps_per_s": B * T * K * steps / wall, "ms_per_replan": ms_per_step,
           "replans_per_s": steps / wall, "latency_ms_p50": round(p50, 4), "latency_ms_p99": round(p99, 4),
           "stage_ms_per_launch": {k: round(v[0] / max(v[1], 1), 4) for k, v in st.items()},
           "roofline": roofline}
    plan.close()
    return rec, info


def mix_flops(cfgs):
    from paper_2505_01059_amd import roofline as RF
    tot = 0
    for c in cfgs:
        n_obs = len(c.task.obstacles) if c.dynamics == 0 else 0
        tot += c.n_samples * c.horizon * c.n_iters * RF.flops_per_sample_step(c.dynamics, c.n_links, n_obs)
    return tot


def bench_mix(args, cfgs):
    """The uneven 256-instance mix: one persistent launch per replan of all instances,
    against the same instances replanned one plan at a time on one stream."""
    import torch
    import mtp_workloads as W
    import paper_2505_01059_amd as mtp
    from paper_2505_01059_amd import roofline as RF
    dev = torch.device("cuda:0")
    x0s = [W.initial_state(c, seed=i) for i, c in enumerate(cfgs)]
    steps_per_replan = sum(c.n_samples * c.horizon * c.n_iters for c in cfgs)
    bt = mtp.Batch(cfgs, device=dev)
    t_tune = time.perf_counter()
    sched, tune_ms, cached = bt.tune(reps=1, cache_path=args.tune_cache)
    t_tune = time.perf_counter() - t_tune
    print(f"[bench] schedule {sched} ({tune_ms:.2f} ms per replan, "
          f"{'from the cache' if cached else f'searched in {t_tune:.1f} s'})", file=sys.stderr, flush=True)
    xp = bt.pack_x0(x0s)
    for _ in range(args.warmup):
        bt.replan(xp, shift=1)
    bt.actions()
    stream = torch.cuda.current_stream(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        bt.replan(xp, shift=1)
        ev[i][1].record(stream)
    bt.actions()
    wall = time.perf_counter() - t0
    launch_ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    lat = []
    for _ in range(max(3, min(args.steps, 10))):
        t = time.perf_counter()
        bt.replan(xp, shift=1)
        bt.actions()
        lat.append((time.perf_counter() - t) * 1e3)
    bt.close()
    del bt
    torch.cuda.empty_cache()

    # per-instance plain launches: one plan per instance, replanned in turn on one stream
    plans = [mtp.Plan(c, device=dev) for c in cfgs]
    xs = [torch.tensor(x, device=dev) for x in x0s]
    for p, x in zip(plans, xs):
        p.replan(x, shift=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_steps = max(1, args.steps // 2)
    for _ in range(plain_steps):
        for p, x in zip(plans, xs):
            p.replan(x, shift=1)
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - t0
    # per-stage kernel time summed over all instances (one replan each, kernels one by one)
    stage_tot = {}
    for p, x in zip(plans, xs):
        p.set_stage_timing(True)
        p.replan(x, shift=1)
    torch.cuda.synchronize()
    for p in plans:
        for k_, (ms, n_) in p.stage_times().items():
            stage_tot[k_] = stage_tot.get(k_, 0.0) + ms
        p.set_stage_timing(False)
    for p in plans:
        p.close()

    value = steps_per_replan * args.steps / wall
    flops = mix_flops(cfgs)
    achieved = flops / (launch_ms * 1e-3) / 1e12
    lat.sort()
    out = {
        "metric": METRIC, "value": value, "unit": "rollout steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mix256", "instances": len(cfgs),
                   "candidates_total": sum(c.n_samples for c in cfgs),
                   "schedule": dict(sched, from_cache=cached)},
        "replans_per_s": len(cfgs) * args.steps / wall,
        "latency_ms_p50": round(statistics.median(lat), 3), "latency_ms_p99": round(lat[-1], 3),
        "plain_stage_ms_sum": {k_: round(v, 3) for k_, v in stage_tot.items()},
        "plain_launches": {"replans_per_s": len(cfgs) * plain_steps / plain_wall,
                           "rollout_steps_per_s": steps_per_replan * plain_steps / plain_wall,
                           "ms_per_round": plain_wall / plain_steps * 1e3},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": RF.PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / RF.PEAK_FP32_VECTOR_TFLOPS, 4),
                     "traffic": None, "kernel": "persistent batched replan (all stages, rollout flops)",
                     "launch_ms": round(launch_ms, 3)},
    }
    print(json.dumps(out), flush=True)


def bench_serve(args, robots):
    """Poisson replan requests from many robots through the continuous-batching
    server, in closed loop: every returned control moves its robot one step of
    its model (float64, on the host), and the robot's next request plans from
    the state it reached (the receding horizon of Alg. 2)."""
    import numpy as np
    import torch
    import mtp_workloads as W
    import paper_2505_01059_amd as mtp
    dev = torch.device("cuda:0")
    state = {i: W.initial_state(c, seed=i).astype(np.float64) for i, c in enumerate(robots)}
    budget = int(args.budget_gb * (1 << 30))
    srv = mtp.Server(budget, len(robots), iters_per_launch=1, max_inflight=2, device=dev, robots=robots)
    work = {i: c.n_samples * c.horizon * c.n_iters for i, c in enumerate(robots)}
    steps_taken = {i: 0 for i in range(len(robots))}

    def deliver(done):
        for d in done:
            r = d["robot"]
            state[r] = mtp.plant_step(robots[r], state[r], d["u"])
            steps_taken[r] += 1

    # warm up: one request per robot
    for i in range(len(robots)):
        srv.submit(i, state[i].astype(np.float32), shift=0)
    n = 0
    while n < len(robots):
        srv.pump(wait_us=1000)
        got = srv.poll()
        deliver(got)
        n += len(got)
    results = []
    for rate in args.rate:
        rng = np.random.Generator(np.random.PCG64(0))
        warm, dur = 2.0, float(args.duration)
        n_req = int(rate * (warm + dur) * 1.2) + 16
        gaps = rng.exponential(1.0 / rate, size=n_req)
        t_rel = np.cumsum(gaps)
        t_rel = t_rel[t_rel < warm + dur]
        who = rng.integers(0, len(robots), size=len(t_rel))
        t0 = srv.now_ns() + 1_000_000
        arrivals = (t0 + (t_rel * 1e9)).astype(np.int64)
        i_next = 0
        done = []
        print(f"[bench] serving {rate:.0f} req/s for {warm + dur:.0f} s ({len(arrivals)} requests)",
              file=sys.stderr, flush=True)
        t_stop = t0 + int((warm + dur) * 1e9)
        last_print = t0
        while True:
            now = srv.now_ns()
            while i_next < len(arrivals) and arrivals[i_next] <= now:
                r = int(who[i_next])
                srv.submit(r, state[r].astype(np.float32), shift=1, t_arrival_ns=int(arrivals[i_next]))
                i_next += 1
            srv.pump(wait_us=200)
            got = srv.poll()
            deliver(got)
            done += got
            if now - last_print > 2_000_000_000:
                st = srv.stats()
                print(f"[bench]   t={(now - t0) / 1e9:5.1f}s done={len(done)} queued={st['queued']} "
                      f"in_flight={st['in_flight']}", file=sys.stderr, flush=True)
                last_print = now
            if now >= t_stop:
                break
        st = srv.stats()
        meas = [d for d in done if d["t_arrival_ns"] >= t0 + int(warm * 1e9)]
        lat = np.array([(d["t_done_ns"] - d["t_arrival_ns"]) / 1e6 for d in meas]) if meas else np.array([np.nan])
        t_lo, t_hi = t0 + int(warm * 1e9), t_stop
        completed_in_window = [d for d in done if t_lo <= d["t_done_ns"] <= t_hi]
        rps = len(completed_in_window) / dur
        steps = sum(work[d["robot"]] for d in completed_in_window) / dur
        results.append({"offered_req_per_s": rate, "replans_per_s": rps, "rollout_steps_per_s": steps,
                        "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
                        "completed_measured": len(meas), "queued_at_end": st["queued"],
                        "pool_peak_gb": st["pool_peak"] / (1 << 30)})
        # drain what is left before the next rate
        while srv.stats()["queued"] + srv.stats()["in_flight"] > 0:
            srv.pump(wait_us=1000)
            deliver(srv.poll())
    main_r = results[0]
    out = {
        "metric": METRIC, "value": main_r["rollout_steps_per_s"], "unit": "rollout steps/s", "n_gpus": 1,
        "steps": len(args.rate), "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serve512", "robots": len(robots), "budget_gb": args.budget_gb,
                   "iters_per_launch": 1, "max_inflight": 2, "duration_s": args.duration,
                   "closed_loop": True},
        "replans_per_s": main_r["replans_per_s"], "latency_ms_p50": main_r["latency_ms_p50"],
        "latency_ms_p99": main_r["latency_ms_p99"], "load_sweep": results,
        "resident_mb": srv.stats()["resident_bytes"] / (1 << 20),
        "plant_steps_taken": int(sum(steps_taken.values())),
    }
    srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
