"""Seeded synthetic workloads for one MTP replan.

This module only *generates inputs*: planner configurations, start states,
task tables (goals, obstacles, targets, link masses) and per-sample
domain-randomisation tables.  It holds none of the planning arithmetic, so
both the FP64 oracle and the GPU binding may import it.

The paper's experiments run MuJoCo-XLA tasks (Section 4, App. A.3); those
models are not available, so the analytic stand-ins below take their place:

* point mass   -- the Navigation task's planar point mass (state 4, control 2,
                  App. A.3), here a double integrator among circular obstacles;
* chain        -- planar n-link pendulum chain with joint torques;
* chain_contact-- the same chain with penalty-spring ground contact and
                  per-sample randomised link masses and friction (the paper's
                  online domain randomisation, Section 4 "Practical Settings").

All real-valued parameters are stored as float32 values because that is what
the GPU consumes; the oracle widens those exact values to float64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

POINT_MASS, CHAIN, CHAIN_CONTACT = 0, 1, 2
BSPLINE, AKIMA, LINEAR = 0, 1, 2

DYN_NAMES = {POINT_MASS: "point_mass", CHAIN: "chain", CHAIN_CONTACT: "chain_contact"}
INTERP_NAMES = {BSPLINE: "bspline", AKIMA: "akima", LINEAR: "linear"}

f32 = np.float32


@dataclasses.dataclass
class PointMassTask:
    goal: np.ndarray            # (2,) float32
    obstacles: np.ndarray       # (K, 3) float32: centre x, centre y, radius
    goal_weight: np.float32
    obstacle_penalty: np.float32
    ctrl_weight: np.float32


@dataclasses.dataclass
class ChainTask:
    gravity: np.float32
    masses: np.ndarray          # (n,) float32 (nominal; per-sample masses override with DR)
    lengths: np.ndarray         # (n,) float32
    target: np.ndarray          # (2,) float32 end-effector target
    goal_weight: np.float32
    ctrl_weight: np.float32
    # ground contact (chain_contact only)
    ground_y: np.float32 = f32(0.0)
    k_contact: np.float32 = f32(0.0)
    d_contact: np.float32 = f32(0.0)
    v_slip: np.float32 = f32(0.01)


@dataclasses.dataclass
class Config:
    """One MTP planner instance.  Field names follow the C ABI `mtp_config`.

    n_layers (L) is the graph depth and n_width (W) the waypoints per layer;
    the graph has W**L paths.  n_gauss (G) counts the local Gaussian samples
    *including* the nominal mean, so the batch is B = n_tensor + n_gauss.
    """
    name: str
    dynamics: int
    interp: int
    n_links: int
    state_dim: int
    ctrl_dim: int
    horizon: int
    n_layers: int
    n_width: int
    n_tensor: int
    n_gauss: int
    n_elites: int
    n_iters: int
    bspline_degree: int
    temperature: np.float32
    smoothing: np.float32
    sigma_min: np.float32
    sigma_init: np.float32
    u_min: np.float32
    u_max: np.float32
    dt: np.float32
    seed: int
    task: object
    sample_params: Optional[np.ndarray] = None   # (R*B, n+1) float32: link masses, friction
    n_replicas: int = 1                          # R randomised models per candidate (contact chain)
    sample_wor: int = 0                          # 1: tensor paths drawn without replacement
    diagnostics: int = 0                         # bit 0: record the cost entropy per iteration

    @property
    def n_samples(self) -> int:
        return self.n_tensor + self.n_gauss

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


# ----------------------------------------------------------------------------
# task generators
# ----------------------------------------------------------------------------

def point_mass_task(seed: int, n_obstacles: int = 20) -> PointMassTask:
    rng = np.random.default_rng(np.random.PCG64([seed, 4]))
    centres = rng.uniform(-1.0, 1.0, size=(n_obstacles, 2))
    radii = rng.uniform(0.05, 0.15, size=(n_obstacles, 1))
    obs = np.concatenate([centres, radii], axis=1).astype(f32)
    return PointMassTask(goal=np.array([0.8, 0.8], f32), obstacles=obs,
                         goal_weight=f32(1.0), obstacle_penalty=f32(1e3),
                         ctrl_weight=f32(1e-2))


def chain_task(seed: int, n_links: int) -> ChainTask:
    rng = np.random.default_rng(np.random.PCG64([seed, 4]))
    reach = float(n_links)
    rho = rng.uniform(0.2, 0.9) * reach
    theta = rng.uniform(0.0, 2.0 * math.pi)
    target = np.array([rho * math.cos(theta), rho * math.sin(theta)], f32)
    return ChainTask(gravity=f32(9.81), masses=np.ones(n_links, f32),
                     lengths=np.ones(n_links, f32), target=target,
                     goal_weight=f32(1.0), ctrl_weight=f32(1e-3))


def chain_contact_task(seed: int, n_links: int, ground_y: float = -4.0) -> ChainTask:
    rng = np.random.default_rng(np.random.PCG64([seed, 4]))
    ground = float(ground_y)
    target = np.array([rng.uniform(-0.5, 0.5) * n_links,
                       rng.uniform(ground + 1.0, ground + 5.0)], f32)
    return ChainTask(gravity=f32(9.81), masses=np.ones(n_links, f32),
                     lengths=np.ones(n_links, f32), target=target,
                     goal_weight=f32(1.0), ctrl_weight=f32(1e-3),
                     ground_y=f32(ground), k_contact=f32(1e4), d_contact=f32(50.0),
                     v_slip=f32(0.01))


def domain_randomisation(seed: int, n_samples: int, n_links: int,
                         nominal_masses: np.ndarray) -> np.ndarray:
    """Per-sample link masses (nominal x U[0.8,1.2]) and friction U[0.5,1.5]."""
    rng = np.random.default_rng(np.random.PCG64([seed, 5]))
    scale = rng.uniform(0.8, 1.2, size=(n_samples, n_links))
    mu_f = rng.uniform(0.5, 1.5, size=(n_samples, 1))
    masses = scale * nominal_masses[None, :].astype(np.float64)
    return np.concatenate([masses, mu_f], axis=1).astype(f32)


# ----------------------------------------------------------------------------
# start states
# ----------------------------------------------------------------------------

def initial_state(cfg: Config, seed: Optional[int] = None) -> np.ndarray:
    """Start state x0 (float32).  seed=None gives the canonical start."""
    if cfg.dynamics == POINT_MASS:
        x = np.array([-0.8, -0.8, 0.0, 0.0], f32)
        if seed is not None:
            rng = np.random.default_rng(np.random.PCG64([seed, 6]))
            x[:2] += rng.uniform(-0.1, 0.1, size=2).astype(f32)
        return x
    n = cfg.n_links
    if cfg.dynamics == CHAIN_CONTACT:
        phi = np.full(n, math.pi / 2, f32)          # horizontal, at rest
    else:
        phi = np.zeros(n, f32)                      # hanging, at rest
    if seed is not None:
        rng = np.random.default_rng(np.random.PCG64([seed, 6]))
        phi = (phi + rng.uniform(-0.3, 0.3, size=n)).astype(f32)
    return np.concatenate([phi, np.zeros(n, f32)]).astype(f32)


# ----------------------------------------------------------------------------
# named configurations
# ----------------------------------------------------------------------------

def point_mass_config(name="point_mass_c0", *, horizon=50, n_layers=4, n_width=8,
                      n_tensor=256, n_gauss=32, n_elites=16, n_iters=10,
                      interp=BSPLINE, bspline_degree=3, seed=0, temperature=0.1,
                      smoothing=0.0, dt=0.01, n_obstacles=20) -> Config:
    return Config(name=name, dynamics=POINT_MASS, interp=interp, n_links=0,
                  state_dim=4, ctrl_dim=2, horizon=horizon, n_layers=n_layers,
                  n_width=n_width, n_tensor=n_tensor, n_gauss=n_gauss,
                  n_elites=n_elites, n_iters=n_iters, bspline_degree=bspline_degree,
                  temperature=f32(temperature), smoothing=f32(smoothing),
                  sigma_min=f32(0.05), sigma_init=f32(0.5), u_min=f32(-1.0),
                  u_max=f32(1.0), dt=f32(dt), seed=seed,
                  task=point_mass_task(seed, n_obstacles))


def chain_config(name="chain7_c1", *, n_links=7, horizon=128, n_layers=8, n_width=32,
                 n_tensor=8192, n_gauss=1024, n_elites=128, n_iters=8, interp=AKIMA,
                 bspline_degree=3, seed=0, temperature=0.1, smoothing=0.0,
                 dt=0.005, u_max=5.0) -> Config:
    return Config(name=name, dynamics=CHAIN, interp=interp, n_links=n_links,
                  state_dim=2 * n_links, ctrl_dim=n_links, horizon=horizon,
                  n_layers=n_layers, n_width=n_width, n_tensor=n_tensor,
                  n_gauss=n_gauss, n_elites=n_elites, n_iters=n_iters,
                  bspline_degree=bspline_degree, temperature=f32(temperature),
                  smoothing=f32(smoothing), sigma_min=f32(0.05 * u_max),
                  sigma_init=f32(0.5 * u_max), u_min=f32(-u_max), u_max=f32(u_max),
                  dt=f32(dt), seed=seed, task=chain_task(seed, n_links))


def chain_contact_config(name="chain24_contact_c4", *, n_links=24, horizon=256,
                         n_layers=12, n_width=64, n_tensor=65536, n_gauss=4096,
                         n_elites=512, n_iters=6, interp=BSPLINE, bspline_degree=3,
                         seed=0, temperature=0.1, smoothing=0.0, dt=0.005,
                         u_max=5.0, n_replicas=1, ground_y=-4.0) -> Config:
    """Contact chain; with n_replicas = R every candidate is rolled out under R
    randomised models (rows r*B + b of sample_params) and its cost averaged.
    ground_y is the ground height below the pinned base (the workload's -4 m;
    a raised ground lets short horizons reach it)."""
    task = chain_contact_task(seed, n_links, ground_y)
    B = n_tensor + n_gauss
    return Config(name=name, dynamics=CHAIN_CONTACT, interp=interp, n_links=n_links,
                  state_dim=2 * n_links, ctrl_dim=n_links, horizon=horizon,
                  n_layers=n_layers, n_width=n_width, n_tensor=n_tensor,
                  n_gauss=n_gauss, n_elites=n_elites, n_iters=n_iters,
                  bspline_degree=bspline_degree, temperature=f32(temperature),
                  smoothing=f32(smoothing), sigma_min=f32(0.05 * u_max),
                  sigma_init=f32(0.5 * u_max), u_min=f32(-u_max), u_max=f32(u_max),
                  dt=f32(dt), seed=seed, task=task,
                  sample_params=domain_randomisation(seed, n_replicas * B, n_links, task.masses),
                  n_replicas=n_replicas)


def c0() -> Config:
    """Point mass, 4x8 graph, 256 tensor + 32 Gaussian, cubic B-spline, T=50."""
    return point_mass_config()


def c1() -> Config:
    """7-link chain, 8x32 graph, 8192 tensor + 1024 Gaussian, Akima, T=128."""
    return chain_config()


def c4() -> Config:
    """24-link chain with contact and per-sample DR, 12x64 graph, 65536 + 4096."""
    return chain_contact_config()


def c4_share(n_gpus: int = 8) -> Config:
    """One GPU's share of the 24-link contact chain split over n_gpus: B/n_gpus
    candidates (tensor and Gaussian counts both divided) at the same T, n, L, W."""
    full = chain_contact_config()
    return chain_contact_config(name=f"chain24_contact_share{n_gpus}", n_tensor=full.n_tensor // n_gpus,
                                n_gauss=full.n_gauss // n_gpus, n_elites=full.n_elites)


def p0() -> Config:
    """Point mass at the sizes of the paper's Navigation runs (Section 5.1, Tab. 3):
    B = 256 all from the tensor (beta = 1, the nominal kept as the one Gaussian
    slot), L = 5, W = 30, T = 20, dt = 0.05."""
    return point_mass_config(name="point_mass_paper", n_tensor=255, n_gauss=1, n_layers=5, n_width=30,
                             horizon=20, dt=0.05, n_elites=16, n_iters=10)


def mix_instance(seed: int) -> Config:
    """One instance of the uneven batching mix (256 of these form the batch).

    samples log-uniform in [1024, 16384]; horizon in {32,64,128,256}; control
    dim in {2, 7, 12, 24} (point mass or 7/12/24-link chain); graph depth
    uniform 4..12 and width uniform 8..64; tensor/Gaussian split 8:1;
    cubic B-spline for even seeds, Akima for odd seeds.
    """
    rng = np.random.default_rng(np.random.PCG64([seed, 7]))
    B = int(round(math.exp(rng.uniform(math.log(1024), math.log(16384)))))
    T = int(rng.choice([32, 64, 128, 256]))
    n = int(rng.choice([2, 7, 12, 24]))
    L = int(rng.integers(4, 13))
    W = int(rng.integers(8, 65))
    P = (8 * B) // 9
    G = B - P
    E = int(min(max(B // 64, 16), 256))
    interp = BSPLINE if seed % 2 == 0 else AKIMA
    common = dict(horizon=T, n_layers=L, n_width=W, n_tensor=P, n_gauss=G,
                  n_elites=E, n_iters=6, interp=interp, seed=seed)
    if n == 2:
        return point_mass_config(name=f"mix{seed}_pm", **common)
    return chain_config(name=f"mix{seed}_chain{n}", n_links=n, **common)


def mix(n_instances: int = 256, base_seed: int = 0) -> list:
    return [mix_instance(base_seed + i) for i in range(n_instances)]


def robot_fleet(n_robots: int = 512) -> list:
    """Robots of the serving workload: robot r is the mix instance of seed 10000+r."""
    return [mix_instance(10000 + r) for r in range(n_robots)]
