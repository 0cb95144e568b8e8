"""Pins for the oracle's Alg. 2 pieces: top-E, softmax refit, special cases that
reduce to textbook planners, brute-force path enumeration (CPU)."""
import itertools
import math

import numpy as np
import pytest

import mtp_workloads as W
from oracle import planner as P, sampling, interp, dynamics as D, philox


def small_pm(**kw):
    base = dict(horizon=20, n_layers=4, n_width=5, n_tensor=60, n_gauss=20,
                n_elites=8, n_iters=3, n_obstacles=5)
    base.update(kw)
    return W.point_mass_config(**base)


# ------------------------------------------------------------------ top-E

def test_top_elites_equals_brute_force_sort():
    rng = np.random.default_rng(0)
    s = np.round(rng.normal(size=500), 1)            # many exact ties
    s[[3, 17, 40]] = np.nan
    s[[5, 6]] = np.inf
    got = P.top_elites(s, 100)
    key = [((math.inf if math.isnan(v) else v), i) for i, v in enumerate(s)]
    want = [i for _, i in sorted(key)[:100]]
    assert list(got) == want


# ------------------------------------------------------------------ refit

def test_single_elite_is_predictive_sampling_corner():
    """E = 1 (PS corner of Fig. design ablation): mu' = best candidate, sigma' = sigma_min."""
    cfg = small_pm(n_elites=1)
    rng = np.random.default_rng(1)
    U = rng.uniform(-1, 1, size=(30, cfg.horizon, 2))
    s = rng.uniform(size=30)
    iE = P.top_elites(s, 1)
    mu, sg = P.initial_distribution(cfg)
    mu2, sg2, w = P.refit(U, s, iE, mu, sg, cfg)
    assert np.array_equal(mu2, U[np.argmin(s)])
    assert np.all(sg2 == np.float64(cfg.sigma_min))


def test_uniform_weights_give_cem_moments():
    """lambda = inf, sigma_min = 0, alpha = 0: plain elite mean, and the variance is
    (E-1)/E times the unbiased CEM estimate of Section 2.1."""
    cfg = small_pm(temperature=np.inf).replace(sigma_min=np.float32(0))
    rng = np.random.default_rng(2)
    U = rng.normal(size=(40, cfg.horizon, 2))
    s = rng.uniform(size=40)
    iE = P.top_elites(s, cfg.n_elites)
    mu, sg = P.initial_distribution(cfg)
    mu2, sg2, _ = P.refit(U, s, iE, mu, sg, cfg)
    E = cfg.n_elites
    elites = U[np.argsort(s)[:E]]
    np.testing.assert_allclose(mu2, elites.mean(0), atol=1e-14)
    np.testing.assert_allclose(sg2 ** 2, (E - 1) / E * elites.var(0, ddof=1), atol=1e-13)


def test_all_candidates_give_mppi_weighted_mean():
    """E = B: the update is the MPPI path-integral average over every candidate."""
    cfg = small_pm(temperature=0.5)
    rng = np.random.default_rng(3)
    B = 25
    cfg = cfg.replace(n_elites=B)
    U = rng.normal(size=(B, cfg.horizon, 2))
    s = rng.uniform(0, 3, size=B)
    mu, sg = P.initial_distribution(cfg)
    mu2, _, _ = P.refit(U, s, P.top_elites(s, B), mu, sg, cfg)
    w = np.exp(-s / 0.5)
    w /= w.sum()
    np.testing.assert_allclose(mu2, np.einsum("b,btn->tn", w, U), atol=1e-13)


def test_smoothing_closed_form():
    cfg = small_pm(smoothing=0.25)
    rng = np.random.default_rng(4)
    U = rng.normal(size=(30, cfg.horizon, 2))
    s = rng.uniform(size=30)
    mu = rng.normal(size=(cfg.horizon, 2))
    sg = rng.uniform(0.1, 1, size=(cfg.horizon, 2))
    a = np.float64(np.float32(0.25))
    mu2, sg2, _ = P.refit(U, s, P.top_elites(s, cfg.n_elites), mu, sg, cfg)
    mu0, sg0, _ = P.refit(U, s, P.top_elites(s, cfg.n_elites), mu, sg, cfg.replace(smoothing=np.float32(0)))
    np.testing.assert_allclose(mu2, a * mu + (1 - a) * mu0, atol=1e-14)
    np.testing.assert_allclose(sg2, a * sg + (1 - a) * sg0, atol=1e-14)


def test_softmax_weights_edge_cases():
    w = P.softmax_weights([1.0, 2.0, np.inf], 0.5)
    assert w[2] == 0.0 and w.sum() == pytest.approx(1.0)
    np.testing.assert_allclose(P.softmax_weights([np.inf, np.inf], 0.1), [0.5, 0.5])
    np.testing.assert_allclose(P.softmax_weights([1.0, 5.0, 9.0], np.inf), [1 / 3] * 3)


# ------------------------------------------------------------------ candidates

def test_zero_sigma_local_samples_equal_mean():
    cfg = small_pm()
    mu = np.random.default_rng(5).uniform(-0.5, 0.5, size=(cfg.horizon, 2))
    Z, I, U = P.candidates(cfg, mu, np.zeros_like(mu), 0, 0)
    G = cfg.n_gauss
    assert np.array_equal(U[:G - 1], np.broadcast_to(mu, (G - 1,) + mu.shape))
    assert np.array_equal(U[-1], mu)


def test_local_noise_moments():
    cfg = small_pm(n_gauss=2001, horizon=32)
    eps = P.gaussian_noise(cfg, 3, 1)
    assert eps.shape == (2000, 32, 2)
    assert abs(eps.mean()) < 0.01 and abs(eps.std() - 1) < 0.01


def test_candidate_layout_and_clip():
    cfg = small_pm()
    mu, sg = P.initial_distribution(cfg)
    sg = sg * 10                                           # force clipping of local samples
    Z, I, U = P.candidates(cfg, mu, sg, 2, 1)
    assert U.shape == (cfg.n_samples, cfg.horizon, 2)
    assert U.min() >= -1 and U.max() <= 1
    _, _, UG = P.tensor_samples(cfg, 2, 1)
    G = cfg.n_gauss
    np.testing.assert_array_equal(U[G - 1:G - 1 + cfg.n_tensor], np.clip(UG, -1, 1))


def test_shift_distribution():
    mu = np.arange(10.0).reshape(5, 2)
    sg = np.arange(10.0, 20.0).reshape(5, 2)
    m2, s2 = P.shift_distribution(mu, sg, 2, 0.5)
    np.testing.assert_array_equal(m2, [[4, 5], [6, 7], [8, 9], [8, 9], [8, 9]])
    np.testing.assert_array_equal(s2, [[14, 15], [16, 17], [18, 19], [.5, .5], [.5, .5]])
    m0, s0 = P.shift_distribution(mu, sg, 0, 0.5)
    np.testing.assert_array_equal(m0, mu)


# ------------------------------------------------------------------ brute force

@pytest.mark.parametrize("interp_kind", [W.BSPLINE, W.AKIMA])
def test_cost_is_a_function_of_the_enumerated_path(interp_kind):
    """Tiny graph: enumerate all W^L paths, roll each out with a scalar loop, and
    require every sampled tensor candidate's cost to equal table[path]."""
    cfg = small_pm(n_layers=4, n_width=3, n_tensor=200, n_gauss=4, interp=interp_kind,
                   horizon=16)
    x0 = W.initial_state(cfg)
    mu, sg = P.initial_distribution(cfg)
    r, k = 4, 2
    Z = sampling.waypoints(cfg.seed, r, k, 4, 3, 2, cfg.u_min, cfg.u_max).astype(np.float64)
    table = {}
    model = D.Model(cfg)
    for path in itertools.product(range(3), repeat=4):
        C = np.stack([Z[l, path[l]] for l in range(4)])[None]
        U = interp.bspline_interp(C, 3, 16) if interp_kind == W.BSPLINE else interp.akima_interp(C, 16)
        U = np.clip(U[0], -1, 1)
        x = np.asarray(x0, np.float64)
        cost = 0.0
        for t in range(16):
            x = D.point_mass_step(x, U[t], float(cfg.dt))
            cost += float(D.point_mass_cost(cfg.task, x, U[t]))
        table[path] = cost
    out = P.iterate(cfg, x0, mu, sg, r, k)
    G = cfg.n_gauss
    for p in range(cfg.n_tensor):
        assert out["s"][G - 1 + p] == pytest.approx(table[tuple(out["I"][p])], rel=1e-12, abs=1e-12)
    assert len({tuple(row) for row in out["I"]}) > 50


# ------------------------------------------------------------------ beta = 0 is CEM

def textbook_cem_iteration(cfg, x0, mu, sigma, eps, lam):
    """Section 2.1 CEM with softmax-weighted moments, written independently:
    sample mu + sigma*eps, add the nominal mean, roll out, keep the E best,
    weight them, refit mean and std with the floor."""
    cand = [np.clip(mu + sigma * e, cfg.u_min, cfg.u_max) for e in eps] + [np.clip(mu, cfg.u_min, cfg.u_max)]
    costs = []
    for u_seq in cand:
        x = np.asarray(x0, np.float64)
        c = 0.0
        for t in range(cfg.horizon):
            x = D.point_mass_step(x, u_seq[t], float(cfg.dt))
            c += float(D.point_mass_cost(cfg.task, x, u_seq[t]))
        costs.append(c)
    order = sorted(range(len(cand)), key=lambda i: (costs[i], i))[:cfg.n_elites]
    best = costs[order[0]]
    w = np.array([math.exp(-(costs[i] - best) / lam) for i in order])
    w = w / w.sum()
    new_mu = sum(wi * cand[i] for wi, i in zip(w, order))
    new_var = sum(wi * (cand[i] - new_mu) ** 2 for wi, i in zip(w, order))
    return new_mu, np.maximum(np.sqrt(new_var), float(cfg.sigma_min)), cand[order[0]][0]


def test_beta_zero_reduces_to_cem():
    """P = floor(0 * B) = 0 tensor paths: one MTP iteration is one CEM iteration."""
    cfg = small_pm(n_tensor=0, n_gauss=24, n_elites=6, horizon=12)
    x0 = W.initial_state(cfg)
    mu = np.random.default_rng(6).uniform(-0.3, 0.3, size=(12, 2))
    sg = np.full((12, 2), 0.4)
    out = P.iterate(cfg, x0, mu, sg, 7, 0)
    eps = P.gaussian_noise(cfg, 7, 0)
    m2, s2, a = textbook_cem_iteration(cfg, x0, mu, sg, eps, float(cfg.temperature))
    np.testing.assert_allclose(out["mu"], m2, atol=1e-12)
    np.testing.assert_allclose(out["sigma"], s2, atol=1e-12)
    np.testing.assert_allclose(out["action"], a, atol=1e-15)


# ------------------------------------------------------------------ coverage

def test_linear_path_coverage_improves_with_graph_size():
    """Thm. 1: min over graph paths of |u - g|_inf shrinks as the graph grows
    (linear interpolation between layer knots, tiny enumerable graphs)."""
    rng = np.random.default_rng(8)
    tgrid = np.linspace(0, 1, 200)
    u = 0.6 * np.sin(2 * np.pi * tgrid)
    def best_error(L, Wd, trials=4):
        errs = []
        for _ in range(trials):
            Z = rng.uniform(-1, 1, size=(L, Wd))
            knots = np.linspace(0, 1, L)
            # dynamic programming over layers is exact for the sup norm on linear pieces
            best = None
            for path in itertools.product(range(Wd), repeat=L):
                g = np.interp(tgrid, knots, Z[np.arange(L), path])
                e = np.max(np.abs(u - g))
                best = e if best is None else min(best, e)
            errs.append(best)
        return np.mean(errs)
    e1 = best_error(3, 3)
    e2 = best_error(5, 6)
    assert e2 < e1


# ------------------------------------------------------------------ randomised replicas

def _contact_small(R):
    return W.chain_contact_config(name="contact_r", n_links=4, n_tensor=10, n_gauss=6, horizon=12,
                                  n_layers=4, n_width=4, n_elites=4, n_iters=1, n_replicas=R)


def test_identical_replicas_reduce_to_single_model():
    """Online domain randomisation (Section 4): R copies of one model give that model's cost."""
    one = _contact_small(1)
    B = one.n_samples
    three = _contact_small(3).replace(sample_params=np.tile(one.sample_params, (3, 1)))
    U = np.random.default_rng(4).uniform(-2, 2, (B, one.horizon, one.ctrl_dim))
    x0 = W.initial_state(one)
    s1 = P.rollout(one, x0, U)
    s3 = P.rollout(three, x0, U)
    assert np.allclose(s3, s1, rtol=1e-13, atol=0)


def test_replica_mean_is_permutation_invariant_and_bracketed():
    """The averaged cost does not depend on the order of the R models, and lies
    between the smallest and largest single-model cost of each candidate."""
    cfg = _contact_small(3)
    B = cfg.n_samples
    U = np.random.default_rng(5).uniform(-2, 2, (B, cfg.horizon, cfg.ctrl_dim))
    x0 = W.initial_state(cfg)
    s = P.rollout(cfg, x0, U)
    blocks = cfg.sample_params.reshape(3, B, -1)
    perm = cfg.replace(sample_params=np.ascontiguousarray(blocks[[2, 0, 1]].reshape(3 * B, -1)))
    assert np.allclose(P.rollout(perm, x0, U), s, rtol=1e-13, atol=0)
    singles = np.stack([P.rollout(cfg.replace(n_replicas=1, sample_params=np.ascontiguousarray(blocks[r])), x0, U)
                        for r in range(3)])
    assert np.all(s >= singles.min(0) * (1 - 1e-12)) and np.all(s <= singles.max(0) * (1 + 1e-12))
    # the models differ, so the mean is not any one of them
    assert np.any(np.abs(singles[0] - s) > 1e-6 * np.abs(s))


# ------------------------------------------------------------------ cost entropy (Section 5.1)

def test_cost_entropy_closed_forms():
    from scipy import special, stats
    B = 37
    assert P.cost_entropy(np.full(B, 3.25)) == pytest.approx(math.log(B), rel=1e-14)
    # n1 costs at a, n2 at b: P = e^a / Z on n1 entries, e^b / Z on n2 entries
    n1, n2, a, b = 5, 11, 0.7, -1.3
    Z = n1 * math.exp(a) + n2 * math.exp(b)
    pa, pb = math.exp(a) / Z, math.exp(b) / Z
    H = -(n1 * pa * math.log(pa) + n2 * pb * math.log(pb))
    J = np.array([a] * n1 + [b] * n2)
    assert P.cost_entropy(J) == pytest.approx(H, rel=1e-13)
    J = np.random.default_rng(3).normal(0, 2, 500)
    assert P.cost_entropy(J) == pytest.approx(stats.entropy(special.softmax(J)), rel=1e-12)
    # shift invariance, non-finite costs left out, one dominant cost
    assert P.cost_entropy(J + 1e3) == pytest.approx(P.cost_entropy(J), rel=1e-10)
    assert P.cost_entropy(np.concatenate([J, [np.inf, np.nan]])) == pytest.approx(P.cost_entropy(J), rel=1e-14)
    assert P.cost_entropy(np.array([0.0, 800.0])) < 1e-300 + 1e-12
    assert P.cost_entropy(np.array([np.inf])) == 0.0
