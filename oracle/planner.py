"""Model Tensor Planning, Alg. 2, one replan (oracle side, float64).

One CEM iteration k of replan r, in the paper's order:
  1. sample the graph Z (Def. 1) and P paths C (Alg. 1);
  2. interpolate them into U_G (Def. 2 B-spline or Def. 3 Akima);
  3. draw G-1 local samples U_L ~ N(mu, diag sigma^2);
  4. stack [U_L, U_G, mu] into U (B = P + G candidates), clipped to the box;
  5. roll out every candidate, S[b, t] per-step cost, s = sum_t S;
  6. top-E by ascending cost (ties broken by candidate index);
  7. softmax weights w = softmax(-s[iE] / lambda);
  8. mu' = w U[iE], sigma' = max(sqrt(w (U[iE] - mu')^2), sigma_min);
  9. mu <- mu' + alpha (mu - mu'), sigma <- sigma' + alpha (sigma - sigma').
The action is the first control of the best candidate of the last iteration.

Readings where the paper is silent (shared with the GPU path by
specification, not by code):
  * the candidate counts are given directly (P tensor, G local incl. nominal);
  * sigma' is a standard deviation (Tab. 3 lists sigma_min in the units of
    the noise std) with the softmax weights and no Bessel factor;
  * every candidate is clipped to [u_min, u_max] before the rollout and the
    refit uses the clipped controls;
  * a non-finite rollout cost counts as +inf; when even the best elite is
    +inf the weights fall back to uniform;
  * lambda = +inf means uniform weights;
  * warm start between replans shifts mu and sigma forward by `shift` steps,
    holding mu's last row and resetting sigma's tail to sigma_init.
"""
import numpy as np

from . import philox, sampling, interp, dynamics


def initial_distribution(cfg):
    T, n = cfg.horizon, cfg.ctrl_dim
    mid = 0.5 * (np.float64(cfg.u_min) + np.float64(cfg.u_max))
    return np.full((T, n), mid), np.full((T, n), np.float64(cfg.sigma_init))


def shift_distribution(mu, sigma, shift, sigma_init):
    if shift <= 0:
        return mu.copy(), sigma.copy()
    T = mu.shape[0]
    s = min(shift, T)
    mu2 = np.empty_like(mu)
    sg2 = np.empty_like(sigma)
    mu2[:T - s] = mu[s:]
    mu2[T - s:] = mu[T - 1]
    sg2[:T - s] = sigma[s:]
    sg2[T - s:] = np.float64(sigma_init)
    return mu2, sg2


def gaussian_noise(cfg, r, k):
    """eps[g, t, j] for the G-1 local samples (tag 3 stream, Box-Muller pairs)."""
    T, n, G = cfg.horizon, cfg.ctrl_dim, cfg.n_gauss
    n_loc = G - 1
    Tq = (T + 3) // 4
    words = philox.stream_words(cfg.seed, philox.TAG_EPS, r, k, np.arange(n_loc), n * Tq * 4)
    words = words.reshape(n_loc, n, Tq, 4)
    z0a, z1a = philox.box_muller(words[..., 0], words[..., 1])
    z0b, z1b = philox.box_muller(words[..., 2], words[..., 3])
    eps = np.stack([z0a, z1a, z0b, z1b], axis=-1).reshape(n_loc, n, Tq * 4)[:, :, :T]
    return np.transpose(eps, (0, 2, 1))                      # (G-1, T, n)


def tensor_samples(cfg, r, k):
    Z = sampling.waypoints(cfg.seed, r, k, cfg.n_layers, cfg.n_width, cfg.ctrl_dim,
                           cfg.u_min, cfg.u_max)
    if getattr(cfg, "sample_wor", 0):
        I = sampling.path_indices_without_replacement(cfg.seed, r, k, cfg.n_tensor, cfg.n_layers, cfg.n_width)
    else:
        I = sampling.path_indices(cfg.seed, r, k, cfg.n_tensor, cfg.n_layers, cfg.n_width)
    C = sampling.gather(Z, I).astype(np.float64)
    if cfg.interp == 0:
        UG = interp.bspline_interp(C, cfg.bspline_degree, cfg.horizon)
    elif cfg.interp == 1:
        UG = interp.akima_interp(C, cfg.horizon)
    else:
        UG = interp.linear_interp(C, cfg.horizon)
    return Z, I, UG


def candidates(cfg, mu, sigma, r, k):
    """U in R^{B x T x n}: [local 0..G-2 | tensor | nominal], clipped."""
    Z, I, UG = tensor_samples(cfg, r, k)
    eps = gaussian_noise(cfg, r, k)
    UL = mu[None] + sigma[None] * eps
    U = np.concatenate([UL, UG, mu[None]], axis=0)
    U = np.clip(U, np.float64(cfg.u_min), np.float64(cfg.u_max))
    return Z, I, U


def rollout(cfg, x0, U, sample_index=None, keep_states=False):
    """Costs s[b] = sum_t S[b, t]; optionally the states X[b, t] = x_{t+1}.

    With R > 1 randomised models (online domain randomisation, Section 4
    "Practical Settings") each candidate is rolled out under every model and
    its cost is the mean over the R rollouts; states are those of model 0."""
    R = int(getattr(cfg, "n_replicas", 1))
    if R > 1:
        B = cfg.n_samples
        idx = np.arange(U.shape[0]) if sample_index is None else np.asarray(sample_index)
        outs = [rollout(cfg.replace(n_replicas=1), x0, U, r * B + idx, keep_states and r == 0)
                for r in range(R)]
        if keep_states:
            s = sum(o[0] if isinstance(o, tuple) else o for o in outs) / R
            return np.where(np.isfinite(s), s, np.inf), outs[0][1]
        s = sum(outs) / R
        return np.where(np.isfinite(s), s, np.inf)
    model = dynamics.Model(cfg, sample_index)
    Bn = U.shape[0]
    x = np.broadcast_to(np.asarray(x0, np.float64), (Bn, len(x0))).copy()
    s = np.zeros(Bn)
    X = [] if keep_states else None
    for t in range(U.shape[1]):
        x = model.step(x, U[:, t, :])
        s = s + model.cost(x, U[:, t, :])
        if keep_states:
            X.append(x)
    s = np.where(np.isfinite(s), s, np.inf)
    if keep_states:
        return s, np.stack(X, axis=1)
    return s


def top_elites(s, n_elites):
    """Indices of the E lowest costs, ascending, ties broken by lower index."""
    s = np.where(np.isnan(s), np.inf, np.asarray(s, dtype=np.float64))
    order = np.lexsort((np.arange(len(s)), s))
    return order[:n_elites]


def softmax_weights(s_elite, temperature):
    s_elite = np.asarray(s_elite, dtype=np.float64)
    E = len(s_elite)
    if np.isinf(temperature) or not np.isfinite(s_elite[0]):
        return np.full(E, 1.0 / E)
    z = np.exp(-(s_elite - s_elite[0]) / np.float64(temperature))
    return z / np.sum(z)


def refit(U, s, iE, mu, sigma, cfg):
    """Alg. 2 weighted mean / std, sigma floor and smoothing."""
    w = softmax_weights(s[iE], float(cfg.temperature))
    Ue = U[iE]                                                  # (E, T, n)
    mu_new = np.tensordot(w, Ue, axes=1)
    var = np.tensordot(w, (Ue - mu_new[None]) ** 2, axes=1)
    sd_new = np.maximum(np.sqrt(var), np.float64(cfg.sigma_min))
    a = np.float64(cfg.smoothing)
    return mu_new + a * (mu - mu_new), sd_new + a * (sigma - sd_new), w


def cost_entropy(s):
    """Exploration diagnostic of Section 5.1: H = -sum_j P_j log P_j with
    P_j = exp(J_j) / sum_l exp(J_l) over the batch of rollout costs J (the sign
    as printed).  Non-finite costs are left out; no finite cost gives 0."""
    J = np.asarray(s, dtype=np.float64)
    J = J[np.isfinite(J)]
    if J.size == 0:
        return 0.0
    e = np.exp(J - J.max())
    Pj = e / e.sum()
    nz = Pj > 0
    return float(-np.sum(Pj[nz] * np.log(Pj[nz])))


def iterate(cfg, x0, mu, sigma, r, k, sample_index=None, keep_states=False):
    """One CEM iteration; returns every intermediate in a dict."""
    Z, I, U = candidates(cfg, mu, sigma, r, k)
    if keep_states:
        s, X = rollout(cfg, x0, U, None, True)
    else:
        s, X = rollout(cfg, x0, U), None
    iE = top_elites(s, cfg.n_elites)
    mu2, sg2, w = refit(U, s, iE, mu, sigma, cfg)
    return dict(Z=Z, I=I, U=U, s=s, X=X, iE=iE, w=w, mu=mu2, sigma=sg2,
                action=U[iE[0], 0, :].copy(), entropy=cost_entropy(s))


def replan(cfg, x0, mu, sigma, r, shift=1):
    """Alg. 2 loop body repeated for the configured number of iterations."""
    mu, sigma = shift_distribution(mu, sigma, shift, cfg.sigma_init)
    out = None
    for k in range(cfg.n_iters):
        out = iterate(cfg, x0, mu, sigma, r, k)
        mu, sigma = out["mu"], out["sigma"]
    return out["action"], mu, sigma, out
