"""Control-path interpolation (oracle side): B-spline and Akima spline.

B-spline (Eq. 3-4 and Def. 2).  The L sampled waypoints of a path are the
control points of a degree-p B-spline on the uniform knots t_i = i/(L+p+1),
i = 0..L+p.  Readings taken where the paper is loose:
  * the degree-0 indicator is half-open, [t_i, t_{i+1}), so the basis sums to
    one at knots as well (Eq. 3 writes a closed interval);
  * the horizon j = 0..T-1 is mapped onto the span where the basis is a
    partition of unity, [t_p, t_L), instead of t_j = j/T over the whole knot
    range, which would break the sum-to-one property Eq. 3 states.
B-splines are invariant under an affine change of parameter, so the
recursion below runs in knot-index units (knot i at i) and evaluates at
tau_j = p + (L - p) j / T.  Which half-open interval contains tau_j is
decided with integers, so knot hits are exact.

Linear paths (Section 3.1, "straight-line interpolation"; Thm. 1).  The L
waypoints sit on equally spaced knots t_i = i/(L-1) spanning [0, 1], as in the
statement of Thm. 1, and the path is sampled at t_j = j/T.

Akima spline (Eq. 5-7 and Def. 3).  Knots t_i = i/L for the L waypoints and
evaluation points t_j = j/T.  Slopes follow Eq. 6 with the paper's end rules;
when both weights of Eq. 6 vanish (e.g. on linear data) the slope is the mean
of the two neighbouring secants, Akima's own rule for that case.  Points past
the last knot use the last cubic piece (interval index capped at L-2).
"""
import numpy as np


# ---------------------------------------------------------------- B-spline

def bspline_span_index(n_ctrl, degree, horizon):
    """Index i with knot_i <= tau_j < knot_{i+1}, for every j (integer arithmetic)."""
    j = np.arange(horizon)
    return degree + ((n_ctrl - degree) * j) // horizon


def bspline_eval_points(n_ctrl, degree, horizon):
    j = np.arange(horizon, dtype=np.float64)
    return degree + (n_ctrl - degree) * j / horizon


def bspline_matrix(n_ctrl, degree, horizon):
    """B_p in R^{L x T}: element (i, j) = B_{i,p}(tau_j), by the Cox-de Boor recursion."""
    L, p, T = n_ctrl, degree, horizon
    if L < p + 1:
        raise ValueError("B-spline needs at least degree+1 control points")
    n_knots = L + p + 1
    knots = np.arange(n_knots, dtype=np.float64)
    tau = bspline_eval_points(L, p, T)
    span = bspline_span_index(L, p, T)
    # degree 0: indicator of the half-open interval [knot_i, knot_{i+1})
    B = np.zeros((n_knots - 1, T))
    B[span, np.arange(T)] = 1.0
    for q in range(1, p + 1):
        Bq = np.zeros((n_knots - 1 - q, T))
        for i in range(n_knots - 1 - q):
            left = (tau - knots[i]) / (knots[i + q] - knots[i]) * B[i]
            right = (knots[i + q + 1] - tau) / (knots[i + q + 1] - knots[i + 1]) * B[i + 1]
            Bq[i] = left + right
        B = Bq
    assert B.shape == (L, T)
    return B


def bspline_interp(C, degree, horizon):
    """Def. 2: U[b, t, :] = sum_l B_p[l, t] C[b, l, :]  (C: (P, L, n) -> U: (P, T, n))."""
    Bm = bspline_matrix(C.shape[1], degree, horizon)
    return np.einsum("lt,bln->btn", Bm, np.asarray(C, dtype=np.float64))


# ---------------------------------------------------------------- Akima

def akima_slopes(z, t):
    """Slopes s_i of Eq. 6 with the end rules of Section 2.2.

    z: (..., L, n) values at knots t (L,), returns (..., L, n)."""
    z = np.asarray(z, dtype=np.float64)
    L = z.shape[-2]
    if L < 2:
        raise ValueError("Akima needs at least two knots")
    h = np.diff(t).reshape((1,) * (z.ndim - 2) + (L - 1, 1))
    m = np.diff(z, axis=-2) / h                              # (..., L-1, n)
    s = np.empty_like(z)
    for i in range(L):
        if i == 0:
            s[..., i, :] = m[..., 0, :]
        elif i == L - 1:
            s[..., i, :] = m[..., L - 2, :]
        elif i == 1:
            s[..., i, :] = 0.5 * (m[..., 0, :] + m[..., 1, :])
        elif i == L - 2:
            s[..., i, :] = 0.5 * (m[..., L - 3, :] + m[..., L - 2, :])
        else:
            w1 = np.abs(m[..., i + 1, :] - m[..., i, :])
            w2 = np.abs(m[..., i - 1, :] - m[..., i - 2, :])
            den = w1 + w2
            safe = np.where(den == 0.0, 1.0, den)
            s[..., i, :] = np.where(den == 0.0,
                                    0.5 * (m[..., i - 1, :] + m[..., i, :]),
                                    (w1 * m[..., i - 1, :] + w2 * m[..., i, :]) / safe)
    return s


def akima_knots(n_ctrl):
    return np.arange(n_ctrl, dtype=np.float64) / n_ctrl


def akima_coefficients(C):
    """Def. 3: A in R^{P x (L-1) x 4 x n} holding (a, b, c, d) of Eq. 7 per interval."""
    C = np.asarray(C, dtype=np.float64)
    L = C.shape[1]
    t = akima_knots(L)
    s = akima_slopes(C, t)
    h = np.diff(t).reshape(1, L - 1, 1)
    m = np.diff(C, axis=1) / h
    a = C[:, :-1, :]
    b = s[:, :-1, :]
    c = (3.0 * m - 2.0 * s[:, :-1, :] - s[:, 1:, :]) / h
    d = (s[:, :-1, :] + s[:, 1:, :] - 2.0 * m) / h ** 2
    return np.stack([a, b, c, d], axis=2)


def akima_interval(n_ctrl, horizon):
    j = np.arange(horizon)
    return np.minimum((n_ctrl * j) // horizon, n_ctrl - 2)


def akima_eval(A, horizon):
    """Eq. 5 at t_j = j/T: u = d x^3 + c x^2 + b x + a with x = t_j - t_i."""
    L = A.shape[1] + 1
    t = akima_knots(L)
    i = akima_interval(L, horizon)
    x = (np.arange(horizon, dtype=np.float64) / horizon - t[i]).reshape(1, horizon, 1)
    a, b, c, d = (A[:, i, q, :] for q in range(4))
    return ((d * x + c) * x + b) * x + a


def akima_interp(C, horizon):
    return akima_eval(akima_coefficients(C), horizon)


# ---------------------------------------------------------------- linear

def linear_interp(C, horizon):
    """Piecewise-linear path through the waypoints (knots i/(L-1)) at t_j = j/T."""
    C = np.asarray(C, dtype=np.float64)
    P_, L, n = C.shape
    knots = np.linspace(0.0, 1.0, L)
    t = np.arange(horizon, dtype=np.float64) / horizon
    out = np.empty((P_, horizon, n))
    for p in range(P_):
        for j in range(n):
            out[p, :, j] = np.interp(t, knots, C[p, :, j])
    return out
