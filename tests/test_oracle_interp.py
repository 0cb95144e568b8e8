"""Pins for the oracle's B-spline (Eq. 3-4, Def. 2) and Akima (Eq. 5-7, Def. 3) code."""
import numpy as np
import pytest
from scipy.interpolate import BSpline, Akima1DInterpolator

from oracle import interp


@pytest.mark.parametrize("L,p,T", [(4, 3, 50), (12, 3, 256), (8, 2, 128), (5, 1, 20), (9, 5, 64), (4, 3, 7)])
def test_bspline_partition_of_unity_and_support(L, p, T):
    B = interp.bspline_matrix(L, p, T)
    assert B.shape == (L, T)
    np.testing.assert_allclose(B.sum(axis=0), 1.0, atol=1e-14)     # Eq. 3 side condition
    assert B.min() >= -1e-15
    nnz = (np.abs(B) > 1e-15).sum(axis=0)
    assert np.all(nnz <= p + 1)


@pytest.mark.parametrize("L,p,T", [(4, 3, 50), (12, 3, 256), (8, 2, 33), (6, 4, 40)])
def test_bspline_matches_scipy_design_matrix(L, p, T):
    knots = np.arange(L + p + 1, dtype=np.float64)
    tau = interp.bspline_eval_points(L, p, T)
    D = BSpline.design_matrix(tau, knots, p).toarray()             # (T, L)
    np.testing.assert_allclose(interp.bspline_matrix(L, p, T), D.T, atol=1e-14)


def test_bspline_uniform_cubic_closed_form():
    """On every span the uniform cubic basis is ((1-x)^3, 3x^3-6x^2+4, -3x^3+3x^2+3x+1, x^3)/6."""
    L, p, T = 12, 3, 256
    B = interp.bspline_matrix(L, p, T)
    span = interp.bspline_span_index(L, p, T)
    x = interp.bspline_eval_points(L, p, T) - span
    blend = np.stack([(1 - x) ** 3, 3 * x ** 3 - 6 * x ** 2 + 4,
                      -3 * x ** 3 + 3 * x ** 2 + 3 * x + 1, x ** 3]) / 6.0
    for j in range(T):
        np.testing.assert_allclose(B[span[j] - 3:span[j] + 1, j], blend[:, j], atol=1e-14)


def test_bspline_reproduces_constants_and_lines():
    L, p, T = 7, 3, 64
    C = np.ones((1, L, 1)) * 0.37
    np.testing.assert_allclose(interp.bspline_interp(C, p, T), 0.37, atol=1e-14)
    # control points affine in their index give a trajectory affine in tau (Greville abscissae)
    a, b = 0.25, -0.1
    grev = np.array([(i + 1 + i + 2 + i + 3) / 3.0 for i in range(L)])
    C = (a + b * grev).reshape(1, L, 1)
    tau = interp.bspline_eval_points(L, p, T)
    np.testing.assert_allclose(interp.bspline_interp(C, p, T)[0, :, 0], a + b * tau, atol=1e-13)


def test_bspline_convex_hull():
    rng = np.random.default_rng(0)
    C = rng.uniform(-1, 1, size=(50, 6, 3))
    U = interp.bspline_interp(C, 3, 40)
    assert U.max() <= C.max() + 1e-14 and U.min() >= C.min() - 1e-14


def test_bspline_rejects_too_few_points():
    with pytest.raises(ValueError):
        interp.bspline_matrix(3, 3, 10)


def test_akima_passes_through_knots():
    """Akima interpolates its waypoints (Section 2.2): at grid points that are knots."""
    L, T = 8, 128                                                    # knots at j = 16 i
    rng = np.random.default_rng(1)
    C = rng.uniform(-5, 5, size=(20, L, 3))
    U = interp.akima_interp(C, T)
    for i in range(L):
        np.testing.assert_allclose(U[:, 16 * i, :], C[:, i, :], atol=1e-12)


def test_akima_exact_on_linear_data():
    """Linear data: every slope equals the secant, so c = d = 0 in Eq. 7."""
    L, T = 6, 60
    t = interp.akima_knots(L)
    C = (0.3 - 1.7 * t).reshape(1, L, 1)
    A = interp.akima_coefficients(C)
    np.testing.assert_allclose(A[0, :, 2:, 0], 0.0, atol=1e-12)
    U = interp.akima_interp(C, T)
    np.testing.assert_allclose(U[0, :, 0], 0.3 - 1.7 * np.arange(T) / T, atol=1e-12)


def test_akima_c1_at_interior_knots():
    L = 7
    rng = np.random.default_rng(2)
    C = rng.uniform(-1, 1, size=(10, L, 2))
    A = interp.akima_coefficients(C)
    h = 1.0 / L
    for i in range(L - 2):
        a, b, c, d = (A[:, i, q] for q in range(4))
        val = ((d * h + c) * h + b) * h + a
        der = (3 * d * h + 2 * c) * h + b
        np.testing.assert_allclose(val, A[:, i + 1, 0], atol=1e-12)
        np.testing.assert_allclose(der, A[:, i + 1, 1], atol=1e-10)


def test_akima_end_slopes():
    L = 6
    rng = np.random.default_rng(3)
    z = rng.uniform(-1, 1, size=(1, L, 1))
    t = interp.akima_knots(L)
    s = interp.akima_slopes(z, t)[0, :, 0]
    m = np.diff(z[0, :, 0]) / np.diff(t)
    assert s[0] == pytest.approx(m[0])
    assert s[1] == pytest.approx(0.5 * (m[0] + m[1]))
    assert s[L - 2] == pytest.approx(0.5 * (m[L - 3] + m[L - 2]))
    assert s[L - 1] == pytest.approx(m[L - 2])


@pytest.mark.parametrize("L", [6, 8, 12])
def test_akima_interior_slopes_match_scipy(L):
    rng = np.random.default_rng(L)
    t = interp.akima_knots(L)
    z = rng.uniform(-1, 1, size=L)
    s = interp.akima_slopes(z.reshape(1, L, 1), t)[0, :, 0]
    ref = Akima1DInterpolator(t, z, method="akima").derivative()(t)
    np.testing.assert_allclose(s[2:L - 2], ref[2:L - 2], atol=1e-12)


def test_akima_zero_weights_rule():
    """Both Eq. 6 weights vanish: the slope is the mean of the neighbouring secants."""
    L = 6
    t = interp.akima_knots(L)
    z = np.array([0.0, 1.0, 2.0, 3.0, 3.5, 4.0]) / L                # m = 1,1,1,.5,.5
    s = interp.akima_slopes(z.reshape(1, L, 1), t)[0, :, 0]
    m = np.diff(z) / np.diff(t)
    # i = 2: w1 = |m3 - m2| = .5, w2 = |m1 - m0| = 0 -> slope m1
    assert s[2] == pytest.approx(m[1])
    z2 = np.array([0.0, 1.0, 2.0, 3.0, 4.0, 5.0])
    s2 = interp.akima_slopes(z2.reshape(1, L, 1), t)[0, :, 0]
    np.testing.assert_allclose(s2, L * 1.0)


def test_akima_small_L():
    t = interp.akima_knots(2)
    z = np.array([[[0.0], [1.0]]])
    np.testing.assert_allclose(interp.akima_interp(z, 10)[0, :, 0], np.arange(10) / 10 * 2)


def test_linear_paths_through_waypoints_and_straight_between():
    """Thm. 1's straight-line paths: waypoints on equally spaced knots over [0, 1]."""
    L, T = 5, 64                     # knots at j = 16 i
    rng = np.random.default_rng(9)
    C = rng.uniform(-1, 1, size=(7, L, 2))
    U = interp.linear_interp(C, T)
    for i in range(L - 1):
        np.testing.assert_allclose(U[:, 16 * i], C[:, i], atol=1e-14)
        seg = U[:, 16 * i:16 * (i + 1)]
        np.testing.assert_allclose(np.diff(seg, 2, axis=1), 0.0, atol=1e-13)
    np.testing.assert_allclose(U[:, 63], C[:, 3] + (C[:, 4] - C[:, 3]) * 15 / 16, atol=1e-14)
