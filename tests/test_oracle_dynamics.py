"""Pins for the oracle's dynamics and costs: closed forms, textbook special cases,
invariants (CPU)."""
import math

import numpy as np
import pytest

import mtp_workloads as W
from oracle import dynamics as D


def chain(n, masses=None, lengths=None, g=9.81):
    t = W.chain_task(0, n)
    if masses is not None:
        t.masses = np.asarray(masses, np.float32)
    if lengths is not None:
        t.lengths = np.asarray(lengths, np.float32)
    t.gravity = np.float32(g)
    return t


# ------------------------------------------------------------------ point mass

def test_point_mass_semi_implicit_euler_closed_form():
    rng = np.random.default_rng(0)
    x0 = np.array([0.1, -0.2, 0.3, 0.05])
    U = rng.uniform(-1, 1, size=(40, 2))
    dt = 0.01
    x = x0.copy()
    for u in U:
        x = D.point_mass_step(x, u, dt)
    v = x0[2:] + dt * U.sum(0)
    # p_T = p0 + dt * sum_{t=1..T} v_t with v_t = v0 + dt sum_{k<t} u_k
    vt = x0[2:] + dt * np.cumsum(U, axis=0)
    p = x0[:2] + dt * vt.sum(0)
    np.testing.assert_allclose(x[2:], v, atol=1e-14)
    np.testing.assert_allclose(x[:2], p, atol=1e-14)
    # constant control: p_T = p0 + T dt v0 + dt^2 u T(T+1)/2
    u = np.array([0.4, -0.7]); T = 25
    x = x0.copy()
    for _ in range(T):
        x = D.point_mass_step(x, u, dt)
    np.testing.assert_allclose(x[:2], x0[:2] + T * dt * x0[2:] + dt * dt * u * T * (T + 1) / 2, atol=1e-14)


def test_point_mass_cost_terms():
    task = W.point_mass_task(0)
    task.obstacles = np.array([[0.0, 0.0, 0.5], [0.1, 0.0, 0.5]], np.float32)
    x = np.array([[0.0, 0.0, 0, 0], [0.45, 0.0, 0, 0], [0.7, 0.0, 0, 0]])
    u = np.array([[1.0, 0.0]] * 3)
    c = D.point_mass_cost(task, x, u)
    base = np.sum((x[:, :2] - task.goal.astype(np.float64)) ** 2, axis=1) + 1e-2
    np.testing.assert_allclose(c - base, [2000.0, 2000.0, 0.0], atol=1e-6)  # overlapping obstacles add


# ------------------------------------------------------------------ chain

def test_single_pendulum_reduces_to_textbook():
    t = chain(1, masses=[2.0], lengths=[1.5], g=9.81)
    rng = np.random.default_rng(1)
    for _ in range(10):
        phi, dphi, tau = rng.uniform(-3, 3, 3)
        a = D.chain_accel(np.array([phi, dphi]), np.array([tau]), t, t.masses.astype(np.float64))
        want = -(float(t.gravity) / 1.5) * math.sin(phi) + tau / (2.0 * 1.5 ** 2)
        assert a[0] == pytest.approx(dphi) and a[1] == pytest.approx(want, rel=1e-12)


def test_double_pendulum_reduces_to_textbook():
    """Lagrange equations of the double pendulum written out by hand (no torque)."""
    t = chain(2, masses=[1.3, 0.7], lengths=[1.1, 0.9], g=9.81)
    (m1, m2), (l1, l2), g = map(float, t.masses), map(float, t.lengths), float(t.gravity)
    rng = np.random.default_rng(2)
    for _ in range(10):
        p1, p2, w1, w2 = rng.uniform(-3, 3, 4)
        a = D.chain_accel(np.array([p1, p2, w1, w2]), np.zeros(2), t, np.array([m1, m2]))
        d = p1 - p2
        den = 2 * m1 + m2 - m2 * math.cos(2 * d)
        a1 = (-g * (2 * m1 + m2) * math.sin(p1) - m2 * g * math.sin(p1 - 2 * p2)
              - 2 * math.sin(d) * m2 * (w2 ** 2 * l2 + w1 ** 2 * l1 * math.cos(d))) / (l1 * den)
        a2 = (2 * math.sin(d) * (w1 ** 2 * l1 * (m1 + m2) + g * (m1 + m2) * math.cos(p1)
              + w2 ** 2 * l2 * m2 * math.cos(d))) / (l2 * den)
        assert a[2] == pytest.approx(a1, rel=1e-10, abs=1e-12)
        assert a[3] == pytest.approx(a2, rel=1e-10, abs=1e-12)


def test_mass_matrix_is_kinetic_energy_hessian():
    n = 5
    rng = np.random.default_rng(3)
    t = chain(n, masses=rng.uniform(0.5, 2, n), lengths=rng.uniform(0.5, 1.5, n))
    m = t.masses.astype(np.float64)
    phi = rng.uniform(-3, 3, n)
    M = D.chain_mass_matrix(phi, m, t.lengths.astype(np.float64))
    assert np.allclose(M, M.T)
    assert np.all(np.linalg.eigvalsh(M) > 0)
    def ke(dphi):
        return D.chain_energy(np.concatenate([phi, dphi]), t, m) - D.chain_energy(
            np.concatenate([phi, np.zeros(n)]), t, m)
    h = 1e-3
    H = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            ei, ej = np.eye(n)[i] * h, np.eye(n)[j] * h
            H[i, j] = (ke(ei + ej) - ke(ei - ej) - ke(-ei + ej) + ke(-ei - ej)) / (4 * h * h)
    np.testing.assert_allclose(H, M, atol=1e-6)


@pytest.mark.parametrize("n", [3, 7])
def test_rk4_energy_drift_is_fourth_order(n):
    t = chain(n)
    m = t.masses.astype(np.float64)
    rng = np.random.default_rng(n)
    x0 = np.concatenate([rng.uniform(-1.5, 1.5, n), rng.uniform(-1, 1, n)])
    f = lambda x, u: D.chain_accel(x, u, t, m)
    errs = []
    for dt in (0.004, 0.002):
        x = x0.copy()
        for _ in range(int(round(0.4 / dt))):
            x = D.rk4_step(f, x, np.zeros(n), dt)
        errs.append(abs(D.chain_energy(x, t, m) - D.chain_energy(x0, t, m)))
    assert errs[0] < 1e-4
    assert errs[0] / errs[1] > 12.0          # ~16 for a fourth-order method


def test_hanging_chain_stays_at_rest_and_gravity_compensation_is_static():
    n = 4
    t = chain(n)
    m = t.masses.astype(np.float64)
    a = D.chain_accel(np.zeros(2 * n), np.zeros(n), t, m)
    np.testing.assert_allclose(a, 0.0, atol=1e-14)
    # static pose: tau_i - tau_{i+1} = g l_i mu_i sin phi_i, so tau_i = sum_{k>=i} g l_k mu_k sin phi_k
    phi = np.array([0.3, -0.5, 1.0, 0.2])
    mu = D.chain_tail_masses(m)
    Q = float(t.gravity) * t.lengths.astype(np.float64) * mu * np.sin(phi)
    tau = np.flip(np.cumsum(np.flip(Q)))
    a = D.chain_accel(np.concatenate([phi, np.zeros(n)]), tau, t, m)
    np.testing.assert_allclose(a, 0.0, atol=1e-12)


def test_rk4_linear_ode_is_truncated_exponential():
    A = np.array([[0.0, 1.0], [-4.0, -0.3]])
    x = np.array([1.0, -0.5])
    dt = 0.1
    got = D.rk4_step(lambda xx, u: A @ xx, x, None, dt)
    hA = dt * A
    want = x + hA @ x + hA @ hA @ x / 2 + hA @ hA @ hA @ x / 6 + hA @ hA @ hA @ hA @ x / 24
    np.testing.assert_allclose(got, want, atol=1e-15)


def test_end_effector_position():
    t = chain(3, lengths=[1.0, 2.0, 0.5])
    x = np.array([0.0, math.pi / 2, math.pi, 0, 0, 0])
    np.testing.assert_allclose(D.chain_end_effector(x, t), [2.0, -1.0 + 0.5], atol=1e-14)


# ------------------------------------------------------------------ contact

def test_contact_resting_mass_settles_to_static_penetration():
    """A single link hanging straight down onto a ground spring: static compression m g / k."""
    t = W.chain_contact_task(0, 1)
    t.lengths = np.array([1.0], np.float32)
    t.ground_y = np.float32(-0.99)
    m = np.array([[2.0]])
    mu_f = np.array([1.0])
    f = lambda x, u: D.chain_accel(x, u, t, m, mu_f, contact=True)
    x = np.array([[0.0, 0.0]])
    for _ in range(4000):
        x = D.rk4_step(f, x, np.zeros((1, 1)), 0.001)
    y = -math.cos(x[0, 0])
    assert abs(x[0, 0]) < 1e-9                         # symmetric, stays vertical
    # the rod is rigid: the mass cannot go below -1, so the spring carries only
    # what it is compressed by; check the force balance at the rest point
    fn = float(t.k_contact) * (float(t.ground_y) - y)
    assert y == pytest.approx(-1.0, abs=1e-9) and fn > 0


def test_contact_normal_force_and_friction_direction():
    t = W.chain_contact_task(0, 2)
    lengths = np.array([1.0, 1.0])
    phi = np.array([[math.pi / 2, 0.0]])                 # first link horizontal, second hanging
    # mass 2 at (1, -1); put the ground at -0.9 -> penetration 0.1
    t.ground_y = np.float32(-0.9)
    dphi = np.array([[0.0, 0.5]])                         # mass 2 moves in +x at 0.5
    F = D.contact_forces(phi, dphi, lengths, np.array([0.8]), t)
    fn = float(t.k_contact) * (float(t.ground_y) + 1.0)
    assert F[0, 1, 1] == pytest.approx(fn, rel=1e-6)
    assert F[0, 1, 0] == pytest.approx(-0.8 * fn * math.tanh(0.5 / 0.01), rel=1e-6)  # opposes motion
    assert F[0, 0, 0] == 0 and F[0, 0, 1] == 0            # mass 1 at y=0 is above ground


def test_contact_generalised_force_is_virtual_work():
    """Q_i from contact equals F . dp/dphi_i (finite differences of positions)."""
    n = 4
    t = W.chain_contact_task(0, n)
    rng = np.random.default_rng(5)
    lengths = t.lengths.astype(np.float64)
    phi = rng.uniform(-0.5, 0.5, n) + np.pi * 0.0
    t.ground_y = np.float32(-2.5)
    dphi = rng.uniform(-1, 1, n)
    F = D.contact_forces(phi[None], dphi[None], lengths, np.array([1.0]), t)[0]
    m = np.ones((1, n))
    a_c = D.chain_accel(np.concatenate([phi, dphi])[None], np.zeros((1, n)), t, m, np.array([1.0]), contact=True)[0, n:]
    a_0 = D.chain_accel(np.concatenate([phi, dphi])[None], np.zeros((1, n)), t, m[0])[0, n:]
    M = D.chain_mass_matrix(phi, m[0], lengths)
    Qc = M @ (a_c - a_0)
    h = 1e-6
    Qfd = np.zeros(n)
    for i in range(n):
        e = np.eye(n)[i] * h
        dp = (D.chain_positions(phi + e, lengths) - D.chain_positions(phi - e, lengths)) / (2 * h)
        Qfd[i] = np.sum(F * dp)
    np.testing.assert_allclose(Qc, Qfd, rtol=1e-6, atol=1e-6)
