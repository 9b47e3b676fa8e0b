"""Pins of the oracle's gas-kinetic flux against closed forms of kinetic theory
and of the Euler equations (no GPU).

The paper defers the GKS flux to the literature (Sec. 2); the oracle follows
the standard BGK interface solution. These tests pin it without re-using any
of its arithmetic:

* Gaussian moments against numerical quadrature, and half + half = full;
* equal constant states give the exact Euler flux and no time variation;
* smooth equal states with tau = 0 give F = F_Euler(W) and dF/dt = A W_t with
  W_t = -(A W_x + B W_y), A and B the Euler Jacobians (complex-step
  derivatives of the Euler flux), and W(t) = W + t W_t;
* tau -> infinity gives the free-transport (kinetic flux-vector splitting)
  flux of Mandal & Deshpande;
* continuity of the tau -> 0 limit;
* a y-invariant 2-D flux equals the 1-D flux (one more internal degree of
  freedom in 1-D).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

GAMMA = 1.4


def _maxw(u, U, lam):
    return math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2)


@pytest.mark.parametrize("U,lam", [(0.3, 0.7), (-1.2, 2.5), (0.0, 0.3), (2.0, 1.1)])
def test_moments_vs_quadrature(oracle, U, lam):
    K = 3.0
    full, mv, mz = oracle.moments(U, 0.4, lam, K, 0)
    pos, _, _ = oracle.moments(U, 0.4, lam, K, +1)
    neg, _, _ = oracle.moments(U, 0.4, lam, K, -1)
    for n in range(8):
        qp = integrate.quad(lambda u: u ** n * _maxw(u, U, lam), 0, np.inf, epsabs=1e-14, epsrel=1e-13)[0]
        qn = integrate.quad(lambda u: u ** n * _maxw(u, U, lam), -np.inf, 0, epsabs=1e-14, epsrel=1e-13)[0]
        scale = 1.0 + abs(qp) + abs(qn)
        assert abs(pos[n] - qp) < 1e-11 * scale
        assert abs(neg[n] - qn) < 1e-11 * scale
        assert abs(pos[n] + neg[n] - full[n]) < 1e-13 * scale
    for n in range(6):
        q = integrate.quad(lambda v: v ** n * _maxw(v, 0.4, lam), -np.inf, np.inf, epsabs=1e-14)[0]
        assert abs(mv[n] - q) < 1e-11 * (1 + abs(q))
    # K internal degrees of freedom each with variance 1/(2 lam)
    assert abs(mz[1] - K / (2 * lam)) < 1e-15 * mz[1]
    assert abs(mz[2] - (3 * K + K * (K - 1)) / (4 * lam * lam)) < 1e-14 * mz[2]


def euler_flux_1d(W, g=GAMMA):
    rho, m, E = W
    u = m / rho
    p = (g - 1) * (E - 0.5 * rho * u * u)
    return np.array([m, m * u + p, u * (E + p)])


def euler_flux_2d(W, g=GAMMA, direction=0):
    rho, mx, my, E = W
    u, v = mx / rho, my / rho
    p = (g - 1) * (E - 0.5 * rho * (u * u + v * v))
    if direction == 0:
        return np.array([mx, mx * u + p, my * u, u * (E + p)])
    return np.array([my, mx * v, my * v + p, v * (E + p)])


def jac(f, W):
    """Exact Jacobian by complex-step differentiation."""
    n = len(W)
    J = np.zeros((n, n))
    h = 1e-30
    for k in range(n):
        Wc = np.array(W, dtype=complex)
        Wc[k] += 1j * h
        J[:, k] = f(Wc).imag / h
    return J


def cons1(rho, u, p):
    return np.array([rho, rho * u, p / (GAMMA - 1) + 0.5 * rho * u * u])


def cons2(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)])


@pytest.mark.parametrize("tau_c1", [0.0, 0.05])
def test_constant_state_gives_euler_flux(oracle, tau_c1):
    prm = oracle.params(tau_c1=tau_c1)
    W1 = cons1(1.3, -0.4, 0.8)
    z = np.zeros((1, 3))
    F, Ft, Wi = oracle.gks_points(prm, 1, W1[None], W1[None], z, z, dt=2e-3)
    np.testing.assert_allclose(F[0], euler_flux_1d(W1), rtol=1e-13, atol=1e-14)
    assert np.abs(Ft).max() < 1e-9
    np.testing.assert_allclose(Wi[0], W1, rtol=1e-14)
    W2 = cons2(0.9, 0.3, -0.7, 0.5)
    z = np.zeros((1, 4))
    F, Ft, Wi = oracle.gks_points(prm, 2, W2[None], W2[None], z, z, z, z, dt=2e-3)
    np.testing.assert_allclose(F[0], euler_flux_2d(W2), rtol=1e-13, atol=1e-14)
    assert np.abs(Ft).max() < 1e-9
    np.testing.assert_allclose(Wi[0], W2, rtol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_smooth_state_gives_euler_time_derivative_2d(oracle, seed):
    rng = np.random.default_rng(seed)
    W = cons2(rng.uniform(0.5, 1.5), rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8), rng.uniform(0.3, 1.2))
    Wx = rng.normal(size=4) * 0.3
    Wy = rng.normal(size=4) * 0.3
    dt = 1e-3
    prm = oracle.params(tau_c1=0.0, tau_c2=1.0)   # equal pressures: tau = 0
    F, Ft, Wi = oracle.gks_points(prm, 2, W[None], W[None], Wx[None], Wx[None], Wy[None], Wy[None], dt=dt)
    A = jac(lambda w: euler_flux_2d(w, direction=0), W)
    B = jac(lambda w: euler_flux_2d(w, direction=1), W)
    Wt = -(A @ Wx + B @ Wy)
    np.testing.assert_allclose(F[0], euler_flux_2d(W), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(Ft[0], A @ Wt, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(Wi[0], W + 0.5 * dt * Wt, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("seed", range(3))
def test_smooth_state_gives_euler_time_derivative_1d(oracle, seed):
    rng = np.random.default_rng(10 + seed)
    W = cons1(rng.uniform(0.5, 1.5), rng.uniform(-0.8, 0.8), rng.uniform(0.3, 1.2))
    Wx = rng.normal(size=3) * 0.3
    dt = 1e-3
    F, Ft, Wi = oracle.gks_points(oracle.params(), 1, W[None], W[None], Wx[None], Wx[None], dt=dt)
    A = jac(euler_flux_1d, W)
    Wt = -(A @ Wx)
    np.testing.assert_allclose(F[0], euler_flux_1d(W), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(Ft[0], A @ Wt, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(Wi[0], W + 0.5 * dt * Wt, rtol=1e-13, atol=1e-14)


def kfvs_1d(W, sign, g=GAMMA):
    """Free-transport half-space flux of one Maxwellian (Mandal & Deshpande)."""
    rho, m, E = W
    U = m / rho
    p = (g - 1) * (E - 0.5 * rho * U * U)
    lam = rho / (2 * p)
    A = 0.5 * special.erfc(-sign * math.sqrt(lam) * U)
    Bf = sign * math.exp(-lam * U * U) / (2 * math.sqrt(math.pi * lam))
    return np.array([rho * (U * A + Bf),
                     (p + rho * U * U) * A + rho * U * Bf,
                     U * (E + p) * A + (E + 0.5 * p) * Bf])


def test_large_tau_gives_free_transport_flux(oracle):
    Wl = cons1(1.0, 0.2, 1.0)
    Wr = cons1(0.3, -0.1, 0.4)
    z = np.zeros((1, 3))
    dt = 1e-3
    prm = oracle.params(tau_c1=1e7, tau_c2=0.0)
    F, _, _ = oracle.gks_points(prm, 1, Wl[None], Wr[None], z, z, dt=dt)
    ref = kfvs_1d(Wl, +1) + kfvs_1d(Wr, -1)
    np.testing.assert_allclose(F[0], ref, rtol=1e-6)


def test_tau_to_zero_is_continuous(oracle):
    # the guarded tau = 0 branch is the limit of the tau > 0 formulas; the
    # deviation of the fitted flux and its time derivative is O(tau / dt^2)
    rng = np.random.default_rng(7)
    Wl = cons2(1.0, 0.2, 0.1, 1.0)
    Wr = cons2(0.8, 0.1, -0.2, 0.9)
    args = [rng.normal(size=(1, 4)) * 0.2 for _ in range(4)]
    dt = 1e-3
    a = oracle.gks_points(oracle.params(tau_c1=0.0, tau_c2=0.0), 2, Wl[None], Wr[None], *args, dt=dt)
    devs = []
    for c1 in (1e-8, 1e-9, 1e-10):
        b = oracle.gks_points(oracle.params(tau_c1=c1, tau_c2=0.0), 2, Wl[None], Wr[None], *args, dt=dt)
        devs.append([np.abs(x - y).max() / np.abs(x).max() for x, y in zip(a, b)])
    devs = np.array(devs)
    assert np.all(devs[2] < 1e-5)
    assert np.all((devs[1] < 0.2 * devs[0]) | (devs[1] < 1e-14))
    assert np.all((devs[2] < 0.2 * devs[1]) | (devs[2] < 1e-14))


@pytest.mark.parametrize("tau_c1", [0.0, 0.1])
def test_y_invariant_2d_equals_1d(oracle, tau_c1):
    # 2-D with V = 0 and no tangential variation carries the y-velocity
    # explicitly: K_1D = K_2D + 1 gives the same distribution moments.
    prm = oracle.params(tau_c1=tau_c1)
    Wl1, Wr1 = cons1(1.1, 0.3, 0.9), cons1(0.7, -0.2, 0.5)
    dl1, dr1 = np.array([[0.1, -0.2, 0.3]]), np.array([[-0.05, 0.1, 0.2]])
    F1, Ft1, Wi1 = oracle.gks_points(prm, 1, Wl1[None], Wr1[None], dl1, dr1, dt=1e-3)
    to2 = lambda w: np.array([w[..., 0], w[..., 1], 0 * w[..., 0], w[..., 2]]).T.reshape(-1, 4)
    z = np.zeros((1, 4))
    F2, Ft2, Wi2 = oracle.gks_points(prm, 2, to2(Wl1[None]), to2(Wr1[None]), to2(dl1), to2(dr1), z, z, dt=1e-3)
    for a, b in ((F1, F2), (Ft1, Ft2), (Wi1, Wi2)):
        np.testing.assert_allclose(b[0, [0, 1, 3]], a[0], rtol=1e-12, atol=1e-13)
        assert abs(b[0, 2]) < 1e-15
