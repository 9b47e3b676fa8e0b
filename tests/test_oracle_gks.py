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
    for n in range(8):
        q = integrate.quad(lambda v: v ** n * _maxw(v, 0.4, lam), -np.inf, np.inf, epsabs=1e-14)[0]
        assert abs(mv[n] - q) < 1e-11 * (1 + abs(q))
    # K internal degrees of freedom each with variance 1/(2 lam): <z> = K s,
    # <z^2> = (3K + K(K-1)) s^2, <z^3> = (15K + 9K(K-1) + K(K-1)(K-2)) s^3
    # with z the sum of K squared Gaussians of variance s = 1/(2 lam)
    s = 1.0 / (2 * lam)
    assert abs(mz[1] - K * s) < 1e-15 * mz[1]
    assert abs(mz[2] - (3 * K + K * (K - 1)) * s * s) < 1e-14 * mz[2]
    assert abs(mz[3] - (15 * K + 9 * K * (K - 1) + K * (K - 1) * (K - 2)) * s ** 3) < 1e-14 * mz[3]


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


def _euler_wtt_symbolic(ndim, g=GAMMA):
    """W, its first and second space derivatives and W_t, W_tt at the origin
    for a smooth analytic primitive field, from the Euler equations by
    symbolic differentiation (Cauchy-Kowalewski): W_t = -(F_x + G_y), W_tt =
    -d_x (F_W W_t) - d_y (G_W W_t)."""
    import sympy as sp
    x, y = sp.symbols("x y")
    rho = 1.1 + 0.3 * sp.sin(1.3 * x + 0.4) + 0.2 * sp.cos(0.7 * y - 0.2) + 0.1 * x * y
    u = 0.4 + 0.5 * sp.sin(0.9 * x - 0.3 * y + 0.1)
    v = -0.3 + 0.4 * sp.cos(0.6 * x + 1.1 * y) if ndim == 2 else sp.Integer(0)
    p = 0.9 + 0.25 * sp.cos(1.7 * x - 0.2) + 0.15 * sp.sin(0.5 * y + 0.3) - 0.05 * x * y
    if ndim == 1:
        rho, u, p = (e.subs(y, 0) for e in (rho, u, p))
    E = p / (g - 1) + rho * (u * u + v * v) / 2
    W = [rho, rho * u, rho * v, E] if ndim == 2 else [rho, rho * u, E]
    w = sp.symbols("w0:%d" % len(W))
    if ndim == 2:
        pw = (g - 1) * (w[3] - (w[1] ** 2 + w[2] ** 2) / (2 * w[0]))
        Fw = [w[1], w[1] ** 2 / w[0] + pw, w[1] * w[2] / w[0], w[1] * (w[3] + pw) / w[0]]
        Gw = [w[2], w[1] * w[2] / w[0], w[2] ** 2 / w[0] + pw, w[2] * (w[3] + pw) / w[0]]
    else:
        pw = (g - 1) * (w[2] - w[1] ** 2 / (2 * w[0]))
        Fw = [w[1], w[1] ** 2 / w[0] + pw, w[1] * (w[2] + pw) / w[0]]
        Gw = [0, 0, 0]
    sub = dict(zip(w, W))
    F = [sp.sympify(f).subs(sub) for f in Fw]
    G = [sp.sympify(f).subs(sub) for f in Gw]
    Wt = [-(sp.diff(F[k], x) + sp.diff(G[k], y)) for k in range(len(W))]
    JF = sp.Matrix(Fw).jacobian(w).subs(sub)
    JG = sp.Matrix(Gw).jacobian(w).subs(sub)
    FtW = JF * sp.Matrix(Wt)
    GtW = JG * sp.Matrix(Wt)
    Wtt = [-(sp.diff(FtW[k], x) + sp.diff(GtW[k], y)) for k in range(len(W))]
    at0 = {x: 0, y: 0}
    ev = lambda e: float(sp.N(sp.sympify(e).subs(at0), 30))
    out = dict(W=[ev(e) for e in W], Wx=[ev(sp.diff(e, x)) for e in W], Wy=[ev(sp.diff(e, y)) for e in W],
               Wxx=[ev(sp.diff(e, x, 2)) for e in W], Wxy=[ev(sp.diff(e, x, y)) for e in W],
               Wyy=[ev(sp.diff(e, y, 2)) for e in W], Wt=[ev(e) for e in Wt], Wtt=[ev(e) for e in Wtt])
    return {k: np.array(v) for k, v in out.items()}


@pytest.mark.parametrize("ndim", [1, 2])
def test_equilibrium_second_time_derivative_vs_euler(oracle, ndim):
    # the kinetic second time derivative of the interface equilibrium (moments
    # of the micro-slope products) equals the Euler equations' W_tt obtained
    # by symbolic differentiation, and W(dt) = W + dt W_t for tau = 0
    d = _euler_wtt_symbolic(ndim)
    W = d["W"][None]
    sec = np.stack([d["Wxx"], d["Wxy"], d["Wyy"]])[None]
    dt = 1e-3
    args = (W, W, d["Wx"][None], d["Wx"][None])
    if ndim == 2:
        args = args + (d["Wy"][None], d["Wy"][None])
    F, Ft, Wh, Wf, Wtt = oracle.gks_points(oracle.params(ndim=ndim), ndim, *args, dt=dt, sec=sec, full=True)
    scale = np.abs(d["Wtt"]).max()
    assert np.abs(Wtt[0] - d["Wtt"]).max() < 1e-12 * scale, (Wtt[0], d["Wtt"])
    np.testing.assert_allclose(Wf[0], d["W"] + dt * d["Wt"], rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(Wh[0], d["W"] + 0.5 * dt * d["Wt"], rtol=1e-14, atol=1e-15)


def _bgk_point_by_quadrature(Wl, Wr, nl, nr, tl, tr, tau, dt, K, g=GAMMA):
    """The BGK interface solution at one 2-D face point (face frame, normal
    velocity u), evaluated independently of the oracle: every velocity moment
    by numerical quadrature (scipy quad in u, Gauss-Hermite in v, the K
    internal degrees of freedom through their Gaussian moments), the
    micro-slopes and time slopes by solving the quadrature moment systems, and
    the time integrals of the solution's weights by quadrature in t:
      f = (1 - e) g_c + ((t + tau) e - tau)(a_c u + b_c v) g_c + (t - tau (1 - e)) A_c g_c
        + e sum_{s = l (u > 0), r (u < 0)} g_s [1 - (t + tau)(a_s u + b_s v) - tau A_s],
    e = exp(-t / tau). Returns F, dF/dt (fitted to the integrals over dt/2 and
    dt), W(dt/2), W(dt)."""
    vh, wh = np.polynomial.hermite.hermgauss(40)

    def prim(W):
        rho, U, V = W[0], W[1] / W[0], W[2] / W[0]
        p = (g - 1) * (W[3] - 0.5 * rho * (U * U + V * V))
        return rho, U, V, rho / (2 * p)

    def psi(u, v, z):
        return [np.ones_like(u * v), u * np.ones_like(v), v * np.ones_like(u), 0.5 * (u * u + v * v + z)]

    def moment(st, fn, half):
        """<fn(u, v, z) psi_k> over the normalised Maxwellian of st (u-half-space
        half = +1, -1, or 0 for all u); fn is polynomial of degree <= 2 in z."""
        rho, U, V, lam = st
        zm = [1.0, K / (2 * lam), K * (K + 2) / (4 * lam * lam)]
        vv = V + vh / math.sqrt(lam)

        def integrand(u, k):
            q = [np.asarray(fn(u, vv, z) * psi(u, vv, z)[k]) for z in (0.0, 1.0, 2.0)]
            a0, a1, a2 = q[0], (-3 * q[0] + 4 * q[1] - q[2]) / 2, (q[0] - 2 * q[1] + q[2]) / 2
            ez = a0 + a1 * zm[1] + a2 * zm[2]
            return float(np.sum(wh * ez)) / math.sqrt(math.pi) * _maxw(u, U, lam)
        lo, hi = (0.0, np.inf) if half > 0 else ((-np.inf, 0.0) if half < 0 else (-np.inf, np.inf))
        return np.array([integrate.quad(integrand, lo, hi, args=(k,), epsabs=1e-14, epsrel=1e-13, limit=200)[0]
                         for k in range(4)])

    def slope_fn(a):
        return lambda u, v, z: a[0] + a[1] * u + a[2] * v + a[3] * 0.5 * (u * u + v * v + z)

    def solve_slope(st, w):
        M = np.stack([moment(st, (lambda i: (lambda u, v, z: psi(u, v, z)[i]))(i), 0) for i in range(4)])
        return np.linalg.solve(M, w)

    def time_slope(st, a, b):
        fa, fb = slope_fn(a), slope_fn(b)
        return solve_slope(st, -moment(st, lambda u, v, z: u * fa(u, v, z) + v * fb(u, v, z), 0))

    sl, sr = prim(Wl), prim(Wr)
    one = lambda u, v, z: np.ones_like(u * v)
    Wc = sl[0] * moment(sl, one, +1) + sr[0] * moment(sr, one, -1)
    sc = prim(Wc)
    al, ar = solve_slope(sl, nl / sl[0]), solve_slope(sr, nr / sr[0])
    bl, br = solve_slope(sl, tl / sl[0]), solve_slope(sr, tr / sr[0])
    ac, bc = solve_slope(sc, 0.5 * (nl + nr) / sc[0]), solve_slope(sc, 0.5 * (tl + tr) / sc[0])
    Al, Ar, Ac = time_slope(sl, al, bl), time_slope(sr, ar, br), time_slope(sc, ac, bc)

    def parts(ufac):
        """velocity moments of the pieces of f, times u^ufac"""
        uf = (lambda u: u) if ufac else (lambda u: 1.0)
        out = {}
        fa, fb, fA = slope_fn(ac), slope_fn(bc), slope_fn(Ac)
        out["c1"] = sc[0] * moment(sc, lambda u, v, z: uf(u) * one(u, v, z), 0)
        out["cs"] = sc[0] * moment(sc, lambda u, v, z: uf(u) * (u * fa(u, v, z) + v * fb(u, v, z)), 0)
        out["cA"] = sc[0] * moment(sc, lambda u, v, z: uf(u) * fA(u, v, z), 0)
        for name, st, a, b, A, half in (("l", sl, al, bl, Al, +1), ("r", sr, ar, br, Ar, -1)):
            fa_, fb_, fA_ = slope_fn(a), slope_fn(b), slope_fn(A)
            out[name + "1"] = st[0] * moment(st, lambda u, v, z: uf(u) * one(u, v, z), half)
            out[name + "s"] = st[0] * moment(st, lambda u, v, z: uf(u) * (u * fa_(u, v, z) + v * fb_(u, v, z)), half)
            out[name + "A"] = st[0] * moment(st, lambda u, v, z: uf(u) * fA_(u, v, z), half)
        return out

    def weights(t):
        e = math.exp(-t / tau)
        return dict(c1=1 - e, cs=(t + tau) * e - tau, cA=t - tau * (1 - e),
                    n1=e, ns=-(t + tau) * e, nA=-tau * e)

    def combine(P, w):
        return (w["c1"] * P["c1"] + w["cs"] * P["cs"] + w["cA"] * P["cA"]
                + sum(w["n1"] * P[s + "1"] + w["ns"] * P[s + "s"] + w["nA"] * P[s + "A"] for s in "lr"))

    Pu, P0 = parts(1), parts(0)
    Fd = []
    for d in (0.5 * dt, dt):
        wi = {k: integrate.quad(lambda t, k=k: weights(t)[k], 0.0, d, epsabs=1e-18, epsrel=1e-13)[0]
              for k in ("c1", "cs", "cA", "n1", "ns", "nA")}
        Fd.append(combine(Pu, wi))
    F = (4 * Fd[0] - Fd[1]) / dt
    Ft = 4 * (Fd[1] - 2 * Fd[0]) / dt ** 2
    return F, Ft, combine(P0, weights(0.5 * dt)), combine(P0, weights(dt))


@pytest.mark.parametrize("ratio", [0.1, 1.0, 10.0])
def test_finite_tau_point_vs_quadrature(oracle, ratio):
    # a 2-D point with different states and non-zero normal and tangential
    # slopes at a fixed collision time tau = ratio * dt: flux, flux time
    # derivative and the interface states at dt/2 and dt of the oracle equal
    # the BGK solution evaluated by quadrature (this pins the finite-tau time
    # coefficients and the interface-state weights with non-zero slopes)
    K = (4.0 - 2.0 * GAMMA) / (GAMMA - 1.0)
    def cons(rho, u, v, p):
        return np.array([rho, rho * u, rho * v, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)])
    Wl, Wr = cons(1.0, 0.3, -0.2, 1.0), cons(0.7, 0.1, 0.15, 0.6)
    nl, nr = np.array([0.3, -0.2, 0.1, 0.5]), np.array([-0.4, 0.25, 0.05, -0.3])
    tl, tr = np.array([0.1, 0.2, -0.3, 0.15]), np.array([0.2, -0.1, 0.1, 0.25])
    dt = 0.02
    ref = _bgk_point_by_quadrature(Wl, Wr, nl, nr, tl, tr, ratio * dt, dt, K)
    prm = oracle.params(ndim=2, tau_c1=ratio, tau_c2=0.0)
    F, Ft, Wh, Wf, _ = oracle.gks_points(prm, 2, Wl[None], Wr[None], nl[None], nr[None], tl[None], tr[None],
                                         dt=dt, full=True)
    for got, want, name in ((F[0], ref[0], "F"), (Ft[0], ref[1], "Ft"), (Wh[0], ref[2], "W(dt/2)"),
                            (Wf[0], ref[3], "W(dt)")):
        assert np.abs(got - want).max() < 1e-9 * (1.0 + np.abs(want).max()), (name, got, want)


def test_second_order_weight_of_the_interface_value(oracle):
    # The weight phi(r) of the interface value's second-order term (reading):
    # with equal side states and a jump of the density's normal slope only,
    # the averaged derivatives, hence the unweighted W_tt, are the same for
    # every jump size, and r = dt c |dn_l - dn_r|_rho / (rho_l + rho_r).
    # r <= 1e-2 keeps phi = 1, r = 0.055 gives phi = 1 - (0.045 / 0.09)^2 =
    # 0.75, r >= 0.1 gives 0; a state jump of r = 0.5 gives 0 as well;
    # rounding-size state differences keep phi = 1
    d = _euler_wtt_symbolic(2)
    W = d["W"][None]
    sec = np.stack([d["Wxx"], d["Wxy"], d["Wyy"]])[None]
    dt = 1e-3
    prm = oracle.params(ndim=2)
    rho, U, V = d["W"][0], d["W"][1] / d["W"][0], d["W"][2] / d["W"][0]
    p = (GAMMA - 1) * (d["W"][3] - 0.5 * rho * (U * U + V * V))
    c = math.sqrt(GAMMA * p / rho)

    def w2(r_slope, Wr=None):
        delta = np.zeros(4)
        delta[0] = r_slope * rho / (dt * c)       # |dn_l - dn_r|_rho = 2 delta
        nl, nr = d["Wx"] + delta, d["Wx"] - delta
        out = oracle.gks_points(prm, 2, W, W if Wr is None else Wr, nl[None], nr[None],
                                d["Wy"][None], d["Wy"][None], dt=dt, sec=sec, full=True)
        return out[4][0]
    ref = w2(0.0)
    scale = np.abs(ref).max()
    assert np.abs(ref - d["Wtt"]).max() < 1e-12 * np.abs(d["Wtt"]).max()
    for r, phi in ((0.005, 1.0), (0.01, 1.0), (0.055, 0.75), (0.1, 0.0), (0.3, 0.0)):
        got = w2(r)
        assert np.abs(got - phi * ref).max() <= 1e-12 * scale, (r, phi, got / ref)
    # a jump of the states (pressure ratio giving r = 0.5): the term is off
    Wj = d["W"].copy()
    Wj[3] += (3.0 * p) / (GAMMA - 1)                 # p_r = 4 p_l: r = 3/5
    assert np.all(w2(0.0, Wj[None]) == 0.0)
    # rounding-size state differences: phi = 1
    Wn = d["W"] * (1.0 + 4e-16 * np.array([1.0, -1.0, 1.0, -1.0]))
    assert np.abs(w2(0.0, Wn[None]) - ref).max() < 1e-11 * scale
