"""Pins of the sixth-order non-compact oracle (Sec. 4.1 GENO, HLLC, classical
Runge-Kutta) against facts fixed outside it: textbook reconstruction
coefficients, hand-integrated smoothness indicators, exactness on
polynomials, the closed-form amplification of the linear scheme on a Fourier
mode, the order of accuracy, the exact Euler flux and contact, mirror
symmetry, conservation and the mirror-doubled domain."""
import math

import numpy as np
import pytest

from oracle import geno6 as o6
from paper_2507_20461_amd import inputs

GAMMA = 1.4


def face_weights(lo, n, xi):
    """Weights mapping the averages of cells lo..lo+n-1 to the value at xi."""
    w = []
    for m in range(n):
        e = np.zeros(n)
        e[m] = 1.0
        a = o6.poly(e, lo)
        w.append(sum(a[k] * xi ** k for k in range(n)))
    return np.array(w)


def test_candidate_face_weights_are_the_textbook_ones():
    # sixth-order interface formula of the symmetric six-cell stencil
    assert np.allclose(face_weights(-2, 6, 0.5) * 60.0, [1, -8, 37, 37, -8, 1], atol=1e-12)
    # third-order (ENO) and fourth-order stencils of the reconstruction tables
    assert np.allclose(face_weights(-2, 3, 0.5), [1 / 3, -7 / 6, 11 / 6], atol=1e-13)
    assert np.allclose(face_weights(-1, 3, 0.5), [-1 / 6, 5 / 6, 1 / 3], atol=1e-13)
    assert np.allclose(face_weights(-1, 4, 0.5), [-1 / 12, 7 / 12, 7 / 12, -1 / 12], atol=1e-13)
    assert np.allclose(face_weights(0, 4, 0.5), [1 / 4, 13 / 12, -5 / 12, 1 / 12], atol=1e-13)


def test_smoothness_by_hand():
    # p = xi: 1; xi^2: int (2 xi)^2 + int 2^2 = 1/3 + 4; xi^3: 9/80 + 3 + 36
    assert o6.smoothness([0, 1], 1) == pytest.approx(1.0, abs=1e-15)
    assert o6.smoothness([0, 0, 1], 2) == pytest.approx(13 / 3, abs=1e-14)
    assert o6.smoothness([0, 0, 0, 1], 3) == pytest.approx(9 / 80 + 3 + 36, abs=1e-13)
    # cross term of xi and xi^3: int 1 * 3 xi^2 * 2 = 1/2
    assert o6.smoothness([0, 1, 0, 1], 3) == pytest.approx(1 + 0.5 + 9 / 80 + 3 + 36, abs=1e-13)


def test_quadratic_indicators_are_jiang_shu():
    rng = np.random.default_rng(4)
    prm = o6.params()
    for _ in range(20):
        u = rng.normal(size=6)
        a, b, c, d = u[0], u[1], u[2], u[3]
        is1 = 13 / 12 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2
        is2 = 13 / 12 * (b - 2 * c + d) ** 2 + 0.25 * (b - d) ** 2
        s = o6.side(prm, u, 0)
        assert s["IS1"] == pytest.approx(is1, rel=1e-12, abs=1e-14)
        assert s["IS2"] == pytest.approx(is2, rel=1e-12, abs=1e-14)


def avg_of_poly(coef, n, lo=-2):
    """Averages of sum coef[k] x^k over cells lo..lo+n-1 (unit cells, cell 0 = [-1/2, 1/2])."""
    out = []
    for m in range(lo, lo + n):
        xl, xr = m - 0.5, m + 0.5
        out.append(sum(c * (xr ** (k + 1) - xl ** (k + 1)) / (k + 1) for k, c in enumerate(coef)))
    return np.array(out)


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4, 5])
def test_polynomial_exactness(deg):
    rng = np.random.default_rng(deg)
    coef = rng.normal(size=deg + 1)
    u6 = avg_of_poly(coef, 6)
    prm = o6.params()
    for side, xf in ((0, 0.5), (1, 0.5)):
        s = o6.side(prm, u6, side)
        exact = sum(c * xf ** k for k, c in enumerate(coef))
        # p^5 is exact up to degree 5, S_1, S_2 up to 2 and S_3, S_4 up to 3
        assert s["p5"] == pytest.approx(exact, abs=1e-11)
        for k, dmax in ((1, 2), (2, 2), (3, 3), (4, 3)):
            if deg <= dmax:
                assert s["p%d" % k] == pytest.approx(exact, abs=1e-11)


def test_linear_data_keeps_the_linear_reconstruction():
    # every candidate has IS = slope^2, so IS^tau = 0, alpha = 1, chi = 1 and
    # the low-order weights are the linear ones d_k / sum d
    prm = o6.params()
    u6 = 0.3 + 0.7 * np.arange(6)
    s = o6.side(prm, u6, 0)
    assert s["chi"] == 1.0 and s["alpha"] == 1.0
    assert np.allclose([s["w1"], s["w2"], s["w3"], s["w4"]], np.array([1, 8, 1, 1]) / 11, rtol=1e-12)
    assert s["value"] == pytest.approx(0.3 + 0.7 * 2.5, abs=1e-13)


def test_step_picks_the_smooth_side():
    # a jump between cells j and j+1: the left state is the left constant and
    # the right state the right one (only S_1 is smooth for the left side)
    prm = o6.params()
    u6 = np.array([1.0, 1.0, 1.0, 5.0, 5.0, 5.0])
    left, right = o6.side(prm, u6, 0), o6.side(prm, u6, 1)
    assert left["chi"] < 1e-20 and right["chi"] < 1e-20
    assert left["value"] == pytest.approx(1.0, abs=1e-12)
    assert right["value"] == pytest.approx(5.0, abs=1e-12)
    # a jump between j-1 and j: S_4 is the only smooth stencil on the left side
    u6 = np.array([1.0, 1.0, 5.0, 5.0, 5.0, 5.0])
    assert o6.side(prm, u6, 0)["value"] == pytest.approx(5.0, abs=1e-12)


def test_worked_examples_of_the_stencil_indicator():
    prm = o6.params()
    eps = 1e-15
    # (a) a jump inside cell j+3 only: S_1..S_3 are flat, so IS^tau = 0 and
    # the linear six-cell value is kept (chi = 1): 1/60 of the jump
    s = o6.side(prm, [0, 0, 0, 0, 0, 1.0], 0)
    assert s["chi"] == 1.0 and s["value"] == pytest.approx(1 / 60, abs=1e-15)
    # (b) a jump inside cell j-2 only: IS_1 = 13/12 + 1/4 = 4/3, the others 0;
    # IS^tau = IS_1 / 2 = 2/3, IS^H = 4/3, IS^L = 0
    s = o6.side(prm, [1.0, 0, 0, 0, 0, 0], 0)
    assert s["IS1"] == pytest.approx(4 / 3, rel=1e-13)
    aH, aL = 1 + ((2 / 3) / (4 / 3 + eps)) ** 2, 1 + ((2 / 3) / eps) ** 2
    assert s["alpha"] == pytest.approx(2 * aH / (aH + aL), rel=1e-12)
    assert s["value"] == pytest.approx(0.0, abs=1e-25)
    # (c) a jump inside cell j+2: S_3 and S_4 see it, S_1 and S_2 do not;
    # IS^tau = IS_3 / 2 with IS_3, IS_4 from the pinned candidate helpers
    s = o6.side(prm, [0, 0, 0, 0, 1.0, 0], 0)
    is3 = o6.smoothness(o6.poly([0, 0, 0, 1.0], -1), 3)
    is4 = o6.smoothness(o6.poly([0, 0, 1.0, 0], 0), 3)
    assert s["IS3"] == pytest.approx(is3, rel=1e-12) and s["IS4"] == pytest.approx(is4, rel=1e-12)
    aH, aL = 1 + ((is3 / 2) / (max(is3, is4) + eps)) ** 2, 1 + ((is3 / 2) / eps) ** 2
    assert s["alpha"] == pytest.approx(2 * aH / (aH + aL), rel=1e-12)


def test_mirror_symmetry_of_the_two_sides():
    rng = np.random.default_rng(11)
    prm = o6.params()
    for _ in range(30):
        u6 = rng.normal(size=6) * rng.choice([1e-3, 1.0, 10.0]) + (rng.random(6) < 0.3) * 3.0
        a = o6.side(prm, u6, 0)
        b = o6.side(prm, u6[::-1].copy(), 1)
        for key in o6.SIDE_FIELDS:
            assert a[key] == pytest.approx(b[key], rel=1e-12, abs=1e-13), key


def test_path_function_bounds_and_limits():
    prm = o6.params()
    rng = np.random.default_rng(3)
    for _ in range(200):
        u6 = rng.normal(size=6)
        s = o6.side(prm, u6, int(rng.integers(2)))
        assert 0.0 < s["alpha"] <= 1.0
        assert 0.0 <= s["chi"] <= 1.0 + 1e-15
        assert sum(s["w%d" % k] for k in range(1, 5)) == pytest.approx(1.0, abs=1e-14)
        lo, hi = min(s["p5"], s["p1"], s["p2"], s["p3"], s["p4"]), max(s["p5"], s["p1"], s["p2"], s["p3"], s["p4"])
        assert lo - 1e-12 <= s["value"] <= hi + 1e-12


def cons(rho, u, p):
    return np.array([rho, rho * u, p / (GAMMA - 1) + 0.5 * rho * u * u])


def euler_flux(rho, u, p):
    E = p / (GAMMA - 1) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, (E + p) * u])


def test_hllc_consistency_upwinding_and_contacts():
    prm = o6.params()
    rng = np.random.default_rng(5)
    for _ in range(20):
        rho, u, p = rng.uniform(0.2, 2), rng.uniform(-2, 2), rng.uniform(0.2, 2)
        assert np.allclose(o6.hllc(prm, cons(rho, u, p), cons(rho, u, p)), euler_flux(rho, u, p), rtol=1e-13)
    # supersonic to the right / left: the upwind Euler flux
    L, R = (1.0, 3.0, 1.0), (0.5, 3.5, 0.8)
    assert np.allclose(o6.hllc(prm, cons(*L), cons(*R)), euler_flux(*L), rtol=1e-13)
    L, R = (1.0, -3.0, 1.0), (0.5, -3.5, 0.8)
    assert np.allclose(o6.hllc(prm, cons(*L), cons(*R)), euler_flux(*R), rtol=1e-13)
    # isolated contacts are resolved exactly: stationary and moving
    assert np.allclose(o6.hllc(prm, cons(1.0, 0.0, 0.7), cons(0.2, 0.0, 0.7)), [0.0, 0.7, 0.0], atol=1e-14)
    for u in (0.4, -0.4):
        F = o6.hllc(prm, cons(1.0, u, 0.7), cons(0.2, u, 0.7))
        up = (1.0, u, 0.7) if u > 0 else (0.2, u, 0.7)
        assert np.allclose(F, euler_flux(*up), rtol=1e-13)


def test_hllc_mirror_symmetry():
    prm = o6.params()
    rng = np.random.default_rng(6)
    for _ in range(30):
        L = (rng.uniform(0.1, 3), rng.uniform(-2, 2), rng.uniform(0.1, 3))
        R = (rng.uniform(0.1, 3), rng.uniform(-2, 2), rng.uniform(0.1, 3))
        F = o6.hllc(prm, cons(*L), cons(*R))
        G = o6.hllc(prm, cons(R[0], -R[1], R[2]), cons(L[0], -L[1], L[2]))
        assert np.allclose(F, [-G[0], G[1], -G[2]], rtol=1e-12, atol=1e-13)


def test_one_step_matches_the_fourier_amplification():
    # On the density wave (U = p = 1) the reconstruction stays linear (chi = 1
    # to rounding), both sides equal the sixth-order central value and HLLC is
    # the exact contact flux: the scheme is linear advection of rho with the
    # Fourier symbol of the six-cell formula and classical Runge-Kutta, whose
    # one-step amplification is the degree-4 Taylor polynomial of exp(z).
    n, dt = 16, 0.05
    U = inputs.density_wave_noncompact(n)
    h = 2.0 / n
    U1, _, g = o6.step(o6.params(dt_fixed=dt), U, h, 1)
    assert g == 0
    k = math.pi
    c = np.array([1, -8, 37, 37, -8, 1]) / 60.0
    S = sum(c[m + 2] * np.exp(1j * k * m * h) for m in range(-2, 4))
    z = -(S / h) * (1 - np.exp(-1j * k * h)) * dt
    G = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    xc = (np.arange(n) + 0.5) * h
    amp = 0.2 * math.sin(k * h / 2) / (k * h / 2)
    rho = 1.0 + amp * np.imag(G * np.exp(1j * k * xc))
    assert np.abs(U1[0] - rho).max() < 1e-13
    assert np.abs(U1[1] - rho).max() < 1e-13
    assert np.abs(U1[2] - (2.5 + 0.5 * rho)).max() < 1e-13


def test_sixth_order_convergence_on_the_density_wave():
    # t = 2 (one period); dt ~ h^1.5 so that the fourth-order time error
    # stays below the sixth-order space error
    errs = []
    for n in (12, 24, 48):
        h = 2.0 / n
        steps = int(math.ceil(2.0 / (0.25 * h ** 1.5)))
        dt = 2.0 / steps
        U, _, _ = o6.step(o6.params(dt_fixed=dt), inputs.density_wave_noncompact(n), h, steps)
        errs.append(np.abs(U[0] - inputs.density_wave_noncompact(n, t=2.0)[0]).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] > 5.6, (errs, orders)


def test_periodic_run_conserves_totals():
    n = 64
    U = inputs.shocks_noncompact(n, seed=2, cells_per_segment=16)
    U1, dts, g = o6.step(o6.params(cfl=0.4), U, 1.0 / n, 20)
    assert np.all(np.isfinite(U1))
    for v in range(3):
        assert abs(U1[v].sum() - U[v].sum()) <= 1e-12 * np.abs(U[v]).sum()


def test_reflecting_walls_equal_the_mirror_doubled_periodic_run():
    n = 40
    U = inputs.smooth_noncompact(n, seed=9)
    U[:, 10:14] *= 1.7   # a bump with jumps
    prm_w = o6.params(bc=o6.REFLECTING, dt_fixed=2e-3)
    Uw, _, _ = o6.step(prm_w, U, 1.0 / n, 15)
    # mirror-doubled domain: cells reversed, momentum negated, periodic
    M = U[:, ::-1].copy()
    M[1] *= -1
    D = np.concatenate([U, M], axis=1)
    Dp, _, _ = o6.step(o6.params(bc=o6.PERIODIC, dt_fixed=2e-3), D, 1.0 / n, 15)
    assert np.allclose(Uw, Dp[:, :n], rtol=1e-11, atol=1e-12)
    for v in (0, 2):
        assert abs(Uw[v].sum() - U[v].sum()) <= 1e-12 * np.abs(U[v]).sum()


def test_transmissive_constant_state_is_steady():
    U = np.repeat(cons(0.8, 0.3, 1.1)[:, None], 20, axis=1)
    U1, _, g = o6.step(o6.params(bc=o6.TRANSMISSIVE), U, 0.05, 5)
    assert g == 0 and np.allclose(U1, U, rtol=1e-14, atol=1e-14)


def test_guard_replaces_a_non_physical_state():
    # a cold, fast flow (p = 1e-9, |u| up to 2): reconstructing rho, rho U and
    # rho E separately leaves the face pressure as the difference of nearly
    # equal numbers, negative at many faces; guarded sides take the target
    # cell's average, which is admissible
    n = 12
    x = np.arange(n) / n
    u = 2.0 * np.sin(2 * np.pi * x)
    rho = 1.0 + 0.5 * np.cos(2 * np.pi * x)
    U = np.stack([rho, rho * u, 1e-9 / (GAMMA - 1) + 0.5 * rho * u * u])
    UL, UR, F, chi, g = o6.faces(o6.params(bc=o6.PERIODIC), U)
    assert g >= 1
    assert np.all(np.isfinite(F))
    replaced = 0
    for s in range(n + 1):
        for W, cell in ((UL[:, s], (s - 1) % n), (UR[:, s], s % n)):
            assert W[0] > 0 and (GAMMA - 1) * (W[2] - 0.5 * W[1] ** 2 / W[0]) > 0
            replaced += bool(np.array_equal(W, U[:, cell]))
    assert replaced >= g


def test_roe_eigenstructure_satisfies_the_roe_property():
    # A(U~) = R diag(lambda) L is the Roe matrix: A (U_R - U_L) = F(U_R) - F(U_L)
    # exactly, and L R = I; the speeds are u~ -+ c~ and u~
    prm = o6.params()
    rng = np.random.default_rng(12)
    for _ in range(20):
        a = (rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(0.2, 3))
        b = (rng.uniform(0.2, 3), rng.uniform(-2, 2), rng.uniform(0.2, 3))
        R, L, lam = o6.eigen(prm, cons(*a), cons(*b))
        assert np.allclose(L @ R, np.eye(3), atol=1e-12)
        A = R @ np.diag(lam) @ L
        dF = euler_flux(*b) - euler_flux(*a)
        assert np.allclose(A @ (cons(*b) - cons(*a)), dF, rtol=1e-11, atol=1e-11)
        # each column of R is an eigenvector of the flux Jacobian at the Roe state
        sa, sb = math.sqrt(a[0]), math.sqrt(b[0])
        u = (sa * a[1] + sb * b[1]) / (sa + sb)
        assert lam[1] == pytest.approx(u, rel=1e-12, abs=1e-13)
        assert lam[0] < lam[1] < lam[2]


def test_characteristic_reconstruction_equals_the_conservative_one_on_smooth_data():
    # where every path function is 1 the reconstruction is the linear p^5,
    # which commutes with the (face-wise constant) projection
    # (compared on the faces where all twelve path functions are 1)
    n = 64
    U = inputs.smooth_noncompact(n, seed=4)
    a = o6.faces(o6.params(), U)
    b = o6.faces(o6.params(characteristic=True), U)
    lin = np.all(a[3] == 1.0, axis=(0, 1)) & np.all(b[3] == 1.0, axis=(0, 1))
    assert lin.sum() > n // 2
    for x, y in zip(a[:3], b[:3]):
        assert np.allclose(x[:, lin], y[:, lin], rtol=1e-12, atol=1e-12)


def test_characteristic_reconstruction_of_an_isolated_contact():
    # a contact (u, p equal, rho jumps) moves only the entropy field: the
    # characteristic states keep u and p exactly constant, and the flux is
    # the exact contact flux
    n = 24
    rho = np.where(np.arange(n) < 12, 1.0, 0.3)
    U = np.stack([rho, 0.5 * rho, 1.0 / (GAMMA - 1) + 0.125 * rho])
    UL, UR, F, chi, g = o6.faces(o6.params(bc=o6.TRANSMISSIVE, characteristic=True), U)
    for W in (UL, UR):
        u = W[1] / W[0]
        p = (GAMMA - 1) * (W[2] - 0.5 * W[1] * u)
        assert np.allclose(u, 0.5, atol=1e-12) and np.allclose(p, 1.0, atol=1e-12)
    # u > 0: the contact flux carries the left state's density
    assert np.allclose(F[0], 0.5 * UL[0], rtol=1e-12)
    assert np.allclose(F[1], 0.25 * UL[0] + 1.0, rtol=1e-12)


def test_characteristic_step_conserves_and_mirrors():
    n = 40
    U = inputs.smooth_noncompact(n, seed=9)
    U[:, 10:14] *= 1.7
    prm = o6.params(bc=o6.REFLECTING, dt_fixed=2e-3, characteristic=True)
    Uw, _, _ = o6.step(prm, U, 1.0 / n, 10)
    M = U[:, ::-1].copy()
    M[1] *= -1
    Dp, _, _ = o6.step(o6.params(bc=o6.PERIODIC, dt_fixed=2e-3, characteristic=True),
                       np.concatenate([U, M], axis=1), 1.0 / n, 10)
    assert np.allclose(Uw, Dp[:, :n], rtol=1e-11, atol=1e-12)
    for v in (0, 2):
        assert abs(Uw[v].sum() - U[v].sum()) <= 1e-12 * np.abs(U[v]).sum()


def test_fixed_ends_reproduce_the_other_kinds():
    # fixed ghost states equal to the copies of the end cells give the
    # transmissive right-hand side, equal to the periodic images the
    # periodic one (a run differs afterwards: fixed ghosts do not follow
    # the end cells)
    n = 30
    U = inputs.smooth_noncompact(n, seed=6)
    g = np.zeros((2, 3, 3))
    g[0] = np.repeat(U[:, :1].T, 3, axis=0)
    g[1] = np.repeat(U[:, -1:].T, 3, axis=0)
    a, _ = o6.rhs(o6.params(bc=o6.FIXED, ghost=g), U, 1.0 / n)
    b, _ = o6.rhs(o6.params(bc=o6.TRANSMISSIVE), U, 1.0 / n)
    assert np.array_equal(a, b)
    g[0] = U[:, [-1, -2, -3]].T      # cells -1, -2, -3 are n-1, n-2, n-3
    g[1] = U[:, [0, 1, 2]].T         # cells n, n+1, n+2 are 0, 1, 2
    La, _ = o6.rhs(o6.params(bc=o6.FIXED, ghost=g), U, 1.0 / n)
    Lb, _ = o6.rhs(o6.params(bc=o6.PERIODIC), U, 1.0 / n)
    assert np.array_equal(La, Lb)


def test_titarev_toro_data():
    U, g = inputs.titarev_toro_noncompact(1000)
    rho = U[0]
    assert np.allclose(rho[:100], 1.515695) and abs(rho[100:].mean() - 1.0) < 1e-3
    # exact averages of 1 + 0.1 sin(20 pi x) over the 10 cells of a period sum to 10
    assert abs(rho[100:110].sum() - 10.0) < 1e-12
    assert np.allclose(g[0, :, 0], 1.515695) and np.allclose(g[1, :, 1], 0.0)


def test_jump_in_s4_only_under_both_indicators():
    # the printed IS^tau of Sec. 4.1 is blind to a jump that lies only in S_4
    # (cells j..j+3 on the left side): chi = 1 and the linear value carries
    # 1/60 of the jump. The large-stencil reading (the fifth-derivative
    # indicator of p^5) sees it; both see a jump that S_3 holds
    printed, large = o6.params(), o6.params(istau=o6.ISTAU_LARGE_STENCIL)
    u = [0, 0, 0, 0, 0, 1.0]
    assert o6.side(printed, u, 0)["chi"] == 1.0
    s = o6.side(large, u, 0)
    assert s["chi"] < 1e-20 and abs(s["value"]) < 1e-12
    # by hand: p^5 of this data has a fifth-derivative coefficient a_5 with
    # 5! a_5 = (the fifth difference of the averages) = 1, so IS^tau = 1
    a = o6.poly(u, -2)
    assert 120.0 * a[5] == pytest.approx(1.0, rel=1e-12)
    for prm in (printed, large):
        assert o6.side(prm, [0, 0, 0, 0, 1.0, 0], 0)["chi"] < 1e-20


def test_large_stencil_indicator_keeps_smooth_data_linear():
    # the density wave of Sec. 6.1: from 12 cells up chi = 1 exactly at every
    # face with either indicator; on 6 cells both stay within 1e-9 of 1
    large = o6.params(istau=o6.ISTAU_LARGE_STENCIL)
    for n in (6, 12, 24):
        h = 2.0 / n
        xl = np.arange(n) * h
        rho = 1 + 0.2 * (np.cos(np.pi * xl) - np.cos(np.pi * (xl + h))) / (np.pi * h)
        for j in range(n):
            u6 = [rho[(j + k) % n] for k in range(-2, 4)]
            for sd in (0, 1):
                chi = o6.side(large, u6, sd)["chi"]
                assert chi == 1.0 if n >= 12 else chi > 1.0 - 1e-9


@pytest.mark.parametrize("istau,survives", [(0, False), (1, True)], ids=["printed", "large-stencil"])
def test_blast_wave_at_cfl_half_with_each_indicator(istau, survives):
    # the Woodward-Colella blast waves (400 cells, reflecting walls) at CFL
    # 0.5: with the printed indicator the cell two to the right of the
    # p = 1000 / 0.01 jump goes negative in the first step; with the
    # large-stencil indicator the run reaches t = 0.038
    from paper_2507_20461_amd import inputs
    W, _ = inputs.blast_wave_1d(400)
    U = W[:, 0, :].copy()
    dx = 1.0 / 400
    t, k, ok = 0.0, 0, True
    while t < 0.038 and k < 5000:
        dt = min(o6.cfl_dt(o6.params(bc=2, istau=istau), U, dx), 0.038 - t)
        U, _, _ = o6.step(o6.params(bc=2, dt_fixed=dt, istau=istau), U, dx, 1)
        t += dt
        k += 1
        p = 0.4 * (U[2] - 0.5 * U[1] ** 2 / U[0])
        if not (np.isfinite(U).all() and U[0].min() > 0 and p.min() > 0):
            ok = False
            break
    assert ok == survives, (k, t)
    if survives:
        assert abs(U[0].sum() - W[0].sum()) < 1e-12 * W[0].sum()
