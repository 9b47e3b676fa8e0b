"""Pins of the oracle's fourth-order compact GENO reconstruction on triangles
(Sec. 4.3 with Sec. 3), no GPU: exactness of the candidate polynomials on
polynomial data, closed forms of the indicators, the path function's smooth
limit, the measured order on smooth data, and the ENO behaviour at a jump.
"""
import math

import numpy as np
import pytest

from paper_2507_20461_amd import inputs


@pytest.fixture(scope="module")
def T():
    from oracle import geno_tri
    return geno_tri


def _poly_data(mesh, coef, exps):
    def f(x, y):
        return sum(c * x ** a * y ** b for c, (a, b) in zip(coef, exps))

    def g(x, y):
        gx = sum(c * a * x ** max(a - 1, 0) * y ** b for c, (a, b) in zip(coef, exps))
        gy = sum(c * b * x ** a * y ** max(b - 1, 0) for c, (a, b) in zip(coef, exps))
        return gx, gy

    W, dW = inputs.tri_cell_data(mesh, f, g)
    return W, dW, f, g


def _interior(mesh, margin=2):
    # cells whose stencil does not cross the periodic boundary
    nx, ny = mesh["nx"], mesh["ny"]
    out = []
    for j in range(margin, ny - margin):
        for i in range(margin, nx - margin):
            out += [2 * (j * nx + i), 2 * (j * nx + i) + 1]
    return out


ALL = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]


def test_cubic_reproduced_by_the_high_order_candidate(T):
    mesh = inputs.tri_mesh(9, 8, 3)
    coef = np.random.default_rng(1).normal(size=10)
    W, dW, f, g = _poly_data(mesh, coef, ALL)
    for c in _interior(mesh):
        fit = T.cell_fit(mesh, W, dW, c)
        pts = T.edge_points(fit["tri"]).reshape(6, 2)
        v, gx, gy = T.p3_at(fit, W[:, c], pts[:, 0], pts[:, 1])
        ex, ey = g(pts[:, 0], pts[:, 1])
        assert np.allclose(v[0], f(pts[:, 0], pts[:, 1]), rtol=0, atol=1e-12)
        assert np.allclose(gx[0], ex, rtol=0, atol=1e-11) and np.allclose(gy[0], ey, rtol=0, atol=1e-11)
        # IS^tau is the third-derivative part alone: h^4 |Omega| sum (D^l q)^2
        # over |l| = 3, with h^2 = |Omega|
        _, _, IStau, _ = T.indicators(fit)
        want = fit["area"] ** 3 * (36 * coef[6] ** 2 + 4 * coef[7] ** 2 + 4 * coef[8] ** 2 + 36 * coef[9] ** 2)
        assert IStau[0] == pytest.approx(want, rel=1e-9)


def test_quadratic_data_gives_chi_one_and_exact_states(T):
    mesh = inputs.tri_mesh(8, 8, 4)
    coef = np.random.default_rng(2).normal(size=6)
    W, dW, f, g = _poly_data(mesh, coef, ALL[:6])
    out, chi, info = T.reconstruct(mesh, W, dW)
    for c in _interior(mesh):
        assert info["IStau"][c, 0] <= 1e-13 * info["ISH"][c, 0]
        assert chi[c, 0] == 1.0
        tri = mesh["xv"][c]
        d1, d2 = tri[1] - tri[0], tri[2] - tri[0]
        h = math.sqrt(0.5 * abs(d1[0] * d2[1] - d1[1] * d2[0]))
        pts = T.edge_points(tri)
        for e in range(3):
            for q in range(2):
                x, y = pts[e, q]
                gx, gy = g(x, y)
                assert out[c, e, q, 0, 0] == pytest.approx(f(x, y), abs=1e-12)
                assert out[c, e, q, 0, 1] == pytest.approx(h * gx, abs=1e-12)
                assert out[c, e, q, 0, 2] == pytest.approx(h * gy, abs=1e-12)


def test_linear_data_closed_forms(T):
    # linear data: every candidate is the data itself; IS_k = IS^H =
    # |Omega| |grad|^2 (first derivatives only), IS^tau = 0
    mesh = inputs.tri_mesh(6, 6, 5)
    W, dW, f, g = _poly_data(mesh, [0.7, -1.3, 0.4], ALL[:3])
    for c in _interior(mesh, 2):
        fit = T.cell_fit(mesh, W, dW, c)
        ISH, ISH2, IStau, ISk = T.indicators(fit)
        want = fit["area"] * (1.3 ** 2 + 0.4 ** 2)
        assert np.allclose(ISk[:, 0], want, rtol=1e-12)
        assert ISH[0] == pytest.approx(want, rel=1e-12) and ISH2[0] == pytest.approx(want, rel=1e-12)
        assert IStau[0] <= 1e-14 * want
        assert np.allclose(fit["b"][:, 0], fit["h"] * np.array([-1.3, 0.4]), atol=1e-13)


def test_constant_state(T):
    mesh = inputs.tri_mesh(4, 5, 6)
    W = np.tile(np.array([1.2, -0.3, 0.5, 2.8])[:, None], (1, 40))
    out, chi, _ = T.reconstruct(mesh, W, np.zeros((2, 4, 40)))
    assert np.all(chi == 1.0)
    assert np.allclose(out[..., 0], np.array([1.2, -0.3, 0.5, 2.8]), rtol=0, atol=1e-14)
    assert np.abs(out[..., 1:]).max() < 1e-14


def test_fourth_order_on_smooth_data(T):
    # point values at the edge Gauss points converge at 4th order (the cubic
    # candidate) where the path function keeps chi = 1
    k = 2 * math.pi

    def f(x, y):
        return np.sin(k * x) * np.cos(k * y) + 0.5 * np.cos(k * (x + y))

    def g(x, y):
        return (k * np.cos(k * x) * np.cos(k * y) - 0.5 * k * np.sin(k * (x + y)),
                -k * np.sin(k * x) * np.sin(k * y) - 0.5 * k * np.sin(k * (x + y)))

    errs = []
    for n in (8, 16, 32):
        mesh = inputs.tri_mesh(n, n, 7)
        W, dW = inputs.tri_cell_data(mesh, f, g)
        out, chi, _ = T.reconstruct(mesh, W, dW)
        pts = np.stack([T.edge_points(t) for t in mesh["xv"]])
        errs.append(np.abs(out[..., 0, 0] - f(pts[..., 0], pts[..., 1])).max())
        if n == 32:
            assert (chi == 1.0).mean() > 0.9
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert orders[-1] > 3.5, (errs, orders)


def test_eno_at_a_jump(T):
    # a step along the lattice line x = 1/2 of an unperturbed mesh: no state
    # leaves the data range, the path function switches off next to the
    # jump, and cells whose edge neighbours are all on their side keep their
    # own (flat) value to rounding
    n = 8
    mesh = inputs.tri_mesh(n, n, 0, jitter=0.0)
    cen = mesh["xv"].mean(axis=1)
    W = np.where((cen[:, 0] > 0.5) & (cen[:, 0] < 1.0), 0.2, 1.0)[None, :]
    out, chi, _ = T.reconstruct(mesh, W, np.zeros((2, 1, W.shape[1])))
    assert out[..., 0, 0].min() > 0.2 - 1e-9 and out[..., 0, 0].max() < 1.0 + 1e-9
    nbr = mesh["nbr"]
    for c in range(W.shape[1]):
        near = [W[0, d] != W[0, c] for d in nbr[c]]
        if any(near):
            assert chi[c, 0] < 1e-6
            # the two candidates on the own side are flat and take the weight
            assert np.abs(out[c, ..., 0, 0] - W[0, c]).max() < 1e-9


def test_quarter_turn_symmetry(T):
    # turning mesh and data by 90 degrees, (x, y) -> (-y, x), turns every
    # state: the momenta and gradients rotate, the rest is unchanged (the
    # indicators sum each partial derivative once, which a quarter turn
    # permutes up to sign)
    mesh = inputs.tri_mesh(6, 5, 8)
    W, dW = inputs.tri_euler_jumps(mesh, 8)
    rot = lambda a: np.stack([-a[..., 1], a[..., 0]], axis=-1)
    m2 = {"xv": rot(mesh["xv"]), "nbr": mesh["nbr"], "shift": rot(mesh["shift"]), "nx": 6, "ny": 5}
    W2 = np.stack([W[0], -W[2], W[1], W[3]])
    # gradient of the turned field at the turned point: (d/dx', d/dy') = (-d/dy, d/dx)
    g = np.stack([-dW[1], dW[0]])
    dW2 = np.stack([g[:, 0], -g[:, 2], g[:, 1], g[:, 3]], axis=1)
    out, chi, _ = T.reconstruct(mesh, W, dW)
    out2, chi2, _ = T.reconstruct(m2, W2, dW2)
    assert np.allclose(chi2[:, [0, 3]], chi[:, [0, 3]], atol=1e-9)
    assert np.allclose(chi2[:, 1], chi[:, 2], atol=1e-9) and np.allclose(chi2[:, 2], chi[:, 1], atol=1e-9)
    # values: momenta turned
    v, v2 = out[..., 0], out2[..., 0]
    assert np.allclose(v2[..., [0, 3]], v[..., [0, 3]], atol=1e-12)
    assert np.allclose(v2[..., 1], -v[..., 2], atol=1e-12) and np.allclose(v2[..., 2], v[..., 1], atol=1e-12)
    # h-gradients: (d/dx', d/dy') = (-d/dy, d/dx), then the momenta turned
    gx2, gy2 = out2[..., 1], out2[..., 2]
    tx, ty = -out[..., 2], out[..., 1]
    assert np.allclose(gx2[..., [0, 3]], tx[..., [0, 3]], atol=1e-11)
    assert np.allclose(gy2[..., [0, 3]], ty[..., [0, 3]], atol=1e-11)
    assert np.allclose(gx2[..., 1], -tx[..., 2], atol=1e-11) and np.allclose(gx2[..., 2], tx[..., 1], atol=1e-11)
