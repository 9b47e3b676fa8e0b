"""Pins of the oracle's characteristic-variable reconstruction on the compact
path (no GPU). The paper does not say which variables its reconstruction
works on; the option projects each face's normal stencil on the eigenvectors
of the Euler flux Jacobian at the Roe average of the two cells at the face.
Each test checks a fact fixed by the Euler equations or by a path already
pinned: the Roe property and the flux Jacobian (by complex-step
differentiation of the flux), linear commutation where every path function
is 1, the 1-D path on y-invariant data, transpose symmetry and isolated
contacts.
"""
import numpy as np
import pytest

from paper_2507_20461_amd import inputs

GAMMA = 1.4


def _flux(W, direction):
    # Euler flux of the state W (rho, rho U, [rho V,] rho E) along x or y
    nv = len(W)
    e = nv - 1
    n = 1 + direction
    rho = W[0]
    ke = sum(W[k] * W[k] for k in range(1, e)) / rho
    p = (GAMMA - 1.0) * (W[e] - 0.5 * ke)
    un = W[n] / rho
    F = [W[n]] + [W[k] * un for k in range(1, e)] + [(W[e] + p) * un]
    F[n] = F[n] + p
    return np.array(F)


def _state(rng, nv):
    rho = rng.uniform(0.2, 2.0)
    vel = rng.uniform(-1.5, 1.5, size=nv - 2)
    p = rng.uniform(0.1, 3.0)
    return np.array([rho, *(rho * vel), p / (GAMMA - 1.0) + 0.5 * rho * (vel @ vel)])


@pytest.mark.parametrize("ndim,direction", [(1, 0), (2, 0), (2, 1)])
def test_roe_eigen_structure(oracle, ndim, direction):
    rng = np.random.default_rng(11 + direction + 3 * ndim)
    nv = 3 if ndim == 1 else 4
    prm = oracle.params(ndim=ndim)
    for _ in range(20):
        Wa, Wb = _state(rng, nv), _state(rng, nv)
        R, L, lam = oracle.roe_eigen(prm, ndim, direction, Wa, Wb)
        assert np.allclose(R @ L, np.eye(nv), atol=1e-12)
        A = R @ np.diag(lam) @ L
        # Roe's property: the averaged matrix maps the state jump to the flux jump
        dF = _flux(Wb, direction) - _flux(Wa, direction)
        assert np.allclose(A @ (Wb - Wa), dF, rtol=1e-11, atol=1e-11 * np.abs(dF).max())
        # equal states: the matrix is the flux Jacobian there (complex step,
        # exact to rounding for the analytic flux)
        R0, L0, lam0 = oracle.roe_eigen(prm, ndim, direction, Wa, Wa)
        A0 = R0 @ np.diag(lam0) @ L0
        h = 1e-30
        J = np.stack([_flux(Wa + 1j * h * np.eye(nv)[k], direction).imag / h for k in range(nv)], axis=1)
        assert np.allclose(A0, J, rtol=1e-11, atol=1e-11 * np.abs(J).max())
        # speeds of the Jacobian: un - c, un (twice in 2-D), un + c
        rho = Wa[0]
        vel = Wa[1:nv - 1] / rho
        c = np.sqrt(GAMMA * (GAMMA - 1.0) * (Wa[-1] - 0.5 * rho * vel @ vel) / rho)
        un = vel[direction]
        want = [un - c, un, un + c] if nv == 3 else [un - c, un, un, un + c]
        assert np.allclose(lam0, want, rtol=1e-13, atol=1e-13)


def test_roe_eigen_rejects_imaginary_sound_speed(oracle):
    # a state of negative pressure on both sides: no real sound speed
    W = np.array([1.0, 2.0, 0.0, 1.0])
    with pytest.raises(Exception):
        oracle.roe_eigen(oracle.params(ndim=2), 2, 0, W, W)


def _transpose(W, dW):
    Wt = np.stack([W[0].T, W[2].T, W[1].T, W[3].T])
    dWt = np.concatenate([np.stack([dW[4 + k].T for k in (0, 2, 1, 3)]),
                          np.stack([dW[k].T for k in (0, 2, 1, 3)])])
    return Wt, dWt


@pytest.mark.parametrize("direction", [0, 1])
def test_characteristic_commutes_where_linear_2d(oracle, direction):
    # where every path function is 1 the normal reconstruction of values and
    # h-derivatives is linear, so it commutes with the face-wise projection
    W, dW = inputs.random_smooth_2d(48, 40, 7, modes=2)
    a, ca = oracle.normal_faces(oracle.params(ndim=2, bc=oracle.PERIODIC), W, dW, direction)
    b, cb = oracle.normal_faces(oracle.params(ndim=2, bc=oracle.PERIODIC, characteristic=True), W, dW,
                                direction)
    lin = np.all(ca == 1.0, axis=(0, 1)) & np.all(cb == 1.0, axis=(0, 1))
    assert lin.mean() > 0.4
    assert np.allclose(a[..., lin], b[..., lin], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("case", ["sine", "jump"])
def test_characteristic_y_invariant_equals_1d(oracle, case):
    # 2-D data without y-dependence and with V = 0 decouples the shear field:
    # the x-faces of every row carry the 1-D characteristic reconstruction
    n, ny = 48, 4
    if case == "sine":
        W1, dW1 = inputs.sine_1d(n)
        bc = oracle.PERIODIC
    else:
        W1, dW1, _ = inputs.jump_1d(n, 2)
        bc = oracle.TRANSMISSIVE
    W2 = np.zeros((4, ny, n))
    dW2 = np.zeros((8, ny, n))
    for v2, v1 in ((0, 0), (1, 1), (3, 2)):
        W2[v2] = W1[v1, 0]
        dW2[v2] = dW1[v1, 0]
    o1, c1 = oracle.normal_faces(oracle.params(ndim=1, bc=bc, characteristic=True), W1, dW1)
    o2, c2 = oracle.normal_faces(oracle.params(ndim=2, bc=bc, characteristic=True), W2, dW2, 0,
                                 dx=1.0 / n, dy=1.0 / ny)
    sc = np.abs(W1).max()
    for a in range(ny + 2):
        got = o2[:, :, [0, 1, 3], a, :]
        assert np.allclose(got, o1[:, :, :, 0, :], rtol=1e-12, atol=1e-12 * sc)
        assert np.abs(o2[:, :, 2, a, :]).max() < 1e-13 * sc
        # chi of the acoustic and entropy fields; the shear field is zero
        assert np.abs(c2[:, [0, 1, 3], a, :] - c1[:, :, 0, :]).max() < 1e-8


def test_characteristic_transpose_symmetry(oracle):
    W, dW, _ = inputs.quadrants_2d(16, 12, 4)
    Ws, dWs = inputs.random_smooth_2d(16, 12, 5)
    W = W + 0.1 * (Ws - Ws.mean(axis=(1, 2), keepdims=True))
    dW = dW + 0.1 * dWs
    prm = oracle.params(ndim=2, bc=oracle.TRANSMISSIVE, characteristic=True)
    ox, _ = oracle.normal_faces(prm, W, dW, 0, dx=1.0 / 16, dy=1.0 / 12)
    Wt, dWt = _transpose(W, dW)
    oy, _ = oracle.normal_faces(prm, Wt, dWt, 1, dx=1.0 / 12, dy=1.0 / 16)
    # y-faces of the transposed data are the transposed x-faces, momentum swapped
    want = ox[:, :, [0, 2, 1, 3]].transpose(0, 1, 2, 4, 3)
    assert np.allclose(oy, want, rtol=1e-12, atol=1e-12 * np.abs(W).max())
    # whole steps too (tangential step, flux, update)
    a, da, _, _ = oracle.step(prm, W, dW, 2)
    b, db, _, _ = oracle.step(prm, Wt, dWt, 2)
    assert np.allclose(b, np.stack([a[0].T, a[2].T, a[1].T, a[3].T]), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("direction", [0, 1])
def test_characteristic_oblique_contact_2d(oracle, direction):
    # a density jump carried by uniform (U, V) and p is a multiple of the
    # entropy eigenvector at every Roe average along the normal, so the
    # characteristic face states keep U, V and p exactly
    n = 24
    idx = np.arange(n)
    jump = np.where(idx < n // 2, 1.0, 0.25)
    rho = np.broadcast_to(jump[None, :] if direction == 0 else jump[:, None], (n, n)).copy()
    U, V, p = 0.4, -0.3, 1.0
    W = np.stack([rho, rho * U, rho * V, p / (GAMMA - 1.0) + 0.5 * rho * (U * U + V * V)])
    o, _ = oracle.normal_faces(oracle.params(ndim=2, bc=oracle.TRANSMISSIVE, characteristic=True),
                               W, np.zeros((8, n, n)), direction)
    for side in range(2):
        S = o[side, 0]
        assert np.allclose(S[1] / S[0], U, atol=1e-12)
        assert np.allclose(S[2] / S[0], V, atol=1e-12)
        pf = (GAMMA - 1.0) * (S[3] - 0.5 * (S[1] ** 2 + S[2] ** 2) / S[0])
        assert np.allclose(pf, p, atol=1e-12)
        # the jump itself is reconstructed without overshoot
        assert S[0].min() > 0.25 - 1e-12 and S[0].max() < 1.0 + 1e-12
