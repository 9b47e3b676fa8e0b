"""CPU FP64 oracle of the fourth-order compact GENO reconstruction on
triangular meshes (Sec. 4.3, with the GENO blend, path function, smoothness
indicators and ENO weights of Sec. 3).

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import this module. It shares no
code with the HIP library or its binding; plain numpy, per cell, in the
paper's steps.

Per cell Omega_j (the target) and per conserved variable:
  * S_0 = Omega_j, its three edge neighbours Omega_{j_k} and their other
    neighbours (six cells); q^H = p^3 is the cubic whose average on
    Omega_j is exact and which fits, in least squares, the averages of the
    other nine cells and the h-scaled averaged gradients of Omega_j and of
    the three edge neighbours (reading: the paper defers the compact
    least-squares reconstruction to its references);
  * S_k = {Omega_j, Omega_{j_k}}, k = 1..3: the linear polynomial whose
    average on Omega_j is exact and which fits, in least squares, the
    average and the h-scaled averaged gradient of Omega_{j_k};
  * IS^H = sum_{|l|=1..3} h^{2|l|-m} int (D^l q^H)^2 (Eq. IS-highorder-1,
    m = 2), IS~^H the same over |l| = 1, 2, IS^tau = |IS^H - IS~^H|;
    IS_k of the linear p_k (|l| = 1); IS^L = (sum IS_k - min - max)/(k_0 - 2);
    alpha from Eq. (5) with r = 3; chi = tanh(C alpha)/tanh(C);
    w_k = d_k/(IS_k + eps)^2 normalised, d_k = 1 (no central sub-stencil);
  * R = chi p^3 + (1 - chi) sum_k w_k p_k, value and h-scaled gradient at
    the two Gauss points of each edge.
h = sqrt(|Omega_j|) (reading: the paper names the mesh cell size).
Sums over l run over multi-indices, each partial derivative once.
"""
from __future__ import annotations

import math

import numpy as np

# monomials xi^a eta^b of degree 1..3 (the constant is fixed by the average)
EXPS = [(1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]
# multi-indices of the smoothness indicator, by order
MULTI = {1: [(1, 0), (0, 1)], 2: [(2, 0), (1, 1), (0, 2)], 3: [(3, 0), (2, 1), (1, 2), (0, 3)]}
GAUSS_T = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))

# collapsed Gauss-Legendre rule on the reference triangle (7 x 7 points,
# exact to degree 13), barycentric coordinates and weights summing to 1
_g = np.polynomial.legendre.leggauss(7)
_s, _t = np.meshgrid(0.5 * (_g[0] + 1.0), 0.5 * (_g[0] + 1.0), indexing="ij")
_w = (np.outer(0.5 * _g[1], 0.5 * _g[1]) * 2.0 * (1.0 - _s)).ravel()
_B1 = _s.ravel()
_B2 = ((1.0 - _s) * _t).ravel()
_B0 = 1.0 - _B1 - _B2


def params(C=20.0, eps=1e-15, r=3.0, rL=2.0, d=(1.0, 1.0, 1.0)):
    """Method constants: C = 20, eps = 1e-15 (Sec. 3), r = 3 on unstructured
    meshes (Sec. 3), r^L = 2, d_k = 1."""
    return {"C": C, "eps": eps, "r": r, "rL": rL, "d": np.asarray(d, dtype=np.float64)}


def _quad(tri):
    """Quadrature points [npts, 2] and weights (sum 1) on triangle tri [3, 2]."""
    pts = _B0[:, None] * tri[0] + _B1[:, None] * tri[1] + _B2[:, None] * tri[2]
    return pts, _w


def _area(tri):
    return 0.5 * ((tri[1, 0] - tri[0, 0]) * (tri[2, 1] - tri[0, 1])
                  - (tri[2, 0] - tri[0, 0]) * (tri[1, 1] - tri[0, 1]))


def _mono(x, y, a, b, da=0, db=0):
    """d^(da+db)/dxi^da deta^db of xi^a eta^b at (x, y) already scaled."""
    if da > a or db > b:
        return np.zeros_like(x)
    ca = math.factorial(a) // math.factorial(a - da)
    cb = math.factorial(b) // math.factorial(b - db)
    return ca * cb * x ** (a - da) * y ** (b - db)


def stencil(mesh, c):
    """Cells of S_0 of cell c with their translations: the edge neighbours
    (k = 0..2, across edge k) and then their other neighbours (two each)."""
    nbr, sh = mesh["nbr"], mesh["shift"]
    face = [(int(nbr[c, k]), sh[c, k].copy()) for k in range(3)]
    second = []
    for d, s in face:
        for f in range(3):
            e, t = int(nbr[d, f]), s + sh[d, f]
            if e == c and np.allclose(t, 0.0):
                continue
            second.append((e, t))
    return face, second


def cell_fit(mesh, W, dW, c):
    """The polynomials of cell c for every variable: p^3 coefficients a
    [nv, 9] (of xi^a eta^b minus their averages on the cell, in EXPS order),
    the linear p_k gradients b [3, nv, 2] (in xi, eta) and the geometry."""
    xv = mesh["xv"]
    tri = xv[c]
    area = _area(tri)
    h = math.sqrt(area)
    xc = tri.mean(axis=0)
    face, second = stencil(mesh, c)

    def scaled_pts(t):
        p, w = _quad(t)
        return (p[:, 0] - xc[0]) / h, (p[:, 1] - xc[1]) / h, w

    xi, eta, w = scaled_pts(tri)
    m = np.array([(w * _mono(xi, eta, a, b)).sum() for a, b in EXPS])
    rows, rhs = [], []
    for d, s in face + second:
        x2, y2, w2 = scaled_pts(xv[d] + s)
        rows.append([(w2 * _mono(x2, y2, a, b)).sum() - m[k] for k, (a, b) in enumerate(EXPS)])
        rhs.append(W[:, d] - W[:, c])
    for d, s in [(c, np.zeros(2))] + face:
        x2, y2, w2 = scaled_pts(xv[d] + s)
        # h * d/dx of (xi^a eta^b) = d/dxi of it
        rows.append([(w2 * _mono(x2, y2, a, b, 1, 0)).sum() for a, b in EXPS])
        rhs.append(h * dW[0, :, d])
        rows.append([(w2 * _mono(x2, y2, a, b, 0, 1)).sum() for a, b in EXPS])
        rhs.append(h * dW[1, :, d])
    A = np.array(rows)
    a = np.linalg.lstsq(A, np.array(rhs), rcond=None)[0].T     # [nv, 9]
    b = np.zeros((3, W.shape[0], 2))
    for k, (d, s) in enumerate(face):
        cen = ((xv[d] + s).mean(axis=0) - xc) / h
        Ak = np.array([cen, [1.0, 0.0], [0.0, 1.0]])
        rk = np.stack([W[:, d] - W[:, c], h * dW[0, :, d], h * dW[1, :, d]])
        b[k] = np.linalg.lstsq(Ak, rk, rcond=None)[0].T
    return {"a": a, "b": b, "m": m, "h": h, "area": area, "xc": xc, "tri": tri}


def p3_at(fit, Wc, x, y):
    """Value and gradient (d/dx, d/dy) of p^3 at physical points."""
    h, xc, a, m = fit["h"], fit["xc"], fit["a"], fit["m"]
    xi, eta = (np.asarray(x) - xc[0]) / h, (np.asarray(y) - xc[1]) / h
    val = Wc[:, None] + sum(a[:, k, None] * (_mono(xi, eta, p, q) - m[k]) for k, (p, q) in enumerate(EXPS))
    gx = sum(a[:, k, None] * _mono(xi, eta, p, q, 1, 0) for k, (p, q) in enumerate(EXPS)) / h
    gy = sum(a[:, k, None] * _mono(xi, eta, p, q, 0, 1) for k, (p, q) in enumerate(EXPS)) / h
    return val, gx, gy


def indicators(fit):
    """IS^H, IS~^H, IS^tau [nv] and IS_k [3, nv] of a cell (Eq. IS-highorder-1
    and -2 on the unstructured mesh, Eq. IS-tau)."""
    h, area, a, tri, xc = fit["h"], fit["area"], fit["a"], fit["tri"], fit["xc"]
    p, w = _quad(tri)
    xi, eta = (p[:, 0] - xc[0]) / h, (p[:, 1] - xc[1]) / h
    terms = {}
    for order, ls in MULTI.items():
        tot = 0.0
        for la, lb in ls:
            # physical derivative: h^-|l| times the derivative in (xi, eta)
            D = sum(a[:, k, None] * _mono(xi, eta, p_, q_, la, lb) for k, (p_, q_) in enumerate(EXPS)) / h ** order
            tot = tot + h ** (2 * order - 2) * area * (w * D * D).sum(axis=1)
        terms[order] = tot
    ISH = terms[1] + terms[2] + terms[3]
    ISH2 = terms[1] + terms[2]
    IStau = np.abs(ISH - ISH2)
    # linear p_k: |l| = 1 only, h^0, constant gradient b_k / h
    ISk = np.stack([area * ((fit["b"][k] / h) ** 2).sum(axis=1) for k in range(3)])
    return ISH, ISH2, IStau, ISk


def path(prm, IStau, ISH, ISL):
    """chi of Eq. (4) from alpha of Eq. (5) with exponent r."""
    aH = 1.0 + (IStau / (ISH + prm["eps"])) ** prm["r"]
    aL = 1.0 + (IStau / (ISL + prm["eps"])) ** prm["r"]
    alpha = 2.0 * aH / (aH + aL)
    return np.tanh(prm["C"] * alpha) / math.tanh(prm["C"]), alpha


def edge_points(tri):
    """The two Gauss points of each edge e (from vertex e to e + 1): [3, 2, 2]."""
    out = np.zeros((3, 2, 2))
    for e in range(3):
        p, q = tri[e], tri[(e + 1) % 3]
        for g, t in enumerate(GAUSS_T):
            out[e, g] = p + t * (q - p)
    return out


def p3_second_at(fit, x, y):
    """h^2 times the second derivatives (d_xx, d_xy, d_yy) of p^3 at physical
    points: [nv, npts, 3] (the second derivatives in xi, eta)."""
    h, xc, a = fit["h"], fit["xc"], fit["a"]
    xi, eta = (np.asarray(x) - xc[0]) / h, (np.asarray(y) - xc[1]) / h
    out = [sum(a[:, k, None] * _mono(xi, eta, p, q, da, db) for k, (p, q) in enumerate(EXPS))
           for da, db in ((2, 0), (1, 1), (0, 2))]
    return np.stack(out, axis=-1)


def reconstruct(mesh, W, dW, prm=None, cells=None, second=False):
    """GENO states of every cell (or of the listed cells) at the Gauss points
    of its edges. W [nv, ncell] cell averages, dW [2, nv, ncell] averaged
    gradients. Returns out [ncell, 3 edges, 2 points, nv, 3 (value, h d/dx,
    h d/dy)], chi [ncell, nv] and info: the indicators {ISH, IStau, ISL}
    [ncell, nv] and the two candidates of the blend, high (the cubic q^H) and
    low (q^L), in the layout of out (rows of cells not listed stay zero).
    With second=True, info also holds "second" [ncell, 3, 2, nv, 3]: h^2 times
    the second derivatives (d_xx, d_xy, d_yy) of the blend, chi times those
    of the cubic (the linear candidates have none; Eq. (3) applied to the
    second derivatives), and "second_high", those of the cubic."""
    prm = params() if prm is None else prm
    W = np.asarray(W, dtype=np.float64)
    dW = np.asarray(dW, dtype=np.float64)
    nv, n = W.shape
    out = np.zeros((n, 3, 2, nv, 3))
    chi = np.zeros((n, nv))
    info = {"ISH": np.zeros((n, nv)), "IStau": np.zeros((n, nv)), "ISL": np.zeros((n, nv)),
            "high": np.zeros((n, 3, 2, nv, 3)), "low": np.zeros((n, 3, 2, nv, 3))}
    if second:
        info["second"] = np.zeros((n, 3, 2, nv, 3))
        info["second_high"] = np.zeros((n, 3, 2, nv, 3))
    for c in (range(n) if cells is None else cells):
        fit = cell_fit(mesh, W, dW, c)
        ISH, _, IStau, ISk = indicators(fit)
        k0 = ISk.shape[0]
        ISL = (ISk.sum(axis=0) - ISk.min(axis=0) - ISk.max(axis=0)) / (k0 - 2)
        x, _ = path(prm, IStau, ISH, ISL)
        wt = prm["d"][:, None] / (ISk + prm["eps"]) ** prm["rL"]
        wt = wt / wt.sum(axis=0)
        chi[c] = x
        info["ISH"][c], info["IStau"][c], info["ISL"][c] = ISH, IStau, ISL
        h, xc = fit["h"], fit["xc"]
        pts = edge_points(fit["tri"]).reshape(6, 2)
        v3, gx3, gy3 = p3_at(fit, W[:, c], pts[:, 0], pts[:, 1])
        # p_k = W_j + b_k . (x - x_j) / h
        rel = (pts - xc) / h
        vL = sum(wt[k, :, None] * (W[:, c, None] + fit["b"][k] @ rel.T) for k in range(k0))
        gL = sum(wt[k, :, None] * fit["b"][k] for k in range(k0))      # h * gradient, [nv, 2]
        val = x[:, None] * v3 + (1.0 - x[:, None]) * vL
        hgx = x[:, None] * h * gx3 + (1.0 - x[:, None]) * gL[:, 0, None]
        hgy = x[:, None] * h * gy3 + (1.0 - x[:, None]) * gL[:, 1, None]
        o = np.stack([val, hgx, hgy], axis=-1)      # [nv, 6, 3]
        out[c] = o.transpose(1, 0, 2).reshape(3, 2, nv, 3)
        hi = np.stack([v3, h * gx3, h * gy3], axis=-1)
        lo = np.stack([vL, np.broadcast_to(gL[:, 0, None], vL.shape), np.broadcast_to(gL[:, 1, None], vL.shape)],
                      axis=-1)
        info["high"][c] = hi.transpose(1, 0, 2).reshape(3, 2, nv, 3)
        info["low"][c] = lo.transpose(1, 0, 2).reshape(3, 2, nv, 3)
        if second:
            s3 = p3_second_at(fit, pts[:, 0], pts[:, 1])                       # [nv, 6, 3]
            s2 = x[:, None, None] * s3
            info["second"][c] = s2.transpose(1, 0, 2).reshape(3, 2, nv, 3)
            info["second_high"][c] = s3.transpose(1, 0, 2).reshape(3, 2, nv, 3)
    return out, chi, info
