"""CPU FP64 oracle of the compact GKS step on triangular meshes: the GENO
reconstruction of Sec. 4.3 (oracle/geno_tri.py), the gas-kinetic flux at the
two Gauss points of every edge (the point solution of oracle/oracle.py), the
finite-volume update of the cell averages (Eq. (1)) and of the cell-averaged
gradients by the Gauss theorem (Eq. (2)), advanced by the two-stage
fourth-order method as on the structured grids.

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import this module. It shares no
code with the HIP library or its binding: numpy over edges and cells, in the
order of the steps below.

One stage from cell averages W [4, ncell] and averaged gradients dW [2, 4,
ncell] (x then y rows), conserved variables (rho, rho u, rho v, rho E):
  1. GENO states of every cell at the Gauss points of its edges: value,
     gradient and second derivatives (those of the cubic candidate times chi).
  2. Per edge, once (from its owner cell, the one with the smaller (cell,
     edge) pair), at each Gauss point: the owner's state on the left, the
     neighbour's on the right (its Gauss points run the other way along the
     edge); a side whose state has rho <= 0, p <= 0 or a non-finite value
     takes its own cell average with zero derivatives, and the mean second
     derivative is then zero. In the frame of the owner's outward unit normal
     n and t = (-n_y, n_x) (momentum components rotated, derivatives along n
     and t, second derivatives n.H.n, n.H.t, t.H.t): the point flux F, its
     time derivative dF/dt (two-point time fit), the interface states W(dt/2)
     and W(dt) and the weighted equilibrium second time derivative phi W_tt,
     then rotated back and averaged over the two points (weights 1/2).
  3. Per cell: L = -(1/|Omega|) sum_edges |e| F.n_out (the owner's F with a
     minus sign on the other cell), the same for dF/dt, and the gradient of
     an interface field w by the Gauss theorem, (1/|Omega|) sum_edges |e| w
     n_out.
The step: stage 1 W* = W + dt/2 L + dt^2/8 L_t, R = W + dt L + dt^2/6 L_t,
grad W* from W(dt/2) + dt^2/8 phi W_tt, and RG = the gradient of W(dt) +
dt^2/6 phi W_tt; stage 2 (from W*, grad W*) W^{n+1} = R + dt^2/3 L_t*,
grad W^{n+1} = RG + dt^2/3 (gradient of phi* W_tt*).
dt = CFL min over cells of d / (|u| + c), d = 4 |Omega| / perimeter (the
inscribed circle's diameter; reading, the paper gives no mesh measure for
the time step on triangles).
"""
from __future__ import annotations

import math

import numpy as np

from . import geno_tri as T
from . import oracle as O

GAMMA = 1.4


def geometry(mesh):
    """Per cell: area, h = sqrt(area), d = 4 area / perimeter; per (cell,
    edge): outward unit normal, length, neighbour, the neighbour's edge index
    of the same edge (rev) and whether the cell owns the edge."""
    xv, nbr, sh = np.asarray(mesh["xv"], dtype=np.float64), np.asarray(mesh["nbr"]), np.asarray(mesh["shift"])
    n = xv.shape[0]
    area = 0.5 * ((xv[:, 1, 0] - xv[:, 0, 0]) * (xv[:, 2, 1] - xv[:, 0, 1])
                  - (xv[:, 2, 0] - xv[:, 0, 0]) * (xv[:, 1, 1] - xv[:, 0, 1]))
    normal = np.zeros((n, 3, 2))
    length = np.zeros((n, 3))
    for e in range(3):
        d = xv[:, (e + 1) % 3] - xv[:, e]
        length[:, e] = np.hypot(d[:, 0], d[:, 1])
        normal[:, e, 0] = d[:, 1] / length[:, e]
        normal[:, e, 1] = -d[:, 0] / length[:, e]
    rev = np.full((n, 3), -1, dtype=np.int64)
    for c in range(n):
        for e in range(3):
            m = int(nbr[c, e])
            for f in range(3):
                if int(nbr[m, f]) == c and np.allclose(sh[m, f], -sh[c, e]):
                    rev[c, e] = f
    if np.any(rev < 0):
        raise ValueError("mesh: an edge without its reverse")
    owner = np.zeros((n, 3), dtype=bool)
    for c in range(n):
        for e in range(3):
            owner[c, e] = (c, e) < (int(nbr[c, e]), int(rev[c, e]))
    perim = length.sum(axis=1)
    return {"area": area, "h": np.sqrt(area), "d": 4.0 * area / perim, "normal": normal,
            "length": length, "nbr": nbr.astype(np.int64), "rev": rev, "owner": owner}


def primitives(W, gamma=GAMMA):
    rho = W[0]
    u, v = W[1] / rho, W[2] / rho
    p = (gamma - 1.0) * (W[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def cfl_dt(geo, W, cfl=0.5, gamma=GAMMA):
    rho, u, v, p = primitives(W, gamma)
    c = np.sqrt(gamma * p / rho)
    return cfl * float(np.min(geo["d"] / (np.hypot(u, v) + c)))


def _rot(Q, n):
    """xy frame -> face frame of normal n: momentum (q1, q2) -> (q.n, q.t),
    t = (-n_y, n_x). Q [..., 4], n [..., 2]."""
    out = Q.copy()
    out[..., 1] = Q[..., 1] * n[..., 0] + Q[..., 2] * n[..., 1]
    out[..., 2] = -Q[..., 1] * n[..., 1] + Q[..., 2] * n[..., 0]
    return out


def _unrot(Q, n):
    out = Q.copy()
    out[..., 1] = Q[..., 1] * n[..., 0] - Q[..., 2] * n[..., 1]
    out[..., 2] = Q[..., 1] * n[..., 1] + Q[..., 2] * n[..., 0]
    return out


def _admissible(Wp, gamma=GAMMA):
    rho, _, _, p = primitives(Wp.T, gamma)
    return np.isfinite(Wp).all(axis=1) & (rho > 0.0) & (p > 0.0)


def edge_fluxes(mesh, geo, W, dW, dt, prm_gks, prm_geno=None, stage=1):
    """Step 2 on every owned edge. Returns per (cell, edge) arrays [n, 3, 4]
    (xy frame; rows of edges the cell does not own stay zero): F, dF/dt and
    the two interface fields (stage 1: W(dt/2) + dt^2/8 phi W_tt and
    W(dt) + dt^2/6 phi W_tt; stage 2: phi W_tt and zero), and the number of
    guarded sides."""
    out, _, info = T.reconstruct(mesh, W, dW, prm_geno, second=True)
    sec = info["second"]
    n = W.shape[1]
    h = geo["h"]
    cs, es = np.nonzero(geo["owner"])
    res = [np.zeros((n, 3, 4)) for _ in range(4)]
    guard = 0
    acc = [np.zeros((cs.size, 4)) for _ in range(4)]
    for g in range(2):
        nb, rv = geo["nbr"][cs, es], geo["rev"][cs, es]
        nrm = geo["normal"][cs, es]
        tng = np.stack([-nrm[:, 1], nrm[:, 0]], axis=-1)
        sides = []
        for cell, edge, gp in ((cs, es, g), (nb, rv, 1 - g)):
            o = out[cell, edge, gp]                        # [npts, nv, 3]
            s2 = sec[cell, edge, gp]                       # [npts, nv, 3]
            hh = h[cell][:, None]
            val, gx, gy = o[..., 0], o[..., 1] / hh, o[..., 2] / hh
            xx, xy, yy = (s2[..., k] / (hh * hh) for k in range(3))
            ok = _admissible(val)
            val = np.where(ok[:, None], val, W[:, cell].T)
            gx = np.where(ok[:, None], gx, 0.0)
            gy = np.where(ok[:, None], gy, 0.0)
            nx_, ny_ = nrm[:, 0:1], nrm[:, 1:2]
            tx, ty = tng[:, 0:1], tng[:, 1:2]
            dn = gx * nx_ + gy * ny_
            dtg = gx * tx + gy * ty
            snn = xx * nx_ * nx_ + 2.0 * xy * nx_ * ny_ + yy * ny_ * ny_
            snt = xx * nx_ * tx + xy * (nx_ * ty + ny_ * tx) + yy * ny_ * ty
            stt = xx * tx * tx + 2.0 * xy * tx * ty + yy * ty * ty
            sides.append((ok, _rot(val, nrm), _rot(dn, nrm), _rot(dtg, nrm),
                          [_rot(q, nrm) for q in (snn, snt, stt)]))
        (okl, Wl, nl, tl, sl), (okr, Wr, nr, tr, sr) = sides
        guard += int((~okl).sum() + (~okr).sum())
        both = (okl & okr)[:, None]
        s2m = np.stack([np.where(both, 0.5 * (a + b), 0.0) for a, b in zip(sl, sr)], axis=1)
        F, Ft, Wh, Wf, W2 = O.gks_points(prm_gks, 2, Wl, Wr, nl, nr, tl, tr, dt=dt, sec=s2m, full=True)
        if stage == 1:
            parts = (F, Ft, Wh + dt * dt / 8.0 * W2, Wf + dt * dt / 6.0 * W2)
        else:
            parts = (np.zeros_like(F), Ft, W2, np.zeros_like(F))
        for a, q in zip(acc, parts):
            a += 0.5 * _unrot(q, nrm)
    for r, a in zip(res, acc):
        r[cs, es] = a
    return res, guard


def cell_terms(geo, res):
    """Step 3: L and dL/dt [4, n] and the Gauss-theorem gradients [2, 4, n] of
    the two interface fields."""
    n = geo["area"].size
    F, Ft, Wa, Wb = res
    L, Lt = np.zeros((4, n)), np.zeros((4, n))
    Ga, Gb = np.zeros((2, 4, n)), np.zeros((2, 4, n))
    for e in range(3):
        own = geo["owner"][:, e]
        nb, rv = geo["nbr"][:, e], geo["rev"][:, e]
        sgn = np.where(own, 1.0, -1.0)[:, None]
        pick = lambda A: np.where(own[:, None], A[:, e], A[nb, rv])
        ln = geo["length"][:, e][:, None]
        nrm = geo["normal"][:, e]
        L -= (sgn * ln * pick(F)).T
        Lt -= (sgn * ln * pick(Ft)).T
        for G, A in ((Ga, Wa), (Gb, Wb)):
            w = ln * pick(A)
            G[0] += (w * nrm[:, 0:1]).T
            G[1] += (w * nrm[:, 1:2]).T
    ia = 1.0 / geo["area"]
    return L * ia, Lt * ia, Ga * ia, Gb * ia


def step(mesh, W, dW, nsteps, cfl=0.5, gamma=GAMMA, tau_c1=0.0, tau_c2=1.0, fixed_dt=None, geo=None):
    """nsteps two-stage steps. Returns W, dW, the dt of each step and the
    guarded sides."""
    geo = geometry(mesh) if geo is None else geo
    prm = O.params(ndim=2, gamma=gamma, tau_c1=tau_c1, tau_c2=tau_c2, cfl=cfl)
    W = np.array(W, dtype=np.float64)
    dW = np.array(dW, dtype=np.float64)
    dts, guard = [], 0
    for _ in range(nsteps):
        dt = float(fixed_dt) if fixed_dt else cfl_dt(geo, W, cfl, gamma)
        dts.append(dt)
        res, g1 = edge_fluxes(mesh, geo, W, dW, dt, prm, stage=1)
        L, Lt, Ga, Gb = cell_terms(geo, res)
        Ws = W + 0.5 * dt * L + dt * dt / 8.0 * Lt
        R = W + dt * L + dt * dt / 6.0 * Lt
        dWs, RG = Ga, Gb
        res2, g2 = edge_fluxes(mesh, geo, Ws, dWs, dt, prm, stage=2)
        _, Lt2, Ga2, _ = cell_terms(geo, res2)
        W = R + dt * dt / 3.0 * Lt2
        dW = RG + dt * dt / 3.0 * Ga2
        guard += g1 + g2
    return W, dW, np.array(dts), guard
