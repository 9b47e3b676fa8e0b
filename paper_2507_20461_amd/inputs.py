"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds initial data only (cell averages and cell-averaged
gradients of analytic or seeded piecewise-constant states); it contains none
of the reconstruction, flux or time-stepping arithmetic.

Arrays are interior-only SoA, ``W[field, y, x]`` and ``dW[d * nv + field, y, x]``
(``d`` = 0 for d/dx, 1 for d/dy), float64. In 1-D, ``ny = 1``.
Fields: 1-D ``(rho, rhoU, rhoE)``; 2-D ``(rho, rhoU, rhoV, rhoE)``.

Workloads (sizes of the paper's structured tests are 1-D; the 2-D and batched
recipes are synthetic stand-ins for throughput measurement):

* ``sine_1d``: density wave rho = 1 + 0.2 sin(2 pi x), U = 1, p = 1 on [0, 1],
  periodic (the 1-D accuracy test of Sec. 6.1 rescaled from [0, 2]).
* ``jump_1d``: one jump at x = 1/2 between two seeded states.
* ``quadrants_2d``: four seeded constant quadrants, jumps on the lines x = 1/2
  and y = 1/2.
* ``vortex_2d``: ``quadrants_2d`` plus a smooth vortex perturbation of the
  velocity.
* ``batched_grids``: many independent quadrant grids of seeded sizes.
* ``blast_wave_1d``: the Woodward-Colella interacting blast waves on [0, 1]
  with reflecting walls (p = 1000 | 0.01 | 100, rho = 1, u = 0).
* ``shu_osher_1d``: a Mach-3 shock running into the density wave
  rho = 1 + 0.2 sin(5 x) on [-5, 5] (transmissive).
  Both are the analytic robustness problems of the paper's Sec. 6.2.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4


def _cons_1d(rho, u, p, gamma=GAMMA):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def _cons_2d(rho, u, v, p, gamma=GAMMA):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def sine_1d(nx: int, amp: float = 0.2, gamma: float = GAMMA):
    """Exact cell averages and averaged gradients of rho = 1 + amp sin(2 pi x), U = p = 1."""
    h = 1.0 / nx
    xl = np.arange(nx) * h
    xr = xl + h
    k = 2.0 * math.pi
    rho_avg = 1.0 + amp * (np.cos(k * xl) - np.cos(k * xr)) / (k * h)
    W = _cons_1d(rho_avg, np.ones(nx), np.ones(nx), gamma)
    # rhoU = rho and rhoE = p/(g-1) + rho/2 are affine in rho: averages are exact.
    W[1] = rho_avg
    W[2] = 1.0 / (gamma - 1.0) + 0.5 * rho_avg

    def point(x):
        r = 1.0 + amp * np.sin(k * x)
        return np.stack([r, r, 1.0 / (gamma - 1.0) + 0.5 * r])

    dW = (point(xr) - point(xl)) / h
    return W.reshape(3, 1, nx), dW.reshape(3, 1, nx)


def sine_1d_exact(nx: int, t: float, amp: float = 0.2, gamma: float = GAMMA):
    """Exact cell averages of the advected sine at time t (U = 1, period 1)."""
    h = 1.0 / nx
    xl = np.arange(nx) * h - t
    xr = xl + h
    k = 2.0 * math.pi
    rho_avg = 1.0 + amp * (np.cos(k * xl) - np.cos(k * xr)) / (k * h)
    return np.stack([rho_avg, rho_avg, 1.0 / (gamma - 1.0) + 0.5 * rho_avg]).reshape(3, 1, nx)


def jump_1d(nx: int, seed: int, gamma: float = GAMMA):
    """Jump at x = 1/2 between (rho, u, p)_L and (rho, u, p)_R; rho, p ~ U[0.1, 1.5],
    u ~ U[-0.5, 0.5], drawn left state first in the order (rho, u, p)."""
    rng = np.random.default_rng(seed)
    states = []
    for _ in range(2):
        rho = rng.uniform(0.1, 1.5)
        u = rng.uniform(-0.5, 0.5)
        p = rng.uniform(0.1, 1.5)
        states.append((rho, u, p))
    xc = (np.arange(nx) + 0.5) / nx
    left = xc < 0.5
    rho = np.where(left, states[0][0], states[1][0])
    u = np.where(left, states[0][1], states[1][1])
    p = np.where(left, states[0][2], states[1][2])
    W = _cons_1d(rho, u, p, gamma).reshape(3, 1, nx)
    return W, np.zeros_like(W), states


def quadrant_states(rng):
    """Four (rho, u, v, p) states in the order q1 (x>1/2, y>1/2), q2 (x<1/2, y>1/2),
    q3 (x<1/2, y<1/2), q4 (x>1/2, y<1/2); rho ~ U[0.5,1.5], u, v ~ U[-0.5,0.5],
    p ~ U[0.1,1.0]."""
    out = []
    for _ in range(4):
        rho = rng.uniform(0.5, 1.5)
        u = rng.uniform(-0.5, 0.5)
        v = rng.uniform(-0.5, 0.5)
        p = rng.uniform(0.1, 1.0)
        out.append((rho, u, v, p))
    return out


def _quadrant_fields(nx, ny, states):
    xc = (np.arange(nx) + 0.5) / nx
    yc = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(xc, yc)
    q = np.where(Y > 0.5, np.where(X > 0.5, 0, 1), np.where(X < 0.5, 2, 3))
    st = np.array(states)
    return [st[q, k] for k in range(4)], q


def quadrants_2d(nx: int, ny: int, seed: int, gamma: float = GAMMA):
    """Four seeded constant quadrants on [0,1]^2 (jumps on cell faces when nx, ny are even)."""
    rng = np.random.default_rng(seed)
    states = quadrant_states(rng)
    (rho, u, v, p), _ = _quadrant_fields(nx, ny, states)
    W = _cons_2d(rho, u, v, p, gamma)
    return W, np.zeros((8, ny, nx)), states


def quadrants_2d_strong(nx: int, ny: int, seed: int, gamma: float = GAMMA):
    """Four seeded constant quadrants with strong jumps (robustness runs):
    rho ~ U[0.1, 1.5], p ~ U[0.03, 1.5], u, v ~ U[-1.2, 1.2] per quadrant,
    drawn in the order of quadrant_states."""
    rng = np.random.default_rng(seed)
    states = [(rng.uniform(0.1, 1.5), rng.uniform(-1.2, 1.2), rng.uniform(-1.2, 1.2), rng.uniform(0.03, 1.5))
              for _ in range(4)]
    (rho, u, v, p), _ = _quadrant_fields(nx, ny, states)
    return _cons_2d(rho, u, v, p, gamma), np.zeros((8, ny, nx)), states


_GL4_X = np.array([-0.8611363115940526, -0.3399810435848563, 0.3399810435848563, 0.8611363115940526])
_GL4_W = np.array([0.3478548451374538, 0.6521451548625461, 0.6521451548625461, 0.3478548451374538])


def vortex_2d(nx: int, ny: int, seed: int, amp: float = 0.1, centre=(0.25, 0.25),
              radius: float = 0.05, gamma: float = GAMMA):
    """Seeded quadrants plus the velocity perturbation
    du = -A (y - yc)/R exp((1 - r^2/R^2)/2), dv = +A (x - xc)/R exp((1 - r^2/R^2)/2);
    rho and p keep their quadrant values. Cell averages by 4x4 Gauss-Legendre,
    averaged gradients by the Gauss theorem with 4-point face quadrature; each
    cell takes the constant state of the quadrant that contains its centre."""
    rng = np.random.default_rng(seed)
    states = quadrant_states(rng)
    (rho_q, u_q, v_q, p_q), _ = _quadrant_fields(nx, ny, states)
    hx, hy = 1.0 / nx, 1.0 / ny
    xl = (np.arange(nx) * hx)[None, :]
    yl = (np.arange(ny) * hy)[:, None]

    def cons_at(x, y):
        rx, ry = x - centre[0], y - centre[1]
        e = np.exp(0.5 * (1.0 - (rx * rx + ry * ry) / (radius * radius)))
        u = u_q - amp * ry / radius * e
        v = v_q + amp * rx / radius * e
        return _cons_2d(rho_q, u, v, p_q, gamma)

    W = np.zeros((4, ny, nx))
    for a, wa in zip(_GL4_X, _GL4_W):
        for b, wb in zip(_GL4_X, _GL4_W):
            W += 0.25 * wa * wb * cons_at(xl + hx * (0.5 + 0.5 * a), yl + hy * (0.5 + 0.5 * b))
    dW = np.zeros((8, ny, nx))
    for a, wa in zip(_GL4_X, _GL4_W):
        ys = yl + hy * (0.5 + 0.5 * a)
        xs = xl + hx * (0.5 + 0.5 * a)
        dW[0:4] += 0.5 * wa * (cons_at(xl + hx, ys) - cons_at(xl, ys)) / hx
        dW[4:8] += 0.5 * wa * (cons_at(xs, yl + hy) - cons_at(xs, yl)) / hy
    return W, dW, states


BATCH_SIDES = (128, 256, 512, 1024)


def batched_grids(seed: int, n: int = 64, sides=BATCH_SIDES):
    """``n`` independent square quadrant grids: the sides are drawn first (uniform over
    ``sides``), then the four quadrant states of each grid in order."""
    rng = np.random.default_rng(seed)
    picks = rng.integers(0, len(sides), size=n)
    grids = []
    for k in range(n):
        s = int(sides[picks[k]])
        states = quadrant_states(rng)
        (rho, u, v, p), _ = _quadrant_fields(s, s, states)
        grids.append((s, _cons_2d(rho, u, v, p), np.zeros((8, s, s)), states))
    return grids


def random_smooth_2d(nx: int, ny: int, seed: int, gamma: float = GAMMA, modes: int = 3):
    """Smooth periodic 2-D state (a few seeded Fourier modes per primitive) with exact
    cell averages (by 4x4 Gauss-Legendre) and Gauss-theorem gradients; used for
    parity on smooth data."""
    rng = np.random.default_rng(seed)
    coef = rng.uniform(-1.0, 1.0, size=(4, modes, modes, 2))
    base = np.array([1.0, 0.3, -0.2, 1.0])
    scale = np.array([0.1, 0.1, 0.1, 0.1])
    hx, hy = 1.0 / nx, 1.0 / ny
    xl = (np.arange(nx) * hx)[None, :]
    yl = (np.arange(ny) * hy)[:, None]

    def prim(x, y):
        out = []
        for f in range(4):
            s = base[f] + 0.0 * x * y
            for a in range(modes):
                for b in range(modes):
                    ph = 2 * math.pi * ((a + 1) * x + b * y)
                    s = s + scale[f] / (1 + a + b) * (coef[f, a, b, 0] * np.sin(ph) + coef[f, a, b, 1] * np.cos(ph))
            out.append(s)
        return out

    def cons_at(x, y):
        rho, u, v, p = prim(x, y)
        return _cons_2d(rho, u, v, p, gamma)

    W = np.zeros((4, ny, nx))
    for a, wa in zip(_GL4_X, _GL4_W):
        for b, wb in zip(_GL4_X, _GL4_W):
            W += 0.25 * wa * wb * cons_at(xl + hx * (0.5 + 0.5 * a), yl + hy * (0.5 + 0.5 * b))
    dW = np.zeros((8, ny, nx))
    for a, wa in zip(_GL4_X, _GL4_W):
        ys = yl + hy * (0.5 + 0.5 * a)
        xs = xl + hx * (0.5 + 0.5 * a)
        dW[0:4] += 0.5 * wa * (cons_at(xl + hx, ys) - cons_at(xl, ys)) / hx
        dW[4:8] += 0.5 * wa * (cons_at(xs, yl + hy) - cons_at(xs, yl)) / hy
    return W, dW


def blast_wave_1d(nx: int, gamma: float = GAMMA):
    """Woodward-Colella blast waves on [0, 1]: rho = 1, u = 0 and p = 1000 on
    x < 0.1, 0.01 on 0.1 < x < 0.9, 100 on x > 0.9. The jumps sit on cell
    faces when nx is a multiple of 10; cells are then constant and their
    averaged gradients zero. End time 0.038."""
    if nx % 10:
        raise ValueError("nx must be a multiple of 10 (jumps on faces)")
    xc = (np.arange(nx) + 0.5) / nx
    p = np.where(xc < 0.1, 1000.0, np.where(xc > 0.9, 100.0, 0.01))
    rho = np.ones(nx)
    u = np.zeros(nx)
    W = _cons_1d(rho, u, p, gamma)[:, None, :]
    return W, np.zeros_like(W)


SHU_OSHER_LEFT = (3.857143, 2.629369, 10.33333)   # (rho, u, p) behind the shock


def shu_osher_1d(nx: int, gamma: float = GAMMA):
    """Shu-Osher problem on [-5, 5]: (rho, u, p) = SHU_OSHER_LEFT on x < -4,
    rho = 1 + 0.2 sin(5 x), u = 0, p = 1 on x > -4. Exact cell averages of the
    density wave (analytic integral) and exact averaged gradients (Gauss
    theorem: face values over h); the jump sits on a face when nx is a
    multiple of 10. End time 1.8."""
    if nx % 10:
        raise ValueError("nx must be a multiple of 10 (jump on a face)")
    h = 10.0 / nx
    xl = -5.0 + np.arange(nx) * h
    xr = xl + h
    left = xr <= -4.0 + 1e-12
    # density average of 1 + 0.2 sin(5x) over [xl, xr] and its face values
    rho_avg = 1.0 + 0.2 * (np.cos(5.0 * xl) - np.cos(5.0 * xr)) / (5.0 * h)
    rho_grad = 0.2 * (np.sin(5.0 * xr) - np.sin(5.0 * xl)) / h
    rl, ul, pl = SHU_OSHER_LEFT
    rho = np.where(left, rl, rho_avg)
    u = np.where(left, ul, 0.0)
    p = np.where(left, pl, 1.0)
    W = _cons_1d(rho, u, p, gamma)
    # u = 0 and p = 1 on the right: d(rho E)/dx = 0, d(rho u)/dx = 0; the
    # left state is constant
    dW = np.zeros_like(W)
    dW[0] = np.where(left, 0.0, rho_grad)
    return W[:, None, :], dW[:, None, :]


# ---------------------------------------------------------------------------
# Inputs of the sixth-order non-compact scheme: U[field, n] (no y axis).
# ---------------------------------------------------------------------------

def density_wave_noncompact(n: int, t: float = 0.0, gamma: float = GAMMA):
    """The 1-D accuracy test of Sec. 6.1 as stated: rho = 1 + 0.2 sin(pi (x - t)),
    U = p = 1 on [0, 2], periodic. Exact cell averages (rho U and rho E are
    affine in rho) at time t of the advected wave."""
    h = 2.0 / n
    xl = np.arange(n) * h - t
    xr = xl + h
    rho = 1.0 + 0.2 * (np.cos(math.pi * xl) - np.cos(math.pi * xr)) / (math.pi * h)
    return np.stack([rho, rho, 1.0 / (gamma - 1.0) + 0.5 * rho])


def density_wave_compact(n: int, t: float = 0.0, gamma: float = GAMMA):
    """The 1-D accuracy test of Sec. 6.1 for the compact scheme: rho = 1 +
    0.2 sin(pi (x - t)), U = p = 1 on [0, 2], periodic, at time t of the
    advected wave. Exact cell averages and exact averaged gradients (the
    difference of the point values at the cell faces over h); rho U and rho E
    are affine in rho. Returns (W[3, 1, n], dW[3, 1, n])."""
    h = 2.0 / n
    xl = np.arange(n) * h - t
    xr = xl + h
    rho = 1.0 + 0.2 * (np.cos(math.pi * xl) - np.cos(math.pi * xr)) / (math.pi * h)
    W = np.stack([rho, rho, 1.0 / (gamma - 1.0) + 0.5 * rho])
    drho = 0.2 * (np.sin(math.pi * xr) - np.sin(math.pi * xl)) / h
    dW = np.stack([drho, drho, 0.5 * drho])
    return W.reshape(3, 1, n), dW.reshape(3, 1, n)


def diagonal_wave_2d(n: int, t: float = 0.0, amp: float = 0.2, gamma: float = GAMMA):
    """An oblique density wave on the periodic unit square: rho = 1 + amp
    sin(2 pi (x + y - 2t)), U = V = p = 1, at time t. Exact cell averages and
    exact cell-averaged gradients (face averages of the point values by the
    Gauss theorem). Returns (W[4, n, n], dW[8, n, n])."""
    h = 1.0 / n
    k = 2.0 * math.pi
    ph = -2.0 * k * t
    x0 = np.arange(n) * h
    X, Y = np.meshgrid(x0, x0, indexing="xy")

    def cell(xa, ya):
        s = np.sin
        return -(s(k * (xa + h + ya + h) + ph) - s(k * (xa + h + ya) + ph)
                 - s(k * (xa + ya + h) + ph) + s(k * (xa + ya) + ph)) / (k * h) ** 2

    def face(xf, ya):   # average over [ya, ya + h] of sin(k (xf + y) + ph)
        return -(np.cos(k * (xf + ya + h) + ph) - np.cos(k * (xf + ya) + ph)) / (k * h)

    rho = 1.0 + amp * cell(X, Y)
    drx = amp * (face(X + h, Y) - face(X, Y)) / h
    dry = amp * (face(Y + h, X) - face(Y, X)) / h
    W = np.stack([rho, rho, rho, 1.0 / (gamma - 1.0) + rho])
    dW = np.stack([drx, drx, drx, drx, dry, dry, dry, dry])
    return W, dW


def entropy_wave_noncompact(n: int = 1800, gamma: float = GAMMA, b: float = 1.5):
    """The entropy-wave advection of Sec. 6.1: rho = 1 + 0.5 exp(-ln2 x^2 / b^2),
    U = p = 1 on [-800, 1000], periodic; 1800 cells in the paper. Exact cell
    averages through the error function."""
    h = 1800.0 / n
    xl = -800.0 + np.arange(n) * h
    xr = xl + h
    s = math.sqrt(math.log(2.0)) / b
    erf = np.vectorize(math.erf)
    rho = 1.0 + 0.5 * (math.sqrt(math.pi) / (2.0 * s)) * (erf(s * xr) - erf(s * xl)) / h
    return np.stack([rho, rho, 1.0 / (gamma - 1.0) + 0.5 * rho])


def smooth_noncompact(n: int, seed: int, gamma: float = GAMMA, modes: int = 3):
    """Seeded smooth periodic state on [0, 1]: rho, u, p each a constant plus
    `modes` Fourier modes with seeded amplitudes (rho, p in [0.5, 1.5],
    |u| <= 0.6), sampled at the cell centres."""
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    fields = []
    for base, amp in ((1.0, 0.4), (0.0, 0.5), (1.0, 0.4)):
        f = np.full(n, base)
        for m in range(1, modes + 1):
            a, ph = rng.uniform(-1.0, 1.0) * amp / modes, rng.uniform(0.0, 2.0 * math.pi)
            f += a * np.sin(2.0 * math.pi * m * x + ph)
        fields.append(f)
    return _cons_1d(fields[0], fields[1], fields[2], gamma)


def shocks_noncompact(n: int, seed: int, gamma: float = GAMMA, cells_per_segment: int = 1000):
    """Seeded piecewise-smooth stand-in for the paper's 1-D shock problems at
    any size: segments of seeded lengths in [cells_per_segment / 2,
    3 cells_per_segment / 2] (the paper's runs use 200 to 1800 cells with one
    to three discontinuities between wide constant or smooth regions), each a
    seeded constant state (rho, p in [10^-0.5, 10^0.5], |u| <= 0.5: jumps of
    up to a factor 10, as the density and pressure jumps of the Shu-Osher and
    Titarev-Toro data, and velocity jumps below the sound speeds, so that no
    Riemann problem opens a near-vacuum) times a density wave
    1 + a sin(2 pi i / P) with a in [0, 0.2] and P in [8, 64] cells; sampled
    at the cell centres."""
    rng = np.random.default_rng(seed)
    half = max(1, cells_per_segment // 2)
    lens = rng.integers(half, 3 * half + 1, n // half + 2)
    edges = np.cumsum(lens)
    edges = edges[edges < n]
    nseg = len(edges) + 1
    seg = np.searchsorted(edges, np.arange(n), side="right")
    rho0 = 10.0 ** rng.uniform(-0.5, 0.5, nseg)
    u0 = rng.uniform(-0.5, 0.5, nseg)
    p0 = 10.0 ** rng.uniform(-0.5, 0.5, nseg)
    amp = rng.uniform(0.0, 0.2, nseg)
    period = rng.uniform(8.0, 64.0, nseg)
    i = np.arange(n)
    rho = rho0[seg] * (1.0 + amp[seg] * np.sin(2.0 * math.pi * i / period[seg]))
    return _cons_1d(rho, u0[seg], p0[seg], gamma)


TITAREV_TORO_LEFT = (1.515695, 0.523346, 1.805)   # (rho, u, p) behind the shock


def titarev_toro_noncompact(n: int = 1000, gamma: float = GAMMA):
    """The Titarev-Toro problem of Sec. 6.2 on [-5, 5]: (rho, u, p) =
    TITAREV_TORO_LEFT on x <= -4, rho = 1 + 0.1 sin(20 pi x), u = 0, p = 1 on
    x > -4 (exact cell averages; the jump sits on a face when n is a
    multiple of 10); end time 5. Returns U and the ghost states [2, 3, 3] of
    the paper's boundaries: the inflow state on the left and the fixed wave
    profile (the cell averages of the three cells beyond x = 5) on the
    right."""
    if n % 10:
        raise ValueError("n must be a multiple of 10 (jump on a face)")
    h = 10.0 / n

    def averages(xl):
        xr = xl + h
        return 1.0 + 0.1 * (np.cos(20.0 * math.pi * xl) - np.cos(20.0 * math.pi * xr)) / (20.0 * math.pi * h)

    xl = -5.0 + np.arange(n) * h
    left = xl + h <= -4.0 + 1e-12
    rl, ul, pl = TITAREV_TORO_LEFT
    rho = np.where(left, rl, averages(xl))
    U = _cons_1d(rho, np.where(left, ul, 0.0), np.where(left, pl, 1.0), gamma)
    ghost = np.zeros((2, 3, 3))
    ghost[0] = np.asarray(_cons_1d(np.full(3, rl), np.full(3, ul), np.full(3, pl), gamma)).T
    xg = 5.0 + np.arange(3) * h
    ghost[1] = np.asarray(_cons_1d(averages(xg), np.zeros(3), np.ones(3), gamma)).T
    return U, ghost


def titarev_toro_1d(nx: int = 800, gamma: float = GAMMA):
    """The Titarev-Toro problem for the compact scheme (800 cells in the
    paper) on [-5, 5]: cell averages and averaged gradients (Gauss theorem:
    face-value differences over h) of TITAREV_TORO_LEFT on x <= -4 and
    rho = 1 + 0.1 sin(20 pi x), u = 0, p = 1 beyond; end time 5. Also
    returns the ghost states [end][layer 0 = next to the grid][W (3), dW (3)]
    of the paper's boundaries: the constant inflow state on the left and the
    fixed wave profile (averages and averaged gradients of the two cells
    beyond x = 5) on the right."""
    if nx % 10:
        raise ValueError("nx must be a multiple of 10 (jump on a face)")
    h = 10.0 / nx
    k = 20.0 * math.pi

    def avg_grad(xl):
        xr = xl + h
        rho = 1.0 + 0.1 * (np.cos(k * xl) - np.cos(k * xr)) / (k * h)
        drho = 0.1 * (np.sin(k * xr) - np.sin(k * xl)) / h
        return rho, drho

    xl = -5.0 + np.arange(nx) * h
    left = xl + h <= -4.0 + 1e-12
    rho_w, drho_w = avg_grad(xl)
    rl, ul, pl = TITAREV_TORO_LEFT
    rho = np.where(left, rl, rho_w)
    W = _cons_1d(rho, np.where(left, ul, 0.0), np.where(left, pl, 1.0), gamma)
    dW = np.zeros_like(W)
    # u = 0, p = 1 on the right: rho U and rho E are constant there, and rho E
    # carries no kinetic part, so only d rho / dx is non-zero
    dW[0] = np.where(left, 0.0, drho_w)
    ghost = np.zeros((2, 2, 6))
    ghost[0, :, :3] = np.asarray(_cons_1d(np.full(2, rl), np.full(2, ul), np.full(2, pl), gamma)).T
    rg, dg = avg_grad(5.0 + np.arange(2) * h)
    ghost[1, :, :3] = np.asarray(_cons_1d(rg, np.zeros(2), np.ones(2), gamma)).T
    ghost[1, :, 3] = dg
    return W[:, None, :], dW[:, None, :], ghost


# ---------------------------------------------------------------------------
# Triangular meshes (the unstructured reconstruction of Sec. 4.3)
# ---------------------------------------------------------------------------
def tri_mesh(nx: int, ny: int, seed: int, jitter: float = 0.2):
    """Periodic triangulation of the unit square: an nx x ny lattice whose
    vertices are moved by up to jitter/2 of the spacing (seeded), each
    quadrilateral split into two counter-clockwise triangles, 2 nx ny cells.

    Returns a dict with
      xv    [ncell, 3, 2]  vertex coordinates, each triangle unwrapped about
                           its own lattice square;
      nbr   [ncell, 3]     the cell across edge e (from vertex e to e+1);
      shift [ncell, 3, 2]  translation that places that neighbour, as stored,
                           next to the cell (a period across the boundary).
    Cell 2 (j nx + i) is the lower triangle of square (i, j), cell + 1 the
    upper one."""
    if nx < 2 or ny < 2:
        raise ValueError("the periodic mesh needs at least 2 x 2 squares")
    rng = np.random.default_rng(seed)
    hx, hy = 1.0 / nx, 1.0 / ny
    jit = rng.uniform(-0.5, 0.5, size=(ny, nx, 2)) * jitter * np.array([hx, hy])
    base = np.stack(np.meshgrid(np.arange(nx) * hx, np.arange(ny) * hy), axis=-1) + jit

    def vert(i, j):
        return base[j % ny, i % nx] + np.array([(i // nx) * 1.0, (j // ny) * 1.0])

    n = 2 * nx * ny
    xv = np.zeros((n, 3, 2))
    nbr = np.zeros((n, 3), dtype=np.int64)
    shift = np.zeros((n, 3, 2))

    def lower(i, j):
        return 2 * ((j % ny) * nx + (i % nx))

    def wrap(i, j):
        # translation of the canonical square of (i, j) to position (i, j)
        return np.array([(i // nx) * 1.0, (j // ny) * 1.0])

    for j in range(ny):
        for i in range(nx):
            c = lower(i, j)
            v00, v10, v11, v01 = vert(i, j), vert(i + 1, j), vert(i + 1, j + 1), vert(i, j + 1)
            xv[c] = (v00, v10, v11)
            xv[c + 1] = (v00, v11, v01)
            # lower: bottom edge, right edge, diagonal
            nbr[c] = (lower(i, j - 1) + 1, lower(i + 1, j) + 1, c + 1)
            shift[c] = (wrap(i, j - 1), wrap(i + 1, j), (0.0, 0.0))
            # upper: diagonal, top edge, left edge
            nbr[c + 1] = (c, lower(i, j + 1), lower(i - 1, j))
            shift[c + 1] = ((0.0, 0.0), wrap(i, j + 1), wrap(i - 1, j))
    return {"xv": xv, "nbr": nbr, "shift": shift, "nx": nx, "ny": ny}


def _tri_points(xv, npts=8):
    """Points and weights (summing to 1) of the collapsed npts x npts Gauss
    rule on each triangle of xv [n, 3, 2] (exact for polynomials of degree
    <= 2 npts - 2)."""
    gx, gw = np.polynomial.legendre.leggauss(npts)
    gx, gw = 0.5 * (gx + 1.0), 0.5 * gw
    s, t = np.meshgrid(gx, gx, indexing="ij")
    ws = np.outer(gw, gw) * 2.0 * (1.0 - s)   # Jacobian of (s, t) -> (b1, b2)
    b1 = s.ravel()
    b2 = ((1.0 - s) * t).ravel()
    w = ws.ravel()
    b0 = 1.0 - b1 - b2
    pts = (b0[None, :, None] * xv[:, None, 0] + b1[None, :, None] * xv[:, None, 1]
           + b2[None, :, None] * xv[:, None, 2])
    return pts, w


def tri_cell_data(mesh, f, grad, npts=8):
    """Cell averages of f(x, y) and of its gradient grad(x, y) -> (gx, gy)
    over every triangle (collapsed npts x npts Gauss rule); f may return
    several fields stacked on axis 0. Returns W [nf, ncell] and dW [2, nf,
    ncell] (x then y derivatives)."""
    pts, w = _tri_points(mesh["xv"], npts)
    x, y = pts[..., 0], pts[..., 1]
    fv = np.asarray(f(x, y))
    single = fv.ndim == 2
    fv = fv[None] if single else fv
    gx, gy = grad(x, y)
    gx, gy = np.asarray(gx), np.asarray(gy)
    if single:
        gx, gy = gx[None], gy[None]
    W = (fv * w).sum(axis=-1)
    dW = np.stack([(gx * w).sum(axis=-1), (gy * w).sum(axis=-1)])
    return W, dW


def tri_euler_smooth(mesh, seed: int, gamma: float = GAMMA, npts: int = 8):
    """Smooth periodic Euler state (a few seeded Fourier modes per primitive)
    as conservative cell averages and averaged gradients on a triangle mesh."""
    rng = np.random.default_rng(seed)
    coef = rng.uniform(-1.0, 1.0, size=(4, 2, 2, 2))
    base = np.array([1.0, 0.3, -0.2, 1.0])

    def prim(x, y):
        out, dx, dy = [], [], []
        for fidx in range(4):
            s = base[fidx] + 0.0 * x
            sx = 0.0 * x
            sy = 0.0 * x
            for a in range(2):
                for b in range(2):
                    kx, ky = 2 * math.pi * (a + 1), 2 * math.pi * b
                    ph = kx * x + ky * y
                    c0, c1 = 0.1 * coef[fidx, a, b, 0] / (1 + a + b), 0.1 * coef[fidx, a, b, 1] / (1 + a + b)
                    s = s + c0 * np.sin(ph) + c1 * np.cos(ph)
                    d = c0 * np.cos(ph) - c1 * np.sin(ph)
                    sx = sx + kx * d
                    sy = sy + ky * d
            out.append(s)
            dx.append(sx)
            dy.append(sy)
        return out, dx, dy

    def cons(x, y):
        (rho, u, v, p), _, _ = prim(x, y)
        return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])

    def cons_grad(x, y):
        (rho, u, v, p), dx, dy = prim(x, y)
        out = []
        for d in (dx, dy):
            dr, du, dv, dp = d
            out.append(np.stack([dr, dr * u + rho * du, dr * v + rho * dv,
                                 dp / (gamma - 1.0) + 0.5 * dr * (u * u + v * v) + rho * (u * du + v * dv)]))
        return out[0], out[1]

    return tri_cell_data(mesh, cons, cons_grad, npts)


def tri_euler_jumps(mesh, seed: int, gamma: float = GAMMA, npts: int = 8):
    """Piecewise-constant Euler state on a triangle mesh: the four quadrant
    states of the structured Riemann data, drawn the same way, on the cells
    whose centroid lies in each quadrant (jumps along cell edges, zero
    gradients), plus a small smooth part so that no stencil is flat
    (averaged with the collapsed npts x npts rule; large meshes take 2)."""
    rng = np.random.default_rng(seed)
    states = quadrant_states(rng)
    cen = mesh["xv"].mean(axis=1)
    right, top = cen[:, 0] > 0.5, cen[:, 1] > 0.5
    q = np.where(right & top, 0, np.where(top, 1, np.where(right, 3, 2)))
    prim = np.asarray(states)[q].T   # rho, u, v, p per cell
    W = _cons_2d(prim[0], prim[1], prim[2], prim[3], gamma)
    Ws, dWs = tri_euler_smooth(mesh, seed + 1, gamma, npts)
    W = W + 0.02 * (Ws - Ws.mean(axis=1, keepdims=True))
    return W, 0.02 * dWs
