"""ctypes wrapper of the CPU FP64 oracle (``geno_gks_oracle.c``).

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import this module. It shares no
code with the HIP library or its binding.

Every function takes and returns interior-only SoA float64 arrays
``W[field, y, x]``, ``dW[d * nv + field, y, x]`` (see ``inputs.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "geno_gks_oracle.c")
_SO = os.path.join(_HERE, "libgeno_gks_oracle.so")
_lib = None

# Parameter vector layout of the C oracle.
P_GAMMA, P_CPATH, P_EPS, P_R, P_RL, P_D1, P_D2, P_D3, P_TAUC1, P_TAUC2, P_CFL = range(11)
P_BC = 11  # four boundary codes follow: x-lo, x-hi, y-lo, y-hi (0 periodic, 1 transmissive)
P_GHOST = 15  # 24 values: 1-D fixed ends [end][layer][W (3), dW (3)]
P_CHAR = 39   # 1 = characteristic-variable reconstruction in the normal step
P_GUPD = 40   # time stepping of the gradients: 0 two-stage structure on the interface values, 1 earlier reading
N_PARAMS = 41
GUPD_S2O4, GUPD_STAGE_HALF = 0, 1
PERIODIC, TRANSMISSIVE, REFLECTING, FIXED = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP over rows)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        llp = ctypes.POINTER(ctypes.c_longlong)
        L.oracle_init.restype = i
        L.oracle_linear_weights.argtypes = [dp, dp]
        L.oracle_geno_face.argtypes = [dp, dp, dp, dp]
        L.oracle_moments.argtypes = [d, d, d, d, i, i, dp]
        L.oracle_geno_side_detail.argtypes = [dp, dp, i, d, d, dp]
        L.oracle_gks_points.argtypes = [dp, i, i, dp, dp, dp, dp, dp, dp, dp, d, dp, dp, dp, dp, dp]
        L.oracle_normal_faces.argtypes = [dp, i, i, i, d, d, dp, dp, i, dp, dp]
        L.oracle_roe_eigen.argtypes = [dp, i, i, dp, dp, dp, dp, dp]
        L.oracle_face_states.argtypes = [dp, i, i, i, d, d, dp, dp, i, dp, llp]
        L.oracle_step.argtypes = [dp, i, i, i, d, d, dp, dp, i, d, dp, llp]
        L.oracle_stage_faces.argtypes = [dp, i, i, i, d, d, dp, dp, d, i, dp, dp, dp, dp, dp]
        L.oracle_weights.argtypes = [dp, dp, d, dp]
        L.oracle_linearity_faces.argtypes = [dp, i, i, i, d, d, dp, dp, i, d, dp]
        L.oracle_cfl_dt.argtypes = [dp, i, i, i, d, d, dp]
        L.oracle_cfl_dt.restype = d
        for name in ("oracle_linear_weights", "oracle_geno_face", "oracle_geno_side_detail", "oracle_moments",
                     "oracle_gks_points", "oracle_normal_faces", "oracle_face_states",
                     "oracle_step", "oracle_stage_faces", "oracle_weights", "oracle_linearity_faces",
                     "oracle_roe_eigen"):
            getattr(L, name).restype = i
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params(ndim: int = 2, bc=TRANSMISSIVE, gamma=1.4, C=20.0, eps=1e-15, r=2.0, rL=2.0,
           d=(1.0, 8.0, 1.0), tau_c1=0.0, tau_c2=1.0, cfl=0.5, ghost=None,
           characteristic=False, gradient_update=GUPD_S2O4) -> np.ndarray:
    """Oracle parameter vector. Paper constants (Sec. 3): C = 20, eps = 1e-15,
    r = 2 (structured), r^L = 2, central weight C_0 = 8. ghost: [2, 2, 6]
    states of the ghost cells of 1-D FIXED ends ([end][layer 0 = next to the
    grid][W (3), dW (3)]); characteristic: the normal step reconstructs the
    characteristic variables of the normal flux Jacobian at the Roe average
    of the two cells at each face (values and h-derivatives projected alike);
    the tangential step of 2-D faces works on the conservative face values.
    gradient_update: GUPD_S2O4 applies the two-stage fourth-order structure to
    the interface values that update the gradients (Eq. (2)); GUPD_STAGE_HALF
    takes the BGK interface state at dt/2 of each stage (earlier reading)."""
    p = np.zeros(N_PARAMS)
    p[P_CHAR] = 1.0 if characteristic else 0.0
    p[P_GUPD] = float(gradient_update)
    if ghost is not None:
        p[P_GHOST:P_GHOST + 24] = np.asarray(ghost, dtype=np.float64).reshape(24)
    p[P_GAMMA], p[P_CPATH], p[P_EPS], p[P_R], p[P_RL] = gamma, C, eps, r, rL
    p[P_D1:P_D3 + 1] = d
    p[P_TAUC1], p[P_TAUC2], p[P_CFL] = tau_c1, tau_c2, cfl
    bcs = [bc] * 4 if np.isscalar(bc) else list(bc)
    p[P_BC:P_BC + 4] = bcs
    return p


def _check(rc, name):
    if rc != 0:
        raise RuntimeError("%s failed with code %d" % (name, rc))


def linear_weights():
    hv, hd = np.zeros(8), np.zeros(8)
    _check(lib().oracle_linear_weights(_p(hv), _p(hd)), "oracle_linear_weights")
    return hv, hd


def geno_face(prm, q, g):
    """GENO at one face for one component; q, g: averages and h-scaled averaged
    derivatives of cells j-1..j+2. Returns (val_l, hder_l, chi_l, val_r, hder_r, chi_r,
    h2der_l, h2der_r) with h2der = h^2 times the second derivative."""
    q, g, out = _c(q), _c(g), np.zeros(8)
    _check(lib().oracle_geno_face(_p(_c(prm)), _p(q), _p(g), _p(out)), "oracle_geno_face")
    return out


def geno_side_detail(prm, dat, side, qH, hqH):
    """Internals of one GENO side. dat: (Q, G) pairs of cells c-2..c+2 (10 values);
    side 0 = left state, 1 = right state. Returns a dict of IS, p, hp, omega, chi,
    qL, hqL, R, hR."""
    out = np.zeros(17)
    _check(lib().oracle_geno_side_detail(_p(_c(prm)), _p(_c(dat)), int(side), float(qH), float(hqH),
                                         _p(out)), "oracle_geno_side_detail")
    return dict(IS=out[0:3], p=out[3:6], hp=out[6:9], omega=out[9:12], chi=out[12],
                qL=out[13], hqL=out[14], R=out[15], hR=out[16])


TENO_CT = 1e-6   # the paper's cut-off of the TENO scale separation


def weights(prm, IS, ct=TENO_CT):
    """WENO-Z and TENO weights and the linearity measures of the paper's
    comparison from three sub-stencil indicators IS (IS_1, IS_2, IS_3).
    Returns dict(wz, chi_z, wt, chi_t, chi_geno)."""
    out = np.zeros(9)
    _check(lib().oracle_weights(_p(_c(prm)), _p(_c(IS)), float(ct), _p(out)), "oracle_weights")
    return dict(wz=out[0:3], chi_z=out[3], wt=out[4:7], chi_t=out[7], chi_geno=out[8])


def linearity_faces(prm, W, dW, direction=0, ct=TENO_CT, dx=None, dy=None):
    """chi of GENO, WENO-Z and TENO on every face-side of a direction:
    [method][side][var][a][b] (layout of normal_faces' chi)."""
    W, dW = _c(W), _c(dW)
    ndim, nv, ny, nx = _dims(W)
    dx = 1.0 / nx if dx is None else dx
    dy = 1.0 / ny if dy is None else dy
    if ndim == 1:
        n0, n1 = 1, nx + 1
    elif direction == 0:
        n0, n1 = ny + 2, nx + 1
    else:
        n0, n1 = ny + 1, nx + 2
    out = np.zeros((3, 2, nv, n0, n1))
    _check(lib().oracle_linearity_faces(_p(_c(prm)), ndim, nx, ny, dx, dy, _p(W), _p(dW), direction,
                                        float(ct), _p(out)), "oracle_linearity_faces")
    return out


def moments(U, V, lam, K, half, has_v=True):
    """Normalised Maxwellian moments <u^n> (n < 8), <v^n> (n < 8), <xi^(2n)> (n < 4)."""
    out = np.zeros(8 + 8 + 4)
    lib().oracle_moments(U, V, lam, K, int(half), int(has_v), _p(out))
    return out[:8], out[8:16], out[16:]


def gks_points(prm, ndim, Wl, Wr, dnl, dnr, dtl=None, dtr=None, dt=1e-3, sec=None, full=False):
    """GKS flux at points in the face frame; arrays [npts, nv]. sec: [npts, 3, nv]
    physical second derivatives (d_nn, d_nt, d_tt) of the points, or None.
    Returns F, Ft, W(dt/2) (and with full=True also W(dt) and W_tt)."""
    Wl, Wr, dnl, dnr = map(_c, (Wl, Wr, dnl, dnr))
    npts, nv = Wl.shape
    dtl = _c(dtl) if dtl is not None else np.zeros_like(Wl)
    dtr = _c(dtr) if dtr is not None else np.zeros_like(Wl)
    sec = _c(sec) if sec is not None else np.zeros((npts, 3, nv))
    F, Ft, Wh, Wf, W2 = (np.zeros_like(Wl) for _ in range(5))
    _check(lib().oracle_gks_points(_p(_c(prm)), ndim, npts, _p(Wl), _p(Wr), _p(dnl), _p(dnr),
                                   _p(dtl), _p(dtr), _p(sec), dt, _p(F), _p(Ft), _p(Wh), _p(Wf),
                                   _p(W2)), "oracle_gks_points")
    return (F, Ft, Wh, Wf, W2) if full else (F, Ft, Wh)


def _dims(W):
    nv, ny, nx = W.shape
    ndim = 1 if nv == 3 else 2
    return ndim, nv, ny, nx


def normal_faces(prm, W, dW, direction=0, dx=None, dy=None):
    """Normal GENO on every face of a direction (rows -1..ny for x-faces,
    columns -1..nx for y-faces). Returns out[side, quant, var, a, b] (quant = value,
    h d_n, h^2 d_nn), chi[side, var, a, b]."""
    W, dW = _c(W), _c(dW)
    ndim, nv, ny, nx = _dims(W)
    dx = 1.0 / nx if dx is None else dx
    dy = 1.0 / ny if dy is None else dy
    if ndim == 1:
        n0, n1 = 1, nx + 1
    elif direction == 0:
        n0, n1 = ny + 2, nx + 1
    else:
        n0, n1 = ny + 1, nx + 2
    out = np.zeros((2, 3, nv, n0, n1))
    chi = np.zeros((2, nv, n0, n1))
    _check(lib().oracle_normal_faces(_p(_c(prm)), ndim, nx, ny, dx, dy, _p(W), _p(dW), direction,
                                     _p(out), _p(chi)), "oracle_normal_faces")
    return out, chi


def roe_eigen(prm, ndim, direction, Wa, Wb):
    """Right eigenvectors R (columns), L = R^-1 and speeds of the normal flux
    Jacobian at the Roe average of the states Wa, Wb."""
    nv = 3 if ndim == 1 else 4
    R, Lm, lam = np.zeros(nv * nv), np.zeros(nv * nv), np.zeros(nv)
    _check(lib().oracle_roe_eigen(_p(_c(prm)), ndim, direction, _p(_c(Wa)), _p(_c(Wb)), _p(R), _p(Lm),
                                  _p(lam)), "oracle_roe_eigen")
    return R.reshape(nv, nv), Lm.reshape(nv, nv), lam


def face_states(prm, W, dW, direction=0, dx=None, dy=None, second=False):
    """Point states on faces after the tangential step and positivity guard.
    Returns (out[side, gauss, quant, var, nfy, nfx], guard_count); with
    second=True also the points' h-scaled second derivatives
    sec[gauss, (h_n^2 d_nn, h_n h_t d_nt, h_t^2 d_tt), var, nfy, nfx] (1-D: one
    point and d_nn only): (out, sec, guard_count)."""
    W, dW = _c(W), _c(dW)
    ndim, nv, ny, nx = _dims(W)
    dx = 1.0 / nx if dx is None else dx
    dy = 1.0 / ny if dy is None else dy
    if ndim == 1:
        nfy, nfx, npl, nsec = 1, nx + 1, 4, 1
        shape, sshape = (2, 1, 2, nv, 1, nx + 1), (1, 1, nv, 1, nx + 1)
    else:
        nfx, nfy = (nx + 1, ny) if direction == 0 else (nx, ny + 1)
        npl, nsec = 12, 6
        shape, sshape = (2, 2, 3, nv, nfy, nfx), (2, 3, nv, nfy, nfx)
    buf = np.zeros((npl + nsec) * nv * nfy * nfx)
    g = ctypes.c_longlong(0)
    _check(lib().oracle_face_states(_p(_c(prm)), ndim, nx, ny, dx, dy, _p(W), _p(dW), direction,
                                    _p(buf), ctypes.byref(g)), "oracle_face_states")
    n = npl * nv * nfy * nfx
    out, sec = buf[:n].reshape(shape), buf[n:].reshape(sshape)
    return (out, sec, g.value) if second else (out, g.value)


def stage_faces(prm, W, dW, dt, direction=0, dx=None, dy=None, full=False):
    """Gauss-averaged F, dF/dt and W_int(dt/2) on every face of a direction:
    [nv, nfy, nfx]; with full=True also W_int(dt) and the equilibrium W_tt."""
    W, dW = _c(W), _c(dW)
    ndim, nv, ny, nx = _dims(W)
    dx = 1.0 / nx if dx is None else dx
    dy = 1.0 / ny if dy is None else dy
    if ndim == 1 or direction == 0:
        shape = (nv, ny, nx + 1)
    else:
        shape = (nv, ny + 1, nx)
    F, Ft, Wh, Wf, W2 = (np.zeros(shape) for _ in range(5))
    _check(lib().oracle_stage_faces(_p(_c(prm)), ndim, nx, ny, dx, dy, _p(W), _p(dW), dt, direction,
                                    _p(F), _p(Ft), _p(Wh), _p(Wf), _p(W2)), "oracle_stage_faces")
    return (F, Ft, Wh, Wf, W2) if full else (F, Ft, Wh)


def step(prm, W, dW, nsteps, dx=None, dy=None, fixed_dt=0.0):
    """nsteps S2O4 steps; returns (W, dW, dt_history, guard_count) (inputs untouched)."""
    W, dW = _c(W).copy(), _c(dW).copy()
    ndim, nv, ny, nx = _dims(W)
    dx = 1.0 / nx if dx is None else dx
    dy = 1.0 / ny if dy is None else dy
    dts = np.zeros(max(nsteps, 1))
    g = ctypes.c_longlong(0)
    _check(lib().oracle_step(_p(_c(prm)), ndim, nx, ny, dx, dy, _p(W), _p(dW), nsteps,
                             float(fixed_dt), _p(dts), ctypes.byref(g)), "oracle_step")
    return W, dW, dts[:nsteps], g.value


def conserved_totals(W, dx=None, dy=None):
    """Sum over the cells of each conserved field times the cell size (dx in
    1-D, dx dy in 2-D): the quantities the conservation form of the update
    (Eq. (1)) keeps fixed on periodic grids. Each sum is the exactly rounded
    one (math.fsum), then multiplied by the cell size."""
    import math
    W = _c(W)
    ndim, nv, ny, nx = _dims(W)
    dx = 1.0 / nx if dx is None else dx
    dy = 1.0 / ny if dy is None else dy
    area = dx * dy if ndim == 2 else dx
    return np.array([math.fsum(W[f].ravel().tolist()) * area for f in range(nv)])


def cfl_dt(prm, W, dx=None, dy=None):
    W = _c(W)
    ndim, nv, ny, nx = _dims(W)
    dx = 1.0 / nx if dx is None else dx
    dy = 1.0 / ny if dy is None else dy
    return lib().oracle_cfl_dt(_p(_c(prm)), ndim, nx, ny, dx, dy, _p(W))
