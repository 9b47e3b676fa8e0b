"""ctypes wrapper of the CPU FP64 oracle of the sixth-order non-compact
scheme (``geno6_oracle.c``): GENO reconstruction on the six-cell stencil of
Sec. 4.1, HLLC flux and classical four-stage Runge-Kutta (Sec. 2).

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import this module. It shares no
code with the HIP library or its binding.

State arrays are SoA float64 ``U[field, n]``, fields (rho, rho U, rho E),
interior cells only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "geno6_oracle.c")
_SO = os.path.join(_HERE, "libgeno6_oracle.so")
_lib = None

PERIODIC, TRANSMISSIVE, REFLECTING, FIXED = 0, 1, 2, 3
# parameter vector: gamma, C, eps, d1..d4, cfl, bc_lo, bc_hi, dt_fixed, characteristic,
# then 18 ghost values [end][cell k][field] of fixed ends
N_PARAMS = 31


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP over faces)."""
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
        i, d, ll = ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        L.o6_nparams.restype = i
        L.o6_poly.argtypes = [dp, i, i, dp]
        L.o6_poly.restype = i
        L.o6_smoothness.argtypes = [dp, i, i]
        L.o6_smoothness.restype = d
        L.o6_side.argtypes = [dp, dp, i, dp]
        L.o6_side.restype = i
        L.o6_eigen.argtypes = [dp, dp, dp, dp, dp, dp]
        L.o6_eigen.restype = i
        L.o6_hllc.argtypes = [dp, dp, dp, dp]
        L.o6_hllc.restype = i
        L.o6_faces.argtypes = [dp, i, dp, dp, dp, dp, dp]
        L.o6_faces.restype = ll
        L.o6_rhs.argtypes = [dp, i, d, dp, dp]
        L.o6_rhs.restype = ll
        L.o6_cfl_dt.argtypes = [dp, i, d, dp]
        L.o6_cfl_dt.restype = d
        L.o6_step.argtypes = [dp, i, d, dp, i, dp]
        L.o6_step.restype = ll
        assert L.o6_nparams() == N_PARAMS
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


ISTAU_PRINTED, ISTAU_LARGE_STENCIL = 0, 1


def params(bc=PERIODIC, gamma=1.4, C=20.0, eps=1e-15, d=(1.0, 8.0, 1.0, 1.0), cfl=0.5,
           dt_fixed=0.0, characteristic=False, ghost=None, istau=ISTAU_PRINTED) -> np.ndarray:
    """Method constants of Sec. 3 and 4.1 (C = 20, eps = 1e-15, C_0 = 8 on the
    central sub-stencil S_2). bc: one code or a (low, high) pair;
    characteristic: reconstruct characteristic instead of conservative
    variables; ghost: [2, 3, 3] states of the ghost cells of FIXED ends
    ([end][cell k][field], cell -1-k or n+k); istau: the printed IS^tau of
    Sec. 4.1, or ISTAU_LARGE_STENCIL, the fifth-derivative indicator of p^5
    (a reading of Sec. 3, built as Sec. 4.3 builds IS^tau on triangles)."""
    lo, hi = (bc, bc) if np.isscalar(bc) else bc
    g = np.zeros(18) if ghost is None else np.asarray(ghost, dtype=np.float64).reshape(18)
    return np.array([gamma, C, eps, *d, cfl, lo, hi, dt_fixed, 1.0 if characteristic else 0.0, *g,
                     float(istau)], dtype=np.float64)


def eigen(prm, Ua, Ub):
    """Roe-averaged right eigenvectors R, their inverse L (3x3) and the
    speeds (u - c, u, u + c) of the face between states Ua and Ub."""
    R, L, lam = np.zeros(9), np.zeros(9), np.zeros(3)
    if lib().o6_eigen(_p(_c(prm)), _p(_c(Ua)), _p(_c(Ub)), _p(R), _p(L), _p(lam)):
        raise ValueError("no eigen-structure (non-physical average)")
    return R.reshape(3, 3), L.reshape(3, 3), lam


def poly(avg, lo: int) -> np.ndarray:
    """Coefficients (in xi = (x - x_j)/h) of the polynomial whose averages over
    cells lo, lo+1, ... (offsets from the target cell j) are avg."""
    avg = _c(avg)
    a = np.zeros(len(avg))
    if lib().o6_poly(_p(avg), lo, len(avg), _p(a)):
        raise ValueError("singular cell-average system")
    return a


def smoothness(a, lmax: int) -> float:
    """sum_{l=1..lmax} integral over the target cell of (d^l p / d xi^l)^2."""
    a = _c(a)
    return lib().o6_smoothness(_p(a), len(a), lmax)


SIDE_FIELDS = ("value", "chi", "alpha", "p5", "IS1", "IS2", "IS3", "IS4", "w1", "w2", "w3", "w4",
               "p1", "p2", "p3", "p4")


def side(prm, u6, side_: int) -> dict:
    """GENO state of one side of the face x_{j+1/2} from the averages of
    cells j-2..j+3 (side 0: left of the face, 1: right of it)."""
    u6 = _c(u6)
    out = np.zeros(16)
    if lib().o6_side(_p(_c(prm)), _p(u6), side_, _p(out)):
        raise ValueError("side reconstruction failed")
    return dict(zip(SIDE_FIELDS, out))


def hllc(prm, UL, UR) -> np.ndarray:
    F = np.zeros(3)
    lib().o6_hllc(_p(_c(prm)), _p(_c(UL)), _p(_c(UR)), _p(F))
    return F


def faces(prm, U):
    """Every face s = 0..n (between cells s-1 and s): UL, UR, F [3, n+1] and
    chi [2, 3, n+1]; plus the guard count."""
    U = _c(U)
    n = U.shape[1]
    UL, UR, F = (np.zeros((3, n + 1)) for _ in range(3))
    chi = np.zeros((2, 3, n + 1))
    g = lib().o6_faces(_p(_c(prm)), n, _p(U), _p(UL), _p(UR), _p(F), _p(chi))
    if g < 0:
        raise ValueError("oracle faces failed (%d)" % g)
    return UL, UR, F, chi, int(g)


def rhs(prm, U, dx: float):
    U = _c(U)
    L = np.zeros_like(U)
    g = lib().o6_rhs(_p(_c(prm)), U.shape[1], dx, _p(U), _p(L))
    if g < 0:
        raise ValueError("oracle rhs failed (%d)" % g)
    return L, int(g)


def cfl_dt(prm, U, dx: float) -> float:
    U = _c(U)
    return lib().o6_cfl_dt(_p(_c(prm)), U.shape[1], dx, _p(U))


def step(prm, U, dx: float, nsteps: int):
    """nsteps Runge-Kutta steps; returns (U, dts, guard)."""
    U = _c(U).copy()
    dts = np.zeros(max(nsteps, 1))
    g = lib().o6_step(_p(_c(prm)), U.shape[1], dx, _p(U), nsteps, _p(dts))
    if g < 0:
        raise ValueError("oracle step failed (%d)" % g)
    return U, dts[:nsteps], int(g)
