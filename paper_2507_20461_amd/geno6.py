"""Python binding of the sixth-order non-compact scheme (C ABI in
``include/geno6.h``; the entry points live in ``libgeno_gks.so``).

Argument marshalling only: reconstruction, flux and Runge-Kutta stages run in
the library's kernels. torch provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import geno_gks as G

ABI_VERSION = 3
VARS_CONSERVATIVE, VARS_CHARACTERISTIC = 0, 1
BC_FIXED = 3
KERNELS = ("init", "dt", "stage", "small")
EXPORTS = ("geno6_params_default", "geno6_grid_init", "geno6_workspace_bytes", "geno6_faces", "geno6_rhs",
           "geno6_step", "geno6_timing_enable", "geno6_timing_read", "geno6_op_costs",
           "geno6_batch_workspace_bytes", "geno6_step_batch")


class geno6_params(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int), ("gamma", ctypes.c_double), ("C", ctypes.c_double),
                ("eps", ctypes.c_double), ("d", ctypes.c_double * 4), ("cfl", ctypes.c_double),
                ("bc", ctypes.c_int * 2), ("dt_fixed", ctypes.c_double), ("variables", ctypes.c_int),
                ("ghost", ctypes.c_double * 18)]


class geno6_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("pitch", ctypes.c_int), ("x0", ctypes.c_double),
                ("x1", ctypes.c_double), ("dx", ctypes.c_double), ("params", geno6_params)]


_ready = False


def lib():
    global _ready
    L = G.lib()
    if not _ready:
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        gp = ctypes.POINTER(geno6_grid)
        L.geno6_params_default.argtypes = [ctypes.POINTER(geno6_params)]
        L.geno6_grid_init.argtypes = [gp, i, d, d, ctypes.POINTER(geno6_params)]
        L.geno6_workspace_bytes.argtypes = [gp]
        L.geno6_workspace_bytes.restype = ctypes.c_size_t
        L.geno6_faces.argtypes = [gp, vp, vp, vp, vp, vp, vp]
        L.geno6_rhs.argtypes = [gp, vp, vp, vp]
        L.geno6_step.argtypes = [gp, vp, vp, i, vp, ctypes.POINTER(G.geno_stats), vp]
        L.geno6_timing_enable.argtypes = [i]
        L.geno6_timing_read.argtypes = [i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]
        L.geno6_op_costs.argtypes = [ctypes.POINTER(ctypes.c_double)]
        L.geno6_batch_workspace_bytes.argtypes = [gp, i]
        L.geno6_batch_workspace_bytes.restype = ctypes.c_size_t
        L.geno6_step_batch.argtypes = [gp, i, vp, vp, i, vp, ctypes.POINTER(G.geno_stats), vp]
        for name in EXPORTS:
            if name not in ("geno6_workspace_bytes", "geno6_batch_workspace_bytes"):
                getattr(L, name).restype = i
        _ready = True
    return L


def default_params(**kw) -> geno6_params:
    p = geno6_params()
    G._check(lib().geno6_params_default(ctypes.byref(p)))
    for k, v in kw.items():
        if k == "bc":
            bcs = [v] * 2 if np.isscalar(v) else list(v)
            p.bc[0], p.bc[1] = int(bcs[0]), int(bcs[1])
        elif k == "d":
            for j in range(4):
                p.d[j] = float(v[j])
        elif k == "ghost":   # [end][cell k][field], see geno6.h
            for j, x in enumerate(np.asarray(v, dtype=np.float64).reshape(18)):
                p.ghost[j] = float(x)
        else:
            setattr(p, k, v)
    return p


class Grid6:
    """n uniform cells on [x0, x1]; state U[3, pitch] float64 on the device."""

    def __init__(self, n, x0=0.0, x1=1.0, params=None, **kw):
        self.params = params if params is not None else default_params(**kw)
        self.g = geno6_grid()
        G._check(lib().geno6_grid_init(ctypes.byref(self.g), int(n), float(x0), float(x1),
                                       ctypes.byref(self.params)))
        self.n, self.pitch, self.dx = self.g.n, self.g.pitch, self.g.dx

    def workspace(self, device="cuda"):
        return torch.empty(lib().geno6_workspace_bytes(ctypes.byref(self.g)), dtype=torch.uint8,
                           device=device)

    def to_device(self, U, device="cuda"):
        U = np.asarray(U, dtype=np.float64)
        out = np.zeros((3, self.pitch))
        out[:, :self.n] = U
        return torch.from_numpy(out).to(device)

    def interior(self, T):
        return T.detach().cpu().numpy()[:, :self.n].copy()


def _state(grid, U, name="U"):
    G._need(U, torch.float64, 3 * grid.pitch, name)


def faces(grid, U, UL=None, UR=None, F=None, chi=None, stream=None):
    """Reconstructed states, HLLC fluxes [3, n+1] and path functions [2, 3, n+1]."""
    _state(grid, U)
    nf = grid.n + 1
    for t, name, m in ((UL, "UL", 3), (UR, "UR", 3), (F, "F", 3), (chi, "chi", 6)):
        G._need(t, torch.float64, m * nf, name, optional=True)
    G._check(lib().geno6_faces(ctypes.byref(grid.g), G._ptr(U), G._ptr(UL), G._ptr(UR), G._ptr(F),
                               G._ptr(chi), G._stream(stream)))


def rhs(grid, U, L, stream=None):
    _state(grid, U)
    _state(grid, L, "L")
    G._check(lib().geno6_rhs(ctypes.byref(grid.g), G._ptr(U), G._ptr(L), G._stream(stream)))


def step(grid, U, ws, nsteps, dt_out=None, stats=False, stream=None):
    """nsteps Runge-Kutta steps of U in place; returns geno_stats if stats."""
    _state(grid, U)
    G._need(ws, torch.uint8, lib().geno6_workspace_bytes(ctypes.byref(grid.g)), "ws")
    G._need(dt_out, torch.float64, nsteps, "dt_out", optional=True)
    st = G.geno_stats() if stats else None
    G._check(lib().geno6_step(ctypes.byref(grid.g), G._ptr(U), G._ptr(ws), int(nsteps), G._ptr(dt_out),
                              ctypes.byref(st) if st is not None else None, G._stream(stream)))
    return st


def timing_enable(max_launches):
    G._check(lib().geno6_timing_enable(int(max_launches)))


def timing_read():
    """{kernel: (total ms, launches)} since the last read."""
    n = len(KERNELS)
    ms = (ctypes.c_double * n)()
    nl = (ctypes.c_longlong * n)()
    G._check(lib().geno6_timing_read(n, ms, nl))
    return {KERNELS[k]: (ms[k], nl[k]) for k in range(n)}


def op_costs():
    """Operations per face (both sides, three variables, guard tests, HLLC),
    per low-order side (chi < 1) and per cell (flux difference and stage)."""
    c = (ctypes.c_double * 3)()
    G._check(lib().geno6_op_costs(c))
    return {"face": c[0], "low_side": c[1], "cell": c[2]}


def batch_workspace(grid, ngrids, device="cuda"):
    return torch.empty(lib().geno6_batch_workspace_bytes(ctypes.byref(grid.g), int(ngrids)), dtype=torch.uint8,
                       device=device)


def step_batch(grid, U, ws, nsteps, dt_out=None, stats=False, stream=None):
    """nsteps steps of every grid of U [ngrids, 3, pitch] in place, one launch."""
    ngrids = U.shape[0]
    G._need(U, torch.float64, ngrids * 3 * grid.pitch, "U")
    G._need(ws, torch.uint8, lib().geno6_batch_workspace_bytes(ctypes.byref(grid.g), int(ngrids)), "ws")
    G._need(dt_out, torch.float64, ngrids * nsteps, "dt_out", optional=True)
    st = G.geno_stats() if stats else None
    G._check(lib().geno6_step_batch(ctypes.byref(grid.g), int(ngrids), G._ptr(U), G._ptr(ws), int(nsteps),
                                    G._ptr(dt_out), ctypes.byref(st) if st is not None else None,
                                    G._stream(stream)))
    return st
