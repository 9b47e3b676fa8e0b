"""Python binding of the fourth-order compact GENO reconstruction on
triangular meshes (C ABI in ``include/geno_tri.h``; the entry points live in
``libgeno_gks.so``).

Argument marshalling only: the operator table is built by the library's
host mesh layer, the reconstruction runs in its kernel. torch provides
device memory and the current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import geno_gks as G

EXPORTS = ("geno_tri_table_doubles", "geno_tri_build", "geno_tri_reconstruct", "geno_tri_op_cost",
           "geno_tri_workspace_bytes", "geno_tri_step")
MAXV = 4
_ready = False


def lib():
    global _ready
    L = G.lib()
    if not _ready:
        vp, i, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        L.geno_tri_table_doubles.restype = ctypes.c_size_t
        L.geno_tri_table_doubles.argtypes = []
        L.geno_tri_build.argtypes = [i, dp, ctypes.POINTER(ctypes.c_int), dp, dp]
        L.geno_tri_build.restype = i
        L.geno_tri_reconstruct.argtypes = [i, i, vp, vp, vp, vp, vp, vp, vp]
        L.geno_tri_reconstruct.restype = i
        L.geno_tri_workspace_bytes.argtypes = [i]
        L.geno_tri_workspace_bytes.restype = ctypes.c_size_t
        L.geno_tri_step.argtypes = [i, vp, vp, vp, vp, i, ctypes.POINTER(G.geno_params), vp,
                                    ctypes.POINTER(G.geno_stats), vp]
        L.geno_tri_step.restype = i
        L.geno_tri_op_cost.restype = ctypes.c_double
        L.geno_tri_op_cost.argtypes = []
        _ready = True
    return L


def build_table(mesh) -> np.ndarray:
    """Host operator table of a mesh dict (xv, nbr, shift): table_doubles *
    ncell doubles, entry e of cell c at ((e // 2) * ncell + c) * 2 + e % 2."""
    xv = np.ascontiguousarray(mesh["xv"], dtype=np.float64)
    nbr = np.ascontiguousarray(mesh["nbr"], dtype=np.int32)
    sh = np.ascontiguousarray(mesh["shift"], dtype=np.float64)
    n = xv.shape[0]
    nt = lib().geno_tri_table_doubles()
    ops = np.zeros(nt * n)
    dp = ctypes.POINTER(ctypes.c_double)
    G._check(lib().geno_tri_build(n, xv.ctypes.data_as(dp), nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                  sh.ctypes.data_as(dp), ops.ctypes.data_as(dp)))
    return ops


class TriMesh:
    """A triangle mesh with its operator table on the device."""

    def __init__(self, mesh, device="cuda"):
        self.ncell = int(np.asarray(mesh["xv"]).shape[0])
        self.table_host = build_table(mesh)
        self.table = torch.from_numpy(self.table_host).to(device)

    def out_shape(self, nv):
        return (6, 3, nv, self.ncell)

    def workspace(self, device="cuda"):
        """Device workspace of step()."""
        return torch.empty(lib().geno_tri_workspace_bytes(self.ncell), dtype=torch.uint8, device=device)


def reconstruct(tm, W, dW, out, chi=None, sec=None, stream=None):
    """W [nv, ncell], dW [2, nv, ncell] float64 on the device; out [6, 3, nv,
    ncell]; chi [nv, ncell] or None; sec [6, 3, nv, ncell] (h^2 second
    derivatives) or None."""
    nv = W.shape[0]
    G._need(W, torch.float64, nv * tm.ncell, "W")
    G._need(dW, torch.float64, 2 * nv * tm.ncell, "dW")
    G._need(out, torch.float64, 18 * nv * tm.ncell, "out")
    G._need(chi, torch.float64, nv * tm.ncell, "chi", optional=True)
    G._need(sec, torch.float64, 18 * nv * tm.ncell, "sec", optional=True)
    G._check(lib().geno_tri_reconstruct(tm.ncell, nv, G._ptr(tm.table), G._ptr(W), G._ptr(dW), G._ptr(out),
                                        G._ptr(chi), G._ptr(sec), G._stream(stream)))


def step(tm, W, dW, ws, nsteps, dt_out=None, stats=False, stream=None, **params):
    """nsteps compact GKS steps in place: W [4, ncell], dW [2, 4, ncell] float64
    on the device; params: geno_params fields (gamma, cfl, tau_c1, tau_c2,
    dt_fixed). Returns a geno_stats if stats=True (synchronises)."""
    G._need(W, torch.float64, 4 * tm.ncell, "W")
    G._need(dW, torch.float64, 8 * tm.ncell, "dW")
    G._need(ws, torch.uint8, lib().geno_tri_workspace_bytes(tm.ncell), "ws")
    if dt_out is not None:
        G._need(dt_out, torch.float64, int(nsteps), "dt_out")
    p = G.geno_params()
    G._check(G.lib().geno_params_default(ctypes.byref(p)))
    for key, val in params.items():
        if not hasattr(p, key):
            raise TypeError("unknown parameter " + key)
        setattr(p, key, val)
    st = G.geno_stats() if stats else None
    G._check(lib().geno_tri_step(tm.ncell, G._ptr(tm.table), G._ptr(W), G._ptr(dW), G._ptr(ws), int(nsteps),
                                 ctypes.byref(p), G._ptr(dt_out), ctypes.byref(st) if st is not None else None,
                                 G._stream(stream)))
    return st


def op_cost():
    return lib().geno_tri_op_cost()
