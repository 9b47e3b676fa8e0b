"""Python binding of the HIP library ``libgeno_gks.so`` (C ABI in ``include/geno_gks.h``).

Argument marshalling only: every step of the method runs in the library's
kernels. torch provides device memory and the current HIP stream. The
library is required: importing this module on a machine without the built
library, or calling it without a GPU, raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgeno_gks.so")

GENO_OK, GENO_EINVAL, GENO_EVERSION, GENO_EHIP, GENO_ENONPHYS = 0, -1, -2, -3, -4
BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTING, BC_FIXED = 0, 1, 2, 3
F64, MIXED = 0, 1
ABI_VERSION = 5
NG = 2
VARS_CONSERVATIVE, VARS_CHARACTERISTIC = 0, 1


class geno_params(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int), ("precision", ctypes.c_int), ("gamma", ctypes.c_double),
                ("C", ctypes.c_double), ("eps", ctypes.c_double), ("r", ctypes.c_double),
                ("rL", ctypes.c_double), ("d", ctypes.c_double * 3), ("tau_c1", ctypes.c_double),
                ("tau_c2", ctypes.c_double), ("cfl", ctypes.c_double), ("bc", ctypes.c_int * 4),
                ("dt_fixed", ctypes.c_double), ("eps_ulps", ctypes.c_double), ("gate_delta", ctypes.c_double),
                ("variables", ctypes.c_int), ("fuse", ctypes.c_int)]


class geno_grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("pitch", ctypes.c_int), ("rows", ctypes.c_int), ("x0", ctypes.c_double),
                ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("params", geno_params)]


class geno_tuning(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int), ("block_normal", ctypes.c_int), ("block_faces", ctypes.c_int),
                ("block_slow", ctypes.c_int), ("block_update", ctypes.c_int),
                ("slow_faces_per_block", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "version"}


class geno_stats(ctypes.Structure):
    _fields_ = [("guard", ctypes.c_longlong), ("nonfinite", ctypes.c_longlong),
                ("last_dt", ctypes.c_double)]


EXPORTS = ("geno_abi_version", "geno_last_error", "geno_params_default", "geno_grid_init",
           "geno_state_elems", "gks_workspace_bytes", "geno_reconstruct", "gks_flux", "gks_step",
           "gks_step_noalloc", "geno_timing_enable", "geno_count_enable", "geno_timing_read", "geno_work_read", "geno_op_costs",
           "geno_kernel_name", "geno_tuning_default", "gks_batched_workspace_bytes", "gks_step_batched",
           "geno_autotune_batched", "geno_harvest", "geno_mlp_train_workspace_bytes", "geno_mlp_grad",
           "geno_mlp_adam", "geno_mlp_forward", "geno_mlp_load", "geno_mlp_infer", "geno_gate_prob",
           "geno_conserved_totals", "geno_linearity", "geno_batched_graphs_built")
KERNELS = ("init", "normal_x", "normal_y", "faces_x", "faces_y", "slow", "update_1", "update_2", "faces_1d",
           "gate", "normal_xy", "fused_x", "fused_y")
WORK_CLASSES = ("units", "equal", "low", "fast", "slow", "guard", "gated")
MLP_NIN, MLP_NPARAM = 40, 6849

_lib = None


class GenoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("geno error %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.geno_abi_version.restype = i
        L.geno_last_error.restype = ctypes.c_char_p
        L.geno_params_default.argtypes = [ctypes.POINTER(geno_params)]
        L.geno_grid_init.argtypes = [ctypes.POINTER(geno_grid), i, i, i, d, d, d, d,
                                     ctypes.POINTER(geno_params)]
        L.geno_state_elems.argtypes = [ctypes.POINTER(geno_grid), i]
        L.geno_state_elems.restype = ctypes.c_size_t
        L.gks_workspace_bytes.argtypes = [ctypes.POINTER(geno_grid)]
        L.gks_workspace_bytes.restype = ctypes.c_size_t
        L.geno_reconstruct.argtypes = [ctypes.POINTER(geno_grid), vp, vp, i, vp, vp, vp, vp]
        L.gks_flux.argtypes = [ctypes.POINTER(geno_grid), vp, d, i, vp, vp, vp, vp]
        L.gks_step.argtypes = [ctypes.POINTER(geno_grid), vp, vp, vp, i, vp,
                               ctypes.POINTER(geno_stats), vp]
        L.gks_step_noalloc.argtypes = [ctypes.POINTER(geno_grid), vp, vp, i, vp,
                                       ctypes.POINTER(geno_stats), vp]
        L.geno_timing_enable.argtypes = [i]
        L.geno_count_enable.argtypes = [i]
        L.geno_timing_read.argtypes = [i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]
        L.geno_kernel_name.argtypes = [i]
        L.geno_kernel_name.restype = ctypes.c_char_p
        L.geno_work_read.argtypes = [i, i, ctypes.POINTER(ctypes.c_longlong), vp]
        L.geno_op_costs.argtypes = [ctypes.POINTER(geno_grid), i, i, ctypes.POINTER(ctypes.c_double)]
        L.geno_tuning_default.argtypes = [ctypes.POINTER(geno_tuning)]
        L.gks_batched_workspace_bytes.argtypes = [i, ctypes.POINTER(geno_grid)]
        L.gks_batched_workspace_bytes.restype = ctypes.c_size_t
        L.gks_step_batched.argtypes = [i, ctypes.POINTER(geno_grid), ctypes.POINTER(vp), ctypes.POINTER(vp), vp, i,
                                       ctypes.POINTER(geno_tuning), i, ctypes.POINTER(ctypes.c_float),
                                       ctypes.POINTER(geno_stats), vp]
        L.geno_autotune_batched.argtypes = [i, ctypes.POINTER(geno_grid), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                            vp, i, ctypes.POINTER(geno_tuning), vp]
        for name in ("geno_tuning_default", "gks_step_batched", "geno_autotune_batched"):
            getattr(L, name).restype = i
        L.geno_harvest.argtypes = [ctypes.POINTER(geno_grid), vp, vp, i, vp, vp, vp, vp]
        L.geno_mlp_train_workspace_bytes.argtypes = [i]
        L.geno_mlp_train_workspace_bytes.restype = ctypes.c_size_t
        L.geno_mlp_grad.argtypes = [vp, vp, vp, i, vp, vp, vp, vp]
        L.geno_mlp_adam.argtypes = [vp, vp, vp, vp, i, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, vp]
        L.geno_mlp_forward.argtypes = [vp, vp, i, vp, vp]
        L.geno_mlp_load.argtypes = [vp, vp]
        L.geno_mlp_infer.argtypes = [vp, i, vp, vp]
        L.geno_gate_prob.argtypes = [ctypes.POINTER(geno_grid), vp, vp, i, vp, vp, vp]
        L.geno_conserved_totals.argtypes = [ctypes.POINTER(geno_grid), vp, vp, vp]
        L.geno_linearity.argtypes = [ctypes.POINTER(geno_grid), vp, vp, i, vp, d, vp, vp]
        L.geno_batched_graphs_built.argtypes = []
        L.geno_batched_graphs_built.restype = ctypes.c_longlong
        for name in ("geno_harvest", "geno_mlp_grad", "geno_mlp_adam", "geno_mlp_forward", "geno_mlp_load",
                     "geno_mlp_infer", "geno_gate_prob", "geno_conserved_totals", "geno_linearity"):
            getattr(L, name).restype = i
        for name in ("geno_params_default", "geno_grid_init", "geno_reconstruct", "gks_flux", "gks_step",
                     "gks_step_noalloc", "geno_timing_enable", "geno_count_enable", "geno_timing_read", "geno_work_read",
                     "geno_op_costs"):
            getattr(L, name).restype = i
        if L.geno_abi_version() != ABI_VERSION:
            raise RuntimeError("library ABI %d != binding ABI %d" % (L.geno_abi_version(), ABI_VERSION))
        _lib = L
    return _lib


def _check(rc):
    if rc != GENO_OK:
        raise GenoError(rc, lib().geno_last_error().decode())


def default_params(**kw) -> geno_params:
    p = geno_params()
    _check(lib().geno_params_default(ctypes.byref(p)))
    for k, v in kw.items():
        if k == "bc":
            bcs = [v] * 4 if np.isscalar(v) else list(v)
            for j in range(4):
                p.bc[j] = int(bcs[j])
        elif k == "d":
            for j in range(3):
                p.d[j] = float(v[j])
        else:
            setattr(p, k, v)
    return p


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _need(t, dtype, nelem, name, optional=False):
    """The library takes plain pointers: check type, device, contiguity and size here."""
    if t is None:
        if optional:
            return
        raise ValueError("%s is required" % name)
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() < nelem:
        raise ValueError("%s must be a contiguous CUDA %s tensor of >= %d elements (got %s %s %s)"
                         % (name, dtype, nelem, t.dtype, tuple(t.shape), t.device))


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Grid:
    """A uniform 1-D or 2-D grid and its padded state layout."""

    def __init__(self, ndim, nx, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, params=None, **kw):
        self.params = params if params is not None else default_params(**kw)
        self.g = geno_grid()
        _check(lib().geno_grid_init(ctypes.byref(self.g), ndim, nx, ny, x0, x1, y0, y1,
                                    ctypes.byref(self.params)))
        self.ndim, self.nx, self.ny = ndim, nx, self.g.ny
        self.nv = 3 if ndim == 1 else 4
        self.pitch, self.rows = self.g.pitch, self.g.rows
        self.yoff = NG if ndim == 2 else 0
        self.mixed = self.params.precision == MIXED
        # element type of dW, face states and face fluxes (W is always float64)
        self.fdtype = torch.float32 if self.mixed else torch.float64

    @property
    def dx(self):
        return self.g.dx

    @property
    def dy(self):
        return self.g.dy

    def workspace(self, device="cuda"):
        n = lib().gks_workspace_bytes(ctypes.byref(self.g))
        return torch.empty(n, dtype=torch.uint8, device=device)

    def empty_state(self, nfields, device="cuda"):
        return torch.zeros((nfields, self.rows, self.pitch), dtype=torch.float64, device=device)

    def to_device(self, A, device="cuda", dtype=torch.float64):
        """Interior array [f, ny, nx] -> padded device tensor [f, rows, pitch]."""
        A = np.asarray(A, dtype=np.float64)
        out = np.zeros((A.shape[0], self.rows, self.pitch))
        out[:, self.yoff:self.yoff + self.ny, NG:NG + self.nx] = A
        return torch.from_numpy(out).to(device=device, dtype=dtype)

    def grad_to_device(self, A, device="cuda"):
        """Interior gradients [ndim * nv, ny, nx] -> padded device tensor of the grid's dW type."""
        return self.to_device(A, device, self.fdtype)

    def set_fixed_ghosts(self, W, dW, ghost):
        """1-D fixed ends: write the ghost states [end][layer 0 = next to the
        grid][W (3), dW (3)] into the padded device tensors W and dW."""
        if self.ndim != 1:
            raise ValueError("fixed-state ends are 1-D only")
        ghost = np.asarray(ghost, dtype=np.float64).reshape(2, NG, 6)
        for end in range(2):
            if self.params.bc[end] != BC_FIXED:
                continue
            for layer in range(NG):
                col = NG - 1 - layer if end == 0 else NG + self.nx + layer
                W[:, 0, col] = torch.as_tensor(ghost[end, layer, :3], dtype=W.dtype, device=W.device)
                dW[:, 0, col] = torch.as_tensor(ghost[end, layer, 3:], dtype=dW.dtype, device=dW.device)

    def interior(self, T):
        """Padded tensor -> interior numpy array [f, ny, nx]."""
        A = T.detach().cpu().numpy()
        return A[:, self.yoff:self.yoff + self.ny, NG:NG + self.nx].copy()

    def face_state_shape(self, direction=0):
        """Planes of geno_reconstruct's output: the point states
        [side][gauss][quant][var] then the points' second derivatives
        [gauss][quant2][var], over [nfy][nfx]."""
        if self.ndim == 1:
            return (2 * 1 * 2 * 3 + 1 * 1 * 3, 1, self.nx + 1)
        nfx, nfy = (self.nx + 1, self.ny) if direction == 0 else (self.nx, self.ny + 1)
        return (2 * 2 * 3 * 4 + 2 * 3 * 4, nfy, nfx)

    def face_state_parts(self, fs):
        """Split a face_state array (numpy) into the point states
        [side, gauss, quant, var, nfy, nfx] and the second derivatives
        [gauss, quant2, var, nfy, nfx]."""
        fs = np.asarray(fs)
        if self.ndim == 1:
            return fs[:12].reshape(2, 1, 2, 3, 1, self.nx + 1), fs[12:].reshape(1, 1, 3, 1, self.nx + 1)
        _, nfy, nfx = fs.shape
        return fs[:48].reshape(2, 2, 3, 4, nfy, nfx), fs[48:].reshape(2, 3, 4, nfy, nfx)

    def chi_shape(self, direction=0):
        if self.ndim == 1:
            return (2, 3, 1, self.nx + 1)
        return (2, 4, self.ny + 2, self.nx + 1) if direction == 0 else (2, 4, self.ny + 1, self.nx + 2)

    def flux_shape(self, direction=0):
        if self.ndim == 1:
            return (3, 1, self.nx + 1)
        return (4, self.ny, self.nx + 1) if direction == 0 else (4, self.ny + 1, self.nx)


def _prod(shape):
    return int(np.prod(shape))


def _check_state(grid, W, dW, ws=None):
    _need(W, torch.float64, grid.nv * grid.rows * grid.pitch, "W")
    _need(dW, grid.fdtype, grid.ndim * grid.nv * grid.rows * grid.pitch, "dW")
    if ws is not None:
        _need(ws, torch.uint8, lib().gks_workspace_bytes(ctypes.byref(grid.g)), "ws")


def geno_reconstruct(grid, W, dW, direction, face_state, chi, ws, stream=None):
    _check_state(grid, W, dW, ws)
    _need(face_state, grid.fdtype, _prod(grid.face_state_shape(direction)), "face_state")
    _need(chi, torch.float64, _prod(grid.chi_shape(direction)), "chi", optional=True)
    _check(lib().geno_reconstruct(ctypes.byref(grid.g), _ptr(W), _ptr(dW), int(direction),
                                  _ptr(face_state), _ptr(chi), _ptr(ws), _stream(stream)))


def gks_flux(grid, face_state, dt, direction, F, Ft, Wint, stream=None):
    """F, Ft: flux_shape; Wint: 3 x flux_shape (W(dt/2), W(dt), W_tt)."""
    _need(face_state, grid.fdtype, _prod(grid.face_state_shape(direction)), "face_state")
    for name, t, m in (("F", F, 1), ("Ft", Ft, 1), ("Wint", Wint, 3)):
        _need(t, grid.fdtype, m * _prod(grid.flux_shape(direction)), name, optional=True)
    _check(lib().gks_flux(ctypes.byref(grid.g), _ptr(face_state), float(dt), int(direction),
                          _ptr(F), _ptr(Ft), _ptr(Wint), _stream(stream)))


def gks_step(grid, W, dW, ws, nsteps, dt_out=None, stats=False, stream=None):
    """nsteps S2O4 steps in place. Returns a geno_stats if stats=True (synchronises)."""
    _check_state(grid, W, dW, ws)
    if dt_out is not None:
        _need(dt_out, torch.float64, int(nsteps), "dt_out")
    st = geno_stats() if stats else None
    rc = lib().gks_step(ctypes.byref(grid.g), _ptr(W), _ptr(dW), _ptr(ws), int(nsteps), _ptr(dt_out),
                        ctypes.byref(st) if st is not None else None, _stream(stream))
    _check(rc)
    return st


NOALLOC_SCRATCH_BYTES = 64 << 20   # GENO_NOALLOC_SCRATCH_BYTES


def gks_step_noalloc(grid, W, dW, nsteps, dt_out=None, stats=False, stream=None):
    """gks_step with the library's own per-device scratch as workspace (no
    allocation by the library; calls overlapping on one device race).
    Returns a geno_stats if stats=True (synchronises)."""
    _check_state(grid, W, dW)
    if dt_out is not None:
        _need(dt_out, torch.float64, int(nsteps), "dt_out")
    st = geno_stats() if stats else None
    rc = lib().gks_step_noalloc(ctypes.byref(grid.g), _ptr(W), _ptr(dW), int(nsteps), _ptr(dt_out),
                                ctypes.byref(st) if st is not None else None, _stream(stream))
    _check(rc)
    return st


LINEARITY_METHODS = ("geno", "weno_z", "teno")


def linearity(grid, W, dW, direction, ws, teno_ct=1e-6, out=None, stream=None):
    """chi of GENO, WENO-Z and TENO at every face-side of a direction:
    device float64 tensor [3][2][nvar][n0][n1] (layout of geno_reconstruct's chi)."""
    _check_state(grid, W, dW, ws)
    shape = (3,) + tuple(grid.chi_shape(direction))
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=W.device)
    _need(out, torch.float64, _prod(shape), "chi3")
    _check(lib().geno_linearity(ctypes.byref(grid.g), _ptr(W), _ptr(dW), int(direction), _ptr(out),
                                float(teno_ct), _ptr(ws), _stream(stream)))
    return out


def conserved_totals(grid, W, out=None, stream=None):
    """|cell| * sum of the interior cells of every field (device float64 tensor of nv)."""
    _need(W, torch.float64, grid.nv * grid.rows * grid.pitch, "W")
    if out is None:
        out = torch.empty(grid.nv, dtype=torch.float64, device=W.device)
    _need(out, torch.float64, grid.nv, "totals")
    _check(lib().geno_conserved_totals(ctypes.byref(grid.g), _ptr(W), _ptr(out), _stream(stream)))
    return out


def timing_enable(max_launches):
    _check(lib().geno_timing_enable(int(max_launches)))


def count_enable(on=True):
    _check(lib().geno_count_enable(1 if on else 0))


def timing_read():
    """{kernel name: (total ms, launches)} of the launches recorded since the last read."""
    n = len(KERNELS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_longlong * n)()
    _check(lib().geno_timing_read(n, ms, cnt))
    return {lib().geno_kernel_name(k).decode(): (ms[k], cnt[k]) for k in range(n)}


def work_read(stream=None):
    """{kernel: {class: count}} counted during the last gks_step made with counting enabled."""
    nk, nc = len(KERNELS), len(WORK_CLASSES)
    out = (ctypes.c_longlong * (nk * nc))()
    _check(lib().geno_work_read(nk, nc, out, _stream(stream)))
    return {KERNELS[a]: {WORK_CLASSES[c]: out[a * nc + c] for c in range(nc)} for a in range(nk)}


def op_costs(grid):
    """{kernel: {class: floating-point operations per counted item}} (host-side count)."""
    nk, nc = len(KERNELS), len(WORK_CLASSES)
    out = (ctypes.c_double * (nk * nc))()
    _check(lib().geno_op_costs(ctypes.byref(grid.g), nk, nc, out))
    return {KERNELS[a]: {WORK_CLASSES[c]: out[a * nc + c] for c in range(nc)} for a in range(nk)}


# ------------------------------------------------------------------ batched form
def default_tuning():
    t = geno_tuning()
    _check(lib().geno_tuning_default(ctypes.byref(t)))
    return t


BATCH_EAGER, BATCH_GRAPH, BATCH_PERSISTENT = 0, 1, 2


def batched_graphs_built():
    """Batched-step graphs instantiated by this process so far."""
    return int(lib().geno_batched_graphs_built())


class Batch:
    """Independent 2-D grids advanced together by gks_step_batched. Grids may
    differ in size and boundary conditions; all other parameters must match."""

    def __init__(self, grids):
        self.grids = list(grids)
        n = len(self.grids)
        self.garr = (geno_grid * n)(*[g.g for g in self.grids])
        self.n = n

    def workspace(self, device="cuda"):
        nb = lib().gks_batched_workspace_bytes(self.n, self.garr)
        if nb == 0:
            raise GenoError(GENO_EINVAL, lib().geno_last_error().decode())
        return torch.empty(nb, dtype=torch.uint8, device=device)

    def _ptrs(self, Ws, dWs, ws):
        if len(Ws) != self.n or len(dWs) != self.n:
            raise ValueError("one W and one dW per grid")
        for g, W, dW in zip(self.grids, Ws, dWs):
            _check_state(g, W, dW)
        _need(ws, torch.uint8, lib().gks_batched_workspace_bytes(self.n, self.garr), "ws")
        pw = (ctypes.c_void_p * self.n)(*[W.data_ptr() for W in Ws])
        pd = (ctypes.c_void_p * self.n)(*[d.data_ptr() for d in dWs])
        return pw, pd

    def step(self, Ws, dWs, ws, nsteps, tuning=None, graph=True, step_times=False, stats=False, stream=None,
             mode=None):
        """nsteps steps of every grid in place; returns (step_ms array or None, geno_stats or None).
        mode: BATCH_EAGER, BATCH_GRAPH or BATCH_PERSISTENT (default: BATCH_GRAPH if graph else
        BATCH_EAGER). The graph modes run on a side stream (the NULL stream cannot be captured)."""
        if mode is None:
            mode = BATCH_GRAPH if graph else BATCH_EAGER
        pw, pd = self._ptrs(Ws, dWs, ws)
        if stream is None:
            stream = torch.cuda.Stream() if mode != BATCH_EAGER else torch.cuda.current_stream()
        stream.wait_stream(torch.cuda.current_stream())
        ms = (ctypes.c_float * max(int(nsteps), 1))() if step_times else None
        st = geno_stats() if stats else None
        _check(lib().gks_step_batched(self.n, self.garr, pw, pd, _ptr(ws), int(nsteps),
                                      ctypes.byref(tuning) if tuning is not None else None, int(mode),
                                      ms, ctypes.byref(st) if st is not None else None,
                                      ctypes.c_void_p(stream.cuda_stream)))
        torch.cuda.current_stream().wait_stream(stream)
        return (np.array(ms[:nsteps], dtype=np.float64) if step_times else None), st

    def autotune(self, Ws, dWs, ws, trial_steps=3, stream=None):
        """Autotuned work-group shapes (the trials advance the given state: pass copies)."""
        pw, pd = self._ptrs(Ws, dWs, ws)
        if stream is None:
            stream = torch.cuda.current_stream()
        t = geno_tuning()
        _check(lib().geno_autotune_batched(self.n, self.garr, pw, pd, _ptr(ws), int(trial_steps),
                                           ctypes.byref(t), ctypes.c_void_p(stream.cuda_stream)))
        return t


# ------------------------------------------------------------------ learned gate
def harvest(grid, W, dW, ws, direction, with_target=True, stream=None):
    """(X[ncell, 40], y[ncell] or None) float32 device tensors for one direction."""
    _check_state(grid, W, dW, ws)
    nc = grid.nx * grid.ny
    X = torch.empty((nc, MLP_NIN), dtype=torch.float32, device=W.device)
    y = torch.empty(nc, dtype=torch.float32, device=W.device) if with_target else None
    _check(lib().geno_harvest(ctypes.byref(grid.g), _ptr(W), _ptr(dW), int(direction), _ptr(X), _ptr(y),
                              _ptr(ws), _stream(stream)))
    return X, y


def _need_mlp(params):
    _need(params, torch.float32, MLP_NPARAM, "params")


def mlp_train_workspace(n, device="cuda"):
    return torch.empty(lib().geno_mlp_train_workspace_bytes(int(n)), dtype=torch.uint8, device=device)


def mlp_grad(params, X, y, grad, loss, ws, stream=None):
    _need_mlp(params)
    n = X.shape[0]
    _need(X, torch.float32, n * MLP_NIN, "X")
    _need(y, torch.float32, n, "y")
    _need(grad, torch.float32, MLP_NPARAM, "grad")
    _need(loss, torch.float32, 1, "loss", optional=True)
    _need(ws, torch.uint8, lib().geno_mlp_train_workspace_bytes(int(n)), "ws")
    _check(lib().geno_mlp_grad(_ptr(params), _ptr(X), _ptr(y), int(n), _ptr(grad), _ptr(loss), _ptr(ws),
                               _stream(stream)))


def mlp_adam(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    for name, x in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        _need(x, torch.float32, MLP_NPARAM, name)
    _check(lib().geno_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t), float(lr), float(beta1),
                               float(beta2), float(eps), _stream(stream)))


def mlp_forward(params, X, stream=None):
    _need_mlp(params)
    n = X.shape[0]
    _need(X, torch.float32, n * MLP_NIN, "X")
    p = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(lib().geno_mlp_forward(_ptr(params), _ptr(X), int(n), _ptr(p), _stream(stream)))
    return p


def mlp_load(params, stream=None):
    _need_mlp(params)
    _check(lib().geno_mlp_load(_ptr(params), _stream(stream)))


def mlp_infer(X, stream=None):
    n = X.shape[0]
    _need(X, torch.float32, n * MLP_NIN, "X")
    p = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(lib().geno_mlp_infer(_ptr(X), int(n), _ptr(p), _stream(stream)))
    return p


def gate_prob(grid, W, dW, ws, direction, stream=None):
    _check_state(grid, W, dW, ws)
    p = torch.empty(grid.nx * grid.ny, dtype=torch.float32, device=W.device)
    _check(lib().geno_gate_prob(ctypes.byref(grid.g), _ptr(W), _ptr(dW), int(direction), _ptr(p), _ptr(ws),
                                _stream(stream)))
    return p

