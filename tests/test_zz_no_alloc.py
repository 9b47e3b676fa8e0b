"""gks_step_noalloc (the allocation-free step, whose workspace is the
library's per-device scratch array) against gks_step with a caller-owned
workspace, through the C ABI: two calls in a row on the same device, the
second on a smaller grid, so that the second call runs over scratch contents
left by the first. Both entry points launch the same kernels on the same
inputs, so the results must be bitwise equal."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2507_20461_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_20461_amd import geno_gks
    geno_gks.lib()
    return geno_gks


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _state(ndim, nx, ny, seed):
    if ndim == 1:
        W, dW, _ = inputs.jump_1d(nx, seed)
        return W, dW
    W, dW, _ = inputs.quadrants_2d(nx, ny, seed)
    return W, dW


def _both(G, grid, W, dW, nsteps):
    """The same run through gks_step (own workspace) and gks_step_noalloc."""
    out = []
    for noalloc in (False, True):
        Wd = grid.to_device(W)
        dWd = grid.grad_to_device(dW)
        dts = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
        if noalloc:
            st = G.gks_step_noalloc(grid, Wd, dWd, nsteps, dt_out=dts, stats=True)
        else:
            st = G.gks_step(grid, Wd, dWd, grid.workspace(), nsteps, dt_out=dts, stats=True)
        torch.cuda.synchronize()
        out.append((Wd.cpu().numpy(), dWd.cpu().numpy(), dts.cpu().numpy(), st.guard, st.last_dt))
    return out


@pytest.mark.parametrize("ndim,prec,big,small", [
    (2, "f64", (96, 80), (40, 36)),
    (2, "mixed", (120, 104), (48, 30)),
    (1, "f64", (4000, 1), (300, 1)),
])
def test_noalloc_matches_gks_step_two_calls(G, ndim, prec, big, small):
    precision = G.MIXED if prec == "mixed" else G.F64
    for call, (nx, ny) in enumerate((big, small)):
        _say("noalloc", ndim, prec, "call", call + 1, nx, ny)
        grid = G.Grid(ndim, nx, ny, bc=1, precision=precision)
        assert G.lib().gks_workspace_bytes(ctypes.byref(grid.g)) <= G.NOALLOC_SCRATCH_BYTES
        W, dW = _state(ndim, nx, ny, 3 + call)
        (a, da, ta, ga, la), (b, db, tb, gb, lb) = _both(G, grid, W, dW, 6)
        assert np.array_equal(a, b) and np.array_equal(da, db), (ndim, prec, call)
        assert np.array_equal(ta, tb) and ga == gb and la == lb
        assert np.all(np.isfinite(b))


def test_noalloc_rejects_grid_beyond_scratch(G):
    # a grid whose workspace exceeds the scratch is refused on the host with
    # GENO_EINVAL before anything is launched; the state is left as it was
    grid = G.Grid(2, 320, 320, bc=1)
    assert G.lib().gks_workspace_bytes(ctypes.byref(grid.g)) > G.NOALLOC_SCRATCH_BYTES
    W, dW = _state(2, 320, 320, 5)
    Wd, dWd = grid.to_device(W), grid.grad_to_device(dW)
    before = Wd.clone()
    with pytest.raises(G.GenoError) as e:
        G.gks_step_noalloc(grid, Wd, dWd, 1)
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(Wd, before)
