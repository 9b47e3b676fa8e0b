"""The fused face kernels of the 2-D gks_step (normal step of each direction
computed inside its face kernel, face-row values kept in LDS; forced with
fuse = 2 on these small grids, where the automatic choice takes the other
form) against the two-launch path (normal step writing the face-row buffer,
face kernels reading it): the same arithmetic, so every result is bitwise
the same. The 2-D parity tests compare the fused path with the oracle.

Cases cover tiles cut by the grid edges in both directions (sizes that are
not multiples of the 16 x 8 and 128-column tiles, single rows and columns),
every boundary kind, both precisions, characteristic variables, the learned
gate's flags, and faces queued for the full BGK solution (their face-row
values are written out by the fused kernels for the queue kernel).
"""
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


def _run(G, W, dW, steps, fuse, bc, precision, count=False, variables=0, gate_delta=0.0):
    nx, ny = W.shape[2], W.shape[1]
    grid = G.Grid(2, nx, ny, bc=bc, fuse=fuse, precision=precision, variables=variables,
                  gate_delta=gate_delta)
    Wd, dWd = grid.to_device(W), grid.grad_to_device(dW)
    ws = grid.workspace()
    dt = torch.zeros(steps, dtype=torch.float64, device="cuda")
    if count:
        G.count_enable(True)
    try:
        st = G.gks_step(grid, Wd, dWd, ws, steps, dt_out=dt, stats=True)
        work = G.work_read() if count else None
    finally:
        if count:
            G.count_enable(False)
    torch.cuda.synchronize()
    return grid.interior(Wd), grid.interior(dWd), dt.cpu().numpy(), st, work


CASES = [
    # kind, nx, ny, bc, precision, steps
    ("quadrants", 67, 45, 0, 0, 8),
    ("quadrants", 130, 33, 1, 1, 8),
    ("vortex", 33, 131, 2, 0, 6),
    ("quadrants", 129, 127, 1, 0, 6),
    ("vortex", 1, 5, 1, 0, 4),
    ("quadrants", 300, 1, 1, 1, 4),
    ("quadrants", 17, 300, 0, 0, 4),
    ("strong", 96, 80, 1, 0, 10),
]


@pytest.mark.parametrize("kind,nx,ny,bc,precision,steps", CASES)
def test_fused_equals_two_launch_path(G, kind, nx, ny, bc, precision, steps):
    _say("fused vs two-launch", kind, nx, ny, "bc", bc, "precision", precision, "steps", steps)
    if kind == "quadrants":
        W, dW, _ = inputs.quadrants_2d(nx, ny, 3)
    elif kind == "strong":
        W, dW, _ = inputs.quadrants_2d_strong(nx, ny, 1)
    else:
        W, dW, _ = inputs.vortex_2d(nx, ny, 3)
    a = _run(G, W, dW, steps, 2, bc, precision)
    b = _run(G, W, dW, steps, 0, bc, precision)
    for x, y, name in zip(a[:3], b[:3], ("W", "dW", "dt")):
        assert np.array_equal(x, y), name
    assert a[3].guard == b[3].guard and a[3].nonfinite == b[3].nonfinite == 0


CHAR_CASES = [
    # kind, nx, ny, bc, precision, steps
    ("quadrants", 67, 45, 0, 0, 6),
    ("quadrants", 130, 33, 1, 1, 6),
    ("strong", 96, 80, 1, 0, 8),
    ("vortex", 33, 131, 2, 1, 4),
]


@pytest.mark.parametrize("kind,nx,ny,bc,precision,steps", CHAR_CASES)
def test_fused_characteristic_equals_two_launch_path(G, kind, nx, ny, bc, precision, steps):
    # characteristic variables: each lane pair projects at the Roe average of
    # its face-row entry, two fields per lane, and maps its side back
    _say("fused vs two-launch, characteristic", kind, nx, ny, "bc", bc, "precision", precision)
    if kind == "quadrants":
        W, dW, _ = inputs.quadrants_2d(nx, ny, 5)
    elif kind == "strong":
        W, dW, _ = inputs.quadrants_2d_strong(nx, ny, 2)
    else:
        W, dW, _ = inputs.vortex_2d(nx, ny, 5)
    a = _run(G, W, dW, steps, 2, bc, precision, variables=1)
    b = _run(G, W, dW, steps, 0, bc, precision, variables=1)
    for x, y, name in zip(a[:3], b[:3], ("W", "dW", "dt")):
        assert np.array_equal(x, y), name
    assert a[3].guard == b[3].guard and a[3].nonfinite == b[3].nonfinite == 0


@pytest.mark.parametrize("precision", [0, 1])
def test_fused_with_learned_gate_equals_two_launch_path(G, precision):
    # a random network whose predictions straddle the threshold: the gated
    # cells take chi = 1 without their indicators in both forms
    rng = np.random.default_rng(11)
    p = 0.2 * rng.standard_normal(G.MLP_NPARAM)
    p[-1] = 0.0
    G.mlp_load(torch.tensor(p, dtype=torch.float32, device="cuda"))
    W, dW, _ = inputs.quadrants_2d(70, 52, 4)
    a = _run(G, W, dW, 5, 2, 1, precision, gate_delta=0.5)
    b = _run(G, W, dW, 5, 0, 1, precision, gate_delta=0.5)
    c = _run(G, W, dW, 5, 0, 1, precision)
    for x, y, name in zip(a[:3], b[:3], ("W", "dW", "dt")):
        assert np.array_equal(x, y), name
    # the gate changed the result (some cells were gated, some not)
    assert not np.array_equal(a[0], c[0])


def test_queued_faces_take_the_spilled_rows(G):
    # a jump case whose faces go to the full-solution queue (counted on the
    # same input): the queue kernel then reads the face-row values that the
    # fused kernels wrote for exactly those faces
    W, dW, _ = inputs.quadrants_2d(129, 127, 3)
    _, _, _, _, work = _run(G, W, dW, 3, 0, 1, 0, count=True)
    _say("queued faces", work["slow"]["units"])
    assert work["slow"]["units"] > 0
    a = _run(G, W, dW, 3, 2, 1, 0)
    b = _run(G, W, dW, 3, 0, 1, 0)
    assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3]))


def test_fused_full_size(G):
    # the 2048^2 quadrants + vortex workload of the benchmark, in its launch
    # configuration, a few steps
    n = 2048
    W, dW, _ = inputs.vortex_2d(n, n, 0)
    for precision in (0, 1):
        _say("full size, precision", precision)
        a = _run(G, W, dW, 3, 1, 1, precision)   # automatic: fused at this size
        b = _run(G, W, dW, 3, 0, 1, precision)
        assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3]))

