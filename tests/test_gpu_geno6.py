"""Parity of the sixth-order non-compact HIP path (geno6_* through the C ABI)
with its CPU FP64 oracle.

Tolerance (FP64): |gpu - oracle| <= 1e-12 * max(|oracle|, scale of the
field), the scale of a field being its largest |value| (fluxes and
right-hand sides on their own scales). The two sides evaluate the same
formulas in different association orders (closed-form stencil coefficients
against per-call Gaussian elimination), so they agree to a few units of
rounding times the conditioning of the blend; path functions are compared
to 1e-9 absolute: chi takes IS^tau = |(IS_1 + IS_3)/2 - IS_2|, a difference
of nearly equal indicators on smooth data, whose rounding the two sides do
not share. Multi-step runs through discontinuities are compared step by
step from the GPU state (a shadow of the trajectory), since rounding-level
differences at a switching path function are not damped.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import geno6 as O6
from paper_2507_20461_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12
CHI_TOL = 1e-9
# The cold-flow case (p = 1e-9 under a kinetic energy of about 2) forms the
# pressure as a difference of numbers 1e9 times larger, so p carries a
# relative rounding of about 1e9 * 2^-53 = 1e-7 on either side, the sound
# speed (3e-5) half of that, and the HLLC wave speeds an absolute 2e-12 that
# the star fluxes inherit. Its fluxes are compared to 1e-10. With
# characteristic variables the left eigenvectors there carry entries
# b1 u^2 / 2 = (gamma - 1) u^2 / (2 c^2) ~ 1e9 (c ~ 4e-5), so the projected
# fields are ~1e9 times the data and cancel back on the way out: the
# states then agree to about 2^-53 * (|u| / c)^2 ~ 3e-7 relative, and the
# cold case with characteristic variables is compared to 1e-6.
TOL_COLD = 1e-10
TOL_COLD_CHAR = 1e-6


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_20461_amd import geno6
    geno6.lib()
    O6.build(force=False)
    return geno6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(g, o):
    g = np.asarray(g, dtype=np.float64).reshape(np.shape(o)[0], -1)
    o = np.asarray(o, dtype=np.float64).reshape(g.shape[0], -1)
    sc = np.abs(o).max(axis=1)
    sc = np.where(sc > 0, sc, 1.0)
    return float((np.abs(g - o) / np.maximum(np.abs(o), sc[:, None])).max())


BCS = {"periodic": (0, 0), "transmissive": (1, 1), "reflecting": (2, 2), "trans_refl": (1, 2)}


def state(kind, n, seed=0):
    if kind == "smooth":
        return inputs.smooth_noncompact(n, seed)
    if kind == "shocks":
        return inputs.shocks_noncompact(n, seed, cells_per_segment=max(4, n // 5))
    if kind == "cold":   # cold fast flow: reconstructed pressures go negative (guard)
        x = np.arange(n) / n
        u = 2.0 * np.sin(2 * np.pi * x)
        rho = 1.0 + 0.5 * np.cos(2 * np.pi * x)
        return np.stack([rho, rho * u, 1e-9 / 0.4 + 0.5 * rho * u * u])
    raise ValueError(kind)


def gpu_faces(S, grid, U):
    nf = grid.n + 1
    Ud = grid.to_device(U)
    UL, UR, F = (torch.zeros(3, nf, dtype=torch.float64, device="cuda") for _ in range(3))
    chi = torch.zeros(2, 3, nf, dtype=torch.float64, device="cuda")
    S.faces(grid, Ud, UL, UR, F, chi)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (UL, UR, F, chi)]


# the cold-flow state is periodic: it runs with periodic ends only
FACE_CASES = [(n, bc, kind) for n in (3, 7, 64, 255, 256, 1021) for bc in BCS
              for kind in ("smooth", "shocks", "cold") if kind != "cold" or bc == "periodic"]


@pytest.mark.parametrize("n,bc,kind", FACE_CASES)
@pytest.mark.parametrize("char", [False, True], ids=["cons", "char"])
def test_faces(S, n, bc, kind, char):
    _say("geno6 faces n=%d bc=%s %s char=%d" % (n, bc, kind, char))
    U = state(kind, n, seed=n)
    grid = S.Grid6(n, 0.0, 1.0, bc=BCS[bc], variables=int(char))
    g = gpu_faces(S, grid, U)
    o = O6.faces(O6.params(bc=BCS[bc], characteristic=char), U)
    for name, a, b in zip(("UL", "UR", "F"), g[:3], o[:3]):
        e = rel_err(a, b)
        tol = TOL
        if kind == "cold":
            tol = TOL_COLD_CHAR if char else (TOL_COLD if name == "F" else TOL)
        assert e <= tol, (name, e)
    assert np.abs(g[3] - o[3]).max() <= (TOL_COLD_CHAR if kind == "cold" and char else CHI_TOL)


@pytest.mark.parametrize("n,bc,kind", [(300, "periodic", "smooth"), (300, "transmissive", "shocks"),
                                       (511, "reflecting", "shocks"), (40, "periodic", "cold")])
@pytest.mark.parametrize("char", [False, True], ids=["cons", "char"])
def test_rhs(S, n, bc, kind, char):
    _say("geno6 rhs n=%d bc=%s %s char=%d" % (n, bc, kind, char))
    U = state(kind, n, seed=3)
    grid = S.Grid6(n, 0.0, 1.0, bc=BCS[bc], variables=int(char))
    L = torch.zeros(3, grid.pitch, dtype=torch.float64, device="cuda")
    S.rhs(grid, grid.to_device(U), L)
    torch.cuda.synchronize()
    Lo, _ = O6.rhs(O6.params(bc=BCS[bc], characteristic=char), U, grid.dx)
    assert rel_err(L.cpu().numpy()[:, :n], Lo) <= (TOL_COLD if kind == "cold" else TOL)


def test_steps_on_the_density_wave(S):
    # smooth periodic data: the trajectories stay together over many steps
    n, steps = 48, 20
    U = inputs.density_wave_noncompact(n)
    grid = S.Grid6(n, 0.0, 2.0)
    Ud = grid.to_device(U)
    dts = torch.zeros(steps, dtype=torch.float64, device="cuda")
    st = S.step(grid, Ud, grid.workspace(), steps, dt_out=dts, stats=True)
    Uo, dto, go = O6.step(O6.params(), U, grid.dx, steps)
    assert st.guard == 0 == go and st.nonfinite == 0
    assert np.abs(dts.cpu().numpy() - dto).max() <= 1e-14 * dto.max()
    assert st.last_dt == pytest.approx(dto[-1], rel=1e-14)
    assert rel_err(grid.interior(Ud), Uo) <= TOL


@pytest.mark.parametrize("bc,kind,n", [("transmissive", "shocks", 600), ("reflecting", "shocks", 257),
                                       ("periodic", "shocks", 1000), ("trans_refl", "smooth", 130)])
@pytest.mark.parametrize("char", [False, True], ids=["cons", "char"])
def test_step_shadow(S, bc, kind, n, char):
    _say("geno6 shadow n=%d bc=%s %s char=%d" % (n, bc, kind, char))
    U = state(kind, n, seed=5)
    grid = S.Grid6(n, 0.0, 1.0, bc=BCS[bc], cfl=0.5, variables=int(char))
    Ud = grid.to_device(U)
    ws = grid.workspace()
    dts = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k in range(8):
        start = grid.interior(Ud)
        S.step(grid, Ud, ws, 1, dt_out=dts)
        torch.cuda.synchronize()
        dt = float(dts.item())
        assert dt == pytest.approx(O6.cfl_dt(O6.params(bc=BCS[bc], cfl=0.5), start, grid.dx), rel=1e-14)
        Uo, _, _ = O6.step(O6.params(bc=BCS[bc], dt_fixed=dt, characteristic=char), start, grid.dx, 1)
        e = rel_err(grid.interior(Ud), Uo)
        assert e <= TOL, (k, e)


@pytest.mark.parametrize("char", [False, True], ids=["cons", "char"])
def test_titarev_toro_fixed_ends(S, char):
    # the paper's inflow / fixed-profile ends: faces at the start and eight
    # shadowed steps
    _say("geno6 titarev-toro char=%d" % char)
    U, ghost = inputs.titarev_toro_noncompact(1000)
    grid = S.Grid6(1000, -5.0, 5.0, bc=S.BC_FIXED, ghost=ghost, variables=int(char))
    prm = dict(bc=O6.FIXED, ghost=ghost, characteristic=char)
    g = gpu_faces(S, grid, U)
    o = O6.faces(O6.params(**prm), U)
    for a, b in zip(g[:3], o[:3]):
        assert rel_err(a, b) <= TOL
    Ud = grid.to_device(U)
    ws = grid.workspace()
    dts = torch.zeros(1, dtype=torch.float64, device="cuda")
    for k in range(8):
        start = grid.interior(Ud)
        S.step(grid, Ud, ws, 1, dt_out=dts)
        torch.cuda.synchronize()
        Uo, _, _ = O6.step(O6.params(dt_fixed=float(dts.item()), **prm), start, grid.dx, 1)
        assert rel_err(grid.interior(Ud), Uo) <= TOL, k


def test_guard_counts(S):
    n = 40
    U = state("cold", n)
    grid = S.Grid6(n, 0.0, 1.0, dt_fixed=1e-4)
    Ud = grid.to_device(U)
    st = S.step(grid, Ud, grid.workspace(), 1, stats=True)
    Uo, _, go = O6.step(O6.params(dt_fixed=1e-4), U, grid.dx, 1)
    assert go > 0 and st.guard == go
    assert rel_err(grid.interior(Ud), Uo) <= TOL_COLD


def test_zero_steps_and_constant_state(S):
    n = 77
    U = np.repeat(np.array([[0.7], [0.21], [2.1]]), n, axis=1)
    grid = S.Grid6(n, bc=(1, 2))
    Ud = grid.to_device(U)
    ws = grid.workspace()
    S.step(grid, Ud, ws, 0)
    torch.cuda.synchronize()
    assert np.array_equal(grid.interior(Ud), U)
    grid = S.Grid6(n, bc=1)
    Ud = grid.to_device(U)
    st = S.step(grid, Ud, ws, 5, stats=True)
    assert st.guard == 0 and st.nonfinite == 0
    assert np.abs(grid.interior(Ud) - U).max() <= 1e-14 * 2.1


def test_periodic_conservation(S):
    n = 4096
    U = inputs.shocks_noncompact(n, seed=8, cells_per_segment=512)
    grid = S.Grid6(n)
    Ud = grid.to_device(U)
    S.step(grid, Ud, grid.workspace(), 50)
    torch.cuda.synchronize()
    V = grid.interior(Ud)
    assert np.all(np.isfinite(V))
    for f in range(3):
        assert abs(V[f].sum() - U[f].sum()) <= 1e-12 * np.abs(U[f]).sum()


def test_nonphysical_state_is_reported(S):
    n = 64
    U = inputs.smooth_noncompact(n, seed=1)
    U[2, 10] = -1.0   # negative energy: p < 0 in the initial state
    grid = S.Grid6(n, dt_fixed=1e-6)
    Ud = grid.to_device(U)
    from paper_2507_20461_amd import geno_gks as G
    with pytest.raises(G.GenoError) as e:
        S.step(grid, Ud, grid.workspace(), 1, stats=True)
    assert e.value.code == G.GENO_ENONPHYS


def test_timing_hooks(S):
    n = 5000
    grid = S.Grid6(n)
    Ud = grid.to_device(inputs.smooth_noncompact(n, 2))
    S.timing_enable(64)
    S.step(grid, Ud, grid.workspace(), 3)
    t = S.timing_read()
    S.timing_enable(0)
    assert t["stage"][1] == 12 and t["dt"][1] == 3 and t["init"][1] == 1
    assert t["stage"][0] > 0.0


# Full size of the benchmark workload (2^24 cells, the launch configuration
# it times) with a ragged tail: sampled faces against the oracle on their
# six-cell stencils, and sampled cells of one step against the oracle on a
# window of 41 cells around them (one step reaches 12 cells: four stages of
# three), with the GPU's dt.
FULL_N = 1 << 24


@pytest.mark.parametrize("n", [FULL_N, FULL_N - 77])
def test_full_size_sampled(S, n):
    _say("geno6 full size n=%d" % n)
    U = inputs.shocks_noncompact(n, seed=21)
    grid = S.Grid6(n, 0.0, 1.0, bc=(1, 1))
    Ud = grid.to_device(U)
    nf = n + 1
    UL, UR, F = (torch.zeros(3, nf, dtype=torch.float64, device="cuda") for _ in range(3))
    S.faces(grid, Ud, UL, UR, F, None)
    torch.cuda.synchronize()
    rng = np.random.default_rng(n)
    faces = np.concatenate([[3, 4, n - 3, n - 4], rng.integers(3, n - 3, 200)])
    gUL, gUR, gF = (t.cpu().numpy() for t in (UL, UR, F))
    prm = O6.params(bc=(1, 1))
    for s in faces:
        w = U[:, s - 3:s + 3]
        oUL, oUR, oF, _, _ = O6.faces(prm, w)
        for a, b in ((gUL[:, s], oUL[:, 3]), (gUR[:, s], oUR[:, 3]), (gF[:, s], oF[:, 3])):
            sc = np.maximum(np.abs(b), np.abs(w).max(axis=1))
            assert np.all(np.abs(a - b) <= TOL * sc), s
    # one step
    dts = torch.zeros(1, dtype=torch.float64, device="cuda")
    S.step(grid, Ud, grid.workspace(), 1, dt_out=dts)
    torch.cuda.synchronize()
    dt = float(dts.item())
    V = Ud[:, :n]
    cells = np.concatenate([[20, n - 21], rng.integers(20, n - 20, 40)])
    got = V[:, torch.as_tensor(cells, device="cuda")].cpu().numpy()
    prm = O6.params(bc=(1, 1), dt_fixed=dt)
    for q, c in enumerate(cells):
        w = U[:, c - 20:c + 21]
        Wo, _, _ = O6.step(prm, w, grid.dx, 1)
        sc = np.maximum(np.abs(Wo[:, 20]), np.abs(w).max(axis=1))
        assert np.all(np.abs(got[:, q] - Wo[:, 20]) <= TOL * sc), c
    # the CFL dt of the whole state
    assert dt == pytest.approx(O6.cfl_dt(O6.params(), U, grid.dx), rel=1e-14)


@pytest.mark.parametrize("n", [3, 200, 511, 1023, 1024, 1800, 2047])
@pytest.mark.parametrize("char", [False, True], ids=["cons", "char"])
def test_batch_equals_single_grid_steps(S, n, char):
    # one launch for several grids: each grid bit for bit as geno6_step on it
    _say("geno6 batch n=%d char=%d" % (n, char))
    ngr, steps = 5, 7
    bcs = [(1, 1), (0, 0), (2, 2), (1, 2), (0, 0)]
    for bc in bcs[:2] if n < 6 else bcs:
        grid = S.Grid6(n, 0.0, 1.0, bc=bc, variables=int(char))
        states = [inputs.shocks_noncompact(n, seed, cells_per_segment=max(4, n // 3)) for seed in range(ngr)]
        Ub = torch.stack([grid.to_device(U) for U in states])
        dtb = torch.zeros(ngr, steps, dtype=torch.float64, device="cuda")
        st = S.step_batch(grid, Ub, S.batch_workspace(grid, ngr), steps, dt_out=dtb, stats=True)
        assert st.nonfinite == 0
        ws = grid.workspace()
        guard = 0
        for gi, U in enumerate(states):
            Ud = grid.to_device(U)
            dts = torch.zeros(steps, dtype=torch.float64, device="cuda")
            guard += S.step(grid, Ud, ws, steps, dt_out=dts, stats=True).guard
            assert torch.equal(Ub[gi], Ud), (bc, gi)
            assert torch.equal(dtb[gi], dts), (bc, gi)
        assert st.guard == guard


def test_batch_reports_nonphysical_states(S):
    n = 64
    U = inputs.smooth_noncompact(n, seed=1)
    U[2, 10] = -1.0
    grid = S.Grid6(n, dt_fixed=1e-6)
    Ub = torch.stack([grid.to_device(U), grid.to_device(inputs.smooth_noncompact(n, seed=2))])
    from paper_2507_20461_amd import geno_gks as G
    with pytest.raises(G.GenoError) as e:
        S.step_batch(grid, Ub, S.batch_workspace(grid, 2), 1, stats=True)
    assert e.value.code == G.GENO_ENONPHYS


def test_batch_fixed_ends_and_zero_steps(S):
    # Titarev-Toro states with fixed ends in a batch of 3 (the ghost states
    # are part of the shared grid description), and a call of zero steps
    U, ghost = inputs.titarev_toro_noncompact(1000)
    grid = S.Grid6(1000, -5.0, 5.0, bc=S.BC_FIXED, ghost=ghost)
    states = [U, U * np.array([[1.01], [1.0], [1.02]]), U]
    Ub = torch.stack([grid.to_device(x) for x in states])
    ws = S.batch_workspace(grid, 3)
    before = Ub.clone()
    S.step_batch(grid, Ub, ws, 0)
    torch.cuda.synchronize()
    assert torch.equal(Ub, before)
    S.step_batch(grid, Ub, ws, 6)
    for gi, x in enumerate(states):
        Ud = grid.to_device(x)
        S.step(grid, Ud, grid.workspace(), 6)
        assert torch.equal(Ub[gi], Ud), gi
