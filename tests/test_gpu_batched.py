"""The batched form (gks_step_batched) through the C ABI: identical results to
gks_step on each grid alone, in eager and graph mode, for every work-group
shape, graphs kept across calls, and a working autotuner. (The persistent
mode is switched off; its tests are kept, skipped.)

The batched launches run the same per-cell arithmetic as the single-grid
launches (only the mapping of work-groups to grids differs, and the CFL
minimum does not depend on the order of its reduction), so the comparison is
bitwise.
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


# (nx, ny, bc, seed): uneven sizes, one periodic grid
SHAPES = [(32, 32, 1, 0), (48, 40, 1, 1), (64, 24, 0, 2), (20, 56, 1, 3), (72, 72, 1, 4)]


def _make(G, prec, variables=0, fuse=1):
    grids, data = [], []
    for nx, ny, bc, seed in SHAPES:
        W, dW, _ = inputs.quadrants_2d(nx, ny, seed)
        Ws, dWs = inputs.random_smooth_2d(nx, ny, seed + 5)
        W = W + 0.05 * (Ws - Ws.mean(axis=(1, 2), keepdims=True))
        dW = dW + 0.05 * dWs
        grids.append(G.Grid(2, nx, ny, bc=bc, precision=prec, variables=variables, fuse=fuse))
        data.append((W, dW))
    return grids, data


def _upload(grids, data):
    return ([g.to_device(W) for g, (W, _) in zip(grids, data)],
            [g.grad_to_device(dW) for g, (_, dW) in zip(grids, data)])


def _single(G, grids, data, nsteps):
    out = []
    for g, (W, dW) in zip(grids, data):
        Wd, dWd = g.to_device(W), g.grad_to_device(dW)
        st = G.gks_step(g, Wd, dWd, g.workspace(), nsteps, stats=True)
        assert st.nonfinite == 0
        out.append((g.interior(Wd), g.interior(dWd)))
    return out


def _same(grids, Ws, dWs, ref):
    for g, W, dW, (rW, rdW) in zip(grids, Ws, dWs, ref):
        if not (np.array_equal(g.interior(W), rW) and np.array_equal(g.interior(dW), rdW)):
            return False
    return True


@pytest.mark.parametrize("mixed,char,fuse", [(False, False, 2), (True, False, 2), (False, True, 2),
                                             (True, True, 2), (False, False, 0), (True, False, 0)],
                         ids=["fp64", "mixed", "fp64-char", "mixed-char", "fp64-two-launch",
                              "mixed-two-launch"])
def test_batched_equals_single_grid(G, mixed, char, fuse):
    # fuse 2: the fused face kernels; 0: normal step and faces in two launches
    prec = G.MIXED if mixed else G.F64
    grids, data = _make(G, prec, G.VARS_CHARACTERISTIC if char else G.VARS_CONSERVATIVE, fuse)
    ref = _single(G, grids, data, 4)
    B = G.Batch(grids)
    ws = B.workspace()
    for mode in (G.BATCH_EAGER, G.BATCH_GRAPH):
        Ws, dWs = _upload(grids, data)
        _say("batched (%s, mode %d) vs single grids" % ("mixed" if mixed else "fp64", mode))
        _, st = B.step(Ws, dWs, ws, 4, mode=mode, stats=True)
        assert st.nonfinite == 0
        assert _same(grids, Ws, dWs, ref)


def test_graph_replays_match_eager(G):
    # every replay count 1..4 of the captured step equals as many eager steps;
    # eager work and synchronisations of the program run between the calls
    grids, data = _make(G, G.MIXED)
    B = G.Batch(grids)
    ws = B.workspace()
    scratch = torch.randn(1 << 20, device="cuda")
    for n in range(1, 5):
        Ws, dWs = _upload(grids, data)
        B.step(Ws, dWs, ws, n, graph=False)
        ref = [(g.interior(W), g.interior(dW)) for g, W, dW in zip(grids, Ws, dWs)]
        scratch.mul_(1.0001).add_(0.5)
        torch.cuda.synchronize()
        Ws, dWs = _upload(grids, data)
        ms, _ = B.step(Ws, dWs, ws, n, graph=True, step_times=True)
        assert len(ms) == n and np.all(ms > 0)
        assert _same(grids, Ws, dWs, ref), n


PERSISTENT_OFF = ("the persistent batched launch did not finish on the device in its test run and "
                  "in the run after a fix; the mode is switched off (GENO_EINVAL) until a cause is shown")


def test_persistent_mode_is_refused(G):
    grids, data = _make(G, G.F64)
    B = G.Batch(grids)
    Ws, dWs = _upload(grids, data)
    before = [W.clone() for W in Ws]
    with pytest.raises(G.GenoError):
        B.step(Ws, dWs, B.workspace(), 1, mode=G.BATCH_PERSISTENT)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(Ws, before))


def test_graph_is_kept_across_calls(G):
    # the calls after the first (same batch, workspace and constants) replay
    # the graph the first one captured; each still equals the eager steps
    grids, data = _make(G, G.MIXED)
    B = G.Batch(grids)
    ws = B.workspace()
    built = None
    for n in (2, 1, 3):
        Ws, dWs = _upload(grids, data)
        B.step(Ws, dWs, ws, n, mode=G.BATCH_EAGER)
        ref = [(g.interior(W), g.interior(dW)) for g, W, dW in zip(grids, Ws, dWs)]
        Ws, dWs = _upload(grids, data)
        B.step(Ws, dWs, ws, n, mode=G.BATCH_GRAPH)
        assert _same(grids, Ws, dWs, ref), n
        if built is None:
            built = G.batched_graphs_built()
        else:
            assert G.batched_graphs_built() == built, n


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_persistent_replays_match_eager_and_reuse_one_graph(G):
    # the persistent step's graph: every replay count 1..4 equals as many
    # eager steps, with eager work of the program between the calls, and the
    # calls after the first reuse the graph kept by the first
    grids, data = _make(G, G.F64)
    B = G.Batch(grids)
    ws = B.workspace()
    scratch = torch.randn(1 << 20, device="cuda")
    built = None
    for n in range(1, 5):
        _say("persistent replays", n)
        Ws, dWs = _upload(grids, data)
        B.step(Ws, dWs, ws, n, mode=G.BATCH_EAGER)
        ref = [(g.interior(W), g.interior(dW)) for g, W, dW in zip(grids, Ws, dWs)]
        scratch.mul_(1.0001).add_(0.5)
        torch.cuda.synchronize()
        Ws, dWs = _upload(grids, data)
        ms, _ = B.step(Ws, dWs, ws, n, mode=G.BATCH_PERSISTENT, step_times=True)
        assert len(ms) == n and np.all(ms > 0)
        assert _same(grids, Ws, dWs, ref), n
        if built is None:
            built = G.batched_graphs_built()
        else:
            assert G.batched_graphs_built() == built, n


@pytest.mark.skip(reason=PERSISTENT_OFF)
def test_persistent_many_small_grids(G):
    # 40 grids of 8..40 cells a side (many work items per phase, grids
    # finishing their phases at different times) equal gks_step per grid
    rng = np.random.default_rng(11)
    grids, data = [], []
    for i in range(40):
        nx, ny = (int(x) for x in rng.integers(8, 41, size=2))
        W, dW, _ = inputs.quadrants_2d(nx, ny, 100 + i)
        grids.append(G.Grid(2, nx, ny, bc=int(i % 2)))
        data.append((W, dW))
    ref = _single(G, grids, data, 3)
    B = G.Batch(grids)
    Ws, dWs = _upload(grids, data)
    _say("persistent, 40 small grids")
    B.step(Ws, dWs, B.workspace(), 3, mode=G.BATCH_PERSISTENT)
    assert _same(grids, Ws, dWs, ref)


def test_every_work_group_shape_gives_the_same_result(G):
    grids, data = _make(G, G.MIXED)
    B = G.Batch(grids)
    ws = B.workspace()
    ref = None
    for bs, fpb in ((128, 512), (256, 2048), (512, 8192), (512, 64)):
        t = G.default_tuning()
        t.block_normal = t.block_faces = t.block_slow = t.block_update = bs
        t.slow_faces_per_block = fpb
        Ws, dWs = _upload(grids, data)
        B.step(Ws, dWs, ws, 3, tuning=t, graph=True)
        got = [(g.interior(W), g.interior(dW)) for g, W, dW in zip(grids, Ws, dWs)]
        if ref is None:
            ref = got
        else:
            assert all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) for a, b in zip(got, ref)), bs


def test_autotune_gives_a_valid_tuning(G):
    grids, data = _make(G, G.MIXED)
    B = G.Batch(grids)
    ws = B.workspace()
    Ws, dWs = _upload(grids, data)
    t = B.autotune(Ws, dWs, ws, trial_steps=2)
    _say("autotuned:", t.as_dict())
    assert t.block_normal in (128, 256, 512) and t.block_faces in (128, 256, 512)
    assert t.block_slow in (128, 256, 512) and t.block_update in (128, 256, 512)
    assert t.slow_faces_per_block in (512, 2048, 8192)
    ref = _single(G, grids, data, 2)
    Ws, dWs = _upload(grids, data)
    B.step(Ws, dWs, ws, 2, tuning=t, graph=True)
    assert _same(grids, Ws, dWs, ref)


def test_batched_rejects_mismatched_parameters(G):
    a = G.Grid(2, 16, 16, bc=1)
    b = G.Grid(2, 16, 16, bc=1, cfl=0.4)
    B = G.Batch([a, b])
    with pytest.raises(G.GenoError):
        B.workspace()


def test_batched_grids_match_oracle(G):
    # each grid of an FP64 batch against the CPU oracle run alone: two steps
    # from the same state, per cell at 1e-12 of the value for density and
    # energy, of the field's scale for the momenta, and of the field's scale
    # over the cell size for the gradients (plus the path-function term of
    # the second-order part of the gradients, 1e-8 CFL^2/3, at the jumps)
    from oracle import oracle as O
    grids, data = _make(G, G.F64)
    B = G.Batch(grids)
    Ws, dWs = _upload(grids, data)
    _, st = B.step(Ws, dWs, B.workspace(), 2, graph=False, stats=True)
    assert st.nonfinite == 0
    for (nx, ny, bc, _), g, W, dW, (W0, dW0) in zip(SHAPES, grids, Ws, dWs, data):
        _say("batched grid %dx%d bc %d vs oracle" % (nx, ny, bc))
        oW, odW, _, _ = O.step(O.params(ndim=2, bc=bc), W0, dW0, 2, dx=g.dx, dy=g.dy)
        gW, gdW = g.interior(W), g.interior(dW)
        sc = np.abs(oW).reshape(4, -1).max(axis=1)
        den = np.abs(oW).reshape(4, -1).copy()
        den[1:3] = np.maximum(den[1:3], sc[1:3, None])
        assert (np.abs(gW - oW).reshape(4, -1) / den).max() < 1e-12
        gsc = np.concatenate([sc / g.dx, sc / g.dy])
        eg = (np.abs(gdW - odW).reshape(8, -1) / np.maximum(np.abs(odW).reshape(8, -1), gsc[:, None])).max()
        assert eg < 1e-12 + 1e-8 * 0.5 ** 2 / 3.0, eg
