"""The C-ABI library builds for gfx950, loads without a GPU and exports every
function that include/*.h declares (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M):
            names.append(m.group(1))
    return names


@pytest.fixture(scope="module")
def so():
    from paper_2507_20461_amd import build
    if build.stale():
        build.build()
    return ctypes.CDLL(build.LIB)


def test_header_declares_the_boundary():
    names = set(_declared())
    for n in ("geno_reconstruct", "gks_flux", "gks_step", "gks_workspace_bytes", "geno_grid_init"):
        assert n in names


def test_library_exports_every_declared_symbol(so):
    missing = [n for n in _declared() if not hasattr(so, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2507_20461_amd import geno6, geno_gks, geno_tri
    assert set(geno_gks.EXPORTS) | set(geno6.EXPORTS) | set(geno_tri.EXPORTS) == set(_declared())
    assert not set(geno_gks.EXPORTS) & set(geno6.EXPORTS)
    assert not (set(geno_gks.EXPORTS) | set(geno6.EXPORTS)) & set(geno_tri.EXPORTS)


def test_host_side_validation(so):
    # host-only entry points: parameter and grid validation, sizes
    from paper_2507_20461_amd import geno_gks as G
    G._lib = None
    p = G.default_params()
    assert p.C == 20.0 and p.eps == 1e-15 and list(p.d) == [1.0, 8.0, 1.0]
    g = G.Grid(2, 64, 48)
    assert g.pitch % 16 == 0 and g.pitch >= 68 and g.rows == 52
    assert G.lib().gks_workspace_bytes(ctypes.byref(g.g)) > 0
    with pytest.raises(G.GenoError):
        G.Grid(2, 0, 4)
    with pytest.raises(G.GenoError):
        G.Grid(1, 16, params=G.default_params(r=3.0))
    bad = G.default_params()
    bad.version = 99
    with pytest.raises(G.GenoError) as e:
        G.Grid(1, 16, params=bad)
    assert e.value.code == G.GENO_EVERSION
    with pytest.raises(G.GenoError):
        G.Grid(2, 8, 8, params=G.default_params(bc=(0, 1, 1, 1)))
    # fixed-state ends: 1-D only
    G.Grid(1, 16, params=G.default_params(bc=(3, 3, 0, 0)))
    with pytest.raises(G.GenoError):
        G.Grid(2, 8, 8, params=G.default_params(bc=(3, 3, 1, 1)))
    # characteristic variables in both dimensions, not with the learned gate
    G.Grid(2, 8, 8, params=G.default_params(variables=G.VARS_CHARACTERISTIC))
    with pytest.raises(G.GenoError):
        G.Grid(2, 8, 8, params=G.default_params(variables=G.VARS_CHARACTERISTIC, gate_delta=0.1))
    with pytest.raises(G.GenoError):
        G.Grid(1, 16, params=G.default_params(variables=7))
    # the fused face kernels: automatic by default; 0 never, 2 always
    assert p.fuse == 1
    G.Grid(2, 8, 8, fuse=0)
    G.Grid(2, 8, 8, fuse=2)
    with pytest.raises(G.GenoError):
        G.Grid(2, 8, 8, fuse=3)
    # null pointers are rejected before any launch
    assert G.lib().gks_step(ctypes.byref(g.g), None, None, None, 1, None, None, None) == G.GENO_EINVAL
    assert G.lib().geno_reconstruct(ctypes.byref(g.g), None, None, 0, None, None, None, None) == G.GENO_EINVAL


def test_batched_host_side_validation(so):
    from paper_2507_20461_amd import geno_gks as G
    t = G.default_tuning()
    assert (t.block_normal, t.block_faces, t.block_slow, t.block_update, t.slow_faces_per_block) == (256, 256, 256, 256, 2048)
    a, b = G.Grid(2, 32, 24, bc=1), G.Grid(2, 40, 16, bc=0)
    B = G.Batch([a, b])
    single = sum(G.lib().gks_workspace_bytes(ctypes.byref(g.g)) for g in (a, b))
    assert G.lib().gks_batched_workspace_bytes(2, B.garr) >= single
    # mismatched method parameters, 1-D grids and empty batches are rejected
    for bad in ([a, G.Grid(2, 8, 8, cfl=0.3)], [G.Grid(1, 16)]):
        assert G.lib().gks_batched_workspace_bytes(len(bad), G.Batch(bad).garr) == 0
    assert G.lib().gks_batched_workspace_bytes(0, B.garr) == 0
    # null pointers and graph mode on the NULL stream fail before any launch
    assert G.lib().gks_step_batched(2, B.garr, None, None, None, 1, None, 0, None, None, None) == G.GENO_EINVAL
    assert G.lib().gks_step_batched(2, B.garr, None, None, None, 1, None, 1, None, None, None) == G.GENO_EINVAL
    bad_t = G.default_tuning()
    bad_t.block_faces = 96
    vp = (ctypes.c_void_p * 2)(1, 1)
    assert G.lib().gks_step_batched(2, B.garr, vp, vp, ctypes.c_void_p(1), 1, ctypes.byref(bad_t), 0, None, None,
                                    None) == G.GENO_EINVAL


def test_noncompact_host_side_validation(so):
    from paper_2507_20461_amd import geno6 as S
    from paper_2507_20461_amd import geno_gks as G
    p = S.default_params()
    assert (p.C, p.eps, list(p.d), p.cfl, list(p.bc), p.variables) == (20.0, 1e-15, [1.0, 8.0, 1.0, 1.0], 0.5,
                                                                      [0, 0], S.VARS_CONSERVATIVE)
    g = S.Grid6(1000, 0.0, 2.0)
    assert g.pitch == 1024 and g.dx == pytest.approx(0.002)
    # control block, 1024 maxima slots and three stage arrays
    assert S.lib().geno6_workspace_bytes(ctypes.byref(g.g)) >= 3 * 3 * 1024 * 8 + 1024 * 8
    for kw in ({"n": 2}, {"n": 8, "x0": 1.0, "x1": 1.0}):
        with pytest.raises(G.GenoError):
            S.Grid6(**kw)
    S.Grid6(16, bc=(S.BC_FIXED, 1))   # fixed-state ends are a boundary kind of this path
    for bad in ({"bc": (0, 1)}, {"d": (1, 8, 0, 1)}, {"cfl": 0.0}, {"bc": (4, 4)}, {"dt_fixed": -1.0},
                {"variables": 2}):
        with pytest.raises(G.GenoError):
            S.Grid6(16, params=S.default_params(**bad))
    v = S.default_params()
    v.version = 7
    with pytest.raises(G.GenoError) as e:
        S.Grid6(16, params=v)
    assert e.value.code == G.GENO_EVERSION
    # null pointers are rejected before any launch
    assert S.lib().geno6_step(ctypes.byref(g.g), None, None, 1, None, None, None) == G.GENO_EINVAL
    assert S.lib().geno6_rhs(ctypes.byref(g.g), None, None, None) == G.GENO_EINVAL
    assert S.lib().geno6_faces(ctypes.byref(g.g), None, None, None, None, None, None) == G.GENO_EINVAL
    assert S.lib().geno6_batch_workspace_bytes(ctypes.byref(g.g), 4) >= 4 * 3 * 3 * 1024 * 8
    assert S.lib().geno6_batch_workspace_bytes(ctypes.byref(g.g), 0) == 0
    assert S.lib().geno6_step_batch(ctypes.byref(g.g), 0, None, None, 1, None, None, None) == G.GENO_EINVAL
    assert S.lib().geno6_step_batch(ctypes.byref(g.g), 2, None, None, 1, None, None, None) == G.GENO_EINVAL


def test_noncompact_op_costs(so):
    from paper_2507_20461_amd import geno6 as S
    c = S.op_costs()
    # a face: two sides of three variables plus HLLC; a low-order side adds
    # the exponential of chi, the weights and the blend
    assert 300 < c["face"] < 1500 and 10 < c["low_side"] < 100 and c["cell"] == 23.0


def test_triangle_table_host_side(so):
    # the mesh layer runs on the host: the table of a small mesh reproduces a
    # cubic through its least-squares operator, and bad meshes are rejected
    import math
    import numpy as np
    from paper_2507_20461_amd import geno_tri as T
    from paper_2507_20461_amd import inputs
    nt = T.lib().geno_tri_table_doubles()
    assert nt == 226
    mesh = inputs.tri_mesh(8, 8, 3)
    n = 2 * 8 * 8
    flat = T.build_table(mesh)
    # entries are stored in pairs: entry e of cell c at ((e // 2) n + c) 2 + e % 2
    ops = np.stack([flat[((e // 2) * n + np.arange(n)) * 2 + e % 2] for e in range(nt)])
    rng = np.random.default_rng(4)
    co = rng.normal(size=10)
    ex = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]
    f = lambda x, y: sum(c * x ** a * y ** b for c, (a, b) in zip(co, ex))
    g = lambda x, y: (sum(c * a * x ** max(a - 1, 0) * y ** b for c, (a, b) in zip(co, ex)),
                      sum(c * b * x ** a * y ** max(b - 1, 0) for c, (a, b) in zip(co, ex)))
    W, dW = inputs.tri_cell_data(mesh, f, g)
    c = 2 * (4 * 8 + 4)            # a cell whose stencil stays inside the square
    idx = ops[0:9, c].astype(int)
    h = ops[9, c]
    d = np.concatenate([W[0, idx] - W[0, c], h * dW[:, 0, c], (h * dW[:, 0, idx[:3]]).T.ravel()])
    a = ops[10:10 + 170, c].reshape(17, 10)[:, :9].T @ d
    xc = mesh["xv"][c].mean(axis=0)
    # the cell's monomial means (the kernel forms them), by the rule with
    # vertex, edge-midpoint and centroid weights 1/20, 2/15, 9/20 (exact for cubics)
    tri = (mesh["xv"][c] - xc) / h
    pts = [tri[0], tri[1], tri[2], (tri[0] + tri[1]) / 2, (tri[1] + tri[2]) / 2, (tri[2] + tri[0]) / 2,
           tri.mean(axis=0)]
    wts = [1 / 20] * 3 + [2 / 15] * 3 + [9 / 20]
    mono = lambda X, Y: np.array([X, Y, X * X, X * Y, Y * Y, X ** 3, X * X * Y, X * Y * Y, Y ** 3])
    mean = sum(w * mono(*p) for w, p in zip(wts, pts))
    for e in range(3):
        p, q = mesh["xv"][c][e], mesh["xv"][c][(e + 1) % 3]
        for t in (0.5 - 0.5 / math.sqrt(3), 0.5 + 0.5 / math.sqrt(3)):
            X, Y = (p + t * (q - p) - xc) / h
            ph = [X, Y, X * X, X * Y, Y * Y, X ** 3, X * X * Y, X * Y * Y, Y ** 3]
            val = W[0, c] + sum(a[k] * (ph[k] - mean[k]) for k in range(9))
            x, y = p + t * (q - p)
            assert abs(val - f(x, y)) < 1e-11
    # the list of owned edges: every owned (cell, edge) pair once, edge-major
    # then by cell, 3n/2 of them on this periodic mesh, the rest -1
    lst = np.concatenate([ops[nt - 2], ops[nt - 1]])
    used = lst[lst >= 0].astype(int)
    # ownership flags of the per-edge blocks (6 entries per edge, before the list)
    own_flags = np.stack([ops[nt - 2 - 18 + 6 * e + 5] for e in range(3)])   # [edge][cell]
    want = [3 * cc + e for e in range(3) for cc in range(n) if own_flags[e, cc] != 0.0]
    assert list(used) == want and len(want) == 3 * n // 2
    assert np.all(lst[len(want):] == -1.0)
    bad = dict(mesh)
    bad["nbr"] = mesh["nbr"].copy()
    bad["nbr"][3, 1] = 10 ** 6
    from paper_2507_20461_amd import geno_gks as G
    with pytest.raises(G.GenoError):
        T.build_table(bad)
    flip = dict(mesh)
    flip["xv"] = mesh["xv"][:, ::-1].copy()
    with pytest.raises(G.GenoError):
        T.build_table(flip)


def test_triangle_table_geometry_matches_the_oracle(so):
    # the step's geometry entries (area, 4 area / perimeter, per edge the
    # outward normal, length, neighbour, the neighbour's edge index, owner)
    # equal the oracle's own computation of them
    import numpy as np
    from oracle import gks_tri
    from paper_2507_20461_amd import geno_tri as T
    from paper_2507_20461_amd import inputs
    mesh = inputs.tri_mesh(6, 5, 2)
    n = 60
    nt = T.lib().geno_tri_table_doubles()
    flat = T.build_table(mesh)
    ops = np.stack([flat[((e // 2) * n + np.arange(n)) * 2 + e % 2] for e in range(nt)])
    geo = gks_tri.geometry(mesh)
    g0 = nt - 22   # area, d, 3 x 6 per-edge entries, then the 2 slots of the owned-edge list
    np.testing.assert_allclose(ops[g0], geo["area"], rtol=1e-14)
    np.testing.assert_allclose(ops[g0 + 1], geo["d"], rtol=1e-14)
    for e in range(3):
        b = g0 + 2 + 6 * e
        np.testing.assert_allclose(ops[b:b + 2].T, geo["normal"][:, e], rtol=0, atol=1e-15)
        np.testing.assert_allclose(ops[b + 2], geo["length"][:, e], rtol=1e-14)
        assert np.array_equal(ops[b + 3].astype(int), geo["nbr"][:, e])
        assert np.array_equal(ops[b + 4].astype(int), geo["rev"][:, e])
        assert np.array_equal(ops[b + 5] != 0.0, geo["owner"][:, e])


def test_triangle_reconstruct_rejects_bad_arguments(so):
    # argument checks happen on the host, before any launch
    from paper_2507_20461_amd import geno_gks as G
    from paper_2507_20461_amd import geno_tri as T
    L = T.lib()
    fake = 256   # never dereferenced: every call below fails its checks first
    assert L.geno_tri_reconstruct(10, 5, fake, fake, fake, fake, None, None, None) == G.GENO_EINVAL
    assert L.geno_tri_reconstruct(10, 0, fake, fake, fake, fake, None, None, None) == G.GENO_EINVAL
    assert L.geno_tri_reconstruct(0, 4, fake, fake, fake, fake, None, None, None) == G.GENO_EINVAL
    assert L.geno_tri_reconstruct(10, 4, None, fake, fake, fake, None, None, None) == G.GENO_EINVAL
    assert L.geno_tri_reconstruct(10, 4, fake, fake, fake, None, None, None, None) == G.GENO_EINVAL
    assert L.geno_tri_build(0, None, None, None, None) == G.GENO_EINVAL
    # the step: host-side checks of its arguments and parameters
    p = G.geno_params()
    assert L.geno_tri_step(0, fake, fake, fake, fake, 1, ctypes.byref(p), None, None, None) == G.GENO_EINVAL
    assert L.geno_tri_step(10, fake, fake, fake, fake, 1, None, None, None, None) == G.GENO_EINVAL
    assert L.geno_tri_step(10, fake, fake, fake, fake, 1, ctypes.byref(p), None, None, None) == G.GENO_EVERSION
    G.lib().geno_params_default(ctypes.byref(p))
    assert L.geno_tri_step(10, fake, fake, fake, fake, -1, ctypes.byref(p), None, None, None) == G.GENO_EINVAL
    p.cfl = 0.0
    assert L.geno_tri_step(10, fake, fake, fake, fake, 1, ctypes.byref(p), None, None, None) == G.GENO_EINVAL
    assert L.geno_tri_workspace_bytes(0) == 0 and L.geno_tri_workspace_bytes(100) > 0
