"""The seeded triangle meshes and their data (host only): counter-clockwise
cells, every edge shared by exactly one neighbour whose translated edge is
the same segment reversed, and cell data that are exact averages of
polynomial fields."""
import numpy as np
import pytest

from paper_2507_20461_amd import inputs


@pytest.mark.parametrize("nx,ny,jitter", [(2, 2, 0.0), (5, 4, 0.2), (9, 7, 0.3)])
def test_mesh_connectivity(nx, ny, jitter):
    m = inputs.tri_mesh(nx, ny, 3, jitter=jitter)
    xv, nbr, sh = m["xv"], m["nbr"], m["shift"]
    n = 2 * nx * ny
    assert xv.shape == (n, 3, 2) and nbr.shape == (n, 3)
    total = 0.0
    for c in range(n):
        a = xv[c]
        area = 0.5 * ((a[1, 0] - a[0, 0]) * (a[2, 1] - a[0, 1]) - (a[2, 0] - a[0, 0]) * (a[1, 1] - a[0, 1]))
        assert area > 0
        total += area
        for e in range(3):
            p, q = a[e], a[(e + 1) % 3]
            d = nbr[c, e]
            t = xv[d] + sh[c, e]
            hits = [f for f in range(3) if np.allclose(t[f], q) and np.allclose(t[(f + 1) % 3], p)]
            assert len(hits) == 1
            # the neighbour sees c across that edge, with the opposite translation
            f = hits[0]
            assert nbr[d, f] == c and np.allclose(sh[d, f], -sh[c, e])
    assert total == pytest.approx(1.0, rel=1e-12)     # the cells tile the unit square


def test_cell_data_exact_for_polynomials():
    m = inputs.tri_mesh(4, 3, 1)

    def f(x, y):
        return 1.0 + 2.0 * x - y + 3.0 * x * x * y - y ** 4

    def g(x, y):
        return 2.0 + 6.0 * x * y, -1.0 + 3.0 * x * x - 4.0 * y ** 3

    W, dW = inputs.tri_cell_data(m, f, g)
    # the averaged gradient equals the boundary integral of f n over |Omega|
    # (Gauss theorem), by a 5-point Gauss rule on each edge (exact here)
    gx, gw = np.polynomial.legendre.leggauss(5)
    for c in range(W.shape[1]):
        a = m["xv"][c]
        area = 0.5 * ((a[1, 0] - a[0, 0]) * (a[2, 1] - a[0, 1]) - (a[2, 0] - a[0, 0]) * (a[1, 1] - a[0, 1]))
        flux = np.zeros(2)
        for e in range(3):
            p, q = a[e], a[(e + 1) % 3]
            nrm = np.array([q[1] - p[1], p[0] - q[0]])        # outward normal times the edge length
            for t, w in zip(0.5 * (gx + 1.0), 0.5 * gw):
                x, y = p + t * (q - p)
                flux += w * f(x, y) * nrm
        assert np.allclose(dW[:, 0, c], flux / area, rtol=1e-12, atol=1e-12)
