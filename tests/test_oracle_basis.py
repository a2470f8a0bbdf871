"""Pins of the oracle's LGL basis and mesh/geometry against closed forms."""
import numpy as np
import pytest

import workloads as W
from oracle import dg, geometry, lgl, mesh


@pytest.mark.parametrize("n,nodes,weights", [
    (2, [-1, 1], [1, 1]),
    (3, [-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
    (4, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    (5, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
])
def test_lgl_closed_forms(n, nodes, weights):
    x, w = lgl.nodes_weights(n)
    np.testing.assert_allclose(x, nodes, atol=1e-15)
    np.testing.assert_allclose(w, weights, rtol=1e-14)


@pytest.mark.parametrize("n", range(2, 10))
def test_lgl_quadrature_exactness(n):
    x, w = lgl.nodes_weights(n)
    assert abs(w.sum() - 2.0) < 1e-14
    for deg in range(0, 2 * n - 2):  # exact to degree 2n - 3
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.dot(w, x ** deg) - exact) < 1e-13, deg
    # and not exact at degree 2n - 2
    deg = 2 * n - 2
    assert abs(np.dot(w, x ** deg) - 2.0 / (deg + 1)) > 1e-6


@pytest.mark.parametrize("n", range(2, 10))
def test_differentiation_exact_on_polynomials(n):
    x, _ = lgl.nodes_weights(n)
    D = lgl.diff_matrix(x)
    for deg in range(n):
        np.testing.assert_allclose(D @ x ** deg, deg * x ** max(deg - 1, 0) if deg else 0 * x,
                                   atol=1e-11 * max(1, deg))
    # summation by parts: W D + D^T W = diag(-1, 0, ..., 0, 1)
    _, w = lgl.nodes_weights(n)
    B = np.diag(w) @ D + D.T @ np.diag(w)
    Bex = np.zeros((n, n))
    Bex[0, 0], Bex[-1, -1] = -1, 1
    np.testing.assert_allclose(B, Bex, atol=1e-13)


def test_interpolation_reproduces_polynomials():
    x, _ = lgl.nodes_weights(6)
    y = np.linspace(-1, 1, 13)
    I = lgl.interp_matrix(x, y)
    for deg in range(6):
        np.testing.assert_allclose(I @ x ** deg, y ** deg, atol=1e-13)


def test_cylinder_mesh_faces_and_volume():
    spec = W.config1()
    P = dg.Problem(spec)
    m, g = P.mesh, P.geo
    assert P.E == 40
    interior = (m.nbr >= 0).sum()
    assert interior == 2 * 92
    assert (m.bc == W.BC_PRESSURE).sum() == 20
    assert (m.bc == W.BC_DIRICHLET).sum() == 20
    assert (m.bc == W.BC_FREE).sum() == 16
    assert np.all(g.det > 0)
    # matched nodes coincide and normals are opposite
    N = m.N
    for e in range(P.E):
        for f in range(6):
            nb = m.nbr[e, f]
            if nb < 0:
                continue
            fb = m.nbr_face[e, f]
            for d in range(3):
                a = mesh.get_face(m.xyz[e, d], f, N)
                b = mesh.get_face(m.xyz[nb, d], fb, N)[m.perm[e, f]]
                assert np.abs(a - b).max() < 1e-14
            np.testing.assert_allclose(g.normal[e, f], -g.normal[nb, fb][:, m.perm[e, f]], atol=1e-12)
            np.testing.assert_allclose(g.jsig[e, f], g.jsig[nb, fb][m.perm[e, f]], rtol=1e-12)
    # volume converges to pi R^2 H with p (isoparametric geometry)
    errs = []
    for p in (2, 4, 6):
        Pp = dg.Problem(dict(spec, p=p))
        vol = np.sum(Pp.geo.w3[None] * Pp.geo.det)
        errs.append(abs(vol - np.pi))
    assert errs[2] < 1e-6 and errs[1] < errs[0] and errs[2] < errs[1] / 10


def test_box_geometry_is_exact():
    spec = W.box(nx=3, ny=2, Lx=1.5, Ly=0.8, p=3,
                 layers=[{"thickness": 0.3, "n_elem": 2, "ratio": 2.0, "material": 0}])
    P = dg.Problem(spec)
    g = P.geo
    # element widths: x 0.5, y 0.4, z 0.1 and 0.2
    np.testing.assert_allclose(g.h[:, 0], 0.5, rtol=1e-13)
    np.testing.assert_allclose(g.h[:, 2], 0.4, rtol=1e-13)
    hz = np.where(np.arange(P.E) < 6, 0.1, 0.2)
    np.testing.assert_allclose(g.h[:, 4], hz[:, None] * np.ones((1, 16)), rtol=1e-13)
    np.testing.assert_allclose(np.sum(g.w3[None] * g.det), 1.5 * 0.8 * 0.3, rtol=1e-14)
    np.testing.assert_allclose(g.normal[:, 5, 2], 1.0)
    np.testing.assert_allclose(g.normal[:, 0, 0], -1.0)
