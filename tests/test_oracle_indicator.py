"""Pins of the oracle's face-jump indicator (oracle/indicator.py).

* A linear field on a layered box is continuous and exactly represented, so every
  interior jump vanishes and the indicator is the Dirichlet term alone:
  int over the fixed face z = H of |u|^2, a closed form (the LGL face rule
  integrates the quadratic exactly at p = 3).  A wrong face pairing or node
  permutation between neighbours leaves a non-zero jump of the linear field.
* A field constant in the top layer and zero below jumps by c across the one
  interface plane only: c^2 Lx Ly, split half and half between the two layers.
* On the curved cylinder the nodal values of any smooth function match on both
  sides of every face (shared face nodes), so the interior part is zero there too,
  and a constant field gives c^2 times the area of the fixed face, pi R^2 up to
  the geometric approximation of the circle.
* Weighted by the penalty sigma = C (p + 1)^2 / min(h, h'), the same steps give
  sigma times those integrals, with the widths of the box's elements.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dg, indicator


def layered_box(nx=2, ny=2, p=3):
    return W.box(nx=nx, ny=ny, Lx=1.2, Ly=0.8, p=p,
                 layers=[{"thickness": 0.1, "n_elem": 1, "ratio": 1.0, "material": 0},
                         {"thickness": 0.5, "n_elem": 2, "ratio": 1.0, "material": 0}])


def test_linear_field_has_only_the_dirichlet_term():
    spec = layered_box()
    P = dg.Problem(spec)
    x, y, z = (P.node_xyz()[:, d] for d in range(3))
    a = np.array([0.3, -1.1, 0.7])
    b = np.array([0.9, 0.2, -0.4])
    g = np.array([-0.5, 1.3, 0.8])
    d = np.array([0.25, -0.6, 1.5])
    u = np.stack([a[c] * x + b[c] * y + g[c] * z + d[c] for c in range(3)], axis=1)
    eta2 = indicator.jump_indicator(P, u)
    H = z.max()
    Lx, Ly = spec["Lx"], spec["Ly"]
    exact = sum(a[c] ** 2 * Lx ** 3 * Ly / 12 + b[c] ** 2 * Lx * Ly ** 3 / 12 + (g[c] * H + d[c]) ** 2 * Lx * Ly
                for c in range(3))
    assert eta2.sum() == pytest.approx(exact, rel=1e-13)
    # only the elements on the fixed face carry anything
    on_bottom = (P.mesh.bc == 1).any(axis=1)
    assert np.abs(eta2[~on_bottom]).max() < 1e-14 * exact
    assert np.all(eta2[on_bottom] > 0)


def test_layer_step_jumps_on_the_interface_only():
    spec = layered_box()
    P = dg.Problem(spec)
    c = 0.7
    u = np.zeros(P.shape)
    u[P.mesh.layer == 0, 0] = c
    eta2 = indicator.jump_indicator(P, u)
    area = spec["Lx"] * spec["Ly"]
    assert eta2.sum() == pytest.approx(c * c * area, rel=1e-13)
    np.testing.assert_allclose(indicator.layer_indicator(P, u), [0.5 * c * c * area, 0.5 * c * c * area],
                               rtol=1e-13)
    # within the lower layer only its top elements touch the interface
    lower = np.where(P.mesh.layer == 1)[0]
    touching = [e for e in lower if np.any(P.mesh.layer[P.mesh.nbr[e][P.mesh.nbr[e] >= 0]] == 0)]
    assert np.abs(np.delete(eta2, np.concatenate([np.where(P.mesh.layer == 0)[0], touching]))).max() < 1e-15


def test_curved_mesh_continuous_field_and_fixed_face_area():
    spec = W.config1()
    P = dg.Problem(spec)
    x, y, z = (P.node_xyz()[:, d] for d in range(3))
    u = np.stack([np.sin(2 * x) * np.cos(y), x * y * z, np.exp(0.3 * z) - x], axis=1)
    eta2 = indicator.jump_indicator(P, u)
    on_bottom = (P.mesh.bc == 1).any(axis=1)
    assert np.abs(eta2[~on_bottom]).max() < 1e-13 * np.abs(eta2).max()
    const = np.ones(P.shape) * 2.0
    total = indicator.jump_indicator(P, const).sum()
    R = spec.get("R", 1.0)
    assert total == pytest.approx(3 * 4.0 * np.pi * R ** 2, rel=1e-4)


def test_scaling_and_layer_sums():
    spec = layered_box(nx=1, ny=2)
    P = dg.Problem(spec)
    u = np.random.default_rng(5).standard_normal(P.shape)
    e1 = indicator.jump_indicator(P, u)
    np.testing.assert_allclose(indicator.jump_indicator(P, -3.0 * u), 9.0 * e1, rtol=1e-14)
    np.testing.assert_allclose(indicator.layer_indicator(P, u).sum(), e1.sum(), rtol=1e-14)


def test_face_families_add_up_and_separate():
    spec = layered_box()
    P = dg.Problem(spec)
    u = np.random.default_rng(8).standard_normal(P.shape)
    all_ = indicator.jump_indicator(P, u)
    np.testing.assert_allclose(indicator.jump_indicator(P, u, "side") + indicator.jump_indicator(P, u, "z"), all_,
                               rtol=1e-14)
    # a step across the layer interface jumps on z-faces only
    c = 0.7
    v = np.zeros(P.shape)
    v[P.mesh.layer == 0, 1] = c
    assert np.abs(indicator.jump_indicator(P, v, "side")).max() == 0.0
    assert indicator.jump_indicator(P, v, "z").sum() == pytest.approx(c * c * spec["Lx"] * spec["Ly"], rel=1e-13)
    # a step across the vertical plane x = 0 (between the two columns along x): its
    # interior jump lies on side faces only
    x = P.node_xyz()[:, 0]
    w = np.zeros(P.shape)
    right = x.mean(axis=(1, 2, 3)) > 0
    w[right, 2] = c
    # its z-faces carry only the fixed-face term of the right half, c^2 (Lx / 2) Ly
    wz = indicator.jump_indicator(P, w, "z")
    on_bottom = (P.mesh.bc == 1).any(axis=1)
    assert np.abs(wz[~on_bottom]).max() == 0.0
    assert wz.sum() == pytest.approx(c * c * 0.5 * spec["Lx"] * spec["Ly"], rel=1e-13)
    H = P.node_xyz()[:, 2].max() - P.node_xyz()[:, 2].min()
    assert indicator.jump_indicator(P, w, "side").sum() == pytest.approx(c * c * spec["Ly"] * H, rel=1e-13)


def test_penalty_weight_closed_forms():
    """weight="penalty": each face's term times sigma = C (p + 1)^2 / min(h, h'),
    with h the element width normal to the face (h = 2 J / J^Sigma is exactly that
    width on a box).  Closed forms on the layered box: a step across the layer
    interface (widths 0.1 above, 0.25 below), a step across the plane x = 0
    (widths 0.6 on both sides) with its fixed-face part (bottom width 0.25), and
    the linear field whose only term is the fixed face."""
    spec = layered_box()
    P = dg.Problem(spec)
    k = spec["penalty"] * (spec["p"] + 1) ** 2
    Lx, Ly = spec["Lx"], spec["Ly"]
    H = 0.6
    c = 0.7
    v = np.zeros(P.shape)
    v[P.mesh.layer == 0, 1] = c
    assert indicator.jump_indicator(P, v, "z", "penalty").sum() == pytest.approx(k / 0.1 * c * c * Lx * Ly, rel=1e-13)
    np.testing.assert_allclose(indicator.layer_indicator(P, v, "all", "penalty"),
                               [0.5 * k / 0.1 * c * c * Lx * Ly] * 2, rtol=1e-13)
    x = P.node_xyz()[:, 0]
    w = np.zeros(P.shape)
    w[x.mean(axis=(1, 2, 3)) > 0, 2] = c
    assert indicator.jump_indicator(P, w, "side", "penalty").sum() == pytest.approx(k / 0.6 * c * c * Ly * H,
                                                                                    rel=1e-13)
    assert indicator.jump_indicator(P, w, "z", "penalty").sum() == pytest.approx(k / 0.25 * c * c * 0.5 * Lx * Ly,
                                                                                 rel=1e-13)
    # the linear field: only the fixed face, whose elements are 0.25 wide
    xyz = P.node_xyz()
    u = np.stack([0.3 * xyz[:, 0] - 0.5 * xyz[:, 2] + 0.2, 0.9 * xyz[:, 1], 0.1 * xyz[:, 2] - 0.4], axis=1)
    np.testing.assert_allclose(indicator.jump_indicator(P, u, "all", "penalty"),
                               k / 0.25 * indicator.jump_indicator(P, u, "all"), rtol=1e-13, atol=1e-15)
    with pytest.raises(ValueError):
        indicator.jump_indicator(P, u, "all", "sigma")
