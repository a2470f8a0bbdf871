"""Pins of the oracle's energy split by elastic modulus (oracle/dg.energy_parts).

* The parts of every layer sum to the layer energy.
* Uniform strains on a box (exact for any p, with traction-free data irrelevant:
  the energy is evaluated on the prescribed displacement field):
  dilatation u = e x  -> isotropic bulk 9 K e^2 / 2 per volume, shear 0;
  simple shear u = (g y, 0, 0) -> bulk 0, shear mu g^2 / 2 per volume;
  cubic uniaxial u = (e x, 0, 0) -> c11 e^2 / 2, c12 and c44 parts 0;
  cubic biaxial u = (e x, e y, 0) -> c11 e^2, c12 e^2, c44 0;
  cubic shear u = (g y, 0, 0) -> c44 g^2 / 2 only.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dg, material, physics


def box(mat, p=2):
    return W.box(nx=2, ny=1, Lx=1.3, Ly=0.7, p=p,
                 layers=[{"thickness": 0.4, "n_elem": 2, "ratio": 1.5, "material": 0}],
                 materials=[dict(mat)])


def field(P, fn):
    x = P.mesh.xyz
    return np.stack(fn(x[:, 0], x[:, 1], x[:, 2]), axis=1)


def volume(spec):
    return spec["Lx"] * spec["Ly"] * sum(l["thickness"] for l in spec["layers"])


def test_parts_sum_to_energy():
    spec = W.config1()
    spec["p"] = 2
    P = dg.Problem(spec)
    u = W.random_field(spec, 1)
    parts = dg.energy_parts(P, u)
    np.testing.assert_allclose(parts.sum(axis=1), dg.energy_layers(P, u), rtol=1e-12)
    spec = box(W.CRYSTAL_A)
    P = dg.Problem(spec)
    u = W.random_field(spec, 2)
    np.testing.assert_allclose(dg.energy_parts(P, u).sum(axis=1), dg.energy_layers(P, u), rtol=1e-12)


def test_isotropic_dilatation_and_shear():
    spec = box(W.COATING_ISO)
    P = dg.Problem(spec)
    V = volume(spec)
    lam, mu = material.lame(W.COATING_ISO["Y"], W.COATING_ISO["nu"])
    K = lam + 2 * mu / 3
    e, g = 1e-3, 2e-3
    parts = dg.energy_parts(P, field(P, lambda x, y, z: (e * x, e * y, e * z)))[0]
    assert parts[0] == pytest.approx(4.5 * K * e * e * V, rel=1e-12)
    assert abs(parts[1]) < 1e-12 * parts[0] and parts[2] == 0
    parts = dg.energy_parts(P, field(P, lambda x, y, z: (g * y, 0 * x, 0 * x)))[0]
    assert parts[1] == pytest.approx(0.5 * mu * g * g * V, rel=1e-12)
    assert abs(parts[0]) < 1e-12 * parts[1]


def test_cubic_parts():
    m = W.CRYSTAL_B
    spec = box(m)
    P = dg.Problem(spec)
    V = volume(spec)
    e, g = 1e-3, 2e-3
    parts = dg.energy_parts(P, field(P, lambda x, y, z: (e * x, 0 * x, 0 * x)))[0]
    np.testing.assert_allclose(parts, [0.5 * m["c11"] * e * e * V, 0, 0], rtol=1e-12, atol=1e-18)
    parts = dg.energy_parts(P, field(P, lambda x, y, z: (e * x, e * y, 0 * x)))[0]
    np.testing.assert_allclose(parts, [m["c11"] * e * e * V, m["c12"] * e * e * V, 0], rtol=1e-12, atol=1e-18)
    parts = dg.energy_parts(P, field(P, lambda x, y, z: (g * y, 0 * x, 0 * x)))[0]
    np.testing.assert_allclose(parts, [0, 0, 0.5 * m["c44"] * g * g * V], rtol=1e-12, atol=1e-18)


def test_noise_with_equal_part_angles_is_the_layer_formula():
    U = np.array([[1.0, 2.0, 0.0], [3.0, 0.5, 0.25]]) * 1e-12
    phi = np.array([4e-4, 1e-7])
    a = physics.noise_psd_parts(U, np.repeat(phi[:, None], 3, axis=1), 300.0, 100.0, 1.0)
    b = physics.noise_psd(U.sum(axis=1), phi, 300.0, 100.0, 1.0)
    assert a == pytest.approx(b, rel=1e-15)
