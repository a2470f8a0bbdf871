"""Pins of the oracle's energy gradient (oracle/adjoint.py).

* Euler homogeneity: A and the energy form are homogeneous of degree one in
  the elastic constants (the penalty uses averaged moduli), so u scales as 1/s
  and U as 1/s when every constant is multiplied by s:
  sum_m c_m dU/dc_m = -U, and per isotropic material Y dU/dY sums the same way.
* Length scaling: the operator scales as s and the load vector is unchanged
  when every length (box sides, layer thicknesses, beam width and centre) is
  multiplied by s, so U scales as 1/s: sum_l l dU/dl = -U.  The box sides are
  differenced through the whole pipeline, the other lengths come from the
  oracle's gradient.
* Reflection symmetry of the beam-centre derivatives on a square box.
* Finite differences of the whole pipeline (re-mesh, re-assemble, solve,
  energy), which share nothing with the adjoint identity.
* dJ/du: K_w u is the derivative of J at fixed parameters (checked against a
  directional difference of the quadratic form).
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, dg, solve


def tiny_spec():
    # three affine elements, a cubic coating over two substrate elements
    return W.box(nx=1, ny=1, p=3,
                 layers=[{"thickness": 0.1, "n_elem": 1, "ratio": 1.0, "material": 1},
                         {"thickness": 0.9, "n_elem": 2, "ratio": 1.0, "material": 0}],
                 materials=[dict(W.FUSED_SILICA), dict(W.CRYSTAL_A)])


def pipeline_energy(spec, w):
    P = dg.Problem(spec)
    u = solve.pcg(P, dg.rhs(P), rtol=1e-14, maxit=5000)[0]
    return float(np.dot(w, dg.energy_layers(P, u)))


def offset_spec(xc=0.12, yc=-0.07):
    # the tiny box under a wider beam whose centre is off the axis
    s = tiny_spec()
    s["load"] = {"F0": 1.0, "r0": 0.25, "xc": xc, "yc": yc}
    return s


@pytest.fixture(scope="module")
def spec():
    return tiny_spec()


def test_euler_homogeneity(spec):
    params = [(k, m) for m in range(2) for k in ("c11", "c12", "c44")]
    J, g = adjoint.gradient(spec, params)
    vals = np.array([adjoint.get_param(spec, k, m) for k, m in params])
    assert abs(np.dot(vals, g) + J) < 1e-10 * J


def test_euler_homogeneity_isotropic_material():
    # a single isotropic material: Y dU/dY = -U exactly
    spec = W.box(nx=1, ny=1, p=2, layers=[{"thickness": 0.4, "n_elem": 2, "ratio": 1.0, "material": 0}])
    J, g = adjoint.gradient(spec, [("youngs", 0), ("poisson", 0)])
    assert abs(spec["materials"][0]["Y"] * g[0] + J) < 1e-10 * J
    assert g[1] != 0


def test_layer_weights_split(spec):
    # the gradient is linear in the layer weights
    params = [("c44", 1), ("thickness", 1)]
    _, g0 = adjoint.gradient(spec, params, w_layers=[1.0, 0.0])
    _, g1 = adjoint.gradient(spec, params, w_layers=[0.0, 1.0])
    _, g = adjoint.gradient(spec, params, w_layers=[0.3, 1.7])
    np.testing.assert_allclose(g, 0.3 * g0 + 1.7 * g1, rtol=1e-9)


def test_length_scaling():
    spec = offset_spec()
    w = np.array([0.3, 1.7])
    lengths = [("thickness", 0), ("thickness", 1), ("r0", 0), ("xc", 0), ("yc", 0)]
    J, g = adjoint.gradient(spec, lengths, w_layers=w)
    total = sum(adjoint.get_param(spec, k, i) * gi for (k, i), gi in zip(lengths, g))
    for side in ("Lx", "Ly"):
        L0 = spec[side]
        h = 1e-4 * L0
        fp = pipeline_energy(W.with_overrides(spec, **{side: L0 + h}), w)
        fm = pipeline_energy(W.with_overrides(spec, **{side: L0 - h}), w)
        total += L0 * (fp - fm) / (2 * h)
    assert abs(total + J) < 1e-7 * J
    # every term matters: the beam terms alone are a sizeable part of the sum
    assert abs(g[2] * 0.25) > 1e-2 * J and abs(g[3]) > 0 and abs(g[4]) > 0


def test_beam_centre_reflection():
    # x -> -x maps the beam at xc to the beam at -xc; x <-> y swaps xc and yc
    params = [("xc", 0), ("yc", 0)]
    _, ga = adjoint.gradient(offset_spec(0.12, -0.07), params)
    _, gb = adjoint.gradient(offset_spec(-0.12, -0.07), params)
    _, gc = adjoint.gradient(offset_spec(-0.07, 0.12), params)
    _, g0 = adjoint.gradient(offset_spec(0.0, 0.0), params)
    np.testing.assert_allclose(gb, [-ga[0], ga[1]], rtol=1e-9)
    np.testing.assert_allclose(gc, [ga[1], ga[0]], rtol=1e-9)
    assert np.max(np.abs(g0)) < 1e-9 * np.max(np.abs(ga))


@pytest.mark.parametrize("param", [("c11", 1), ("poisson", 0), ("thickness", 0), ("r0", 0), ("xc", 0)])
def test_against_pipeline_differences(param):
    spec = offset_spec() if param[0] in ("r0", "xc") else tiny_spec()
    w = np.array([0.3, 1.7])
    _, g = adjoint.gradient(spec, [param], w_layers=w)
    kind, index = param
    t0 = adjoint.get_param(spec, kind, index)
    h = adjoint.param_step(spec, kind, index, 1e-4)
    fp = pipeline_energy(adjoint.set_param(spec, kind, index, t0 + h), w)
    fm = pipeline_energy(adjoint.set_param(spec, kind, index, t0 - h), w)
    fd = (fp - fm) / (2 * h)
    assert abs(g[0] - fd) < 1e-6 * abs(fd)


def test_energy_grad_is_derivative_of_energy(spec):
    P = dg.Problem(spec)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(P.shape)
    v = rng.standard_normal(P.shape)
    w = np.array([2.0, 0.5])
    g = adjoint.energy_grad_u(P, u, w)

    def J(x):
        return float(np.dot(w, dg.energy_layers(P, x)))
    # J is quadratic: the central difference is exact up to rounding
    fd = (J(u + v) - J(u - v)) / 2
    assert abs(np.sum(g * v) - fd) < 1e-11 * abs(J(u))


def test_set_param_roundtrip(spec):
    s = adjoint.set_param(spec, "c12", 0, 1.0e10)
    assert s["materials"][0]["kind"] == "cubic"
    assert adjoint.get_param(s, "c11", 0) == pytest.approx(adjoint.get_param(spec, "c11", 0), rel=1e-15)
    assert spec["materials"][0]["kind"] == "iso"
