"""Host logic of the design loop (paper_2111_06893_amd/design.py) on the CPU.

* With the oracle as the evaluation engine (dense solves and its own energy
  gradient on a three-element box), the loop recovers a Young's modulus and a
  cubic shear modulus from the layer energies they produce.
* With analytic engines of known optimum: a sum a/x + b/y at fixed x + y
  (minimum at x : y = sqrt(a) : sqrt(b)), on magnitudes of 1e-5 to exercise
  the variable scaling, and an active upper bound.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, dg
from paper_2111_06893_amd import design, with_params


def tiny_spec():
    return W.box(nx=1, ny=1, p=2,
                 layers=[{"thickness": 0.1, "n_elem": 1, "ratio": 1.0, "material": 1},
                         {"thickness": 0.9, "n_elem": 1, "ratio": 1.0, "material": 0}],
                 materials=[dict(W.FUSED_SILICA), dict(W.CRYSTAL_A)])


def oracle_engine(spec, params, x, objective):
    s = with_params(spec, params, x)
    P, u, _ = adjoint.solve_state(s)
    U = dg.energy_layers(P, u)
    J, w = objective(U, s)
    _, g = adjoint.gradient(s, params, w_layers=w)
    return U, J, g


def test_identifies_moduli_with_oracle_engine():
    spec = tiny_spec()
    params = [("youngs", 0), ("c44", 1)]
    truth = np.array([W.FUSED_SILICA["Y"], W.CRYSTAL_A["c44"]])
    P, u, _ = adjoint.solve_state(spec)
    target = dg.energy_layers(P, u)
    r = design.optimize(spec, params, design.TargetObjective(target), x0=truth * [1.2, 0.8],
                        bounds=[(0.5 * t, 2 * t) for t in truth], engine=oracle_engine, maxiter=60)
    np.testing.assert_allclose(r.x, truth, rtol=1e-5)
    assert r.fun < 1e-12
    assert r.n_evals == len(r.history) and r.history[0][1] > r.history[-1][1]


def analytic_engine(a, b):
    def run(spec, params, x, objective):
        U = np.array([a / x[0], b / x[1]])
        J, w = objective(U, spec)
        return U, J, np.array([-w[0] * a / x[0] ** 2, -w[1] * b / x[1] ** 2])
    return run


class Sum:
    def __call__(self, U, spec):
        return float(np.sum(U)), np.ones(len(U))


def test_fixed_sum_constraint_and_scaling():
    a, b, total = 2.0e-12, 0.5e-12, 3.0e-5
    params = [("thickness", 0), ("thickness", 1)]
    r = design.optimize(tiny_spec(), params, Sum(), x0=[1.0e-5, 2.0e-5],
                        bounds=[(1e-7, None), (1e-7, None)], constraints=[design.fixed_sum([0, 1], total)],
                        engine=analytic_engine(a, b), tol=1e-15)
    xa = total * np.sqrt(a) / (np.sqrt(a) + np.sqrt(b))
    np.testing.assert_allclose(r.x, [xa, total - xa], rtol=1e-6)
    assert r.success


def test_active_bound():
    params = [("thickness", 0), ("thickness", 1)]
    r = design.optimize(tiny_spec(), params, Sum(), x0=[1.0, 1.0], bounds=[(0.5, 2.0), (0.5, 3.0)],
                        engine=analytic_engine(1.0, 1.0))
    np.testing.assert_allclose(r.x, [2.0, 3.0], rtol=1e-9)


def test_target_objective_derivative():
    obj = design.TargetObjective([2.0, 4.0], weights=[1.0, 3.0])
    U = np.array([2.5, 3.0])
    J, w = obj(U, None)
    h = 1e-6
    for k in range(2):
        e = np.eye(2)[k] * h
        fd = (obj(U + e, None)[0] - obj(U - e, None)[0]) / (2 * h)
        assert abs(w[k] - fd) < 1e-8


def test_bad_arguments():
    with pytest.raises(ValueError):
        design.TargetObjective([1.0, 0.0])
    with pytest.raises(ValueError):
        design.optimize(tiny_spec(), [("thickness", 0)], Sum(), x0=[1.0, 2.0], engine=analytic_engine(1, 1))
