"""The design loop on the device (paper_2111_06893_amd/design.py).

* Beam centring under a constraint: the noise S_x of the five-block cylinder
  (40 elements, p = 5) over the beam centre (xc, yc) restricted to the line
  xc - yc = 0.2.  The mesh and load are symmetric under (x, y) -> (-y, -x),
  which maps the line onto itself with (0.1, -0.1) as its fixed point, so that
  point is stationary; the loop must find it from (0.25, 0.05).
* Identification: the coating's Young's modulus and the beam width of the
  coated cylinder recovered from the two layer energies they produce, from a
  start 15-20 % off.
* The forty-layer mirror: S_x (loss angles 1e-4 on crystal A, 1e-5 on crystal
  B) over the forty coating thicknesses at fixed total thickness, each within
  [0.5, 1.5] of nominal.  A thin layer's energy is nearly proportional to its
  thickness, so the problem is nearly a linear programme: every B layer ends at
  the upper bound, every A layer at the lower, the total unchanged, and at that
  point the KKT conditions hold: each A layer's derivative of S_x exceeds each
  B layer's (moving thickness from A to B would still lower S_x).
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
import paper_2111_06893_amd as dgtn  # noqa: E402
from paper_2111_06893_amd import design  # noqa: E402

pytestmark = pytest.mark.gpu


def test_beam_centring_on_a_line():
    spec = W.config1()
    spec["load"] = {"F0": 1.0, "r0": 0.2, "xc": 0.25, "yc": 0.05}
    params = [("xc", 0), ("yc", 0)]
    obj = design.NoiseObjective([1e-4, 1e-4], 300.0, 100.0)
    seen = []
    r = design.optimize(spec, params, obj, constraints=[design.fixed_sum([0, 1], 0.2, [1.0, -1.0])],
                        bounds=[(-0.6, 0.6), (-0.6, 0.6)], tol=1e-14, maxiter=40,
                        callback=lambda x, J: seen.append(J))
    print("centring", r.x, r.n_evals, r.message)
    assert abs(r.x[0] - 0.1) < 2e-4 and abs(r.x[1] + 0.1) < 2e-4, r.x
    assert r.fun < seen[0]


def test_identify_coating_modulus_and_beam_width():
    spec = W.config4(d=0.05)
    spec["p"] = 4
    spec["load"]["r0"] = 0.15
    params = [("youngs", 1), ("r0", 0)]
    truth = np.array([spec["materials"][1]["Y"], 0.15])
    P = dgtn.Problem(spec)
    u, _ = P.solve(opts=dgtn.default_opts(rtol=1e-11))
    target = P.energy(u)
    P.close()
    r = design.optimize(spec, params, design.TargetObjective(target), x0=truth * [1.2, 0.85],
                        bounds=[(0.3 * truth[0], 3 * truth[0]), (0.05, 0.4)], tol=1e-14, maxiter=60)
    print("identify", r.x / truth - 1, r.n_evals, r.message)
    np.testing.assert_allclose(r.x, truth, rtol=1e-5)


def test_forty_layer_mirror_thicknesses():
    print("[design] forty-layer mirror", flush=True)
    spec = W.config5(p=5)
    n = len(spec["layers"]) - 1
    is_a = np.array([spec["layers"][k]["material"] == 1 for k in range(n)])
    phi = np.r_[np.where(is_a, 1e-4, 1e-5), 1e-7]
    d0 = np.array([spec["layers"][k]["thickness"] for k in range(n)])
    r = design.optimize(spec, [("thickness", k) for k in range(n)], design.NoiseObjective(phi, 300.0, 100.0),
                        constraints=[design.fixed_sum(range(n), float(d0.sum()))],
                        bounds=[(0.5 * d, 1.5 * d) for d in d0], tol=1e-9, maxiter=30,
                        engine=design.device_engine(dgtn.default_opts(32, rtol=5e-8, max_iter=2000),
                                                    max_rel_res=1e-6))
    assert r.success, r.message
    np.testing.assert_allclose(r.x[~is_a], 1.5 * d0[~is_a], rtol=1e-9)
    np.testing.assert_allclose(r.x[is_a], 0.5 * d0[is_a], rtol=1e-9)
    assert abs(r.x.sum() / d0.sum() - 1.0) < 1e-12
    assert r.grad[is_a].min() > r.grad[~is_a].max()
    assert r.fun < 0.8 * r.history[0][1]          # observed 3.125e-40 -> 2.368e-40
