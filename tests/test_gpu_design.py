"""The design loop on the device (paper_2111_06893_amd/design.py).

* Beam centring under a constraint: the noise S_x of the five-block cylinder
  (40 elements, p = 5) over the beam centre (xc, yc) restricted to the line
  xc - yc = 0.2.  The mesh and load are symmetric under (x, y) -> (-y, -x),
  which maps the line onto itself with (0.1, -0.1) as its fixed point, so that
  point is stationary; the loop must find it from (0.25, 0.05).
* Identification: the coating's Young's modulus and the beam width of the
  coated cylinder recovered from the two layer energies they produce, from a
  start 15-20 % off.
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
