"""GPU checks of the energy gradient (dgtn_energy_grad, dgtn_grad, EnergyFn).

* dJ/du and dJ/dtheta of the library equal the oracle's (dense solves,
  five-point differences of its own operator) on a three-element box with a
  cubic coating: 1e-11 relative for dJ/du, 1e-8 for dJ/dtheta.
* On the coating workload (40 elements, p = 5 and 6) the adjoint gradient with
  respect to (Y_coat, nu_coat, Y_sub, nu_sub, coating thickness) equals
  five-point differences of the library's own solve-and-energy pipeline to
  1e-6 (coating 0.05 thick), and obeys Euler's relation
  Y_coat dU/dY_coat + Y_sub dU/dY_sub = -U (coating 1e-3 thick, to 1e-7).
* The beam width and centre (the load's parameters): the library's
  lambda^T b_theta equals the oracle's gradient on the box under an off-axis
  beam (1e-8), the oracle's five-point difference of the functional given the
  same u and lambda (1e-9), and differences of the library's pipeline on the
  cylinder (1e-6).
* The autograd function returns the oracle's weighted gradient.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint

torch = pytest.importorskip("torch")
import paper_2111_06893_amd as dgtn  # noqa: E402

pytestmark = pytest.mark.gpu

PARAMS = [("c11", 1), ("c12", 1), ("c44", 1), ("youngs", 0), ("poisson", 0), ("thickness", 0), ("thickness", 1)]
W_LAYERS = np.array([0.3, 1.7])


def tiny_spec():
    return W.box(nx=1, ny=1, p=3,
                 layers=[{"thickness": 0.1, "n_elem": 1, "ratio": 1.0, "material": 1},
                         {"thickness": 0.9, "n_elem": 2, "ratio": 1.0, "material": 0}],
                 materials=[dict(W.FUSED_SILICA), dict(W.CRYSTAL_A)])


def opts(rtol=1e-10):
    return dgtn.default_opts(64, rtol=rtol, max_iter=20000)


def gpu_gradient(spec, params, w, rtol=1e-10):
    P = dgtn.Problem(spec)
    o = opts(rtol)
    u, _ = P.solve(opts=o)
    g = P.energy_grad(u, w)
    lam, _ = P.solve(b=g, opts=o)
    return P, u, g, P.grad(u, lam, params, w)


@pytest.fixture(scope="module")
def oracle_tiny():
    spec = tiny_spec()
    P, u, lam = adjoint.solve_state(spec, w_layers=W_LAYERS)
    J, g = adjoint.gradient(spec, PARAMS, w_layers=W_LAYERS)
    return spec, u, J, g


def test_energy_grad_matches_oracle(oracle_tiny):
    spec, u, _, _ = oracle_tiny
    from oracle import dg
    P = dgtn.Problem(spec)
    ud = torch.from_numpy(u).to("cuda")
    g = P.energy_grad(ud, W_LAYERS).cpu().numpy()
    ref = adjoint.energy_grad_u(dg.Problem(spec), u, W_LAYERS)
    assert np.max(np.abs(g - ref)) < 1e-11 * np.max(np.abs(ref))


def test_gradient_matches_oracle(oracle_tiny):
    spec, _, J, ref = oracle_tiny
    P, u, _, g = gpu_gradient(spec, PARAMS, W_LAYERS)
    assert abs(float(np.dot(W_LAYERS, P.energy(u))) - J) < 1e-10 * J
    for (kind, index), a, b in zip(PARAMS, g, ref):
        assert abs(a - b) < 1e-8 * abs(b), (kind, index, a, b)


def test_gradient_with_given_state_is_exact(oracle_tiny):
    # with the oracle's u and lambda the contraction alone is compared
    spec, u, _, _ = oracle_tiny
    _, _, lam = adjoint.solve_state(spec, w_layers=W_LAYERS)
    P = dgtn.Problem(spec)
    g = P.grad(torch.from_numpy(u).to("cuda"), torch.from_numpy(lam).to("cuda"), PARAMS, W_LAYERS)
    for (kind, index), a in zip(PARAMS, g):
        t0 = adjoint.get_param(spec, kind, index)
        h = 1e-3 * abs(t0)
        f = [adjoint.functional(adjoint.set_param(spec, kind, index, t0 + s * h), u, lam, W_LAYERS)
             for s in (-2, -1, 1, 2)]
        fd = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
        assert abs(a - fd) < 1e-9 * abs(fd), (kind, index, a, fd)


def coating_spec(d=0.05):
    return W.config4(d=d)


COATING_PARAMS = [("youngs", 1), ("poisson", 1), ("youngs", 0), ("poisson", 0), ("thickness", 0)]


def gpu_total_energy(spec, rtol=1e-11):
    P = dgtn.Problem(spec)
    u, _ = P.solve(opts=opts(rtol))
    return float(np.sum(P.energy(u)))


@pytest.mark.parametrize("p", [5, 6])
def test_coating_gradient_against_differences(p):
    spec = coating_spec()
    spec["p"] = p
    params = COATING_PARAMS if p == 5 else [("youngs", 1), ("thickness", 0)]
    _, _, _, g = gpu_gradient(spec, params, None, rtol=1e-11)
    for (kind, index), a in zip(params, g):
        t0 = adjoint.get_param(spec, kind, index)
        h = 1e-3 * abs(t0)
        f = [gpu_total_energy(dgtn.with_params(spec, [(kind, index)], [t0 + s * h])) for s in (-2, -1, 1, 2)]
        fd = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
        assert abs(a - fd) < 1e-6 * abs(fd), (kind, index, a, fd)


def test_coating_euler_relation():
    # the 1e-3 coating: FP64 residuals stagnate near 1e-10 here, so solve to 1e-9
    spec = W.config4()
    P, u, _, g = gpu_gradient(spec, [("youngs", 1), ("youngs", 0)], None, rtol=1e-9)
    U = float(np.sum(P.energy(u)))
    s = spec["materials"][1]["Y"] * g[0] + spec["materials"][0]["Y"] * g[1]
    print("euler residual", (s + U) / U)
    assert abs(s + U) < 1e-7 * U


def test_energy_fn_backward(oracle_tiny):
    spec, _, _, _ = oracle_tiny
    params = [("youngs", 0), ("thickness", 0), ("c44", 1)]
    theta = torch.tensor([adjoint.get_param(spec, k, i) for k, i in params], dtype=torch.float64,
                         requires_grad=True)
    U = dgtn.layer_energies(theta, spec, params, opts())
    (U * torch.from_numpy(W_LAYERS)).sum().backward()
    _, ref = adjoint.gradient(spec, params, w_layers=W_LAYERS)
    np.testing.assert_allclose(theta.grad.numpy(), ref, rtol=1e-8)


BEAM_PARAMS = [("r0", 0), ("xc", 0), ("yc", 0)]


def offset_spec():
    s = tiny_spec()
    s["load"] = {"F0": 1.0, "r0": 0.25, "xc": 0.12, "yc": -0.07}
    return s


def test_beam_gradient_matches_oracle():
    spec = offset_spec()
    J, ref = adjoint.gradient(spec, BEAM_PARAMS, w_layers=W_LAYERS)
    P, u, _, g = gpu_gradient(spec, BEAM_PARAMS, W_LAYERS)
    assert abs(float(np.dot(W_LAYERS, P.energy(u))) - J) < 1e-10 * J
    for (kind, _), a, b in zip(BEAM_PARAMS, g, ref):
        assert abs(a - b) < 1e-8 * abs(b), (kind, a, b)


def test_beam_gradient_with_given_state_is_exact():
    spec = offset_spec()
    _, u, lam = adjoint.solve_state(spec, w_layers=W_LAYERS)
    P = dgtn.Problem(spec)
    g = P.grad(torch.from_numpy(u).to("cuda"), torch.from_numpy(lam).to("cuda"), BEAM_PARAMS, W_LAYERS)
    for (kind, index), a in zip(BEAM_PARAMS, g):
        t0 = adjoint.get_param(spec, kind, index)
        h = adjoint.param_step(spec, kind, index, 1e-3)
        f = [adjoint.functional(adjoint.set_param(spec, kind, index, t0 + s * h), u, lam, W_LAYERS)
             for s in (-2, -1, 1, 2)]
        fd = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
        assert abs(a - fd) < 1e-9 * abs(fd), (kind, a, fd)


def test_beam_gradient_on_cylinder_against_differences():
    spec = W.config1()
    spec["load"] = {"F0": 1.0, "r0": 0.2, "xc": 0.3, "yc": 0.1}
    params = [("r0", 0), ("xc", 0)]
    _, _, _, g = gpu_gradient(spec, params, None, rtol=1e-11)
    for (kind, index), a in zip(params, g):
        t0 = adjoint.get_param(spec, kind, index)
        h = 1e-3 * spec["load"]["r0"]
        f = [gpu_total_energy(dgtn.with_params(spec, [(kind, index)], [t0 + s * h])) for s in (-2, -1, 1, 2)]
        fd = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
        assert abs(a - fd) < 1e-6 * abs(fd), (kind, a, fd)


def test_grad_rejects_bad_parameters():
    P = dgtn.Problem(tiny_spec())
    u = P.rhs()
    with pytest.raises(dgtn.DgtnError):
        P.grad(u, u, [("youngs", 1)])       # material 1 is cubic
    with pytest.raises(dgtn.DgtnError):
        P.grad(u, u, [("thickness", 5)])
    with pytest.raises(ValueError):
        P.grad(u, u, [("density", 0)])


# --- the coated cylinder of 40 elements (coating 1e-3 R) -------------------------------
# The oracle's gradients on this topology at p = 3 (tests/golden/make_gradients.py: dense
# solves refined with extended-precision residuals, five-point differences of its own
# operator).  The moduli enter A and K linearly, so the oracle's difference quotient is
# exact up to rounding (1e-10); the Poisson ratios and the thickness enter nonlinearly and
# its five-point step of 1e-3 relative leaves an O(1e-12) truncation and ~1e-10 of rounding
# amplified by the step (1e-9).

def _golden_gradients():
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", "gradients.json")))


@pytest.mark.parametrize("case", [0, 1])
@pytest.mark.parametrize("prec", [64, 32])
def test_coated_cylinder_gradient_matches_oracle(case, prec):
    g = _golden_gradients()
    spec, params = g["spec"], [tuple(p) for p in g["params"]]
    c = g["cases"][case]
    w = np.array(c["w_layers"])
    print(f"[adjoint] coated cylinder p=3 against the oracle, w={w.tolist()}, fp{prec} preconditioner", flush=True)
    P = dgtn.Problem(spec)
    # rtol below the attainable residual of a double-rounded solution: the solves end on
    # stagnation there, with u refined by the double-double residual
    o = dgtn.default_opts(prec, rtol=1e-14, max_iter=20000)
    u, st = P.solve(opts=o, raise_on_noconv=False)
    assert st.rel_res < 1e-9
    J = float(np.dot(w, P.energy(u)))
    lam, st2 = P.solve(b=P.energy_grad(u, w), opts=o, raise_on_noconv=False)
    assert st2.rel_res < 1e-9
    dJ = P.grad(u, lam, params, w)
    print(f"J {J:.15e} vs {c['J']:.15e}; solves {st.iters}/{st2.iters} it, rel.res {st.rel_res:.1e}", flush=True)
    tol_J = 1e-10 if prec == 64 else 1e-8
    assert abs(J / c["J"] - 1) < tol_J
    # per-layer gradients of the oracle (case 1 weighs the coating only): an entry of a
    # weighted sum can cancel between the layers (dU/dd: +5.05e-11 coating, -5.37e-11
    # substrate), so each entry is held relative to the sum of its layer parts' magnitudes
    g_coat = np.array(g["cases"][1]["dJ"])
    g_sub = np.array(g["cases"][0]["dJ"]) - g_coat
    scale = np.abs(w[0] * g_coat) + np.abs(w[1] * g_sub)
    for q, ((kind, index), a, b) in enumerate(zip(params, dJ, c["dJ"])):
        if scale[q] < 1e-12 * scale.max():
            continue                             # a structurally ~zero entry (Y with w = 0 on its layer)
        tol = (1e-10 if kind == "youngs" else 1e-9) if prec == 64 else 1e-8
        print(f"  {kind}[{index}] {a:.12e} oracle {b:.12e} rel {a / b - 1:+.2e} "
              f"(of the layer parts {(a - b) / scale[q]:+.2e})", flush=True)
        assert abs(a - b) < tol * scale[q], (kind, index, a, b)


def test_coated_cylinder_gradient_central_differences():
    # the benchmark's coated cylinder at p = 5 (coating 1e-3 R): central differences of the
    # whole solve-and-energy pipeline with a relative step of 1e-6 against the adjoint; the
    # difference quotient carries ~1e-8 of solve rounding amplified by the step
    spec = W.config4()
    w = np.array([1.0, 1.0])
    params = COATING_PARAMS
    print("[adjoint] coated cylinder p=5, central differences h = 1e-6", flush=True)
    o = opts(1e-14)        # ends on stagnation at the rounding floor of the stored solution
    P = dgtn.Problem(spec)
    u, _ = P.solve(opts=o, raise_on_noconv=False)
    lam, _ = P.solve(b=P.energy_grad(u, w), opts=o, raise_on_noconv=False)
    dJ = P.grad(u, lam, params, w)
    for (kind, index), a in zip(params, dJ):
        t0 = dgtn.param_value(spec, kind, index)
        h = 1e-6 * abs(t0)
        f = []
        for s in (-1, 1):
            Q = dgtn.Problem(dgtn.with_params(spec, [(kind, index)], [t0 + s * h]))
            uq, _ = Q.solve(opts=o, raise_on_noconv=False)
            f.append(float(np.dot(w, Q.energy(uq))))
            Q.close()
        fd = (f[1] - f[0]) / (2 * h)
        print(f"  {kind}[{index}] adjoint {a:.10e} central {fd:.10e} rel {a / fd - 1:+.2e}", flush=True)
        assert abs(a / fd - 1) < 1e-6, (kind, index, a, fd)


def test_gradient_at_the_highest_degree_matches_oracle():
    # p = 7 (N = 8): the dual-number kernels at their largest size (136 KB of LDS) against the
    # oracle's gradient on a three-element box with a cubic coating (dense refined solves)
    g = _golden_gradients()["box_p7"]
    spec, params, w = g["spec"], [tuple(p) for p in g["params"]], np.array(g["w_layers"])
    print("[adjoint] box p=7 against the oracle", flush=True)
    P = dgtn.Problem(spec)
    o = dgtn.default_opts(64, rtol=1e-14, max_iter=20000)
    u, st = P.solve(opts=o, raise_on_noconv=False)
    assert st.rel_res < 1e-9
    J = float(np.dot(w, P.energy(u)))
    lam, st2 = P.solve(b=P.energy_grad(u, w), opts=o, raise_on_noconv=False)
    assert st2.rel_res < 1e-9
    dJ = P.grad(u, lam, params, w)
    assert abs(J / g["J"] - 1) < 1e-11, (J, g["J"])
    for (kind, index), a, b in zip(params, dJ, g["dJ"]):
        print(f"  {kind}[{index}] {a:.12e} oracle {b:.12e} rel {a / b - 1:+.2e}", flush=True)
        assert abs(a / b - 1) < (1e-10 if kind in ("c11", "c12", "c44", "youngs") else 1e-9), (kind, index, a, b)
    # and the double-double residual at this degree agrees with FP64 to its rounding
    b = P.rhs()
    r = P.residual(u, b)
    r64 = b - P.apply(u)
    assert float(torch.linalg.norm(r - r64)) < 1e-2 * float(torch.linalg.norm(r64))
