"""Oracle: gradient of the layer-weighted elastic energy J = sum_k w_k U_k.

Sec. 2.1 defines U_k; with A u = b (Sec. 2.3) the adjoint identity gives
    dJ/dtheta = 1/2 u^T K_w,theta u - lambda^T A_theta u + lambda^T b_theta,
    A^T lambda = K_w u,
K_w the layer-weighted energy form, A^T = A for the weak-form operator.
Materials and thicknesses change A and K_w (the load on z = 0 does not move);
the beam width r0 and centre xc, yc of eq. laserbeam change only b.  The
oracle solves both systems with its own solver (dense on tiny meshes) and
evaluates the three contractions by five-point central differences of its own
operator, energy and load in the parameter (exact up to rounding where they
are linear, i.e. for the moduli; O(step^4) otherwise).

Pinned by tests: Euler homogeneity sum_m c_m dU/dc_m = -U for all moduli;
length scaling sum_l l dU/dl = -U over every length of a box (sides, layer
thicknesses, beam width and centre); reflection symmetry of the beam-centre
derivatives; agreement with finite differences of the whole pipeline.
"""
from __future__ import annotations

import copy

import numpy as np

from . import dg, solve
from .geometry import ref_deriv_T

PARAM_KINDS = ("c11", "c12", "c44", "youngs", "poisson", "thickness", "r0", "xc", "yc")


def energy_grad_u(prob, u, w_layers=None):
    """K_w u = dJ/du: sum_m Dhat_m^T [w J (J^-1)^m_i Y^{ijkl} D_(k u_l)] per element,
    weighted by its layer's w."""
    G = dg.gradient(prob, u)
    T = dg.contract(prob.Yel, dg.sym(G))
    wJ = prob.geo.w3[None] * prob.geo.det
    g = np.zeros(prob.shape)
    for m in range(3):
        Fm = wJ[:, None] * np.einsum("ei...,eij...->ej...", prob.geo.inv[:, m], T)
        g += ref_deriv_T(Fm, prob.geo.D, m)
    w = np.ones(prob.mesh.n_layers) if w_layers is None else np.asarray(w_layers, float)
    return g * w[prob.mesh.layer][:, None, None, None, None]


def get_param(spec, kind, index):
    if kind == "thickness":
        return spec["layers"][index]["thickness"]
    if kind in ("r0", "xc", "yc"):
        return spec["load"][kind]
    m = spec["materials"][index]
    if kind in ("c11", "c12", "c44"):
        if m["kind"] == "cubic":
            return m[kind]
        lam = m["Y"] * m["nu"] / ((1 + m["nu"]) * (1 - 2 * m["nu"]))
        mu = m["Y"] / (2 * (1 + m["nu"]))
        return {"c11": lam + 2 * mu, "c12": lam, "c44": mu}[kind]
    return m["Y"] if kind == "youngs" else m["nu"]


def set_param(spec, kind, index, value):
    """Copy of spec with one parameter changed (an isotropic material whose
    cubic constant is set becomes cubic)."""
    s = copy.deepcopy(spec)
    if kind == "thickness":
        s["layers"][index]["thickness"] = value
        return s
    if kind in ("r0", "xc", "yc"):
        s["load"][kind] = value
        return s
    m = s["materials"][index]
    if kind in ("c11", "c12", "c44"):
        if m["kind"] == "iso":
            c = {k: get_param(spec, k, index) for k in ("c11", "c12", "c44")}
            s["materials"][index] = m = {"kind": "cubic", **c}
        m[kind] = value
    elif kind == "youngs":
        m["Y"] = value
    else:
        m["nu"] = value
    return s


def solve_state(spec, dense=True, w_layers=None):
    P = dg.Problem(spec)
    b = dg.rhs(P)
    if dense:
        # A is symmetric (weak form), so the factorisation serves the adjoint system too
        F = solve.RefinedDense(P)
        u = F.solve(b)[0].reshape(P.shape)
        g = energy_grad_u(P, u, w_layers)
        lam = F.solve(g)[0].reshape(P.shape)
    else:
        u = solve.pcg(P, b, rtol=1e-13)[0]
        g = energy_grad_u(P, u, w_layers)
        lam = solve.pcg(P, g, rtol=1e-13)[0]
    return P, u, lam


def functional(spec, u, lam, w_layers=None):
    """1/2 u^T K_w u - lambda^T A u + lambda^T b for fixed u, lambda under `spec`,
    in extended precision (numpy longdouble): lambda^T A u and lambda^T b are
    large and nearly cancel (the interior-penalty terms of a thin layer), and
    gradient() divides differences of this value by a small step."""
    P = dg.Problem(spec)
    ul = np.asarray(u, dtype=np.longdouble)
    ll = np.asarray(lam, dtype=np.longdouble)
    U = dg.energy_layers(P, ul)
    w = np.ones(len(U)) if w_layers is None else np.asarray(w_layers, float)
    return np.sum(w.astype(np.longdouble) * U) - np.sum(ll * dg.apply(P, ul)) + np.sum(ll * dg.rhs(P))


def param_step(spec, kind, index, rel_step):
    """Difference step: relative to the parameter, for the beam centre relative to r0."""
    if kind in ("xc", "yc"):
        return rel_step * spec["load"]["r0"]
    return rel_step * abs(get_param(spec, kind, index))


def gradient(spec, params, w_layers=None, rel_step=1e-3, dense=True):
    """J and dJ/dtheta for params = [(kind, index)]."""
    P, u, lam = solve_state(spec, dense=dense, w_layers=w_layers)
    U = dg.energy_layers(P, u)
    w = np.ones(len(U)) if w_layers is None else np.asarray(w_layers, float)
    J = float(np.dot(w, U))
    out = []
    for kind, index in params:
        t0 = get_param(spec, kind, index)
        h = param_step(spec, kind, index, rel_step)
        f = [functional(set_param(spec, kind, index, t0 + s * h), u, lam, w_layers) for s in (-2, -1, 1, 2)]
        out.append(float((f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * np.longdouble(h))))
    return J, np.array(out)
