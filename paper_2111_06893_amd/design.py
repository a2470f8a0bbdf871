"""Design loop over mirror, coating and beam parameters, driven by the adjoint
energy gradient.

Sec. 4 proposes using the solver to search realistic mirror configurations,
coatings and beam sizes for low Brownian coating noise; what such a search
needs from the solver is dU_k/dtheta for the per-layer energies U_k of Sec. 2.1,
which the library computes with one extra (adjoint) solve for any number of
parameters.  One evaluation of an objective J(U(theta)) at theta:

  1. forward solve A(theta) u = b(theta) on the device and the layer energies U_k;
  2. J and w_k = dJ/dU_k on the host (the objectives below are cheap in U);
  3. one adjoint solve A lambda = sum_k w_k K_k u and dJ/dtheta = dgtn_grad(u,
     lambda, w), i.e. w . dU/dtheta.

The outer optimiser is scipy's (L-BFGS-B for bounds only, SLSQP when there are
constraints).  It works on theta divided by a per-parameter scale (|theta_0|;
the beam width for a beam centre), and on J divided by its value at the start,
because the physical magnitudes span some forty decades (moduli ~1e11 Pa,
thicknesses ~1e-5 R, S_x ~1e-40).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import Problem, default_opts, noise_psd, param_value, with_params

__all__ = ["NoiseObjective", "TargetObjective", "DesignResult", "optimize", "fixed_sum", "device_engine"]


class NoiseObjective:
    """S_x of eqs. thermalnoise and wdiss with one loss angle per layer: linear in U, so
    dS_x/dU_k is S_x of the k-th unit vector."""

    def __init__(self, phi: Sequence[float], T: float, f: float):
        self.phi = np.asarray(phi, dtype=np.float64)
        self.T, self.f = float(T), float(f)

    def __call__(self, U, spec):
        F0 = spec["load"]["F0"]
        n = len(U)
        if n != len(self.phi):
            raise ValueError("one loss angle per layer expected")
        val = noise_psd(U, self.phi, self.T, self.f, F0)
        grad = np.array([noise_psd(np.eye(n)[k], self.phi, self.T, self.f, F0) for k in range(n)])
        return val, grad


class TargetObjective:
    """1/2 sum_k c_k ((U_k - U*_k) / U*_k)^2: the misfit to given layer energies
    (identifying moduli, thicknesses or the beam from measured energies);
    c_k = 1 by default."""

    def __init__(self, U_target: Sequence[float], weights: Optional[Sequence[float]] = None):
        self.Ut = np.asarray(U_target, dtype=np.float64)
        if np.any(self.Ut == 0):
            raise ValueError("target energies must be non-zero")
        self.c = np.ones_like(self.Ut) if weights is None else np.asarray(weights, dtype=np.float64)

    def __call__(self, U, spec):
        r = (np.asarray(U) - self.Ut) / self.Ut
        return 0.5 * float(np.sum(self.c * r * r)), self.c * r / self.Ut


def fixed_sum(indices: Sequence[int], total: float, weights: Optional[Sequence[float]] = None):
    """Equality constraint sum_i a_i theta_i = total over the given parameter
    positions (a fixed total coating thickness, a beam centre on a line)."""
    idx = list(indices)
    a = np.ones(len(idx)) if weights is None else np.asarray(weights, dtype=np.float64)

    def fun(x):
        return float(np.dot(a, np.asarray(x)[idx]) - total)

    def jac(x):
        g = np.zeros(len(x))
        g[idx] = a
        return g

    return {"type": "eq", "fun": fun, "jac": jac}


Engine = Callable[[dict, List[Tuple[str, int]], np.ndarray, Callable], Tuple[np.ndarray, float, np.ndarray]]


def device_engine(opts=None, max_rel_res: Optional[float] = None) -> Engine:
    """Evaluates (U, J, dJ/dtheta) with the library: forward solve, layer
    energies, adjoint solve and dgtn_grad on the current device.  A solve that
    stagnates above its rtol (at the FP64 residual floor of thin layers) raises,
    unless max_rel_res is given and the relative residual it reached is within
    it: the energies and the gradient then carry an error of first order in that
    residual."""

    def solve(P, o, b=None):
        x, st = P.solve(b=b, opts=o, raise_on_noconv=max_rel_res is None)
        if max_rel_res is not None and not st.converged and st.rel_res > max_rel_res:
            raise RuntimeError(f"design evaluation: solve stalled at relative residual {st.rel_res:.3e}")
        return x

    def run(spec, params, x, objective):
        s = with_params(spec, params, x)
        P = Problem(s)
        try:
            o = opts if opts is not None else default_opts(rtol=1e-10)
            u = solve(P, o)
            U = P.energy(u)
            J, w = objective(U, s)
            w = np.asarray(w, dtype=np.float64)
            if not np.any(w):
                return U, J, np.zeros(len(params))
            lam = solve(P, o, P.energy_grad(u, w))
            return U, J, P.grad(u, lam, params, w)
        finally:
            P.close()

    return run


@dataclass
class DesignResult:
    x: np.ndarray                 # optimal parameter values (physical units)
    fun: float                    # objective at x
    U: np.ndarray                 # layer energies at x
    grad: np.ndarray              # dJ/dtheta at x
    n_evals: int
    success: bool
    message: str
    history: List[Tuple[np.ndarray, float]] = field(default_factory=list)


def _scales(spec, params, x0):
    out = np.empty(len(params))
    for i, ((kind, _), v) in enumerate(zip(params, x0)):
        if kind in ("xc", "yc"):
            out[i] = spec["load"]["r0"]
        else:
            out[i] = abs(v) if v != 0 else 1.0
    return out


def optimize(spec: dict, params: Sequence[Tuple[str, int]], objective, x0: Optional[Sequence[float]] = None,
             bounds: Optional[Sequence[Tuple[Optional[float], Optional[float]]]] = None,
             constraints: Sequence[dict] = (), opts=None, method: Optional[str] = None, maxiter: int = 50,
             tol: float = 1e-10, engine: Optional[Engine] = None, callback=None) -> DesignResult:
    """Minimise objective(U(theta)) over the parameters [(kind, index)] (kinds of
    PARAM_KINDS; x0 defaults to their values in spec).  bounds and constraints
    (scipy dictionaries with 'fun' and 'jac') are in physical units.  engine
    replaces the device evaluation (tests).  Returns the optimiser's final
    point with its energies and gradient."""
    from scipy import optimize as so

    params = [tuple(p) for p in params]
    if x0 is None:
        x0 = [param_value(spec, k, i) for k, i in params]
    x0 = np.asarray(x0, dtype=np.float64)
    if len(x0) != len(params):
        raise ValueError("x0 and params differ in length")
    run = engine if engine is not None else device_engine(opts)
    sc = _scales(spec, params, x0)
    cache = {}
    hist: List[Tuple[np.ndarray, float]] = []
    J0 = [None]

    def evaluate(y):
        key = tuple(np.round(y, 15))
        if key not in cache:
            x = y * sc
            U, J, g = run(spec, params, x, objective)
            if J0[0] is None:
                J0[0] = abs(J) if J != 0 else 1.0
            cache.clear()
            cache[key] = (np.asarray(U), float(J), np.asarray(g, dtype=np.float64))
            hist.append((x.copy(), float(J)))
            if callback is not None:
                callback(x.copy(), float(J))
        return cache[key]

    def fun(y):
        _, J, g = evaluate(y)
        return J / J0[0], g * sc / J0[0]

    b = None
    if bounds is not None:
        b = [(None if lo is None else lo / s, None if hi is None else hi / s) for (lo, hi), s in zip(bounds, sc)]
    cons = []
    for c in constraints:
        f, jf = c["fun"], c["jac"]
        cons.append({"type": c["type"], "fun": (lambda y, f=f: f(y * sc)),
                     "jac": (lambda y, jf=jf: np.asarray(jf(y * sc)) * sc)})
    if method is None:
        method = "SLSQP" if cons else "L-BFGS-B"
    evaluate(x0 / sc)  # fixes the objective's normalisation
    if method == "SLSQP":
        r = so.minimize(fun, x0 / sc, jac=True, method=method, bounds=b, constraints=cons,
                        options={"maxiter": maxiter, "ftol": tol})
    else:
        if cons:
            raise ValueError(f"{method} takes no constraints")
        r = so.minimize(fun, x0 / sc, jac=True, method=method, bounds=b,
                        options={"maxiter": maxiter, "ftol": tol, "gtol": tol})
    U, J, g = evaluate(r.x)
    return DesignResult(x=r.x * sc, fun=J, U=U, grad=g, n_evals=len(hist), success=bool(r.success),
                        message=str(r.message), history=hist)
