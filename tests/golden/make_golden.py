"""Writes tests/golden/energies.json: the oracle's converged layer energies for
small workloads, used by the GPU solve-parity tests.  Calls only the oracle and
the workload descriptions.

    python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import dg, solve  # noqa: E402


def cases():
    out = {"config1": W.config1()}
    for s in range(10):
        out[f"config3_seed{s}"] = W.config3(seed=s)
    # thin-coating cases small enough for a dense direct solve (the block-Jacobi CG of the
    # oracle converges too slowly on 1e-3 coatings)
    c4 = W.config4()
    c4["p"] = 3
    out["config4_p3_dense"] = c4
    tc = W.config2()
    tc["refine"] = 0
    tc["p"] = 3
    tc["layers"][1]["n_elem"] = 4
    tc["layers"][1]["ratio"] = 3.0
    tc["load"]["r0"] = 0.3      # resolved by the 5-column mesh at p = 3
    out["thin_coating_p3_dense"] = tc
    return out


def run(name, spec):
    t0 = time.time()
    P = dg.Problem(spec)
    b = dg.rhs(P)
    if name.endswith("_dense"):
        # dense LU of the assembled matrix refined with the operator's own residual in
        # extended precision (oracle.solve.RefinedDense): the operator's solution to
        # the rounding of u, not that of the matrix's rounded entries
        F = solve.RefinedDense(P)
        u, rel = F.solve(b)
        u = u.reshape(P.shape)
        it = 0
    else:
        u, it, rel = solve.pcg(P, b, rtol=1e-13, maxit=60000)
    U = dg.energy_layers(P, u)
    comp = dg.compliance(P, u, b)
    return {"spec": spec, "U_layers": [float(x) for x in U], "U": float(U.sum()), "compliance": comp,
            "cg_iterations": it, "rel_residual": rel, "seconds": time.time() - t0}


def main():
    path = os.path.join(HERE, "energies.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    want = sys.argv[1:] or list(cases())
    for name, spec in cases().items():
        if name not in want:
            continue
        data[name] = run(name, spec)
        print(name, data[name]["U"], data[name]["cg_iterations"], data[name]["rel_residual"],
              f"{data[name]['seconds']:.0f}s", flush=True)
        with open(path, "w") as f:
            json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
