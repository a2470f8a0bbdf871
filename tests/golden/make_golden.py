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
    out = {"config1": W.config1(), "config4": W.config4()}
    for s in range(3):
        out[f"config3_seed{s}"] = W.config3(seed=s)
    small = W.config2()
    small["refine"] = 1
    small["p"] = 3
    small["layers"][1]["n_elem"] = 6
    small["layers"][1]["ratio"] = 2.5
    out["thin_coating_small"] = small
    return out


def run(name, spec):
    t0 = time.time()
    P = dg.Problem(spec)
    b = dg.rhs(P)
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
