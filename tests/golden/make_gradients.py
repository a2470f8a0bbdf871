"""Writes tests/golden/gradients.json: the oracle's adjoint gradients of the
layer-weighted energy J = sum_k w_k U_k on the coated cylinder of 40 elements
(coating 1e-3 R of 140 GPa / 0.23 on 72 GPa / 0.17 fused silica) at p = 3, with
respect to (Y_coat, nu_coat, Y_sub, nu_sub, coating thickness), from dense
solves refined with extended-precision residuals.  Used by the GPU gradient
parity tests.  Calls only the oracle and the workload descriptions.

    python tests/golden/make_gradients.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import adjoint  # noqa: E402

PARAMS = [("youngs", 1), ("poisson", 1), ("youngs", 0), ("poisson", 0), ("thickness", 0)]


def main():
    spec = W.config4()
    spec["p"] = 3
    out = {"spec": spec, "params": PARAMS, "cases": []}
    for w in ([1.0, 1.0], [1.0, 0.0]):
        t0 = time.time()
        J, g = adjoint.gradient(spec, PARAMS, w_layers=w, dense=True)
        out["cases"].append({"w_layers": w, "J": J, "dJ": [float(x) for x in g], "seconds": time.time() - t0})
        print(w, J, g.tolist(), f"{time.time() - t0:.0f}s", flush=True)
    with open(os.path.join(HERE, "gradients.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
