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


# the highest degree, p = 7, on a box of three elements: a cubic coating over two fused-silica
# elements, every kind of material and thickness parameter
BOX_PARAMS = [("c11", 1), ("c12", 1), ("c44", 1), ("youngs", 0), ("poisson", 0), ("thickness", 0),
              ("thickness", 1)]


def box_p7():
    return W.box(nx=1, ny=1, p=7,
                 layers=[{"thickness": 0.1, "n_elem": 1, "ratio": 1.0, "material": 1},
                         {"thickness": 0.9, "n_elem": 2, "ratio": 1.0, "material": 0}],
                 materials=[dict(W.FUSED_SILICA), dict(W.CRYSTAL_A)])


def main():
    path = os.path.join(HERE, "gradients.json")
    spec = W.config4()
    spec["p"] = 3
    out = {"spec": spec, "params": PARAMS, "cases": []}
    for w in ([1.0, 1.0], [1.0, 0.0]):
        t0 = time.time()
        J, g = adjoint.gradient(spec, PARAMS, w_layers=w, dense=True)
        out["cases"].append({"w_layers": w, "J": J, "dJ": [float(x) for x in g], "seconds": time.time() - t0})
        print(w, J, g.tolist(), f"{time.time() - t0:.0f}s", flush=True)
    spec7 = box_p7()
    w7 = [0.3, 1.7]
    t0 = time.time()
    J, g = adjoint.gradient(spec7, BOX_PARAMS, w_layers=w7, dense=True)
    out["box_p7"] = {"spec": spec7, "params": BOX_PARAMS, "w_layers": w7, "J": J, "dJ": [float(x) for x in g],
                     "seconds": time.time() - t0}
    print("box p=7", J, g.tolist(), f"{time.time() - t0:.0f}s", flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
