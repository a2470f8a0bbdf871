"""Drives every host-side call of the library (no device): problem creation and
validation, workspace planning with the multigrid hierarchy and the smoother
data at overlaps 0, 1 and 2, the hierarchy introspection, node coordinates and
the pure host functions, over the benchmark workloads and a box.  Run by
tests/test_host_sanitizers.py against a build with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code:

    python tests/sanitize_driver.py path/to/libdgtn_sanitized.so
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from paper_2111_06893_amd import _lib  # noqa: E402

_lib.LIB_PATH = sys.argv[1]
import paper_2111_06893_amd as dgtn  # noqa: E402


def main():
    s7 = W.config1()
    s7["p"] = 7
    specs = [W.config1(), W.config2(), W.config4(), W.config5(p=2), s7,
             W.box(nx=3, ny=2, p=4, layers=[{"thickness": 0.3, "n_elem": 3, "ratio": 1.7, "material": 0}])]
    for sp in specs:
        P = dgtn.Problem(sp)
        for ov in (0, 1, 2):
            o = dgtn.default_opts(32, overlap=ov)
            n = P.workspace_bytes(o)
            lv = 0
            while True:
                try:
                    N, E, C = P.level_info(o, lv)
                except dgtn.DgtnError:
                    break
                P.smoother_block(o, lv, E - 1)
                P.patch_table(o, lv)
                lv += 1
        xyz = P.node_coords()
        P.close()
        print(W.n_elements(sp), n, lv, float(np.abs(xyz).max()), flush=True)
    print(dgtn.material_constants(W.COATING_ISO), dgtn.noise_psd([1e-11], [1e-4], 300.0, 100.0, 1.0))
    for bad in ({"p": 9}, {"materials": [{"kind": "iso", "Y": 1e9, "nu": 0.5}]}):
        s = W.config1()
        s.update(bad)
        try:
            dgtn.Problem(s)
            raise SystemExit("an invalid problem was accepted")
        except dgtn.DgtnError:
            pass
    print("SANITIZED HOST CALLS DONE", flush=True)


if __name__ == "__main__":
    main()
