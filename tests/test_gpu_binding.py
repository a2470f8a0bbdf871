"""GPU: the binding works whatever the caller imports first.  Torch ships its
own HIP runtime under the soname of the system one that libdgtn.so links, so
the binding loads torch before the library and the process holds one runtime.
Run in a fresh process, which loads the library before the caller imports
torch, and solves a small problem."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import paper_2111_06893_amd as dgtn
import workloads as W
dgtn._lib.load()
import torch
P = dgtn.Problem(W.config1())
u, st = P.solve(raise_on_noconv=False)
U = P.energy(u)
assert st.rel_res < 1e-6 and U.sum() > 0, (st.rel_res, U)
print("ok", flush=True)
"""


def test_library_loaded_before_torch():
    print("[binding] fresh process, library before torch", flush=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-2000:]
