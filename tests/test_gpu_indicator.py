"""GPU parity of the face-jump indicator (dgtn_jump_indicator) with the oracle's
(oracle/indicator.py, pinned in tests/test_oracle_indicator.py): every element's
value and the per-layer sums on the same seeded fields, over all faces, the
side faces and the z-faces, plain and weighted by the penalty, FP64 to 1e-12
of the largest value; boxes at p = 1, 3, 7 (Dirichlet, pressure and free faces), the
curved cylinder, and the thin-coating workload at full size."""
import numpy as np
import pytest

import workloads as W
from oracle import dg, indicator

torch = pytest.importorskip("torch")
import paper_2111_06893_amd as dgtn  # noqa: E402

pytestmark = pytest.mark.gpu


def _box(p):
    return W.box(nx=2, ny=3, Lx=1.2, Ly=0.8, p=p, materials=[W.FUSED_SILICA, W.CRYSTAL_A],
                 layers=[{"thickness": 0.05, "n_elem": 1, "ratio": 1.0, "material": 1},
                         {"thickness": 0.5, "n_elem": 3, "ratio": 1.5, "material": 0}])


CASES = {"box_p1": lambda: _box(1), "box_p3": lambda: _box(3), "box_p7": lambda: _box(7),
         "cylinder_p5": W.config1, "thin_coating_full": W.config2}


@pytest.mark.parametrize("name", list(CASES))
def test_indicator_matches_oracle(name):
    spec = CASES[name]()
    print(f"[indicator] {name}", flush=True)
    u = W.random_field(spec, seed=11)
    P = dgtn.Problem(spec)
    O = dg.Problem(spec)
    ud = torch.from_numpy(u).to("cuda")
    for weight in ("jump", "penalty"):
        for faces in ("all", "side", "z"):
            eta, lay = P.jump_indicator(ud, faces, weight)
            ref = indicator.jump_indicator(O, u, faces, weight)
            assert np.abs(eta - ref).max() <= 1e-12 * np.abs(ref).max(), (faces, weight)
            np.testing.assert_allclose(lay, indicator.layer_indicator(O, u, faces, weight), rtol=1e-12)


def test_indicator_of_a_linear_field_is_the_fixed_face_integral():
    # the closed form of the oracle pin, through the library
    spec = _box(3)
    O = dg.Problem(spec)
    x, y, z = (O.node_xyz()[:, d] for d in range(3))
    u = np.stack([0.3 * x - 0.5 * z + 0.2, 0.9 * y + 1.1, -0.4 * x + 0.7 * y + 0.1 * z], axis=1)
    P = dgtn.Problem(spec)
    eta, _ = P.jump_indicator(torch.from_numpy(np.ascontiguousarray(u)).to("cuda"))
    H, Lx, Ly = z.max(), spec["Lx"], spec["Ly"]
    a, b, c0 = [0.3, 0.0, -0.4], [0.0, 0.9, 0.7], [-0.5 * H + 0.2, 1.1, 0.1 * H]
    exact = sum(a[k] ** 2 * Lx ** 3 * Ly / 12 + b[k] ** 2 * Lx * Ly ** 3 / 12 + c0[k] ** 2 * Lx * Ly
                for k in range(3))
    assert eta.sum() == pytest.approx(exact, rel=1e-12)


def test_indicator_rejects_bad_arguments():
    import ctypes
    spec = _box(1)
    P = dgtn.Problem(spec)
    u = torch.from_numpy(W.random_field(spec, seed=2)).to("cuda")
    P.jump_indicator(u)      # binds the workspace
    eta = np.zeros(P.info.n_elem)
    dp = ctypes.POINTER(ctypes.c_double)
    for faces in (0, 4, 8, 11, -1):
        st = P.lib.dgtn_jump_indicator(P.ctx, ctypes.c_void_p(u.data_ptr()), faces, eta.ctypes.data_as(dp), None,
                                       P._stream())
        assert st == -1, (faces, st)                  # DGTN_EINVAL
    st = P.lib.dgtn_jump_indicator(P.ctx, ctypes.c_void_p(u.data_ptr()), 3, None, None, P._stream())
    assert st == -1
    with pytest.raises(KeyError):
        P.jump_indicator(u, "top")
