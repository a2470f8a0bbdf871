"""GPU: problems on an explicit 2D mesh (DGTN_DOMAIN_COLUMNS: each column's map
given as node coordinates, extruded through the layers), against the oracle
built from the same column maps.

* A u, every entry, FP64 to 1e-12 and FP32 to 2e-5 of max |A u|: a quadrilateral
  mesh of a box with randomly displaced interior vertices (degree-1 maps), and
  curved annulus sectors (degree-3 maps), with pressure, fixed and free faces.
* Rigid-body modes in the nullspace with every face free.
* Solves: the FP64-preconditioned solution satisfies the oracle's discrete
  system, the FP32-preconditioned one gives the same energies to 1e-8, and the
  undisplaced mesh gives the box description's energies to 1e-11 (its multigrid
  coarsens in degree and across layers only).
"""
import numpy as np
import pytest

import workloads as W
from oracle import dg

torch = pytest.importorskip("torch")
import paper_2111_06893_amd as dgtn  # noqa: E402

pytestmark = pytest.mark.gpu

LAYERS = [{"thickness": 0.05, "n_elem": 1, "ratio": 1.0, "material": 1},
          {"thickness": 0.6, "n_elem": 2, "ratio": 2.0, "material": 0}]
MATS = [dict(W.FUSED_SILICA), dict(W.CRYSTAL_A)]
LOAD = {"F0": 1.0, "r0": 0.25, "xc": 0.05, "yc": -0.03}


def _annulus(order, n_r=2, n_t=6, r_in=0.3, r_out=1.0):
    from oracle import lgl
    xs, _ = lgl.nodes_weights(order + 1)
    out = np.zeros((n_r * n_t, 2, order + 1, order + 1))
    for t in range(n_t):
        for s in range(n_r):
            for j in range(order + 1):
                th = 2 * np.pi * (t + 0.5 * (xs[j] + 1)) / n_t
                for i in range(order + 1):
                    r = r_in + (r_out - r_in) * (s + 0.5 * (xs[i] + 1)) / n_r
                    out[t * n_r + s, 0, j, i] = r * np.cos(th)
                    out[t * n_r + s, 1, j, i] = r * np.sin(th)
    return out


CASES = {
    "jittered_p2": lambda: W.columns_mesh(W.quad_columns(4, 3, 1.2, 0.9, jitter=0.3, seed=1), p=2,
                                          layers=LAYERS, materials=MATS, load=LOAD),
    "jittered_p5": lambda: W.columns_mesh(W.quad_columns(4, 3, 1.2, 0.9, jitter=0.3, seed=2), p=5,
                                          layers=LAYERS, materials=MATS, load=LOAD),
    "annulus_p4": lambda: W.columns_mesh(_annulus(3), order=3, p=4, layers=LAYERS, materials=MATS,
                                         load={"F0": 1.0, "r0": 0.2, "xc": 0.6, "yc": 0.1}),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_apply_on_explicit_mesh_matches_oracle(name):
    spec = CASES[name]()
    print(f"[mesh] apply {name}", flush=True)
    P = dgtn.Problem(spec)
    O = dg.Problem(spec)
    u = W.random_field(spec, seed=11)
    ref = dg.apply(O, u)
    ud = torch.from_numpy(u).cuda()
    got = P.apply(ud).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    got32 = P.apply(ud.float()).double().cpu().numpy()
    assert np.abs(got32 - ref).max() <= 2e-5 * np.abs(ref).max()
    b = P.rhs().cpu().numpy()
    bref = dg.rhs(O)
    assert np.abs(b - bref).max() <= 1e-13 * np.abs(bref).max()


def test_rigid_modes_on_explicit_mesh():
    spec = CASES["jittered_p5"]()
    spec["bc"] = {"top": W.BC_FREE, "bottom": W.BC_FREE, "side": W.BC_FREE}
    P = dgtn.Problem(spec)
    xyz = dg.Problem(spec).mesh.xyz
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    u = np.stack([-y + 0.3 * z + 1.0, x - 0.5 * z - 0.2, -0.3 * x + 0.5 * y], axis=1)   # three rotations, two shifts
    got = P.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    scale = np.abs(dg.apply(dg.Problem(spec), W.random_field(spec, 1))).max()
    assert np.abs(got).max() < 1e-13 * scale


@pytest.mark.parametrize("name", ["jittered_p5", "annulus_p4"])
def test_solve_on_explicit_mesh(name):
    spec = CASES[name]()
    print(f"[mesh] solve {name}", flush=True)
    P = dgtn.Problem(spec)
    u, st = P.solve(opts=dgtn.default_opts(64, rtol=1e-10, max_iter=4000), raise_on_noconv=False)
    assert st.rel_res < 1e-9, st.rel_res
    U = P.energy(u)
    O = dg.Problem(spec)
    b = dg.rhs(O)
    r = np.linalg.norm(b - dg.apply(O, u.cpu().numpy())) / np.linalg.norm(b)
    assert r < 1e-9, r
    u32, st32 = P.solve(opts=dgtn.default_opts(32, rtol=1e-10, max_iter=4000), raise_on_noconv=False)
    assert st32.rel_res < 1e-9
    np.testing.assert_allclose(P.energy(u32), U, rtol=1e-8)


def test_undisplaced_mesh_gives_the_box_energies():
    box = W.box(nx=4, ny=3, Lx=1.2, Ly=0.9, p=4, layers=LAYERS, materials=MATS, load=LOAD)
    cols = W.columns_mesh(W.quad_columns(4, 3, 1.2, 0.9), p=4, layers=LAYERS, materials=MATS, load=LOAD)
    out = []
    for spec in (box, cols):
        P = dgtn.Problem(spec)
        u, st = P.solve(opts=dgtn.default_opts(64, rtol=1e-11, max_iter=4000), raise_on_noconv=False)
        assert st.rel_res < 1e-9
        out.append(P.energy(u))
    np.testing.assert_allclose(out[1], out[0], rtol=1e-11)
