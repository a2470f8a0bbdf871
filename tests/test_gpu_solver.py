"""GPU checks of the preconditioner and of the Krylov solve, through the C ABI.

* One V-cycle of the library equals a NumPy V-cycle assembled from the oracle's
  operators on the same levels (fine p = 3 and coarse p = 1, or fine p = 5 and
  coarse p = 2 with an odd number of coarse unknowns, with the fine level's
  penalty, dense coarse inverse), the library's own Schwarz subdomain data and
  LGL interpolation: FP64 to 1e-10, FP32 to 1e-4.
* The FP64 solve (flexible CG, multigrid with the overlapping column-Schwarz
  smoother) reproduces the oracle's converged layer energies (stored by
  tests/golden/make_golden.py, which calls only the oracle; CG to 1e-13 on the
  isotropic cylinder, dense direct solves on the thin-coating cases) to 1e-10
  relative; the FP32-preconditioned solve, with the FP64 residual recomputed
  periodically, to 1e-8.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import dg, lgl

torch = pytest.importorskip("torch")
import paper_2111_06893_amd as dgtn  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "energies.json")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype=torch.float64)


def _golden(name):
    if not os.path.exists(GOLDEN):
        pytest.skip("golden energies not generated")
    data = json.load(open(GOLDEN))
    if name not in data:
        pytest.skip(f"no golden entry {name}")
    return data[name]


def _interp3(I, u):
    """Apply I (x) I (x) I to u[E, 3, k, j, i]."""
    u = np.einsum("ai,ecgbi->ecgba", I, u)
    u = np.einsum("bj,ecgji->ecgbi", I, u)
    return np.einsum("gk,eckji->ecgji", I, u)


def _fdm_apply(P, opts, r):
    E, _, N, _, _ = r.shape
    out = np.zeros_like(r)
    for e in range(E):
        S, lam = P.smoother_block(opts, 0, e)
        for c in range(3):
            T = np.kron(S[c][2], np.kron(S[c][1], S[c][0]))
            L = (lam[c][2][:, None, None] + lam[c][1][None, :, None] + lam[c][0][None, None, :]).ravel()
            out[e, c] = (T @ ((T.T @ r[e, c].ravel()) / L)).reshape(N, N, N)
    return out


def _vcycle_check(spec, nu, omega, n_coarse):
    """One library V-cycle (two levels, dense coarse inverse, non-overlapping
    smoother) against the same V-cycle from the oracle's operators."""
    P = dgtn.Problem(spec)
    opts = dgtn.default_opts(64, mg_levels=2, smooth_steps=nu, smooth_damping=omega, smoother=0, krylov=0)
    Nf = spec["p"] + 1
    Nc = P.level_info(opts, 1)[0]
    assert Nc == max(1, spec["p"] // 2) + 1
    v = W.random_field(spec, seed=21)
    z = P.precondition(_dev(v), opts).cpu().numpy()
    yref = P.y_ref
    Of = dg.Problem(spec)
    # the finest level's penalty on the coarse level: C Nf^2 = C' Nc^2
    coarse = dict(spec, p=Nc - 1, penalty=spec["penalty"] * (Nf / Nc) ** 2)
    Oc = dg.Problem(coarse)
    Ac = dg.assemble_dense(Oc) / yref
    assert Ac.shape[0] == n_coarse
    xf, _ = lgl.nodes_weights(Nf)
    xc, _ = lgl.nodes_weights(Nc)
    I = lgl.interp_matrix(xc, xf)

    def A(x):
        return dg.apply(Of, x) / yref

    x = omega * _fdm_apply(P, opts, v)
    for _ in range(nu - 1):
        x = x + omega * _fdm_apply(P, opts, v - A(x))
    r = v - A(x)
    rc = _interp3(I.T, r)
    ec = np.linalg.solve(Ac, rc.ravel()).reshape(rc.shape)
    x = x + _interp3(I, ec)
    for _ in range(nu):
        x = x + omega * _fdm_apply(P, opts, v - A(x))
    assert np.abs(z - x).max() <= 1e-10 * np.abs(x).max()
    opts32 = dgtn.default_opts(32, mg_levels=2, smooth_steps=nu, smooth_damping=omega, smoother=0, krylov=0)
    z32 = P.precondition(_dev(v), opts32).cpu().numpy()
    assert np.abs(z32 - x).max() <= 1e-4 * np.abs(x).max()


@pytest.mark.parametrize("nu,omega", [(1, 1.0), (2, 0.7)])
def test_vcycle_matches_numpy_reference(nu, omega):
    mats = [W.FUSED_SILICA, W.CRYSTAL_A]
    spec = W.box(nx=2, ny=2, Lx=1.0, Ly=0.7, p=3, materials=mats,
                 layers=[{"thickness": 0.05, "n_elem": 1, "ratio": 1, "material": 1},
                         {"thickness": 0.6, "n_elem": 2, "ratio": 2.0, "material": 0}])
    print(f"[solver] vcycle reference nu={nu} omega={omega}", flush=True)
    # coarse level p = 1: 12 elements x 3 x 8 = 288 unknowns (the dense product's 16-byte path)
    _vcycle_check(spec, nu, omega, 288)


def test_vcycle_odd_coarse_size():
    # fine p = 5, coarse p = 2 on three elements: 3 x 3 x 27 = 243 unknowns, an odd
    # count, so the dense coarse product takes its scalar-load path in both precisions
    mats = [W.FUSED_SILICA, W.CRYSTAL_A]
    spec = W.box(nx=1, ny=1, Lx=1.0, Ly=0.7, p=5, materials=mats,
                 layers=[{"thickness": 0.05, "n_elem": 1, "ratio": 1, "material": 1},
                         {"thickness": 0.6, "n_elem": 2, "ratio": 2.0, "material": 0}])
    print("[solver] vcycle reference, odd coarse size", flush=True)
    _vcycle_check(spec, 2, 0.7, 243)


def _solve_energy(spec, prec, floor_ok=False, compliance=False, **kw):
    P = dgtn.Problem(spec)
    opts = dgtn.default_opts(prec, **kw)
    u, st = P.solve(opts=opts, raise_on_noconv=not floor_ok)
    if floor_ok:   # stopped at the FP64 residual floor
        assert st.rel_res < 1e-9, st.rel_res
    if compliance:
        U, comp = P.energy(u, compliance=True)
        return U, st, comp
    return P.energy(u), st


# thin-coating goldens come from dense direct oracle solves refined with extended-precision
# residuals.  Their conditioning (1e-3 coating, graded substrate, penalty C N^2 / h) puts the
# FP64 residual floor near 1e-10, where an FP64-residual solve would stagnate 2e-10 away from
# the energies; the library's true residual is double-double, so its solves converge below
# that floor and every case is held to 1e-10 (the thin-coating solves may still stop on
# stagnation of the recurrence once below 1e-9, which floor_ok accepts).
GOLDEN_CASES = ["config1", "config3_seed0", "config3_seed1", "config3_seed2", "config4_p3_dense",
                "thin_coating_p3_dense"]


def _rtol(name):
    return 1e-11


@pytest.mark.parametrize("name", GOLDEN_CASES)
def test_fp64_solve_matches_oracle_energy(name):
    g = _golden(name)
    print(f"[solver] fp64 solve {name}", flush=True)
    U, st, comp = _solve_energy(g["spec"], 64, floor_ok=name.endswith("_dense"), compliance=True,
                                rtol=_rtol(name), max_iter=8000)
    ref = np.array(g["U_layers"])
    tol = 1e-10
    assert abs(U.sum() / ref.sum() - 1) < tol
    np.testing.assert_allclose(U, ref, rtol=tol)
    # the compliance form 1/2 u . b of the same solution against the oracle's
    assert abs(comp / g["compliance"] - 1) < tol, (comp, g["compliance"])


@pytest.mark.parametrize("name", GOLDEN_CASES)
def test_mixed_precision_solve_matches_oracle_energy(name):
    g = _golden(name)
    print(f"[solver] fp32-preconditioned solve {name}", flush=True)
    U, st = _solve_energy(g["spec"], 32, floor_ok=name.endswith("_dense"), rtol=_rtol(name), max_iter=8000)
    ref = np.array(g["U_layers"])
    assert abs(U.sum() / ref.sum() - 1) < 1e-8


def test_mixed_precision_solve_through_residual_replacements():
    # The Schwarz smoother alone (no coarse levels) needs more than the 50 iterations
    # after which the FP64 residual replaces the recurrence; the FP32 preconditioner
    # input is then re-derived from the replaced residual.  The energy must still
    # reach the oracle's golden value.
    g = _golden("config1")
    print("[solver] fp32-preconditioned single-level solve through residual replacements", flush=True)
    U, st = _solve_energy(g["spec"], 32, mg_levels=1, rtol=_rtol("config1"), max_iter=8000)
    assert st.iters > 50 and st.restarts >= 1, (st.iters, st.restarts)
    ref = np.array(g["U_layers"])
    assert abs(U.sum() / ref.sum() - 1) < 1e-8


def test_fgmres_and_fcg_agree_and_solve_reports_status():
    spec = W.config1()
    spec["p"] = 3
    P = dgtn.Problem(spec)
    u1, s1 = P.solve(opts=dgtn.default_opts(64, krylov=1, rtol=1e-11, max_iter=8000))
    U1 = P.energy(u1)
    u2, s2 = P.solve(opts=dgtn.default_opts(64, krylov=0, restart=60, rtol=1e-6, max_iter=20000))
    U2 = P.energy(u2)
    assert s1.converged and s2.converged
    assert abs(U2.sum() / U1.sum() - 1) < 1e-5
    # iteration cap -> DGTN_ENOCONV, reported without raising when asked
    u3, s3 = P.solve(opts=dgtn.default_opts(64, rtol=1e-11, max_iter=5), raise_on_noconv=False)
    assert not s3.converged and s3.iters == 5
    with pytest.raises(dgtn.DgtnError, match="ENOCONV"):
        P.solve(opts=dgtn.default_opts(64, rtol=1e-11, max_iter=5))


def test_extended_residual_matches_fp64_to_its_rounding():
    # on a random field the double-double residual and the FP64 one differ only by the
    # FP64 rounding of A u (no cancellation to hide it)
    spec = W.config2()
    spec["p"] = 4
    print("[solver] double-double residual against FP64 on a random field", flush=True)
    P = dgtn.Problem(spec)
    u = torch.from_numpy(W.random_field(spec, seed=4) * 1e-9).cuda()
    b = P.rhs()
    r = P.residual(u, b)
    r64 = b - P.apply(u)
    scale = float(torch.linalg.norm(r64))
    assert float(torch.linalg.norm(r - r64)) < 1e-12 * scale


@pytest.mark.parametrize("name", ["config4_p3_dense", "thin_coating_p3_dense"])
def test_solve_at_the_rounding_floor_matches_the_oracle_energies(name):
    # A u of the double-rounded exact solution is itself off by eps |A| |u| (about 1e-10
    # of |b| on a 1e-3 coating), so no solve reaches a smaller relative residual; these
    # solves end on stagnation there.  Their energies match the oracle's refined dense
    # solutions (the operator's solution to the rounding of u) to 1e-12, with the FP64
    # true residual and with the double-double one alike, and at the stagnated iterate
    # the two residuals agree: the floor is the rounding of u, not of the arithmetic.
    g = _golden(name)
    ref = np.array(g["U_layers"])
    for rp in (64, 128):
        print(f"[solver] {name}, residual precision {rp}", flush=True)
        P = dgtn.Problem(g["spec"])
        u, st = P.solve(opts=dgtn.default_opts(64, rtol=1e-14, max_iter=8000, residual_precision=rp),
                        raise_on_noconv=False)
        assert not st.converged and 1e-12 < st.rel_res < 1e-9, st.rel_res
        U = P.energy(u)
        err = float(np.max(np.abs(U / ref - 1)))
        b = P.rhs()
        r_dd = float(torch.linalg.norm(P.residual(u, b)))
        r_64 = float(torch.linalg.norm(b - P.apply(u)))
        print(f"  {st.iters} it, rel.res {st.rel_res:.2e}, residual dd/fp64 {r_dd / r_64:.4f}, "
              f"max layer energy error {err:.2e}", flush=True)
        assert err < 1e-12
        assert abs(r_dd / r_64 - 1) < 0.05
        P.close()


def test_noise_from_solved_energies():
    g = _golden("config1")
    P = dgtn.Problem(g["spec"])
    u, st = P.solve(opts=dgtn.default_opts(64, rtol=1e-11, max_iter=8000))
    U = P.energy(u)
    from oracle import physics
    S = P.noise(U, [1e-6] * len(U), 295.0, 100.0)
    assert abs(S / physics.noise_psd(g["U_layers"], [1e-6] * len(U), 295.0, 100.0, 1.0) - 1) < 1e-10


def test_overlap_on_a_single_column_equals_no_overlap():
    # one column: the patch has no neighbours, so the overlapping solve is the plain one
    spec = W.box(nx=1, ny=1, Lx=0.7, Ly=0.4, p=4,
                 layers=[{"thickness": 0.05, "n_elem": 1, "ratio": 1, "material": 1},
                         {"thickness": 0.6, "n_elem": 3, "ratio": 1.5, "material": 0}],
                 materials=[W.FUSED_SILICA, W.CRYSTAL_A])
    P = dgtn.Problem(spec)
    v = _dev(W.random_field(spec, 7))
    out = []
    for ov in (0, 2):
        o = dgtn.default_opts(64, mg_levels=1, smooth_damping=1.0, overlap=ov)
        P.bind(o)
        out.append(P.precondition(v, o).cpu().numpy())
    assert np.max(np.abs(out[0] - out[1])) < 1e-12 * np.max(np.abs(out[0]))


@pytest.mark.parametrize("overlap", [1, 2])
def test_overlapping_preconditioner_is_symmetric_positive(overlap):
    spec = W.config1()
    P = dgtn.Problem(spec)
    o = dgtn.default_opts(64, mg_levels=1, smooth_damping=1.0, overlap=overlap)
    P.bind(o)
    v = _dev(W.random_field(spec, 1))
    w = _dev(W.random_field(spec, 2))
    Mv, Mw = P.precondition(v, o), P.precondition(w, o)
    a, b = float(torch.sum(w * Mv)), float(torch.sum(v * Mw))
    assert abs(a - b) < 1e-12 * float(torch.linalg.norm(v) * torch.linalg.norm(Mw))
    assert float(torch.sum(v * Mv)) > 0 and float(torch.sum(w * Mw)) > 0


@pytest.mark.parametrize("name", ["config1", "config3_seed0"])
def test_overlapping_schwarz_cuts_iterations_and_keeps_the_energy(name):
    g = _golden(name)
    spec = g["spec"]
    P = dgtn.Problem(spec)
    its = {}
    for ov in (0, 1):
        o = dgtn.default_opts(64, rtol=1e-11, max_iter=20000, overlap=ov, mg_levels=1, smooth_damping=1.0)
        P.bind(o)
        u, st = P.solve(opts=o)
        its[ov] = st.iters
        U = P.energy(u)
        np.testing.assert_allclose(U, g["U_layers"], rtol=1e-9)
    assert its[1] * 5 < its[0], its


@pytest.mark.parametrize("prec", [64, 32])
def test_multigrid_with_overlapping_smoother(prec):
    # default preconditioner: V-cycle over p- and h-coarsened levels, weighted
    # overlapping column smoother (damping 0.65), dense coarsest solve
    g = _golden("config1")
    spec = g["spec"]
    P = dgtn.Problem(spec)
    o1 = dgtn.default_opts(prec, rtol=1e-11, max_iter=20000, mg_levels=1, smooth_damping=1.0)
    P.bind(o1)
    _, s1 = P.solve(opts=o1)
    o = dgtn.default_opts(prec, rtol=1e-11, max_iter=20000)
    P.bind(o)
    u, st = P.solve(opts=o)
    np.testing.assert_allclose(P.energy(u), g["U_layers"], rtol=1e-9 if prec == 64 else 1e-8)
    assert st.iters * 2 < s1.iters, (st.iters, s1.iters)
    # the V-cycle is a symmetric positive preconditioner
    v = _dev(W.random_field(spec, 3))
    w = _dev(W.random_field(spec, 4))
    Mv, Mw = P.precondition(v, o), P.precondition(w, o)
    a, b = float(torch.sum(w * Mv)), float(torch.sum(v * Mw))
    tol = 1e-12 if prec == 64 else 1e-5
    assert abs(a - b) < tol * float(torch.linalg.norm(v) * torch.linalg.norm(Mw))
    assert float(torch.sum(v * Mv)) > 0


def _multilayer_box():
    layers = [{"thickness": 0.01, "n_elem": 1, "ratio": 1.0, "material": 1 + (i % 2)} for i in range(12)]
    layers.append({"thickness": 0.88, "n_elem": 4, "ratio": 1.8, "material": 0})
    return W.box(nx=4, ny=4, Lx=2.0, Ly=2.0, p=3, layers=layers,
                 materials=[W.FUSED_SILICA, W.CRYSTAL_A, W.CRYSTAL_B])


def test_fiducial_layer_coarsening():
    # 16 columns x 16 z-elements: the N = 2 level still has 6144 unknowns, so the
    # hierarchy merges z-element pairs (mixed crystal pairs become effective materials)
    spec = _multilayer_box()
    P = dgtn.Problem(spec)
    o = dgtn.default_opts(64, rtol=1e-11, max_iter=4000)
    levels = []
    while True:
        try:
            levels.append(P.level_info(o, len(levels)))
        except dgtn.DgtnError:
            break
    assert levels[-1][1] < levels[-2][1], levels       # the last level merged z-elements
    P.bind(o)
    u, st = P.solve(opts=o, raise_on_noconv=False)      # runs to the FP64 residual floor
    o3 = dgtn.default_opts(64, rtol=1e-11, max_iter=4000, mg_levels=2)   # no merged layers
    P.bind(o3)
    u3, st3 = P.solve(opts=o3, raise_on_noconv=False)
    assert st.rel_res < 1e-9 and st3.rel_res < 1e-9, (st.rel_res, st3.rel_res)
    np.testing.assert_allclose(P.energy(u), P.energy(u3), rtol=1e-9)
    o8 = dgtn.default_opts(64, rtol=1e-8, max_iter=4000)
    P.bind(o8)
    _, s8 = P.solve(opts=o8)
    assert s8.iters < 60, s8.iters
    v = _dev(W.random_field(spec, 5))
    w = _dev(W.random_field(spec, 6))
    Mv, Mw = P.precondition(v, o8), P.precondition(w, o8)
    a, b = float(torch.sum(w * Mv)), float(torch.sum(v * Mw))
    assert abs(a - b) < 1e-12 * float(torch.linalg.norm(v) * torch.linalg.norm(Mw))


def test_solve_at_the_maximum_degree():
    """p = 7 (N = 8, the largest degree the kernels take) on the five-block
    cylinder: the FP64- and FP32-preconditioned solves agree on U, and the
    solution solves the oracle's discrete system (relative residual of the
    oracle's operator below 1e-9)."""
    from oracle import dg
    spec = W.config1()
    spec["p"] = 7
    print("[solve] config1 at p = 7", flush=True)
    P = dgtn.Problem(spec)
    u64, s64 = P.solve(opts=dgtn.default_opts(64, rtol=1e-10, max_iter=4000))
    u32, s32 = P.solve(opts=dgtn.default_opts(32, rtol=1e-10, max_iter=4000))
    np.testing.assert_allclose(P.energy(u32), P.energy(u64), rtol=1e-9)
    O = dg.Problem(spec)
    b = dg.rhs(O)
    r = b - dg.apply(O, u64.cpu().numpy())
    assert np.linalg.norm(r) < 1e-9 * np.linalg.norm(b)


def test_thin_coating_solve_satisfies_the_oracle_system():
    """The benchmark's workload at full size (2,058,000 DoF): the FP32-
    preconditioned solve at the benchmark's stopping tolerance and a tight FP64
    solve, checked with the oracle's operator (relative residuals) and against
    each other on U (1e-8, the mixed-precision target)."""
    from oracle import dg
    spec = W.config2()
    print("[solve] thin-coating cylinder, full size", flush=True)
    P = dgtn.Problem(spec)
    u64, _ = P.solve(opts=dgtn.default_opts(64, rtol=1e-9, max_iter=4000))
    u32, _ = P.solve(opts=dgtn.default_opts(32, rtol=1e-7, max_iter=4000))
    U64, U32 = P.energy(u64), P.energy(u32)
    assert abs(U32.sum() / U64.sum() - 1) < 1e-8
    O = dg.Problem(spec)
    b = dg.rhs(O)
    bn = np.linalg.norm(b)
    r64 = np.linalg.norm(b - dg.apply(O, u64.cpu().numpy())) / bn
    r32 = np.linalg.norm(b - dg.apply(O, u32.cpu().numpy())) / bn
    print(f"oracle residuals: FP64-preconditioned {r64:.2e}, FP32-preconditioned {r32:.2e}", flush=True)
    assert r64 < 2e-9 and r32 < 2e-7


@pytest.mark.parametrize("krylov", ["fcg", "fgmres"])
def test_fp32_preconditioner_input_is_scaled_into_range(krylov):
    """The FP32 V-cycle sees the residual times a power of two chosen from ||b||,
    and its output is divided by it.  So a load scaled by 2^-100 (entries near
    1e-30, whose small residual entries would fall below FP32's normal range)
    gives the solution scaled by exactly 2^-100, in the same iterations: before
    the scaling, such loads (the adjoint load of S_x is ~1e-27 times the layer
    energy operators) stalled the FP32-preconditioned solve near 2e-6."""
    spec = W.config4()
    spec["p"] = 3
    P = dgtn.Problem(spec)
    o = (dgtn.default_opts(32, rtol=1e-9, max_iter=4000) if krylov == "fcg" else
         dgtn.default_opts(32, krylov=0, restart=60, rtol=1e-7, max_iter=20000))
    b = P.rhs()
    u1, st1 = P.solve(b, opts=o)
    tiny = 2.0 ** -100
    u2, st2 = P.solve(b * tiny, opts=o)
    assert st2.iters == st1.iters, (st1.iters, st2.iters)
    assert torch.equal(u2, u1 * tiny)
    P.close()
