"""Pins of the oracle DG operator (Sec. 2.2) against exact algebraic and
analytic properties."""
import numpy as np
import pytest

import workloads as W
from oracle import dg, solve
from tests.manufactured import fields, X, Y, Z

TWO_LAYERS = [{"thickness": 0.5, "n_elem": 1, "ratio": 1.0, "material": 0},
              {"thickness": 0.5, "n_elem": 1, "ratio": 1.0, "material": 1}]


def small_cylinder(p=2, bc=None, materials=None, layers=None):
    spec = W.config1()
    spec["refine"] = 0
    spec["p"] = p
    if layers is not None:
        spec["layers"] = layers
    if materials is not None:
        spec["materials"] = materials
    if bc is not None:
        spec["bc"] = bc
    return spec


def test_symmetric_positive_definite_across_material_interface():
    spec = small_cylinder(p=2, layers=TWO_LAYERS, materials=[W.FUSED_SILICA, W.CRYSTAL_A])
    P = dg.Problem(spec)
    A = dg.assemble_dense(P)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev[0] > 1e-8 * ev[-1]


def test_symmetry_on_config1_random_vectors():
    P = dg.Problem(W.config1())
    u = W.random_field(W.config1(), seed=1)
    v = W.random_field(W.config1(), seed=2)
    a = np.sum(v * dg.apply(P, u))
    b = np.sum(u * dg.apply(P, v))
    scale = np.sqrt(np.sum(u * u) * np.sum(dg.apply(P, v) ** 2))
    assert abs(a - b) < 1e-14 * scale


def test_rigid_body_nullspace_all_neumann():
    free = {"top": W.BC_FREE, "bottom": W.BC_FREE, "side": W.BC_FREE}
    spec = small_cylinder(p=2, bc=free, layers=TWO_LAYERS,
                          materials=[W.FUSED_SILICA, W.CRYSTAL_B])
    P = dg.Problem(spec)
    A = dg.assemble_dense(P)
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert np.all(np.abs(ev[:6]) < 1e-13 * ev[-1])
    assert ev[6] > 1e-8 * ev[-1]
    x, y, z = (P.mesh.xyz[:, d] for d in range(3))
    o = np.ones_like(x)
    modes = [(o, 0 * o, 0 * o), (0 * o, o, 0 * o), (0 * o, 0 * o, o),
             (-y, x, 0 * o), (z, 0 * o, -x), (0 * o, -z, y)]
    Anorm = np.abs(A).max()
    for mode in modes:
        r = dg.apply(P, np.stack(mode, axis=1))
        assert np.abs(r).max() < 1e-13 * Anorm


@pytest.mark.parametrize("mat", [W.FUSED_SILICA, W.CRYSTAL_A])
@pytest.mark.parametrize("form", ["weak", "strong"])
def test_polynomial_solution_reproduced_exactly(mat, form):
    p = 3
    spec = W.box(nx=2, ny=2, p=p, Lx=1.3, Ly=0.7, materials=[mat],
                 layers=[{"thickness": 0.4, "n_elem": 1, "ratio": 1, "material": 0},
                         {"thickness": 0.6, "n_elem": 2, "ratio": 1.5, "material": 0}],
                 bc={"top": W.BC_PRESSURE, "bottom": W.BC_DIRICHLET, "side": W.BC_FREE})
    P = dg.Problem(spec)
    u = [X ** 3 * Y + Z ** 2 - 2 * X * Z, Y ** 2 * Z ** 3 - X, X * Y * Z + Z ** 3 * X ** 2]
    F, U, Tb = fields(u, mat)
    xyz = P.mesh.xyz
    uex = np.moveaxis(U(xyz[:, 0], xyz[:, 1], xyz[:, 2]), 0, 1)
    data = {"f": F, "u_b": U, "t_b": Tb}
    r = dg.residual(P, uex, data, form=form)
    b = dg.rhs(P, data)
    assert np.abs(r).max() < 1e-13 * np.abs(b).max()
    # a polynomial one degree too high is not reproduced
    u2 = [X ** 4 * Y, Y * Z, X]
    F2, U2, T2 = fields(u2, mat)
    r2 = dg.residual(P, np.moveaxis(U2(xyz[:, 0], xyz[:, 1], xyz[:, 2]), 0, 1),
                     {"f": F2, "u_b": U2, "t_b": T2}, form=form)
    assert np.abs(r2).max() > 1e-9 * np.abs(dg.rhs(P, {"f": F2, "u_b": U2, "t_b": T2})).max()


def _layered_exact(P, mats, kind):
    """Piecewise-linear, stress-continuous solution through the layers:
    uniaxial strain u_z = w(z) with Y_zzzz w' = s, or shear u_x = g(z) with
    Y_xzxz g' = s.  Returns the nodal field and the top traction datum."""
    s = 1.0e8
    zs = []
    z = 0.0
    for lay in P.spec["layers"]:
        zs.append((z, z + lay["thickness"], lay["material"]))
        z += lay["thickness"]
    H = z

    def modulus(m):
        if m["kind"] == "iso":
            lam = m["Y"] * m["nu"] / ((1 + m["nu"]) * (1 - 2 * m["nu"]))
            mu = m["Y"] / (2 * (1 + m["nu"]))
            return lam + 2 * mu if kind == "normal" else mu
        return m["c11"] if kind == "normal" else m["c44"]

    def disp(zz):
        # integrate slope s / modulus from the fixed bottom z = H upward
        out = np.zeros_like(zz)
        for (a, b, mi) in zs:
            k = s / modulus(mats[mi])
            inside = np.clip(zz, a, b)
            out += -k * (b - inside)
        return out

    xyz = P.mesh.xyz
    wz = disp(xyz[:, 2])
    u = np.zeros(P.shape)
    comp = 2 if kind == "normal" else 0

    def ub(x, y, z):
        v = np.zeros((3,) + np.shape(x))
        v[comp] = disp(z)
        return v

    def tb(x, y, z, n):
        # top face n = -z: n_i T^{ij} with T = -Y grad u; Y_{zjz?} grad = s
        v = np.zeros((3,) + np.shape(x))
        v[comp] = s * np.where(np.abs(z) < 1e-12, 1.0, 0.0)
        return v

    u[:, comp] = wz
    return u, {"u_b": ub, "t_b": tb}


@pytest.mark.parametrize("kind", ["normal", "shear"])
def test_layered_stress_continuous_solution_is_exact(kind):
    mats = [W.FUSED_SILICA, W.CRYSTAL_A, W.COATING_ISO]
    layers = [{"thickness": 0.05, "n_elem": 1, "ratio": 1, "material": 1},
              {"thickness": 0.02, "n_elem": 1, "ratio": 1, "material": 2},
              {"thickness": 0.93, "n_elem": 2, "ratio": 3.0, "material": 0}]
    spec = W.box(nx=2, ny=1, p=3, materials=mats, layers=layers,
                 bc={"top": W.BC_PRESSURE, "bottom": W.BC_DIRICHLET, "side": W.BC_DIRICHLET})
    P = dg.Problem(spec)
    u, data = _layered_exact(P, mats, kind)
    r = dg.residual(P, u, data)
    b = dg.rhs(P, data)
    # round-off amplified by the penalty C N^2 / h on the thin layers
    assert np.abs(r).max() < 1e-11 * np.abs(b).max()
    # the interior-only moduli in the traction average would break it
    Pbad = dg.Problem(spec)
    Pbad.Yel = Pbad.Yel.copy()
    # swap to a single material everywhere -> the same u is no longer a solution
    Pbad.Yel[:] = Pbad.Ymat[0]
    assert np.abs(dg.residual(Pbad, u, data)).max() > 1e-6 * np.abs(b).max()


def test_weak_equals_strong_on_affine_mesh():
    spec = W.box(nx=2, ny=2, p=4, materials=[W.FUSED_SILICA, W.CRYSTAL_A],
                 layers=[{"thickness": 0.3, "n_elem": 1, "ratio": 1, "material": 1},
                         {"thickness": 0.7, "n_elem": 2, "ratio": 2.0, "material": 0}])
    P = dg.Problem(spec)
    u = W.random_field(spec, seed=3)
    a = dg.apply(P, u, form="weak")
    b = dg.apply(P, u, form="strong")
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


def test_weak_and_strong_differ_only_by_aliasing_on_curved_wedges():
    spec = W.config1()
    spec["p"] = 4
    P = dg.Problem(spec)
    u = W.random_field(spec, seed=3)
    a = dg.apply(P, u, form="weak")
    b = dg.apply(P, u, form="strong")
    rel = np.abs(a - b).max() / np.abs(a).max()
    assert 1e-14 < rel < 1e-2


def test_cubic_with_isotropic_constants_equals_isotropic():
    iso = W.COATING_ISO
    lam = iso["Y"] * iso["nu"] / ((1 + iso["nu"]) * (1 - 2 * iso["nu"]))
    mu = iso["Y"] / (2 * (1 + iso["nu"]))
    cub = {"kind": "cubic", "c11": lam + 2 * mu, "c12": lam, "c44": mu}
    s1 = small_cylinder(p=3, materials=[iso])
    s2 = small_cylinder(p=3, materials=[cub])
    u = W.random_field(s1, seed=5)
    a = dg.apply(dg.Problem(s1), u)
    b = dg.apply(dg.Problem(s2), u)
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


def test_h_convergence_order_p_plus_1():
    """Smooth manufactured solution on refined boxes: L2 error ~ h^(p+1)."""
    p = 2
    u = [0.01 * np.e ** 0 * (X * Z + sp_sin(Y)), 0.01 * sp_cos(X + Z), 0.01 * sp_sin(X * Y + Z)]
    F, U, Tb = fields(u, W.FUSED_SILICA)
    errs = []
    for n in (1, 2, 4):
        spec = W.box(nx=n, ny=n, p=p, layers=[{"thickness": 1.0, "n_elem": n, "ratio": 1, "material": 0}],
                     bc={"top": W.BC_PRESSURE, "bottom": W.BC_DIRICHLET, "side": W.BC_FREE})
        P = dg.Problem(spec)
        data = {"f": F, "u_b": U, "t_b": Tb}
        b = dg.rhs(P, data)
        uh, it, rel = solve.pcg(P, b, rtol=1e-13)
        assert rel < 1e-12
        xyz = P.mesh.xyz
        uex = np.moveaxis(U(xyz[:, 0], xyz[:, 1], xyz[:, 2]), 0, 1)
        wJ = P.geo.w3[None] * P.geo.det
        errs.append(np.sqrt(np.sum(wJ[:, None] * (uh - uex) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 1 - 0.3, rates


def sp_sin(a):
    import sympy
    return sympy.sin(a)


def sp_cos(a):
    import sympy
    return sympy.cos(a)


def test_p_convergence_is_exponential():
    u = [0.01 * sp_sin(X + 2 * Z), 0.01 * sp_cos(Y * Z), 0.01 * sp_sin(X * Y)]
    F, U, Tb = fields(u, W.CRYSTAL_B)
    errs = []
    for p in (2, 4, 6):
        spec = W.box(nx=1, ny=1, p=p, materials=[W.CRYSTAL_B],
                     bc={"top": W.BC_PRESSURE, "bottom": W.BC_DIRICHLET, "side": W.BC_FREE})
        P = dg.Problem(spec)
        data = {"f": F, "u_b": U, "t_b": Tb}
        uh = solve.dense_solve(P, dg.rhs(P, data)) if p <= 4 else solve.pcg(P, dg.rhs(P, data))[0]
        xyz = P.mesh.xyz
        uex = np.moveaxis(U(xyz[:, 0], xyz[:, 1], xyz[:, 2]), 0, 1)
        errs.append(np.abs(uh - uex).max())
    assert errs[1] < errs[0] / 30 and errs[2] < errs[1] / 30, errs


def test_cg_equals_dense_solve():
    spec = small_cylinder(p=2, layers=TWO_LAYERS, materials=[W.FUSED_SILICA, W.COATING_ISO])
    P = dg.Problem(spec)
    b = dg.rhs(P)
    ud = solve.dense_solve(P, b)
    uc, it, rel = solve.pcg(P, b, rtol=1e-14)
    assert np.abs(ud - uc).max() < 1e-11 * np.abs(ud).max()


def test_load_vector_total_force_and_direction():
    spec = W.config1()
    P = dg.Problem(spec)
    b = dg.rhs(P)
    # pushes into the material (+z); total equals F0 (1 - exp(-R^2/r0^2)) up to quadrature
    assert np.all(b[:, 2] >= 0)
    assert abs(b[:, 0].sum()) < 1e-14 and abs(b[:, 1].sum()) < 1e-14
    assert abs(b[:, 2].sum() - 1.0) < 3e-3
    # spectral convergence of the face quadrature of the Gaussian
    spec["p"] = 9
    assert abs(dg.rhs(dg.Problem(spec))[:, 2].sum() - 1.0) < 1e-6
    spec["p"] = 11
    assert abs(dg.rhs(dg.Problem(spec))[:, 2].sum() - 1.0) < 1e-9


def test_energy_of_uniform_strain():
    """A linear field has constant strain; U = 1/2 V eps : Y : eps exactly."""
    mat = W.CRYSTAL_A
    spec = W.box(nx=2, ny=3, Lx=1.2, Ly=0.9, p=2, materials=[mat],
                 layers=[{"thickness": 0.7, "n_elem": 2, "ratio": 1, "material": 0}])
    P = dg.Problem(spec)
    x, y, z = (P.mesh.xyz[:, d] for d in range(3))
    u = np.stack([1e-3 * x + 2e-3 * y, -1e-3 * z, 3e-3 * z + 1e-3 * x], axis=1)
    eps = {(0, 0): 1e-3, (1, 1): 0.0, (2, 2): 3e-3, (0, 1): 1e-3, (1, 2): -0.5e-3, (0, 2): 0.5e-3}
    exx, eyy, ezz = eps[0, 0], eps[1, 1], eps[2, 2]
    exy, eyz, exz = eps[0, 1], eps[1, 2], eps[0, 2]
    c11, c12, c44 = mat["c11"], mat["c12"], mat["c44"]
    dens = (c11 * (exx ** 2 + eyy ** 2 + ezz ** 2) + 2 * c12 * (exx * eyy + eyy * ezz + exx * ezz)
            + 4 * c44 * (exy ** 2 + eyz ** 2 + exz ** 2))
    U = dg.energy_layers(P, u).sum()
    assert abs(U - 0.5 * dens * 1.2 * 0.9 * 0.7) < 1e-13 * U
