"""Pins of the oracle's physics (Sec. 2.1): the noise formula, the closed forms
and the semi-analytic slab against each other."""
import numpy as np
import pytest

import workloads as W
from oracle import physics, slab


def test_noise_formula_reproduces_approx_analytic():
    """Eq. approx_analytic equals S_x = 4 kB T phi U_coat / (pi f F0^2) with the
    closed-form thin-coating energy: this pins the reading of eqs.
    thermalnoise / wdiss (dissipated power 2 pi f U phi)."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        Ys, Yc = rng.uniform(50e9, 200e9, 2)
        nus, nuc = rng.uniform(0.1, 0.4, 2)
        r0, d, T, f, phi, F0 = (rng.uniform(0.01, 0.2), rng.uniform(1e-7, 1e-4),
                                rng.uniform(10, 300), rng.uniform(10, 1000),
                                rng.uniform(1e-5, 1e-3), rng.uniform(0.5, 2))
        Uc = physics.thin_coating_energy(d, r0, Ys, nus, Yc, nuc, F0=F0)
        S = physics.noise_psd([Uc], [phi], T, f, F0)
        ref = physics.approx_analytic_coating_psd(T, f, r0, d, Ys, nus, Yc, nuc, phi)
        assert abs(S / ref - 1) < 1e-13
    # identical coating and substrate: the bracket reduces to (1 + nu)(1 - 2 nu) / Y
    e = physics.thin_coating_energy(1.0, 1.0, 80e9, 0.2, 80e9, 0.2) * 2 * np.pi
    assert abs(e - 1.2 * 0.6 / 80e9) < 1e-12 * e


def test_noise_is_independent_of_F0():
    U = np.array([2e-11, 3e-13])
    phi = np.array([1e-6, 4e-4])
    assert abs(physics.noise_psd(U * 4, phi, 290, 100, 2.0)
               / physics.noise_psd(U, phi, 290, 100, 1.0) - 1) < 1e-15


def test_slab_converges_to_halfspace_closed_form():
    Y, nu, r0 = 72e9, 0.17, 0.1
    Uh = physics.halfspace_energy(Y, nu, r0)
    assert abs(Uh - 2.690367003e-11) < 1e-19
    vals = {}
    for H in (4.0, 8.0, 16.0):
        Ul, comp = slab.energies([(H, Y, nu)], r0)
        assert abs(Ul.sum() / comp - 1) < 1e-10
        vals[H] = comp
    # deficit ~ 1/H: halves when H doubles, extrapolates to the closed form
    d1, d2 = Uh - vals[8.0], Uh - vals[16.0]
    assert 1.9 < d1 / d2 < 2.1
    rich = 2 * vals[16.0] - vals[8.0]
    assert abs(rich / Uh - 1) < 2e-4


def test_slab_thin_coating_converges_to_closed_form():
    r0 = 0.1
    devs = []
    for d in (1e-3, 1e-4, 1e-5):
        Ul, comp = slab.energies([(d, 140e9, 0.23), (16.0, 72e9, 0.17)], r0)
        assert abs(Ul.sum() / comp - 1) < 1e-10
        cf = physics.thin_coating_energy(d, r0, 72e9, 0.17, 140e9, 0.23)
        devs.append(Ul[0] / cf - 1)
    # deviation ~ -5.9 d / r0, shrinking tenfold per decade
    assert devs[2] < 0 and abs(devs[2]) < 1e-3
    assert 8 < devs[0] / devs[1] < 11 and 8 < devs[1] / devs[2] < 11


def _box_energy(H, L, n, p, side, r0=0.1):
    """Compliance 1/2 u.b and volume energy of the oracle's DG solution on a box
    of side L (n x n columns) and height H in one fused-silica element layer,
    fixed bottom, Gaussian load of width r0 at the centre of the top, sides free
    or clamped."""
    from oracle import dg, solve
    spec = W.box(nx=n, ny=n, Lx=L, Ly=L, p=p, layers=[{"thickness": H, "n_elem": 1, "ratio": 1.0, "material": 0}],
                 bc={"top": W.BC_PRESSURE, "bottom": W.BC_DIRICHLET, "side": side},
                 load={"F0": 1.0, "r0": r0, "xc": 0.0, "yc": 0.0})
    O = dg.Problem(spec)
    b = dg.rhs(O)
    u, _, rel = solve.pcg(O, b, rtol=1e-10, maxit=20000)
    assert rel < 1e-9
    return dg.compliance(O, u, b), float(dg.energy_layers(O, u).sum())


@pytest.mark.slow
def test_dg_energy_is_bracketed_by_free_and_clamped_boxes_around_the_slab():
    """The oracle's DG energy against the semi-analytic slab (Sec. 2.1, the energy U
    of the elastostatic problem under the Gaussian pressure of eq. laserbeam).

    In the continuum the compliance of a body is the maximum over admissible
    displacements v of b.v - 1/2 a(v, v).  A box with clamped sides admits fewer
    fields than the slab of the same height with the same fixed bottom (extend by
    zero), so its energy is at most the slab's; a box with free sides admits the
    slab's solution restricted to it, whose functional is at least the slab's, so
    its energy is at least the slab's.  Both hold up to the load that falls
    outside the box, a fraction below 1e-7 for a half-width of 3.5 r0 or more.
    The discrete energies must respect the bracket to within the discretisation
    error (~2e-5 at p = 4 on elements of width r0 to 2 r0), and the bracket must
    close onto the slab as the box grows relative to H: this pins the scale of
    the load, the fixed and free boundary conditions and the resolution of the
    Gaussian, none of which the algebraic pins see."""
    r0 = 0.1
    free, clamped = W.BC_FREE, W.BC_DIRICHLET
    # H = 2 r0, box 8 r0 wide: the bracket is 7.5e-4 wide and holds the slab
    _, Us = slab.energies([(2 * r0, 72e9, 0.17)], r0)
    cf, vf = _box_energy(2 * r0, 8 * r0, 4, 4, free)
    cc, vc = _box_energy(2 * r0, 8 * r0, 4, 4, clamped)
    tol = 3e-5
    assert cf / Us - 1 > -tol and cc / Us - 1 < tol, (cf / Us - 1, cc / Us - 1)
    assert (cf - cc) / Us > 3e-4
    for c, v in ((cf, vf), (cc, vc)):       # the two forms of U agree to the discretisation error
        assert abs(v / c - 1) < 2e-5
    # H = r0, box 7 r0 wide: the side effect has decayed, both boxes give the slab's energy
    _, Us1 = slab.energies([(r0, 72e9, 0.17)], r0)
    c4f, _ = _box_energy(r0, 7 * r0, 7, 4, free)
    c4c, _ = _box_energy(r0, 7 * r0, 7, 4, clamped)
    assert abs(c4f / Us1 - 1) < tol and abs(c4c / Us1 - 1) < tol, (c4f / Us1 - 1, c4c / Us1 - 1)
    # and the DG energy converges to it in p (p = 3 is about a hundred times further off)
    c3f, _ = _box_energy(r0, 7 * r0, 7, 3, free)
    assert abs(c3f / Us1 - 1) > 20 * abs(c4f / Us1 - 1)
