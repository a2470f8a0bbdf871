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
