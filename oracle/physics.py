"""Oracle: thermal-noise relations and closed forms (Sec. 2.1).

* Eq. thermalnoise with eq. wdiss.  As printed, S_q = 2 kB T W / (pi^2 f^2 F0^2)
  with W = U phi is not dimensionally consistent; the reading taken is that the
  dissipated power is W = 2 pi f U phi (energy lost per cycle 2 pi phi U, times
  f), which gives S_x = 4 kB T sum_k phi_k U_k / (pi f F0^2).  With the layer
  split W = U_sub phi_sub + U_coat phi_coat.
* Eq. approx_analytic, the thin-coating half-space noise, transcribed as a
  formula; together with the closed-form coating energy below it pins the
  reading above (the two agree identically).
* Half-space energy under the Gaussian pressure of eq. laserbeam (derived, not
  printed in the paper): with the Boussinesq surface compliance
  2 (1 - nu^2) / (Y k) per Fourier mode, U = (1 - nu^2) F0^2 / (2 sqrt(2 pi) Y r0).
* Thin-coating energy (derived): the coating carries sigma_zz = -p and the
  in-plane strain of the substrate surface, giving
  U_coat = d F0^2 e / (2 pi r0^2),
  e = [Yc^2 (1+ns)^2 (1-2ns)^2 + Ys^2 (1+nc)^2 (1-2nc)] / (2 Ys^2 Yc (1-nc^2)).
"""
from __future__ import annotations

import numpy as np

KB = 1.380649e-23  # J/K, exact SI value


def noise_psd(U_layers, phi, T, f, F0):
    W = float(np.dot(np.asarray(U_layers, float), np.asarray(phi, float)))
    return 4.0 * KB * T * W / (np.pi * f * F0 ** 2)


def approx_analytic_coating_psd(T, f, r0, d, Ys, nus, Yc, nuc, phic):
    """Eq. approx_analytic."""
    pre = KB * T / (np.pi ** 2 * f) * (1 - nus ** 2) / (r0 * Ys) * (d / r0)
    pre *= phic / (Ys * Yc * (1 - nuc ** 2) * (1 - nus ** 2))
    br = Yc ** 2 * (1 + nus) ** 2 * (1 - 2 * nus) ** 2 + Ys ** 2 * (1 + nuc) ** 2 * (1 - 2 * nuc)
    return pre * br


def halfspace_energy(Y, nu, r0, F0=1.0):
    return (1 - nu ** 2) * F0 ** 2 / (2.0 * np.sqrt(2.0 * np.pi) * Y * r0)


def thin_coating_energy(d, r0, Ys, nus, Yc, nuc, F0=1.0):
    e = (Yc ** 2 * (1 + nus) ** 2 * (1 - 2 * nus) ** 2
         + Ys ** 2 * (1 + nuc) ** 2 * (1 - 2 * nuc)) / (2 * Ys ** 2 * Yc * (1 - nuc ** 2))
    return d * F0 ** 2 * e / (2 * np.pi * r0 ** 2)


def noise_psd_parts(U_parts, phi_parts, T, f, F0):
    """S_x with one loss angle per energy part: W = 2 pi f sum_k,p phi_kp U_kp."""
    W = float(np.sum(np.asarray(U_parts, float) * np.asarray(phi_parts, float)))
    return 4.0 * KB * T * W / (np.pi * f * F0 ** 2)
