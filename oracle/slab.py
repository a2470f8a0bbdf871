"""Oracle: semi-analytic layered slab under the Gaussian pressure.

Independent physics reference for the pins, not a discretisation of the
paper's operator.  A laterally infinite stack of isotropic layers (eq.
constrel_iso), the top z = 0 loaded by the pressure of eq. laserbeam (times F0),
the bottom z = H fixed (eq. BCfixed).

Each 2D Fourier mode of wavenumber k is a plane-strain problem
u_x = U(z) sin kx, u_z = W(z) cos kx with s_zz = S(z) cos kx, s_xz = T(z) sin kx
(conventional stress).  Hooke's law and equilibrium give the first-order system
    U' = k W + T / mu
    W' = (S - lambda k U) / (lambda + 2 mu)
    S' = -k T
    T' = 4 mu (lambda + mu) / (lambda + 2 mu) k^2 U + lambda / (lambda + 2 mu) k S
The displacement-to-traction compliance C(z), [U, W] = C [S, T], is carried from
the fixed bottom (C = 0) to the top through sub-layers of thickness <= 1/k with
the exact propagator exp(-M dz) (a stable Riccati update); the top condition is
S = -1, T = 0 (unit pressure pushing into the material).  The energy stored in a
layer per unit mode is half the boundary work, 1/2 [S W + T U] between its
faces, and with Parseval
    U_layer = F0^2 / (2 pi) int_0^inf e^{-k^2 r0^2 / 2} e_layer(k) k dk.
The layer energies sum to the compliance 1/2 int p u_z, checked in the tests.

Pinned by tests: the half-space closed form as H grows; the thin-coating closed
form as d -> 0.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def _lame(Y, nu):
    return Y * nu / ((1 + nu) * (1 - 2 * nu)), Y / (2 * (1 + nu))


def _system(k, lam, mu):
    a = lam + 2 * mu
    return np.array([
        [0.0, k, 0.0, 1.0 / mu],
        [-lam * k / a, 0.0, 1.0 / a, 0.0],
        [0.0, 0.0, 0.0, -k],
        [4 * mu * (lam + mu) / a * k * k, 0.0, lam / a * k, 0.0],
    ])


def mode_energies(k, layers):
    """(W(0), [e_layer]) for a unit pressure mode; layers = [(t, Y, nu)]."""
    steps = []   # per sub-layer: (layer index, Q = exp(-M dz))
    for li, (t, Y, nu) in enumerate(layers):
        lam, mu = _lame(Y, nu)
        n = max(1, int(np.ceil(k * t)))
        Q = expm(-_system(k, lam, mu) * (t / n))
        steps += [(li, Q)] * n
    # upward sweep of the compliance, state order [U, W, S, T]
    C = np.zeros((2, 2))
    Cs = [C]
    for li, Q in reversed(steps):
        C = (Q[:2, :2] @ C + Q[:2, 2:]) @ np.linalg.inv(Q[2:, :2] @ C + Q[2:, 2:])
        Cs.append(C)
    Cs = Cs[::-1]            # Cs[i] = compliance at the top of sub-layer i
    t = np.array([-1.0, 0.0])
    work = []                # S W + T U at the top of each sub-layer, then bottom
    for i, (li, Q) in enumerate(steps):
        d = Cs[i] @ t
        work.append(t[0] * d[1] + t[1] * d[0])
        t = np.linalg.solve(Q[2:, :2] @ Cs[i + 1] + Q[2:, 2:], t)
    d = Cs[-1] @ t
    work.append(t[0] * d[1] + t[1] * d[0])
    W0 = (Cs[0] @ np.array([-1.0, 0.0]))[1]
    e = np.zeros(len(layers))
    for i, (li, _) in enumerate(steps):
        e[li] += 0.5 * (work[i + 1] - work[i])
    return W0, e


def energies(layers, r0, F0=1.0, n_panels=48, n_gauss=10):
    """Per-layer energies and the compliance 1/2 int p u_z of the slab."""
    kmax = 12.0 / r0
    Htot = sum(l[0] for l in layers)
    kmin = min(0.05 / Htot, kmax / 1e4)
    edges = np.concatenate(([0.0], np.geomspace(kmin, kmax, n_panels)))
    xg, wg = np.polynomial.legendre.leggauss(n_gauss)
    Ul = np.zeros(len(layers))
    comp = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        for x, w in zip(xg, wg):
            k = 0.5 * (a + b) + 0.5 * (b - a) * x
            W0, e = mode_energies(k, layers)
            wt = 0.5 * (b - a) * w * np.exp(-k * k * r0 * r0 / 2) * k * F0 ** 2 / (2 * np.pi)
            Ul += wt * e
            comp += wt * 0.5 * W0
    return Ul, comp
