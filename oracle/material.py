"""Oracle: constitutive relations Y^{ijkl}.

Eq. constrel_iso: Y = lambda d^ij d^kl + mu (d^ik d^jl + d^il d^jk), with the
footnote's conversions from Young's modulus and Poisson ratio,
lambda = Y nu / ((1 + nu)(1 - 2 nu)), mu = Y / (2 (1 + nu)).
Eq. constrel_cryst: cubic crystal with c11 (i=j=k=l), c12 (i=j, k=l, i != k),
c44 (i=k, j=l, i != j or i=l, j=k, i != j), crystal axes along x, y, z.

Pinned by tests: the tensor symmetries stated after eq. Hooke; the cubic tensor
with c11 = lambda + 2 mu, c12 = lambda, c44 = mu equals the isotropic one; the
footnote's inverse relations.
"""
from __future__ import annotations

import numpy as np


def lame(Y, nu):
    lam = Y * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = Y / (2.0 * (1.0 + nu))
    return lam, mu


def isotropic(lam, mu):
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def cubic(c11, c12, c44):
    Y = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    if i == j == k == l:
                        Y[i, j, k, l] = c11
                    elif i == j and k == l and i != k:
                        Y[i, j, k, l] = c12
                    elif (i == k and j == l and i != j) or (i == l and j == k and i != j):
                        Y[i, j, k, l] = c44
    return Y


def tensor(m):
    """Y^{ijkl} of a material description."""
    if m["kind"] == "iso":
        return isotropic(*lame(m["Y"], m["nu"]))
    if m["kind"] == "cubic":
        return cubic(m["c11"], m["c12"], m["c44"])
    raise ValueError(m["kind"])


def tensors(spec):
    return np.stack([tensor(m) for m in spec["materials"]])
