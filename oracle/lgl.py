"""Oracle: one-dimensional Legendre-Gauss-Lobatto (LGL) collocation.

Sec. 2.2.1: each element carries N LGL points per dimension; fields are
Lagrange interpolants through them (eqs. field_expansion, lagrprod).

Pinned by tests: closed-form nodes for N = 2, 3, 4; quadrature exact to degree
2N - 3; differentiation exact on polynomials of degree <= N - 1; interpolation
reproduces polynomials.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as leg


def nodes_weights(n: int):
    """LGL nodes (ascending) and quadrature weights for n >= 2 points.

    Nodes: -1, +1 and the roots of P'_{n-1}.  Weights: 2 / (n (n-1) P_{n-1}(x)^2).
    """
    if n < 2:
        raise ValueError("LGL needs at least 2 points")
    p = n - 1
    c = np.zeros(p + 1)
    c[p] = 1.0
    dc = leg.legder(c)
    if p >= 2:
        inner = np.sort(np.real(leg.legroots(dc)))
        ddc = leg.legder(dc)
        for _ in range(4):  # Newton polish of the roots of P'_p
            inner = inner - leg.legval(inner, dc) / leg.legval(inner, ddc)
        x = np.concatenate(([-1.0], inner, [1.0]))
    else:
        x = np.array([-1.0, 1.0])
    Pp = leg.legval(x, c)
    w = 2.0 / (p * (p + 1) * Pp ** 2)
    return x, w


def barycentric_weights(x):
    n = len(x)
    lam = np.ones(n)
    for j in range(n):
        for m in range(n):
            if m != j:
                lam[j] /= (x[j] - x[m])
    return lam


def diff_matrix(x):
    """D[i, j] = l_j'(x_i) for the Lagrange basis through the nodes x."""
    n = len(x)
    lam = barycentric_weights(x)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, :])
    return D


def interp_matrix(x, y):
    """I[a, j] = l_j(y_a): values at points y of the Lagrange basis through x."""
    n = len(x)
    I = np.ones((len(y), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                I[:, j] *= (np.asarray(y) - x[m]) / (x[j] - x[m])
    return I
