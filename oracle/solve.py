"""Oracle: solving A u = b (Sec. 2.3, eq. matrix_eqn).

A is symmetric positive definite whenever a Dirichlet face exists (weak-form
reading of the primal equation), so the oracle uses the conjugate-gradient
method preconditioned by the exact inverses of the element-diagonal blocks of A,
or a dense factorisation on tiny meshes.  Only the converged solution matters:
the paper's GMRES / multigrid / Schwarz choices change iteration counts, never
the discrete solution.

Pinned by tests: CG equals the dense solve on tiny meshes.
"""
from __future__ import annotations

import numpy as np

from . import dg


def dense_solve(prob, b):
    A = dg.assemble_dense(prob)
    return np.linalg.solve(A, b.ravel()).reshape(prob.shape)


class BlockJacobi:
    def __init__(self, prob):
        B = dg.element_blocks(prob)
        self.inv = np.linalg.inv(B)
        self.shape = prob.shape

    def __call__(self, r):
        E = self.shape[0]
        z = np.einsum("eab,eb->ea", self.inv, r.reshape(E, -1))
        return z.reshape(self.shape)


def pcg(prob, b, rtol=1e-13, maxit=20000, precond=None, x0=None, verbose=False,
        stall=400):
    """Preconditioned conjugate gradients on the oracle operator.

    Stops at the relative residual rtol, or once the residual has not halved
    in `stall` iterations (the FP64 rounding floor of the penalty-dominated
    operator lies near 1e-12).  Returns (u, iterations, final relative residual
    ||b - A u|| / ||b||)."""
    M = precond if precond is not None else BlockJacobi(prob)
    x = np.zeros(prob.shape) if x0 is None else x0.copy()
    r = b - dg.apply(prob, x)
    z = M(r)
    p = z.copy()
    rz = np.sum(r * z)
    bn = np.sqrt(np.sum(b * b))
    it = 0
    rel = np.sqrt(np.sum(r * r)) / bn
    best, best_it = rel, 0
    while rel > rtol and it < maxit and not (best < 1e-9 and it - best_it > stall):
        Ap = dg.apply(prob, p)
        alpha = rz / np.sum(p * Ap)
        x += alpha * p
        r -= alpha * Ap
        it += 1
        if it % 50 == 0:   # guard against drift of the recursive residual
            r = b - dg.apply(prob, x)
        rel = np.sqrt(np.sum(r * r)) / bn
        if rel < 0.5 * best:
            best, best_it = rel, it
        if verbose and it % 100 == 0:
            print(it, rel)
        z = M(r)
        rz_new = np.sum(r * z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    r = b - dg.apply(prob, x)
    return x, it, float(np.sqrt(np.sum(r * r)) / bn)
