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


class RefinedDense:
    """Solves the operator's equation A x = b with the dense LU of its assembled
    matrix as the approximate inverse and iterative refinement whose residual
    b - A x is the operator itself (dg.apply) evaluated in extended precision
    (numpy longdouble).

    The assembled matrix is the operator applied to unit vectors in FP64, so
    each of its large interior-penalty entries (C N^2 / h on a thin layer)
    carries its own rounding; the exact solution of those rounded entries
    differs from the operator's by about 1e-10 in the energies of a 1e-3
    coating.  With the operator's extended-precision residual the refined x is
    the operator's solution to the rounding of x."""

    def __init__(self, prob, A=None):
        import scipy.linalg as sla
        self._sla = sla
        self.prob = prob
        self.lu = sla.lu_factor(dg.assemble_dense(prob) if A is None else A)

    def residual(self, b, x):
        """b - A x in extended precision."""
        xl = np.asarray(x, dtype=np.float64).reshape(self.prob.shape).astype(np.longdouble)
        return np.asarray(b, dtype=np.float64).ravel().astype(np.longdouble) - dg.apply(self.prob, xl).ravel()

    def solve(self, b, max_refine=8):
        """(x, relative residual of x computed in extended precision)."""
        bf = np.asarray(b, dtype=np.float64).ravel()
        x = self._sla.lu_solve(self.lu, bf)
        for _ in range(max_refine):
            d = self._sla.lu_solve(self.lu, self.residual(bf, x).astype(np.float64))
            x = (x.astype(np.longdouble) + d.astype(np.longdouble)).astype(np.float64)
            if np.linalg.norm(d) <= 1e-16 * np.linalg.norm(x):
                break
        r = self.residual(bf, x)
        return x, float(np.linalg.norm(r.astype(np.float64)) / np.linalg.norm(bf))


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
