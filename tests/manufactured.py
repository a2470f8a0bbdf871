"""Manufactured solutions for the oracle pins, derived symbolically with sympy
from the continuum equations (eq. elasticity_eqns with the isotropic or cubic
constitutive relation), independently of the oracle's discrete code."""
import numpy as np
import sympy as sp

X, Y, Z = sp.symbols("x y z", real=True)
COORDS = (X, Y, Z)


def stiffness_sym(mat):
    """Y^{ijkl} as a nested sympy list, written from the component rules of
    eqs. constrel_iso / constrel_cryst (not from the oracle)."""
    if mat["kind"] == "iso":
        E, nu = sp.nsimplify(mat["Y"]), sp.nsimplify(mat["nu"])
        mu = E / (2 * (1 + nu))
        lam = E * nu / ((1 + nu) * (1 - 2 * nu))
        c11, c12, c44 = lam + 2 * mu, lam, mu
    else:
        c11, c12, c44 = (sp.nsimplify(mat[k]) for k in ("c11", "c12", "c44"))

    def Yc(i, j, k, l):
        if i == j == k == l:
            return c11
        if i == j and k == l:
            return c12
        if (i == k and j == l) or (i == l and j == k):
            return c44
        return 0
    return Yc


def fields(u_exprs, mat):
    """Return callables f(x,y,z) -> [3, ...], u(x,y,z) -> [3, ...] and
    t(x,y,z,n) -> [3, ...] = n_i T^{ij} with T = -Y grad u."""
    Yc = stiffness_sym(mat)
    grad = [[sp.diff(u_exprs[l], COORDS[k]) for l in range(3)] for k in range(3)]
    stress = [[sum(Yc(i, j, k, l) * grad[k][l] for k in range(3) for l in range(3))
               for j in range(3)] for i in range(3)]          # Y grad u
    f = [-sum(sp.diff(stress[i][j], COORDS[i]) for i in range(3)) for j in range(3)]
    fl = sp.lambdify(COORDS, f, "numpy")
    ul = sp.lambdify(COORDS, list(u_exprs), "numpy")
    sl = sp.lambdify(COORDS, stress, "numpy")

    def bcast(vals, ref):
        return np.array([np.broadcast_to(np.asarray(v, float), np.shape(ref)) for v in vals])

    def F(x, y, z):
        return bcast(fl(x, y, z), x)

    def U(x, y, z):
        return bcast(ul(x, y, z), x)

    def Tb(x, y, z, n):
        s = sl(x, y, z)
        s = np.array([[np.broadcast_to(np.asarray(v, float), np.shape(x)) for v in row] for row in s])
        # n_i T^{ij} with T = -Y grad u
        return -np.einsum("i...,ij...->j...", n, s)

    return F, U, Tb
