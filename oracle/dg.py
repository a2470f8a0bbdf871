"""Oracle: the DG elasticity operator, load vector and energies.

Follows Sec. 2.2.2 - 2.2.4 step by step, in FP64, over all elements at once.

Auxiliary strain (Sec. 2.2.2):
    S_kl = D_(k u_l) + L ((n_(k u_l))* - n_(k u_l)),
with D_k the chain-rule derivative on the nodal values and L = M^-1 ML the
lifting operator (diagonal with LGL quadrature: w_face J^Sigma / (w J) on face
nodes).  Eq. numfluxaux with n_ext = -n_int gives
    (n_(k u_l))* - n_(k u_l)^int = -1/2 n_(k [u]_l),   [u] = u_int - u_ext.

Primal residual, eq. dg_residuals, with T = Y S (the minus sign of eq. Hooke is
carried by the operator):
    strong form   -M D_i T^{ij} - ML ((n_i Y S)* - n_i Y S) = M f^j,
    weak form     sum_m Dhat_m^T [w J (J^-1)^m_i T^{ij}] - ML (n_i Y S)* = M f^j,
identical on affine elements by LGL summation by parts.  The weak form is the
reading used for the operator (it keeps A exactly symmetric on curved
elements); the strong form is kept for the equivalence check.

Numerical flux, eq. numfluxprimal with averaged moduli (eq. constrel_avg):
    (n_i Y S)* = 1/2 n_i (Y_int D u_int + Y_ext D u_ext)^{ij}
                 - sigma n_i Y_*^{ijkl} n_k [u]_l,
    sigma = C (max(p_int, p_ext) + 1)^2 / min(h_int, h_ext)   (eq. penalty).
Boundary conditions, eq. bc: Dirichlet faces take [u] = 2 (u_int - u_b) and the
interior stress; Neumann faces take no jump and (n_i Y S)* = -n_i T_b^{ij}.
Thermal-noise data: n_i T_b^{ij} = n^j p(r) on z = 0 with p of eq. laserbeam
scaled by F0, u_b = 0 on z = H, zero traction on the mantle.

Energy: U = -1/2 int S_ij T^ij dV = 1/2 int D_(i u_j) Y^{ijkl} D_(k u_l) dV with
the unlifted strain, LGL quadrature, summed per layer; and the same integral
split by elastic modulus (Sec. 2.1 allows one loss angle per modulus):
isotropic bulk / shear, cubic c11 / c12 / c44 parts.

Pinned by tests: symmetry, positive definiteness with a Dirichlet face, the
six-mode rigid-body nullspace, exact reproduction of polynomial and of layered
stress-continuous solutions, weak = strong on affine meshes, cubic = isotropic,
O(h^{p+1}) convergence, total force of the load, energy of a uniform strain;
energy parts: they sum to U, closed forms of the parts for uniform dilatation,
shear and uniaxial strains.
"""
from __future__ import annotations

import numpy as np

from . import geometry, material, mesh as mesh_mod
from .geometry import ref_deriv, ref_deriv_T
from .mesh import get_face, add_face

HOMOGENEOUS = "homogeneous"


class Problem:
    def __init__(self, spec):
        self.spec = spec
        self.mesh = mesh_mod.build(spec)
        self.geo = geometry.build(self.mesh)
        self.Ymat = material.tensors(spec)
        self.Yel = self.Ymat[self.mesh.mat]          # [E, 3, 3, 3, 3]
        self.C = float(spec["penalty"])
        self.p = spec["p"]
        self.N = self.mesh.N
        self.E = self.mesh.xyz.shape[0]

    @property
    def shape(self):
        return (self.E, 3, self.N, self.N, self.N)

    def node_xyz(self):
        return self.mesh.xyz


def gradient(prob, u):
    """G[e, k, l] = D_k u_l at every node."""
    D = prob.geo.D
    du = np.stack([ref_deriv(u, D, m) for m in range(3)], axis=1)   # [E, m, l, ...]
    return np.einsum("emk...,eml...->ekl...", prob.geo.inv, du)


def contract(Y, S):
    """T^{ij} = Y^{ijkl} S_kl elementwise; Y [E, 3,3,3,3], S [E, 3, 3, ...]."""
    return np.einsum("eijkl,ekl...->eij...", Y, S)


def sym(G):
    return 0.5 * (G + np.swapaxes(G, 1, 2))


def gaussian_pressure(spec, x, y):
    ld = spec["load"]
    r2 = (x - ld["xc"]) ** 2 + (y - ld["yc"]) ** 2
    return ld["F0"] * np.exp(-r2 / ld["r0"] ** 2) / (np.pi * ld["r0"] ** 2)


def _neighbour_face(prob, arr, f):
    """Values of arr[e', ...] at the face nodes of each element's neighbour
    across face f, reordered to the element's own face-node order.
    arr [E, A..., N, N, N] -> [E, A..., N*N] (zeros where there is no neighbour)."""
    N = prob.N
    m = prob.mesh
    E = prob.E
    allf = np.stack([get_face(arr, g, N) for g in range(6)], axis=1)   # [E, 6, A..., NN]
    nb = m.nbr[:, f]
    ok = nb >= 0
    out = np.zeros(allf.shape[:1] + allf.shape[2:], dtype=allf.dtype)
    src = allf[nb[ok], m.nbr_face[ok, f]]                              # [E', A..., NN]
    idx = m.perm[ok, f]
    idx = idx.reshape((idx.shape[0],) + (1,) * (src.ndim - 2) + (idx.shape[1],))
    out[ok] = np.take_along_axis(src, np.broadcast_to(idx, src.shape), axis=-1)
    return out


def residual(prob, u, data=None, form="weak", couple=True):
    """A u - b for the boundary/source data `data`.

    data = HOMOGENEOUS gives A u.  data = None is the thermal-noise problem.
    Otherwise a dict with optional callables 'f'(x, y, z) -> [3, ...] (source of
    eq. elasticity_eqns), 'u_b'(x, y, z) -> [3, ...] on Dirichlet faces and
    't_b'(x, y, z, n) -> [3, ...] giving n_i T_b^{ij} on Neumann faces
    (n is passed component-first, [3, ...]).
    couple=False drops the neighbours' values (the element-diagonal block of A).
    """
    geo, m, spec = prob.geo, prob.mesh, prob.spec
    N, Y, C = prob.N, prob.Yel, prob.C
    if u is None:
        u = np.zeros(prob.shape)
    G = gradient(prob, u)                       # unlifted derivative
    S = sym(G).copy()
    wJ = geo.w3[None] * geo.det                 # mass matrix diagonal
    xyz = m.xyz
    jumps, fluxes = [], []
    for f in range(6):
        n = geo.normal[:, f]                    # [E, 3, NN]
        ws = geo.wface[f][None] * geo.jsig[:, f]  # w_face J^Sigma  [E, NN]
        uf = get_face(u, f, N)                  # [E, 3, NN]
        Gf = get_face(G, f, N)                  # [E, 3, 3, NN]
        t_int = np.einsum("ei...,eijkl,ekl...->ej...", n, Y, Gf)
        interior = m.nbr[:, f] >= 0
        bc = m.bc[:, f]
        jump = np.zeros_like(uf)
        flux = np.zeros_like(uf)
        # interior faces
        if np.any(interior):
            if couple:
                ue = _neighbour_face(prob, u, f)
                Ge = _neighbour_face(prob, G, f)
            else:
                ue = np.zeros_like(uf)
                Ge = np.zeros_like(Gf)
            Ye = prob.Yel[np.where(interior, m.nbr[:, f], 0)]
            he = _neighbour_h(prob, f)
            hmin = np.where(interior[:, None], np.minimum(geo.h[:, f], he), geo.h[:, f])
            sigma = C * (prob.p + 1) ** 2 / hmin
            Ystar = 0.5 * (Y + Ye)
            t_ext = np.einsum("ei...,eijkl,ekl...->ej...", n, Ye, Ge)
            jmp = uf - ue
            pen = sigma[:, None] * np.einsum("ei...,eijkl,ek...,el...->ej...", n, Ystar, n, jmp)
            sel = interior[:, None, None]
            jump = np.where(sel, jmp, jump)
            flux = np.where(sel, 0.5 * (t_int + t_ext) - pen, flux)
        # Dirichlet faces
        dmask = bc == 1
        if np.any(dmask):
            ub = np.zeros_like(uf)
            if isinstance(data, dict) and "u_b" in data:
                ub = np.moveaxis(np.asarray(
                    data["u_b"](*[get_face(xyz[:, d], f, N) for d in range(3)])), 0, 1)
            jmp = 2.0 * (uf - ub)
            sigma = C * (prob.p + 1) ** 2 / geo.h[:, f]
            pen = sigma[:, None] * np.einsum("ei...,eijkl,ek...,el...->ej...", n, Y, n, jmp)
            sel = dmask[:, None, None]
            jump = np.where(sel, jmp, jump)
            flux = np.where(sel, t_int - pen, flux)
        # Neumann faces: (n Y S)* = -n_i T_b^{ij}
        nmask = (bc == 2) | (bc == 3)
        if np.any(nmask) and data is not HOMOGENEOUS:
            tb = np.zeros_like(uf)
            fx = [get_face(xyz[:, d], f, N) for d in range(3)]
            if isinstance(data, dict):
                if "t_b" in data:
                    tb = np.moveaxis(np.asarray(
                        data["t_b"](*fx, np.moveaxis(n, 1, 0))), 0, 1)
            else:
                p = gaussian_pressure(spec, fx[0], fx[1])
                tb = np.where((bc == 2)[:, None, None], n * p[:, None, :], 0.0)
            flux = np.where(nmask[:, None, None], -tb, flux)
        jumps.append(jump)
        fluxes.append(flux)
        # lift of the auxiliary-variable flux into S at this face's nodes
        lift_scale = ws / get_face(wJ, f, N)
        dS = -0.5 * lift_scale[:, None, None, :] * 0.5 * (
            n[:, :, None, :] * jump[:, None, :, :] + n[:, None, :, :] * jump[:, :, None, :])
        add_face(S, f, N, dS)
    T = contract(Y, S)                          # [E, i, j, ...]
    if form == "weak":
        r = np.zeros(prob.shape, dtype=T.dtype)
        for mdir in range(3):
            Fm = wJ[:, None] * np.einsum("ei...,eij...->ej...", geo.inv[:, mdir], T)
            r += ref_deriv_T(Fm, geo.D, mdir)
        for f in range(6):
            ws = geo.wface[f][None] * geo.jsig[:, f]
            add_face(r, f, N, -ws[:, None, :] * fluxes[f])
    elif form == "strong":
        divT = np.zeros(prob.shape, dtype=T.dtype)
        for mdir in range(3):
            dT = ref_deriv(T, geo.D, mdir)                 # [E, i, j, ...]
            divT += np.einsum("ei...,eij...->ej...", geo.inv[:, mdir], dT)
        r = -wJ[:, None] * divT
        for f in range(6):
            n = geo.normal[:, f]
            ws = geo.wface[f][None] * geo.jsig[:, f]
            nT = np.einsum("ei...,eij...->ej...", n, get_face(T, f, N))
            add_face(r, f, N, -ws[:, None, :] * (fluxes[f] - nT))
    else:
        raise ValueError(form)
    if isinstance(data, dict) and "f" in data:
        fv = data["f"](xyz[:, 0], xyz[:, 1], xyz[:, 2])     # [3, E, ...]
        r -= wJ[:, None] * np.moveaxis(np.asarray(fv), 0, 1)
    return r


def _neighbour_h(prob, f):
    """Normal width h of the neighbour across face f at the matching nodes."""
    m = prob.mesh
    nb = m.nbr[:, f]
    ok = nb >= 0
    out = np.zeros((prob.E, prob.N * prob.N))
    src = prob.geo.h[nb[ok], m.nbr_face[ok, f]]
    out[ok] = np.take_along_axis(src, m.perm[ok, f], axis=-1)
    return out


def apply(prob, u, form="weak", couple=True):
    """A u, in the floating-point type of u (float64, or numpy's extended
    longdouble for the residuals of iterative refinement)."""
    return residual(prob, u, HOMOGENEOUS, form=form, couple=couple)


def rhs(prob, data=None):
    """b, so that A u = b is the discrete problem for `data`."""
    return -residual(prob, None, data)


def energy_layers(prob, u):
    """U_k = 1/2 sum over the elements of layer k of w J D_(i u_j) Y D_(k u_l)."""
    G = gradient(prob, u)
    Su = sym(G)
    dens = np.einsum("eij...,eijkl,ekl...->e...", Su, prob.Yel, Su)
    wJ = prob.geo.w3[None] * prob.geo.det
    per_el = 0.5 * np.sum(wJ * dens, axis=(1, 2, 3))
    out = np.zeros(prob.mesh.n_layers, dtype=per_el.dtype)
    np.add.at(out, prob.mesh.layer, per_el)
    return out


def compliance(prob, u, b):
    """1/2 u . b."""
    return 0.5 * float(np.sum(u * b))


def assemble_dense(prob, form="weak"):
    """A as a dense matrix, column by column (tiny meshes only)."""
    n = int(np.prod(prob.shape))
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        A[:, j] = apply(prob, e.reshape(prob.shape), form=form).ravel()
    return A


def element_blocks(prob):
    """Diagonal blocks of A, one dense [3N^3, 3N^3] matrix per element."""
    nloc = 3 * prob.N ** 3
    B = np.zeros((prob.E, nloc, nloc))
    e = np.zeros((prob.E, nloc))
    for j in range(nloc):
        e[:] = 0.0
        e[:, j] = 1.0
        B[:, :, j] = apply(prob, e.reshape(prob.shape), couple=False).reshape(prob.E, nloc)
    return B


def _part_tensors(m):
    """Stiffness tensors of the parts of one material's energy (they sum to Y).

    Sec. 2.1 notes that each independent elastic modulus may carry its own loss
    angle.  Isotropic (eq. constrel_iso): bulk K d^ij d^kl with K = lambda + 2 mu / 3,
    and shear mu (d^ik d^jl + d^il d^jk - 2/3 d^ij d^kl).  Cubic (eq.
    constrel_cryst): the c11, c12 and c44 terms separately.  A third zero part
    pads the isotropic case."""
    d = np.eye(3)
    if m["kind"] == "iso":
        lam, mu = material.lame(m["Y"], m["nu"])
        K = lam + 2.0 * mu / 3.0
        dd = np.einsum("ij,kl->ijkl", d, d)
        bulk = K * dd
        shear = mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d) - 2.0 / 3.0 * dd)
        return [bulk, shear, np.zeros((3, 3, 3, 3))]
    return [material.cubic(m["c11"], 0.0, 0.0), material.cubic(0.0, m["c12"], 0.0),
            material.cubic(0.0, 0.0, m["c44"])]


def energy_parts(prob, u):
    """[n_layers, 3]: U_k split by modulus (isotropic: bulk, shear, 0; cubic:
    c11, c12, c44 parts), each 1/2 sum w J D_(i u_j) Y_part D_(k u_l)."""
    G = gradient(prob, u)
    Su = sym(G)
    wJ = prob.geo.w3[None] * prob.geo.det
    out = np.zeros((prob.mesh.n_layers, 3))
    parts = [_part_tensors(m) for m in prob.spec["materials"]]
    for p in range(3):
        Yp = np.stack([parts[mi][p] for mi in range(len(parts))])[prob.mesh.mat]
        dens = np.einsum("eij...,eijkl,ekl...->e...", Su, Yp, Su)
        per_el = 0.5 * np.sum(wJ * dens, axis=(1, 2, 3))
        np.add.at(out[:, p], prob.mesh.layer, per_el)
    return out
