"""Oracle: the face-jump indicator that drives adaptive z-refinement.

Test infrastructure only, like the rest of oracle/.

The method is discontinuous across element faces and penalises the jump [u]
(Sec. 2.2.4, eq. penalty), so the size of the jumps is the natural measure of
where the discrete solution is under-resolved; Sec. 4 names adaptive mesh
refinement as the next step.  Per element e, with the face quadrature of the
operator (LGL weights times the surface Jacobian J^Sigma, identical on both
sides of a conforming face):

    eta_e^2 = sum over interior faces f of e   1/2 int_f |u_e - u_nb|^2 dS
            + sum over Dirichlet faces f of e      int_f |u_e - u_b|^2 dS   (u_b = 0)

Neumann faces contribute nothing.  Each interior face's integral is split
equally between its two elements, so sum_e eta_e^2 = sum over faces of
int |[u]|^2 dS.  The sum may be restricted to one family of faces: the side
faces across the disk or the z-faces across the layers; refinement in z acts
on the jumps of the latter only.

With weight="penalty" each face node's term is multiplied by the penalty of
eq. penalty at that node, sigma = C (p + 1)^2 / min(h_int, h_ext) (h_int on a
Dirichlet face), the weight the jump carries in the DG energy norm: a thin
layer's jumps then count in proportion to the penalty that acts on them.
"""
from __future__ import annotations

import numpy as np

from .dg import _neighbour_face, _neighbour_h
from .mesh import get_face


FACES = {"all": range(6), "side": range(4), "z": range(4, 6)}


def jump_indicator(prob, u, faces="all", weight="jump"):
    """eta_e^2 for every element of the oracle Problem `prob`, u [E, 3, N, N, N],
    over the element's faces of the family `faces`: "side" (the four faces across
    the disk, logical xi and eta), "z" (the two faces across the layers, logical
    zeta, where z-refinement acts) or "all"; weight "jump" (plain) or "penalty"
    (each term times sigma of eq. penalty)."""
    if weight not in ("jump", "penalty"):
        raise ValueError(weight)
    geo, m, N = prob.geo, prob.mesh, prob.N
    out = np.zeros(prob.E)
    for f in FACES[faces]:
        ws = geo.wface[f][None] * geo.jsig[:, f]          # w_face J^Sigma  [E, NN]
        uf = get_face(u, f, N)                             # [E, 3, NN]
        ue = _neighbour_face(prob, u, f)                   # neighbour traces (0 on boundaries)
        interior = m.nbr[:, f] >= 0
        dirichlet = m.bc[:, f] == 1
        jump2 = np.sum((uf - ue) ** 2, axis=1)             # [E, NN]
        val2 = np.sum(uf ** 2, axis=1)
        dens = np.where(interior[:, None], 0.5 * jump2, np.where(dirichlet[:, None], val2, 0.0))
        if weight == "penalty":
            hmin = np.where(interior[:, None], np.minimum(geo.h[:, f], _neighbour_h(prob, f)), geo.h[:, f])
            dens = dens * (prob.C * (prob.p + 1) ** 2 / hmin)
        out += np.sum(ws * dens, axis=1)
    return out


def layer_indicator(prob, u, faces="all", weight="jump"):
    """Per-layer sums of eta_e^2."""
    eta2 = jump_indicator(prob, u, faces, weight)
    return np.bincount(prob.mesh.layer, weights=eta2, minlength=prob.mesh.n_layers)
