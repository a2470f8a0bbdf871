"""Oracle: per-element geometric factors.

Sec. 2.2.1: the Jacobian J^i_j = dx^i/dxi^j of the element map, its determinant
and inverse (J^-1)^j_i = dxi^j/dx^i.  The map is taken isoparametric: J is the
LGL derivative of the node coordinates.  Eqs. massmat / stiffmat / liftop, with
LGL quadrature (mass lumping, the reading taken for the integrals): the mass
matrix is diag(w J), the lifting operator on a face is w_face J^Sigma, with the
outward unit normal n_i = s (J^-1)^m_i / |(J^-1)^m| on the face xi^m = s and the
surface Jacobian J^Sigma = J |(J^-1)^m|.  Eq. penalty: h = 2 J / J^Sigma at each
face node, the element width normal to the face.

Pinned by tests: det J > 0, sum of w J equals the volume, normals opposite on
matched faces, h equals the exact width on affine elements.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lgl
from .mesh import FACE_DIR, FACE_SIDE, get_face


def ref_deriv(v, D, m):
    """Derivative along reference direction m (0 = xi, 1 = eta, 2 = zeta) of
    nodal values v[..., k, j, i]."""
    if m == 0:
        return np.einsum("ab,...kjb->...kja", D, v)
    if m == 1:
        return np.einsum("ab,...kbi->...kai", D, v)
    return np.einsum("ab,...bji->...aji", D, v)


def ref_deriv_T(v, D, m):
    """Transposed derivative: sum_a D[a, b] v[a] along direction m."""
    if m == 0:
        return np.einsum("ab,...kja->...kjb", D, v)
    if m == 1:
        return np.einsum("ab,...kai->...kbi", D, v)
    return np.einsum("ab,...aji->...bji", D, v)


@dataclass
class Geometry:
    N: int
    x: np.ndarray          # LGL nodes
    w: np.ndarray          # LGL weights
    D: np.ndarray          # LGL differentiation matrix
    jac: np.ndarray        # [E, 3(i), 3(j), N, N, N]  dx^i/dxi^j
    det: np.ndarray        # [E, N, N, N]
    inv: np.ndarray        # [E, 3(j), 3(i), N, N, N]  dxi^j/dx^i
    w3: np.ndarray         # [N, N, N] tensor-product weights
    # per face f: arrays on the face nodes [E, N*N]
    normal: np.ndarray     # [E, 6, 3, N*N]
    jsig: np.ndarray       # [E, 6, N*N]
    wface: np.ndarray      # [6, N*N] face quadrature weights
    h: np.ndarray          # [E, 6, N*N]


def build(mesh) -> Geometry:
    N = mesh.N
    x, w = lgl.nodes_weights(N)
    D = lgl.diff_matrix(x)
    E = mesh.xyz.shape[0]
    jac = np.zeros((E, 3, 3, N, N, N))
    for i in range(3):
        for j in range(3):
            jac[:, i, j] = ref_deriv(mesh.xyz[:, i], D, j)
    J = np.moveaxis(jac, (1, 2), (-2, -1))          # [E, N, N, N, 3, 3]
    det = np.linalg.det(J)
    inv = np.moveaxis(np.linalg.inv(J), (-2, -1), (1, 2))  # [E, 3(j), 3(i), ...]
    w3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
    normal = np.zeros((E, 6, 3, N * N))
    jsig = np.zeros((E, 6, N * N))
    h = np.zeros((E, 6, N * N))
    wface = np.zeros((6, N * N))
    w2 = np.outer(w, w).reshape(N * N)
    for f in range(6):
        m, s = FACE_DIR[f], FACE_SIDE[f]
        am = np.stack([get_face(inv[:, m, i], f, N) for i in range(3)], axis=1)  # [E, 3, NN]
        nrm = np.sqrt(np.sum(am ** 2, axis=1))
        detf = get_face(det, f, N)
        normal[:, f] = s * am / nrm[:, None, :]
        jsig[:, f] = detf * nrm
        h[:, f] = 2.0 * detf / jsig[:, f]
        wface[f] = w2
    return Geometry(N, x, w, D, jac, det, inv, w3, normal, jsig, wface, h)
