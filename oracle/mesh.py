"""Oracle: element meshes of the layered mirror.

Sec. 2.2.1 (fig. domain_and_elements): a cylinder of radius R and height H,
z = 0 the loaded face, decomposed into a central square block wrapped by four
wedges; in z the cylinder is cut into layers of distinct material; elements are
deformed cubes with an LGL grid.  Readings taken where the paper is silent:

* the central square has half-width a = R / (2 sqrt 2), so its corners lie on
  the circle of radius R/2;
* a wedge is the linear blend, in its radial coordinate xi, between the flat
  inner edge of the square and the outer arc, which is parametrised
  equi-angularly in eta;
* h-refinement splits each block's logical square into 2^r x 2^r sub-squares;
* the z-map of every element is affine; a layer may hold several elements whose
  thicknesses grow geometrically by a stated ratio.

A layered box with affine elements is provided for exactness tests.

Face connectivity is found by matching face node coordinates, independently of
how the blocks were laid out.  Pinned by tests: matched face nodes coincide,
the volume converges to pi R^2 H, det J > 0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.spatial import cKDTree

from . import lgl

# face f -> (reference direction, side): 0 xi-, 1 xi+, 2 eta-, 3 eta+, 4 zeta-, 5 zeta+
FACE_DIR = (0, 0, 1, 1, 2, 2)
FACE_SIDE = (-1, +1, -1, +1, -1, +1)


def face_slice(f, N):
    """Index tuple selecting face f from an array [..., k, j, i]."""
    last = N - 1
    if f == 0:
        return (Ellipsis, slice(None), slice(None), 0)
    if f == 1:
        return (Ellipsis, slice(None), slice(None), last)
    if f == 2:
        return (Ellipsis, slice(None), 0, slice(None))
    if f == 3:
        return (Ellipsis, slice(None), last, slice(None))
    if f == 4:
        return (Ellipsis, 0, slice(None), slice(None))
    return (Ellipsis, last, slice(None), slice(None))


def get_face(arr, f, N):
    """Face values of arr[..., k, j, i], flattened to [..., N*N]."""
    v = arr[face_slice(f, N)]
    return v.reshape(v.shape[:-2] + (N * N,))


def add_face(arr, f, N, vals):
    """arr[face f] += vals (vals flattened [..., N*N])."""
    sl = face_slice(f, N)
    arr[sl] += vals.reshape(vals.shape[:-1] + (N, N))


def cylinder_block_map(block, R, xi, eta):
    a = R / (2.0 * np.sqrt(2.0))
    if block == 0:
        x, y = a * xi, a * eta
    else:
        th = np.pi * eta / 4.0
        x = 0.5 * (1 - xi) * a + 0.5 * (1 + xi) * R * np.cos(th)
        y = 0.5 * (1 - xi) * a * eta + 0.5 * (1 + xi) * R * np.sin(th)
        for _ in range(block - 1):  # quarter turns counter-clockwise
            x, y = -y, x
    return x, y


def columns(spec):
    """List of (xi, eta) -> (x, y) maps of the columns, in column order."""
    cols = []
    if spec["domain"] == "cylinder":
        R = spec["R"]
        m = 2 ** spec["refine"]
        for b in range(5):
            for t in range(m):
                for s in range(m):
                    def fmap(xi, eta, b=b, s=s, t=t):
                        XB = -1.0 + (s + 0.5 * (xi + 1.0)) * (2.0 / m)
                        EB = -1.0 + (t + 0.5 * (eta + 1.0)) * (2.0 / m)
                        return cylinder_block_map(b, R, XB, EB)
                    cols.append(fmap)
    elif spec["domain"] == "box":
        nx, ny, Lx, Ly = spec["nx"], spec["ny"], spec["Lx"], spec["Ly"]
        for t in range(ny):
            for s in range(nx):
                def fmap(xi, eta, s=s, t=t):
                    x = -0.5 * Lx + (s + 0.5 * (xi + 1.0)) * (Lx / nx)
                    y = -0.5 * Ly + (t + 0.5 * (eta + 1.0)) * (Ly / ny)
                    return x, y
                cols.append(fmap)
    elif spec["domain"] == "columns":
        # explicit 2D mesh: each column's map given at the LGL points of degree q,
        # taken anywhere by Lagrange interpolation through those points
        q = int(spec["columns"]["order"])
        xs, _ = lgl.nodes_weights(q + 1)
        maps = np.asarray(spec["columns"]["xy"], dtype=np.float64).reshape(-1, 2, q + 1, q + 1)

        def basis(t):
            t = np.asarray(t, dtype=np.float64)
            out = np.ones(t.shape + (q + 1,))
            for k in range(q + 1):
                for m in range(q + 1):
                    if m != k:
                        out[..., k] *= (t - xs[m]) / (xs[k] - xs[m])
            return out

        for c in range(maps.shape[0]):
            def fmap(xi, eta, m=maps[c]):
                Li, Lj = basis(xi), basis(eta)
                x = np.einsum("...i,...j,ji->...", Li, Lj, m[0])
                y = np.einsum("...i,...j,ji->...", Li, Lj, m[1])
                return x, y
            cols.append(fmap)
    else:
        raise ValueError(spec["domain"])
    return cols


def z_elements(spec):
    """[(z_lo, z_hi, layer, material)] from the loaded face downward."""
    out = []
    z = 0.0
    for li, layer in enumerate(spec["layers"]):
        n, r, t = layer["n_elem"], layer["ratio"], layer["thickness"]
        rel = np.array([r ** i for i in range(n)])
        h = t * rel / rel.sum()
        edges = z + np.concatenate(([0.0], np.cumsum(h)))
        edges[-1] = z + t
        for i in range(n):
            out.append((edges[i], edges[i + 1], li, layer["material"]))
        z = z + t
    return out


@dataclass
class Mesh:
    N: int
    xyz: np.ndarray        # [E, 3, N, N, N]
    layer: np.ndarray      # [E]
    mat: np.ndarray        # [E]
    nbr: np.ndarray        # [E, 6] neighbour element or -1
    nbr_face: np.ndarray   # [E, 6]
    perm: np.ndarray       # [E, 6, N*N] neighbour face-node index matching each own face node
    bc: np.ndarray         # [E, 6] 0 interior, else the boundary condition code
    H: float
    n_layers: int


def build(spec) -> Mesh:
    N = spec["p"] + 1
    x, _ = lgl.nodes_weights(N)
    cols = columns(spec)
    zs = z_elements(spec)
    E = len(cols) * len(zs)
    xyz = np.zeros((E, 3, N, N, N))
    layer = np.zeros(E, dtype=np.int64)
    mat = np.zeros(E, dtype=np.int64)
    XI, ETA = np.meshgrid(x, x, indexing="xy")  # XI[j, i] = x_i, ETA[j, i] = x_j
    for iz, (zlo, zhi, li, mi) in enumerate(zs):
        for c, fmap in enumerate(cols):
            e = iz * len(cols) + c
            X, Y = fmap(XI, ETA)
            xyz[e, 0] = X[None, :, :]
            xyz[e, 1] = Y[None, :, :]
            xyz[e, 2] = (zlo + 0.5 * (x + 1.0) * (zhi - zlo))[:, None, None]
            layer[e] = li
            mat[e] = mi
    H = zs[-1][1]
    nbr, nbr_face, perm, bc = connect(xyz, N, H, spec)
    return Mesh(N, xyz, layer, mat, nbr, nbr_face, perm, bc, H, len(spec["layers"]))


def connect(xyz, N, H, spec):
    """Match faces by coordinates; tag the unmatched ones by position."""
    E = xyz.shape[0]
    scale = max(np.ptp(xyz[:, 0]), np.ptp(xyz[:, 1]), np.ptp(xyz[:, 2]))
    tol = 1e-9 * scale
    fpts = np.zeros((E, 6, N * N, 3))
    for f in range(6):
        for d in range(3):
            fpts[:, f, :, d] = get_face(xyz[:, d], f, N)
    cent = fpts.mean(axis=2).reshape(E * 6, 3)
    tree = cKDTree(cent)
    nbr = -np.ones((E, 6), dtype=np.int64)
    nbr_face = -np.ones((E, 6), dtype=np.int64)
    perm = np.zeros((E, 6, N * N), dtype=np.int64)
    for a, b in tree.query_pairs(tol):
        ea, fa = divmod(a, 6)
        eb, fb = divmod(b, 6)
        if ea == eb:
            continue
        pa, pb = fpts[ea, fa], fpts[eb, fb]
        dist = np.linalg.norm(pa[:, None, :] - pb[None, :, :], axis=2)
        ab = dist.argmin(axis=1)
        ba = dist.argmin(axis=0)
        if dist[np.arange(N * N), ab].max() > tol:
            continue
        nbr[ea, fa], nbr_face[ea, fa], perm[ea, fa] = eb, fb, ab
        nbr[eb, fb], nbr_face[eb, fb], perm[eb, fb] = ea, fa, ba
    bc = np.zeros((E, 6), dtype=np.int64)
    for e in range(E):
        for f in range(6):
            if nbr[e, f] >= 0:
                continue
            z = fpts[e, f, :, 2]
            if np.all(np.abs(z) < tol):
                bc[e, f] = spec["bc"]["top"]
            elif np.all(np.abs(z - H) < tol):
                bc[e, f] = spec["bc"]["bottom"]
            else:
                bc[e, f] = spec["bc"]["side"]
    return nbr, nbr_face, perm, bc
