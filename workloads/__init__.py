"""Problem descriptions and seeded synthetic inputs shared by the oracle and the
HIP library.

This module holds no arithmetic of the method: it only names problem
parameters (geometry, layers, materials, load, boundary conditions, resolution)
as plain dictionaries, and draws seeded random vectors.  Both the oracle and
the library build their own meshes, geometry and operators from these
descriptions.

Conventions every consumer follows (the interface both sides agree on):

* Columns.  Cylinder: block-major over the five blocks of the domain
  decomposition (0 = centre square, 1..4 = wedges at +x, +y, -x, -y), then
  within a block the 2^refine x 2^refine sub-squares with the xi index fastest:
  ``col = block * 4**refine + t * 2**refine + s``.  Box: ``col = t * nx + s``.
* z-elements are numbered from the loaded face z = 0 downward through the
  layers (layer 0 is at z = 0).  Element index ``e = iz * n_cols + col``.
* Nodes.  LGL node (i, j, k) of an element sits at reference coordinates
  (xi_i, eta_j, zeta_k); zeta = -1 is the element side nearer z = 0.
  Fields are stored ``u[e][c][k][j][i]`` (i fastest), c = x, y, z component.
* Faces: 0 = xi-, 1 = xi+, 2 = eta-, 3 = eta+, 4 = zeta-, 5 = zeta+.
* Boundary conditions: 1 = Dirichlet (u = 0), 2 = Neumann with the Gaussian
  pressure, 3 = Neumann traction-free.
"""
from __future__ import annotations

import copy

import numpy as np

BC_DIRICHLET = 1
BC_PRESSURE = 2
BC_FREE = 3

GPA = 1.0e9

FUSED_SILICA = {"kind": "iso", "Y": 72.0 * GPA, "nu": 0.17}
COATING_ISO = {"kind": "iso", "Y": 140.0 * GPA, "nu": 0.23}
CRYSTAL_A = {"kind": "cubic", "c11": 119.0 * GPA, "c12": 53.8 * GPA, "c44": 59.5 * GPA}
CRYSTAL_B = {"kind": "cubic", "c11": 120.0 * GPA, "c12": 57.0 * GPA, "c44": 58.9 * GPA}

# Geometric growth factors of the graded substrate layers: the first substrate
# element is twice as thick as the layer above it and the elements fill the rest
# of the unit height.
RATIO_CFG2 = 1.2157857156003284   # 24 elements, first 2e-3, total 0.999
RATIO_CFG5 = 1.161797272292244    # 60 elements, first 2e-5, total 1 - 4e-4


def _base(**kw):
    spec = {
        "domain": "cylinder",
        "R": 1.0,
        "refine": 1,
        "p": 5,
        "layers": [],
        "materials": [],
        "load": {"F0": 1.0, "r0": 0.1, "xc": 0.0, "yc": 0.0},
        "bc": {"top": BC_PRESSURE, "bottom": BC_DIRICHLET, "side": BC_FREE},
        "penalty": 100.0,
    }
    spec.update(kw)
    return spec


def config1():
    """Isotropic cylinder R = H = 1, 5 blocks x 2 z-layers, one horizontal
    refinement (40 elements), p = 5: 25,920 DoF."""
    return _base(
        refine=1, p=5,
        layers=[{"thickness": 0.5, "n_elem": 1, "ratio": 1.0, "material": 0},
                {"thickness": 0.5, "n_elem": 1, "ratio": 1.0, "material": 0}],
        materials=[dict(FUSED_SILICA)])


def config2():
    """Thin isotropic coating (1e-3, 140 GPa / 0.23) on the fused-silica
    substrate; 80 columns x (1 + 24 graded) = 2000 elements, p = 6:
    2,058,000 DoF."""
    return _base(
        refine=2, p=6,
        layers=[{"thickness": 1e-3, "n_elem": 1, "ratio": 1.0, "material": 1},
                {"thickness": 0.999, "n_elem": 24, "ratio": RATIO_CFG2, "material": 0}],
        materials=[dict(FUSED_SILICA), dict(COATING_ISO)])


def config3(seed=0):
    """Config-1 mesh with a seeded Gaussian width r0 in [0.05, 0.2] R."""
    spec = config1()
    rng = np.random.default_rng(seed)
    spec["load"]["r0"] = float(rng.uniform(0.05, 0.2))
    return spec


def config4(d=1e-3, Yc=140.0 * GPA, nuc=0.23, Ys=72.0 * GPA, nus=0.17):
    """Config-1 topology whose top z-layer is a coating of thickness d;
    the substrate below has thickness 1.  Parameters of the gradient:
    (Y_coat, nu_coat, Y_sub, nu_sub, d)."""
    return _base(
        refine=1, p=5,
        layers=[{"thickness": d, "n_elem": 1, "ratio": 1.0, "material": 1},
                {"thickness": 1.0, "n_elem": 1, "ratio": 1.0, "material": 0}],
        materials=[{"kind": "iso", "Y": Ys, "nu": nus},
                   {"kind": "iso", "Y": Yc, "nu": nuc}])


def config5(p=5, n_coat=40):
    """Forty alternating cubic-crystal layers of 1e-5 each on fused silica;
    80 columns x (40 + 60 graded) = 8000 elements."""
    layers = [{"thickness": 1e-5, "n_elem": 1, "ratio": 1.0, "material": 1 + (i % 2)}
              for i in range(n_coat)]
    layers.append({"thickness": 1.0 - n_coat * 1e-5, "n_elem": 60,
                   "ratio": RATIO_CFG5, "material": 0})
    return _base(refine=2, p=p, layers=layers,
                 materials=[dict(FUSED_SILICA), dict(CRYSTAL_A), dict(CRYSTAL_B)])


def box(nx=2, ny=2, Lx=1.0, Ly=1.0, layers=None, materials=None, p=3, bc=None,
        load=None):
    """Layered rectangular box [-Lx/2, Lx/2] x [-Ly/2, Ly/2] x [0, H]; affine
    elements, used for exactness and convergence checks."""
    spec = _base(domain="box", nx=nx, ny=ny, Lx=Lx, Ly=Ly, p=p)
    spec["layers"] = layers or [{"thickness": 1.0, "n_elem": 1, "ratio": 1.0, "material": 0}]
    spec["materials"] = materials or [dict(FUSED_SILICA)]
    if bc is not None:
        spec["bc"] = dict(bc)
    if load is not None:
        spec["load"] = dict(load)
    return spec


def quad_columns(nx, ny, Lx=1.0, Ly=1.0, jitter=0.0, seed=0):
    """Column maps of degree 1 of an nx x ny quadrilateral mesh of the box
    [-Lx/2, Lx/2] x [-Ly/2, Ly/2] whose interior vertices are displaced by up to
    `jitter` times the cell size (uniform, seeded): array [nx * ny, 2, 2, 2],
    entry [c, d, j, i] the coordinate d of the corner at xi = -1 + 2 i,
    eta = -1 + 2 j of column c = t * nx + s (counter-clockwise)."""
    hx, hy = Lx / nx, Ly / ny
    VX, VY = np.meshgrid(-0.5 * Lx + hx * np.arange(nx + 1), -0.5 * Ly + hy * np.arange(ny + 1), indexing="xy")
    g = np.random.default_rng(seed)
    inner = np.zeros_like(VX, dtype=bool)
    inner[1:-1, 1:-1] = True
    VX = VX + np.where(inner, jitter * hx * g.uniform(-1.0, 1.0, VX.shape), 0.0)
    VY = VY + np.where(inner, jitter * hy * g.uniform(-1.0, 1.0, VY.shape), 0.0)
    out = np.zeros((nx * ny, 2, 2, 2))
    for t in range(ny):
        for s in range(nx):
            for j in range(2):
                for i in range(2):
                    out[t * nx + s, 0, j, i] = VX[t + j, s + i]
                    out[t * nx + s, 1, j, i] = VY[t + j, s + i]
    return out


def columns_mesh(xy, order=1, layers=None, materials=None, p=3, bc=None, load=None):
    """Problem on an explicit 2D mesh: xy [n_columns, 2, order + 1, order + 1],
    each column's map at the LGL points of degree `order` (see quad_columns),
    extruded through the layers."""
    spec = _base(domain="columns", refine=0, p=p)
    spec["columns"] = {"order": int(order), "xy": np.asarray(xy, dtype=np.float64)}
    spec["layers"] = layers or [{"thickness": 1.0, "n_elem": 1, "ratio": 1.0, "material": 0}]
    spec["materials"] = materials or [dict(FUSED_SILICA)]
    if bc is not None:
        spec["bc"] = dict(bc)
    if load is not None:
        spec["load"] = dict(load)
    return spec


def with_overrides(spec, **kw):
    out = copy.deepcopy(spec)
    out.update(kw)
    return out


CONFIGS = {"config1": config1, "config2": config2, "config3": config3,
           "config4": config4, "config5": config5}


def n_columns(spec):
    if spec["domain"] == "cylinder":
        return 5 * 4 ** spec["refine"]
    if spec["domain"] == "columns":
        return len(spec["columns"]["xy"])
    return spec["nx"] * spec["ny"]


def n_elements(spec):
    return n_columns(spec) * sum(l["n_elem"] for l in spec["layers"])


def n_dof(spec):
    N = spec["p"] + 1
    return 3 * n_elements(spec) * N ** 3


def field_shape(spec):
    N = spec["p"] + 1
    return (n_elements(spec), 3, N, N, N)


def random_field(spec, seed=0, dtype=np.float64):
    """Seeded displacement field, uniform in [-1, 1], in the storage layout."""
    g = np.random.default_rng(seed)
    return g.uniform(-1.0, 1.0, size=field_shape(spec)).astype(dtype)
