"""Adaptive refinement across the layers, driven by the face-jump indicator.

Sec. 4 names adaptive mesh refinement as the way to reach a given accuracy with
fewer unknowns.  The mesh here is a 2D disk (or box) mesh extruded through the
layers, so refining in z (more elements across a layer's thickness, each old
element split into graded new ones) keeps every face conforming and needs no
mortar projections, and so does refining the whole disk mesh at once; local refinement across the disk or
per-element degrees would need them (not built).

One step:
  1. solve A u = b on the device and take the layer energies U_k;
  2. eta_e^2, the face-jump indicator of dgtn_jump_indicator over the z-faces
     (the jumps between z-elements and on the fixed face: the side-face jumps
     measure the resolution across the disk, which refinement in z leaves as it
     is), each face's squared jump weighted by the penalty sigma = C N^2 / h
     that acts on it (the jump term of the DG energy norm, so that a thin
     layer's jumps count as much as the operator makes them cost), summed per
     layer;
  3. mark the fewest layers whose indicators hold a fraction theta of the total
     (bulk marking, largest first);
  4. multiply their element counts across the thickness by `factor`, splitting
     every element of a graded layer into `factor` geometrically graded ones, so
     the new z-faces include the old ones (the refined mesh nests the old).
The jumps are what the interior penalty acts on, and they vanish for a field the
discrete space represents exactly, so they measure where u is under-resolved.
"""
from __future__ import annotations

import copy
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import Problem, default_opts

__all__ = ["mark_layers", "refine_layers", "refine_disk", "AdaptStep", "adapt"]


def mark_layers(eta_layers: Sequence[float], theta: float = 0.5) -> List[int]:
    """Indices of the fewest layers whose indicator sum reaches theta times the
    total, largest first (ties keep the lower index)."""
    eta = np.asarray(eta_layers, dtype=np.float64)
    if eta.ndim != 1 or eta.size == 0 or np.any(eta < 0) or not 0 < theta <= 1:
        raise ValueError("non-negative layer indicators and 0 < theta <= 1 expected")
    total = eta.sum()
    if total == 0:
        return []
    order = np.argsort(-eta, kind="stable")
    acc, out = 0.0, []
    for k in order:
        out.append(int(k))
        acc += eta[k]
        if acc >= theta * total:
            break
    return sorted(out)


def refine_layers(spec: dict, layers: Sequence[int], factor: int = 2, max_elem: Optional[int] = None) -> dict:
    """A copy of spec whose listed layers have `factor` times as many elements
    across their thickness.

    A layer of n elements with growth factor q between consecutive element
    thicknesses becomes n * factor elements with growth factor q**(1/factor):
    the `factor` new elements inside an old one then have the old one's
    thickness between them, so every old z-face is kept.  A layer that would
    exceed max_elem elements is left as it is (a partial split would not nest)."""
    if factor < 2:
        raise ValueError("factor must be at least 2")
    s = copy.deepcopy(spec)
    for k in layers:
        lay = s["layers"][k]
        n = lay["n_elem"] * factor
        if max_elem is not None and n > max_elem:
            continue
        lay["n_elem"] = n
        lay["ratio"] = float(lay["ratio"]) ** (1.0 / factor)
    return s


def refine_disk(spec: dict) -> dict:
    """A copy of spec refined once across the disk, everywhere: the cylinder's
    disk mesh one level finer (four times the columns), the box's columns halved
    in both directions.  Conforming, like refinement in z."""
    if spec["domain"] == "columns":
        raise ValueError("an explicit 2D mesh is not refined across the disk here")
    s = copy.deepcopy(spec)
    if s["domain"] == "cylinder":
        s["refine"] += 1
    else:
        s["nx"] *= 2
        s["ny"] *= 2
    return s


@dataclass
class AdaptStep:
    spec: dict                 # the mesh this step solved on
    n_dof: int
    U: np.ndarray              # layer energies (J)
    eta_layers: np.ndarray     # per-layer indicator sums
    marked: List[int]          # layers refined in z for the next step
    iters: int                 # Krylov iterations of the solve
    rel_res: float = 0.0       # final true relative residual of the solve
    eta_side: float = 0.0      # total side-face indicator
    action: str = ""           # "z", "disk" or "" (last step)


def adapt(spec: dict, steps: int = 4, theta: float = 0.5, factor: int = 2, opts=None, tol: Optional[float] = None,
          max_elem: Optional[int] = 64, disk: bool = False, max_dof: Optional[int] = 50_000_000,
          max_rel_res: float = 1e-8, weight: str = "penalty") -> List[AdaptStep]:
    """Solve-estimate-mark-refine for `steps` meshes (fewer if the total
    z-face indicator drops to tol, no layer can be refined further, or the
    next mesh would exceed max_dof unknowns).  With disk=True a step whose
    side-face jumps outweigh its z-face jumps refines across the disk instead
    (refine_disk), so the loop follows the direction in which the solution is
    under-resolved.  A solve that stops above rtol (at the FP64 residual floor
    of a finer mesh) is accepted up to the relative residual max_rel_res, which
    each step records: the layer energies are not stationary in u, so their
    error is of first order in the residual.  weight "penalty" (default) weights
    every face's squared jump by the penalty sigma at its nodes (the jump term of
    the DG energy norm), "jump" leaves it plain."""
    o = opts if opts is not None else default_opts(32, rtol=1e-10)
    s = copy.deepcopy(spec)
    out: List[AdaptStep] = []
    for it in range(steps):
        P = Problem(s)
        try:
            # finer meshes raise the penalty and with it the FP64 residual floor: a
            # solve that stagnates there is accepted up to max_rel_res and its
            # residual recorded, since the layer energies carry an error of first
            # order in it
            u, st = P.solve(opts=o, raise_on_noconv=False)
            if not st.converged and st.rel_res > max_rel_res:
                raise RuntimeError(f"adaptive step {it}: solve stalled at relative residual {st.rel_res:.3e}")
            U = P.energy(u)
            _, lay = P.jump_indicator(u, faces="z", weight=weight)
            side = float(P.jump_indicator(u, faces="side", weight=weight)[1].sum()) if disk else 0.0
            n_dof = int(P.info.n_dof)
        finally:
            P.close()
        last = it == steps - 1 or (tol is not None and lay.sum() <= tol)
        rr = float(st.rel_res)
        if not last and disk and side > lay.sum():
            nxt = refine_disk(s)
            if max_dof is None or _n_dof(nxt) <= max_dof:
                out.append(AdaptStep(s, n_dof, U, lay, [], int(st.iters), rr, side, "disk"))
                s = nxt
                continue
            last = True
        marked = [] if last else mark_layers(lay, theta)
        if max_elem is not None:
            marked = [k for k in marked if s["layers"][k]["n_elem"] * factor <= max_elem]
        nxt = refine_layers(s, marked, factor, max_elem) if marked else None
        if nxt is not None and max_dof is not None and _n_dof(nxt) > max_dof:
            marked, nxt = [], None
        out.append(AdaptStep(s, n_dof, U, lay, marked, int(st.iters), rr, side, "z" if marked else ""))
        if nxt is None:
            break
        s = nxt
    return out


def _n_dof(spec: dict) -> int:
    """Unknowns of a mesh description: 3 (p + 1)^3 per element."""
    if spec["domain"] == "cylinder":
        cols = 5 * 4 ** spec["refine"]
    elif spec["domain"] == "columns":
        cols = len(spec["columns"]["xy"])
    else:
        cols = spec["nx"] * spec["ny"]
    return 3 * cols * sum(l["n_elem"] for l in spec["layers"]) * (spec["p"] + 1) ** 3
