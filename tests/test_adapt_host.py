"""Host logic of the adaptive z-refinement loop (paper_2111_06893_amd/adapt.py):
bulk marking and layer refinement, no device needed."""
import numpy as np
import pytest

import workloads as W
from paper_2111_06893_amd import adapt


def test_bulk_marking_takes_the_fewest_largest_layers():
    assert adapt.mark_layers([1.0, 5.0, 2.0, 2.0], 0.5) == [1]
    assert adapt.mark_layers([1.0, 5.0, 2.0, 2.0], 0.7) == [1, 2]      # ties: lower index first
    assert adapt.mark_layers([1.0, 5.0, 2.0, 2.0], 0.8) == [1, 2, 3]
    assert adapt.mark_layers([1.0, 5.0, 2.0, 2.0], 1.0) == [0, 1, 2, 3]
    assert adapt.mark_layers([0.0, 0.0], 0.5) == []
    with pytest.raises(ValueError):
        adapt.mark_layers([1.0, -1.0], 0.5)
    with pytest.raises(ValueError):
        adapt.mark_layers([1.0], 0.0)


def test_refine_layers_multiplies_marked_counts_only():
    spec = W.config4()
    s = adapt.refine_layers(spec, [1], factor=2)
    assert [l["n_elem"] for l in s["layers"]] == [spec["layers"][0]["n_elem"], 2 * spec["layers"][1]["n_elem"]]
    assert spec["layers"][1]["n_elem"] != s["layers"][1]["n_elem"]      # the input is not modified
    capped = adapt.refine_layers(spec, [0, 1], factor=4, max_elem=3)
    assert [l["n_elem"] for l in capped["layers"]] == [1, 1]            # a split past the cap is skipped
    with pytest.raises(ValueError):
        adapt.refine_layers(spec, [0], factor=1)


def _z_faces(spec):
    """Depths of the z-element faces of the library's mesh (host only, no device)."""
    import paper_2111_06893_amd as dgtn
    P = dgtn.Problem(spec)
    try:
        z = P.node_coords()[::W.n_columns(spec), 2]           # one column, every z-element
        return np.unique(np.round(np.r_[z[:, 0, 0, 0], z[-1, -1, 0, 0]], 14))
    finally:
        P.close()


@pytest.mark.parametrize("factor", [2, 3])
def test_refined_graded_layer_nests_the_old_mesh(factor):
    # the thin-coating workload's graded substrate (24 elements, growth 1.2158 from 2e-3):
    # every old z-face is a face of the refined mesh, and each old element is split into
    # `factor` elements, so the thinnest element shrinks by about the factor, not more
    spec = W.config2()
    spec["p"] = 1
    spec["refine"] = 0
    fine = adapt.refine_layers(spec, [1], factor=factor)
    z0, z1 = _z_faces(spec), _z_faces(fine)
    assert len(z1) == len(z0) + (factor - 1) * spec["layers"][1]["n_elem"]
    assert np.all(np.min(np.abs(z1[None, :] - z0[:, None]), axis=1) < 1e-12), "old faces lost"
    h0, h1 = np.diff(z0)[1:], np.diff(z1)[1:]
    assert np.allclose(h1.reshape(-1, factor).sum(axis=1), h0, rtol=1e-10, atol=1e-15)
    assert h1.min() > 0.9 * h0.min() / factor and h1.max() < 1.1 * h0.max() / factor * spec["layers"][1]["ratio"]


def test_refine_disk_is_global_and_conforming():
    cyl = W.config1()
    assert adapt.refine_disk(cyl)["refine"] == cyl["refine"] + 1
    assert W.n_columns(adapt.refine_disk(cyl)) == 4 * W.n_columns(cyl)
    box = W.box(nx=2, ny=3)
    b2 = adapt.refine_disk(box)
    assert (b2["nx"], b2["ny"]) == (4, 6) and box["nx"] == 2
