"""Host logic of the adaptive z-refinement loop (paper_2111_06893_amd/adapt.py):
bulk marking and layer refinement, no device needed."""
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
    assert s["layers"][1]["ratio"] == spec["layers"][1]["ratio"]
    assert spec["layers"][1]["n_elem"] != s["layers"][1]["n_elem"]      # the input is not modified
    capped = adapt.refine_layers(spec, [0, 1], factor=4, max_elem=3)
    assert all(l["n_elem"] <= 3 for l in capped["layers"])
    with pytest.raises(ValueError):
        adapt.refine_layers(spec, [0], factor=1)


def test_refine_disk_is_global_and_conforming():
    cyl = W.config1()
    assert adapt.refine_disk(cyl)["refine"] == cyl["refine"] + 1
    assert W.n_columns(adapt.refine_disk(cyl)) == 4 * W.n_columns(cyl)
    box = W.box(nx=2, ny=3)
    b2 = adapt.refine_disk(box)
    assert (b2["nx"], b2["ny"]) == (4, 6) and box["nx"] == 2
