"""V-cycles replayed from a recorded HIP graph against eager V-cycles.

The library records the level-0 V-cycle once per precision and smoother
setting and replays it on the caller's stream.  A second problem created with
DGTN_NO_GRAPHS set runs every V-cycle eagerly.  Both launch the same kernels in
the same order, so every replay must agree with the eager result bit for bit:
checked over several replays separated by other eager work and
synchronisations, in FP32 and FP64, and for whole solves.
"""
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
import paper_2111_06893_amd as dgtn  # noqa: E402

pytestmark = pytest.mark.gpu


def _pair(spec, opts):
    os.environ["DGTN_NO_GRAPHS"] = "1"
    try:
        eager = dgtn.Problem(spec)
        eager.bind(opts)
    finally:
        del os.environ["DGTN_NO_GRAPHS"]
    graph = dgtn.Problem(spec)
    graph.bind(opts)
    return eager, graph


@pytest.mark.parametrize("prec", [32, 64])
def test_replays_match_eager(prec):
    spec = W.config4()
    o = dgtn.default_opts(prec)
    eager, graph = _pair(spec, o)
    print(f"[graphs] precondition replays, FP{prec}", flush=True)
    v = torch.from_numpy(W.random_field(spec, seed=21)).cuda()
    u = torch.from_numpy(W.random_field(spec, seed=22)).cuda()
    ref = eager.precondition(v, o).cpu().numpy()
    for rep in range(5):
        z = graph.precondition(v, o)
        graph.apply(u)                      # eager work between the replays
        torch.cuda.synchronize()
        got = z.cpu().numpy()
        assert np.array_equal(got, ref), f"replay {rep} differs: {np.abs(got - ref).max()}"
    # a different input through the same graph
    v2 = torch.from_numpy(W.random_field(spec, seed=23)).cuda()
    assert np.array_equal(graph.precondition(v2, o).cpu().numpy(), eager.precondition(v2, o).cpu().numpy())


def test_solves_match_eager():
    spec = W.config1()
    o = dgtn.default_opts(32, rtol=1e-10)
    eager, graph = _pair(spec, o)
    print("[graphs] solves", flush=True)
    ue, se = eager.solve(opts=o)
    for _ in range(2):
        ug, sg = graph.solve(opts=o)
        assert sg.iters == se.iters
        assert np.array_equal(ug.cpu().numpy(), ue.cpu().numpy())


def test_rebind_drops_recorded_graphs():
    # a new workspace moves every buffer: the recorded V-cycle must not be reused
    spec = W.config1()
    o = dgtn.default_opts(32)
    eager, graph = _pair(spec, o)
    v = torch.from_numpy(W.random_field(spec, seed=24)).cuda()
    ref = eager.precondition(v, o).cpu().numpy()
    assert np.array_equal(graph.precondition(v, o).cpu().numpy(), ref)
    old_ws = graph.ws                      # held, so the new workspace lies elsewhere
    graph.bind(o)
    assert graph.ws.data_ptr() != old_ws.data_ptr()
    assert np.array_equal(graph.precondition(v, o).cpu().numpy(), ref)
    del old_ws
