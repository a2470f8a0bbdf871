"""GPU: dgtn_energy_noalloc, the energy entry point that keeps its partial sums
in the library's fixed device array instead of the bound workspace, called
through the C ABI and compared with dgtn_energy on the same inputs: two calls in
a row on different contexts, the second with fewer elements and layers (the
array then still holds the first call's values past the second's range), and a
third on the first context again.  The two entry points run the same kernels in
the same order, so their outputs agree bit for bit."""
import ctypes

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
import paper_2111_06893_amd as dgtn  # noqa: E402
from paper_2111_06893_amd import _lib  # noqa: E402

pytestmark = pytest.mark.gpu

DP = ctypes.POINTER(ctypes.c_double)


def _both(P, u):
    """(layer energies, compliance) from dgtn_energy and from dgtn_energy_noalloc."""
    lib = dgtn.load()
    out = []
    for fn in (lib.dgtn_energy, lib.dgtn_energy_noalloc):
        U = np.full(P.n_layers, np.nan)
        c = ctypes.c_double(np.nan)
        _lib.check(fn(P.ctx, ctypes.c_void_p(u.data_ptr()), U.ctypes.data_as(DP), ctypes.byref(c),
                      P._stream()))
        out.append((U, c.value))
    return out


def _case(spec, seed):
    P = dgtn.Problem(spec)
    P.bind()
    u = torch.from_numpy(W.random_field(spec, seed=seed) * 1e-9).cuda()
    return P, u


def test_energy_noalloc_matches_energy_on_consecutive_calls():
    big = W.config5(p=2)                               # 8000 elements, 41 layers
    small = W.box(nx=1, ny=1, p=3, materials=[W.FUSED_SILICA, W.CRYSTAL_A],
                  layers=[{"thickness": 0.1, "n_elem": 1, "ratio": 1.0, "material": 1},
                          {"thickness": 0.9, "n_elem": 2, "ratio": 1.0, "material": 0}])
    print("[no-alloc] forty-layer coating at p = 2, then a three-element box, then the first again", flush=True)
    Pb, ub = _case(big, 1)
    Ps, us = _case(small, 2)
    first = _both(Pb, ub)
    second = _both(Ps, us)
    third = _both(Pb, ub)
    for (U_ref, c_ref), (U, c) in (first, second, third):
        assert np.all(np.isfinite(U)) and np.isfinite(c)
        np.testing.assert_array_equal(U, U_ref)
        assert c == c_ref
    np.testing.assert_array_equal(third[1][0], first[0][0])
    assert second[0][0].shape == (2,) and first[0][0].shape == (41,)
    # and the energies are the layer energies of the oracle
    from oracle import dg
    O = dg.Problem(small)
    np.testing.assert_allclose(second[1][0], dg.energy_layers(O, us.cpu().numpy()), rtol=1e-12)


def test_energy_noalloc_rejects_meshes_beyond_its_maximum():
    # 257 x 257 columns x 2 z-elements = 132,098 elements > 131,072: refused before any
    # device work (the workspace is not even bound)
    spec = W.box(nx=257, ny=257, p=1, layers=[{"thickness": 1.0, "n_elem": 2, "ratio": 1.0, "material": 0}])
    P = dgtn.Problem(spec)
    U = np.zeros(1)
    u = torch.zeros(8, dtype=torch.float64, device="cuda")
    st = dgtn.load().dgtn_energy_noalloc(P.ctx, ctypes.c_void_p(u.data_ptr()), U.ctypes.data_as(DP), None,
                                         P._stream())
    assert st == -1
    assert "exceed" in dgtn.load().dgtn_last_error().decode()
