"""Host-side checks of the multigrid hierarchy and of the additive-Schwarz
subdomain solves (no GPU).

On a box element with an isotropic or cubic material the component-diagonal
part of the element block of A is exactly separable,
sum_d kappa_cd K_d (x) M (x) M, so the library's fast-diagonalisation inverse
must equal the inverse of the oracle's exact element block restricted to one
displacement component."""
import numpy as np
import pytest

import workloads as W
import paper_2111_06893_amd as dgtn
from oracle import dg


def fdm_inverse(S, lam):
    """(S_x (x) S_y (x) S_z) diag(1 / sum lambda) (...)^T in node order k, j, i."""
    N = S.shape[-1]
    T = np.kron(S[2], np.kron(S[1], S[0]))
    L = (lam[2][:, None, None] + lam[1][None, :, None] + lam[0][None, None, :]).ravel()
    return T @ np.diag(1.0 / L) @ T.T


@pytest.mark.parametrize("bc_side", [W.BC_FREE, W.BC_DIRICHLET])
def test_fdm_equals_exact_block_inverse_on_box(bc_side):
    mats = [W.FUSED_SILICA, W.CRYSTAL_A]
    spec = W.box(nx=3, ny=2, Lx=1.2, Ly=0.5, p=3, materials=mats,
                 layers=[{"thickness": 0.1, "n_elem": 1, "ratio": 1, "material": 1},
                         {"thickness": 0.6, "n_elem": 2, "ratio": 2.0, "material": 0}],
                 bc={"top": W.BC_PRESSURE, "bottom": W.BC_DIRICHLET, "side": bc_side})
    P = dgtn.Problem(spec)
    opts = dgtn.default_opts(64, mg_levels=1)
    O = dg.Problem(spec)
    B = dg.element_blocks(O)
    N = spec["p"] + 1
    n3 = N ** 3
    yref = P.y_ref
    for e in range(O.E):
        S, lam = P.smoother_block(opts, 0, e)
        for c in range(3):
            Bcc = B[e][c * n3:(c + 1) * n3, c * n3:(c + 1) * n3] / yref
            ref = np.linalg.inv(Bcc)
            got = fdm_inverse(S[c], lam[c])
            assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max(), (e, c)


def test_hierarchy_of_config2():
    P = dgtn.Problem(W.config2())
    opts = dgtn.default_opts(64, mg_levels=6)
    got = [P.level_info(opts, l) for l in range(5)]
    # p 6 -> 3 -> 1, then 80 -> 20 -> 5 columns, 25 z-elements throughout
    assert got == [(7, 2000, 80), (4, 2000, 80), (2, 2000, 80), (2, 500, 20), (2, 125, 5)]
    with pytest.raises(dgtn.DgtnError):
        P.level_info(opts, 5)


def _patch_geometry_faults(P, opts):
    """Checks the overlapping-patch gather table against the node coordinates:
    consecutive patch positions on either side of a column face are the two
    copies of one face node (same point), and never coincide elsewhere."""
    tab = P.patch_table(opts)
    N = P.info.N
    n_cols, Pw, _ = tab.shape
    k = (Pw - N) // 2
    xy = P.node_coords()[:n_cols, :2, 0].reshape(n_cols, 2, N * N)
    pts = np.where(tab[..., None] >= 0, np.moveaxis(xy, 1, 2).reshape(-1, 2)[np.maximum(tab, 0)], np.nan)
    faults = 0
    for axis in (2, 1):      # a (xi) then b (eta)
        d = np.diff(pts, axis=axis)
        dist = np.hypot(d[..., 0], d[..., 1])
        cross = np.zeros(Pw - 1, bool)
        cross[[k - 1, k + N - 1]] = True
        cross = cross[None, None, :] if axis == 2 else cross[None, :, None]
        ok = ~np.isnan(dist)
        faults += int(np.sum(ok & cross & (dist > 1e-12)) + np.sum(ok & ~cross & (dist < 1e-12)))
    return tab, faults


@pytest.mark.parametrize("overlap", [1, 2, 3])
def test_patch_tables_on_the_cylinder(overlap):
    spec = W.config2()
    P = dgtn.Problem(spec)
    opts = dgtn.default_opts(64, overlap=overlap)
    tab, faults = _patch_geometry_faults(P, opts)
    assert faults == 0
    N = P.info.N
    n_cols, Pw, _ = tab.shape
    assert Pw == N + 2 * overlap
    k = overlap
    # own nodes map to themselves
    own = tab[:, k:k + N, k:k + N].reshape(n_cols, -1)
    assert np.array_equal(own, np.arange(n_cols)[:, None] * N * N + np.arange(N * N)[None, :])
    # missing entries: the k lines beyond the arc of the 16 boundary columns
    # (refine 2), and the k x k corner blocks of the three columns at each of
    # the four vertices shared by three columns
    assert int(np.sum(tab < 0)) == 16 * k * Pw + 4 * 3 * k * k


def test_patch_tables_on_a_box():
    spec = W.box(nx=3, ny=2, Lx=1.5, Ly=1.0, p=4)
    P = dgtn.Problem(spec)
    opts = dgtn.default_opts(64, overlap=2)
    tab, faults = _patch_geometry_faults(P, opts)
    assert faults == 0
    # every interior vertex is shared by four columns: only positions beyond the box are missing
    N, k, Pw = 5, 2, 9
    expect = 0
    for t in range(2):
        for s in range(3):
            ax = sum(1 for a in range(Pw) if 0 <= s * N + a - k < 3 * N)
            ay = sum(1 for b in range(Pw) if 0 <= t * N + b - k < 2 * N)
            expect += Pw * Pw - ax * ay
    assert int(np.sum(tab < 0)) == expect
