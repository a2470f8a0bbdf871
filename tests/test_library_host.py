"""Host-side checks of the HIP library (no GPU): it loads, exports every symbol
the header declares, validates its inputs, and its mesh agrees with the
oracle's independently built mesh."""
import ctypes

import numpy as np
import pytest

import workloads as W
import paper_2111_06893_amd as dgtn
from paper_2111_06893_amd import _lib
from oracle import mesh as omesh, physics


def test_library_exports_every_declared_symbol():
    lib = dgtn.load()
    names = _lib.header_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(_lib._SIGS) >= set(names)


@pytest.mark.parametrize("make", [W.config1, W.config2, W.config4,
                                  lambda: W.box(nx=3, ny=2, Lx=1.5, Ly=0.8, p=4,
                                                layers=[{"thickness": 0.3, "n_elem": 3, "ratio": 1.7,
                                                         "material": 0}])])
def test_mesh_matches_oracle(make):
    spec = make()
    if spec["p"] > 5:
        spec["p"] = 3  # keep the oracle mesh small; the topology is unchanged
    P = dgtn.Problem(spec)
    assert P.shape == W.field_shape(spec)
    assert P.n_dof == W.n_dof(spec)
    xyz = P.node_coords()
    ref = omesh.build(spec).xyz
    assert np.abs(xyz - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_config_sizes():
    assert W.n_dof(W.config1()) == 25920
    assert W.n_dof(W.config2()) == 2058000
    assert W.n_elements(W.config5()) == 8000


def test_invalid_problems_are_rejected():
    bad = W.config1()
    bad["p"] = 0
    with pytest.raises(dgtn.DgtnError, match="EINVAL"):
        dgtn.Problem(bad)
    bad = W.config1()
    bad["materials"] = [{"kind": "cubic", "c11": 50e9, "c12": 60e9, "c44": 30e9}]
    with pytest.raises(dgtn.DgtnError, match="positive definite"):
        dgtn.Problem(bad)
    bad = W.config1()
    bad["layers"][0]["thickness"] = -1.0
    with pytest.raises(dgtn.DgtnError):
        dgtn.Problem(bad)
    bad = W.config1()
    bad["layers"][0]["material"] = 3
    with pytest.raises(dgtn.DgtnError):
        dgtn.Problem(bad)


@pytest.mark.parametrize("mat", [W.FUSED_SILICA, W.COATING_ISO, {"kind": "iso", "Y": 3.0e9, "nu": -0.4},
                                 W.CRYSTAL_A])
def test_material_constants_match_oracle_stiffness(mat):
    # the library's constants (eq. constrel_iso for an isotropic material) against the
    # entries of the oracle's full stiffness tensor: Y_xxxx = c11, Y_xxyy = c12, Y_xyxy = c44
    from oracle import material
    c = dgtn.material_constants(mat)
    Y = material.tensor(mat)
    ref = {"c11": Y[0, 0, 0, 0], "c12": Y[0, 0, 1, 1], "c44": Y[0, 1, 0, 1]}
    for k in ref:
        assert abs(c[k] / ref[k] - 1) < 1e-14, (k, c[k], ref[k])
    assert dgtn.param_value(W.config4(), "c12", 1) == pytest.approx(dgtn.material_constants(W.COATING_ISO)["c12"])
    s = dgtn.with_params(W.config4(), [("c44", 0)], [31e9])
    assert s["materials"][0] == {"kind": "cubic", **dgtn.material_constants(W.FUSED_SILICA), "c44": 31e9}


def test_material_constants_reject_invalid_materials():
    for bad in ({"kind": "iso", "Y": 70e9, "nu": 0.5}, {"kind": "iso", "Y": -1.0, "nu": 0.2},
                {"kind": "cubic", "c11": 50e9, "c12": 60e9, "c44": 30e9}):
        with pytest.raises(dgtn.DgtnError, match="positive definite"):
            dgtn.material_constants(bad)


def test_noise_psd_matches_oracle_formula():
    U = [2.4e-11, 1.7e-13]
    phi = [1e-6, 4e-4]
    a = dgtn.noise_psd(U, phi, 295.0, 100.0, 1.0)
    b = physics.noise_psd(U, phi, 295.0, 100.0, 1.0)
    assert abs(a / b - 1) < 1e-14
    with pytest.raises(dgtn.DgtnError):
        dgtn.noise_psd(U, phi, -1.0, 100.0, 1.0)


def test_workspace_size_is_reported():
    P = dgtn.Problem(W.config1())
    n = P.workspace_bytes()
    # at least the two face-traction buffers (FP64 + FP32)
    assert n > 40 * 6 * 3 * 36 * 12


def test_missing_library_fails_loudly(monkeypatch):
    # no fallback: without the built library every entry point raises
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libdgtn.so")
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="is not built"):
        _lib.load()
    with pytest.raises(RuntimeError):
        dgtn.Problem(W.config1())


def test_device_calls_need_a_device():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a HIP device is visible")
    P = dgtn.Problem(W.config1())
    with pytest.raises(dgtn.DgtnError, match="no HIP device"):
        P.bind()


def _annulus_columns(order, n_r=2, n_t=6, r_in=0.3, r_out=1.0):
    """Curved columns of degree `order`: an annulus split into n_r x n_t sectors,
    the map r(xi), theta(eta) sampled at the oracle's LGL points."""
    from oracle import lgl
    xs, _ = lgl.nodes_weights(order + 1)
    out = np.zeros((n_r * n_t, 2, order + 1, order + 1))
    for t in range(n_t):
        for s in range(n_r):
            for j in range(order + 1):
                th = 2 * np.pi * (t + 0.5 * (xs[j] + 1)) / n_t
                for i in range(order + 1):
                    r = r_in + (r_out - r_in) * (s + 0.5 * (xs[i] + 1)) / n_r
                    out[t * n_r + s, 0, j, i] = r * np.cos(th)
                    out[t * n_r + s, 1, j, i] = r * np.sin(th)
    return out


@pytest.mark.parametrize("make", [
    lambda: W.columns_mesh(W.quad_columns(3, 2, 1.2, 0.8, jitter=0.25, seed=3), p=4,
                           layers=[{"thickness": 0.2, "n_elem": 2, "ratio": 1.5, "material": 0}]),
    lambda: W.columns_mesh(_annulus_columns(3), order=3, p=5),
    lambda: W.columns_mesh(_annulus_columns(6), order=6, p=2)])
def test_explicit_mesh_matches_oracle(make):
    # the library's and the oracle's meshes from the same column maps: both interpolate the
    # given nodes at their own LGL points and match neighbours by coordinates
    spec = make()
    P = dgtn.Problem(spec)
    assert P.shape == W.field_shape(spec)
    xyz = P.node_coords()
    ref = omesh.build(spec).xyz
    assert np.abs(xyz - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_explicit_mesh_reproduces_the_box():
    # undisplaced quad columns are the box description's own columns
    box = W.box(nx=3, ny=2, Lx=1.2, Ly=0.8, p=3)
    cols = W.columns_mesh(W.quad_columns(3, 2, 1.2, 0.8), p=3)
    a, b = dgtn.Problem(box).node_coords(), dgtn.Problem(cols).node_coords()
    assert np.abs(a - b).max() < 1e-15


def _quad(x0, x1, y0, y1):
    """Degree-1 map of the rectangle [x0, x1] x [y0, y1] (corners at xi, eta = -1, 1)."""
    return np.array([[[x0, x1], [x0, x1]], [[y0, y0], [y1, y1]]])


def test_explicit_mesh_is_validated():
    import ctypes
    from paper_2111_06893_amd._lib import check
    xy = W.quad_columns(2, 2)
    st, keep = dgtn.problem_struct(W.columns_mesh(xy))
    st.refine = 1
    with pytest.raises(dgtn.DgtnError, match="refine"):
        check(dgtn.load().dgtn_create(ctypes.byref(st), ctypes.byref(ctypes.c_void_p())))
    flipped = xy[:, :, :, ::-1].copy()          # clockwise columns: det J < 0
    with pytest.raises(dgtn.DgtnError, match="EMESH"):
        dgtn.Problem(W.columns_mesh(flipped))
    bad = xy.copy()
    bad[0, 0, 0, 0] = np.nan
    with pytest.raises(dgtn.DgtnError, match="non-finite"):
        dgtn.Problem(W.columns_mesh(bad))
    # a hanging node: two columns on top of one (a T-junction) would be a crack
    tee = np.stack([_quad(-0.5, 0.5, -0.5, 0.0), _quad(-0.5, 0.0, 0.0, 0.5), _quad(0.0, 0.5, 0.0, 0.5)])
    with pytest.raises(dgtn.DgtnError, match="hanging node"):
        dgtn.Problem(W.columns_mesh(tee))
    # a shared edge that the two columns curve differently (degree-2 maps, same end points)
    from oracle import lgl
    xs, _ = lgl.nodes_weights(3)
    two = np.zeros((2, 2, 3, 3))
    for c, (x0, x1) in enumerate(((-0.5, 0.0), (0.0, 0.5))):
        for j in range(3):
            for i in range(3):
                two[c, 0, j, i] = x0 + (x1 - x0) * 0.5 * (xs[i] + 1)
                two[c, 1, j, i] = -0.5 + 0.5 * (xs[j] + 1)
    two[0, 0, 1, 2] += 0.05                     # bulge the right edge of the first column only
    with pytest.raises(dgtn.DgtnError, match="non-conforming"):
        dgtn.Problem(W.columns_mesh(two, order=2))
    two[1, 0, 1, 0] += 0.05                     # the same bulge on both sides: conforming
    dgtn.Problem(W.columns_mesh(two, order=2))
