"""MI355X-native DG elasticity for Brownian coating thermal noise.

Thin Python binding of the C ABI in include/dgtn.h (libdgtn.so, HIP for
gfx950): argument marshalling only.  Every step of the operator, load, solve
and energy runs in the library's kernels; PyTorch provides device memory and
streams.  There is no CPU fallback: without the built library every call
raises.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import DgtnError, check, load

__all__ = ["Problem", "DgtnError", "noise_psd", "noise_psd_parts", "load", "problem_struct", "default_opts", "PARAM_KINDS",
           "with_params", "param_value", "material_constants", "EnergyFn", "layer_energies"]

# Parameter kinds of the energy gradient (dgtn_param.kind)
PARAM_KINDS = {"c11": 0, "c12": 1, "c44": 2, "youngs": 3, "poisson": 4, "thickness": 5,
               "r0": 6, "xc": 7, "yc": 8}
_LOAD_KINDS = ("r0", "xc", "yc")  # beam width and centre of the pressure profile (index unused)

_BC = {"top", "bottom", "side"}


def problem_struct(spec):
    """ctypes problem description from a spec dict (kept alive by the result)."""
    mats = (_lib.Material * len(spec["materials"]))()
    for i, m in enumerate(spec["materials"]):
        mats[i] = _material_struct(m)
    lays = (_lib.Layer * len(spec["layers"]))()
    for i, l in enumerate(spec["layers"]):
        lays[i] = _lib.Layer(l["thickness"], l["n_elem"], l["ratio"], l["material"])
    ld = spec["load"]
    bc = spec["bc"]
    domain = {"cylinder": 0, "box": 1, "columns": 2}[spec["domain"]]
    cxy, n_columns, order = None, 0, 0
    if domain == 2:
        order = int(spec["columns"]["order"])
        cxy = np.ascontiguousarray(spec["columns"]["xy"], dtype=np.float64)
        if cxy.ndim != 4 or cxy.shape[1:] != (2, order + 1, order + 1):
            raise ValueError("columns xy must be [n_columns, 2, order + 1, order + 1]")
        n_columns = cxy.shape[0]
    p = _lib.ProblemC(
        domain=domain, R=spec.get("R", 1.0), refine=spec["refine"] if domain == 0 else 0,
        Lx=spec.get("Lx", 1.0), Ly=spec.get("Ly", 1.0), nx=spec.get("nx", 1), ny=spec.get("ny", 1),
        p=spec["p"], n_layers=len(lays), layers=lays, n_materials=len(mats), materials=mats,
        F0=ld["F0"], r0=ld["r0"], xc=ld["xc"], yc=ld["yc"],
        bc_top=bc["top"], bc_bottom=bc["bottom"], bc_side=bc["side"], penalty=spec["penalty"],
        n_columns=n_columns, map_order=order,
        columns_xy=cxy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if cxy is not None else None)
    return p, (mats, lays, cxy)


def _material_struct(m):
    if m["kind"] == "iso":
        return _lib.Material(0, m["Y"], m["nu"], 0.0, 0.0, 0.0)
    if m["kind"] == "cubic":
        return _lib.Material(1, 0.0, 0.0, m["c11"], m["c12"], m["c44"])
    raise ValueError(m["kind"])


def material_constants(m):
    """Cubic constants {c11, c12, c44} (Pa) of a material dict, from the
    library (dgtn_material_constants: an isotropic material's from its Young's
    modulus and Poisson ratio)."""
    out = (ctypes.c_double * 3)()
    check(load().dgtn_material_constants(ctypes.byref(_material_struct(m)), out))
    return {"c11": out[0], "c12": out[1], "c44": out[2]}


def with_params(spec, params, values):
    """Copy of spec with the parameters [(kind, index)] set to values.  Setting
    a cubic constant of an isotropic material turns it into the equivalent
    cubic material first."""
    import copy
    s = copy.deepcopy(spec)
    for (kind, index), v in zip(params, values):
        v = float(v)
        if kind == "thickness":
            s["layers"][index]["thickness"] = v
            continue
        if kind in _LOAD_KINDS:
            s["load"][kind] = v
            continue
        m = s["materials"][index]
        if kind in ("c11", "c12", "c44"):
            if m["kind"] != "cubic":
                m = s["materials"][index] = {"kind": "cubic", **material_constants(m)}
            m[kind] = v
        elif kind in ("youngs", "poisson"):
            if m["kind"] != "iso":
                raise ValueError(f"material {index} is not isotropic")
            m["Y" if kind == "youngs" else "nu"] = v
        else:
            raise ValueError(f"unknown parameter kind {kind!r}")
    return s


def param_value(spec, kind, index):
    """Value of the parameter (kind, index) in spec (see with_params)."""
    if kind == "thickness":
        return float(spec["layers"][index]["thickness"])
    if kind in _LOAD_KINDS:
        return float(spec["load"][kind])
    m = spec["materials"][index]
    if kind in ("c11", "c12", "c44"):
        return float(m[kind] if m["kind"] == "cubic" else material_constants(m)[kind])
    if kind in ("youngs", "poisson"):
        if m["kind"] != "iso":
            raise ValueError(f"material {index} is not isotropic")
        return float(m["Y"] if kind == "youngs" else m["nu"])
    raise ValueError(f"unknown parameter kind {kind!r}")


def noise_psd_parts(U_parts, phi_parts, T, f, F0):
    """S_x with one loss angle per energy part (arrays [n_layers, 3])."""
    lib = load()
    U = np.ascontiguousarray(U_parts, dtype=np.float64)
    ph = np.ascontiguousarray(phi_parts, dtype=np.float64)
    if U.shape != ph.shape or U.ndim != 2 or U.shape[1] != 3:
        raise ValueError("expected [n_layers, 3] energy parts and loss angles")
    out = ctypes.c_double()
    check(lib.dgtn_noise_psd_parts(U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), U.shape[0], T, f, F0,
                                   ctypes.byref(out)))
    return out.value


def default_opts(precision=64, **kw):
    o = dict(precond_precision=precision, restart=30, max_iter=20000, rtol=1e-11,
             mg_levels=16, smooth_steps=1, smooth_damping=0.65, smoother=1, krylov=1, overlap=1,
             residual_precision=64)
    o.update(kw)
    return _lib.SolveOpts(**o)


def noise_psd(U_layers, phi, T, f, F0):
    """S_x = 4 kB T sum_k phi_k U_k / (pi f F0^2) (host function of the library)."""
    lib = load()
    U = np.ascontiguousarray(U_layers, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    if U.shape != ph.shape:
        raise ValueError("U_layers and phi differ in length")
    out = ctypes.c_double()
    check(lib.dgtn_noise_psd(U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(U), T, f, F0,
                             ctypes.byref(out)))
    return out.value


class Problem:
    """One problem on the current HIP device.

    spec: a problem description dict (see the workloads package).  The mesh
    and host geometry are built at construction; the device workspace is
    allocated as a torch uint8 tensor and bound when first needed.
    """

    def __init__(self, spec, opts=None, device=None):
        self.lib = load()
        self.spec = spec
        self._struct, self._keep = problem_struct(spec)
        ctx = ctypes.c_void_p()
        check(self.lib.dgtn_create(ctypes.byref(self._struct), ctypes.byref(ctx)))
        self.ctx = ctx
        info = _lib.Info()
        check(self.lib.dgtn_get_info(self.ctx, ctypes.byref(info)))
        self.info = info
        self.n_dof = info.n_dof
        self.shape = (info.n_elem, 3, info.N, info.N, info.N)
        self.n_layers = info.n_layers
        self.y_ref = info.y_ref
        self.ws = None
        self.opts = opts
        self.device = device

    # --- host-only queries -------------------------------------------------
    def workspace_bytes(self, opts=None):
        n = ctypes.c_size_t()
        check(self.lib.dgtn_workspace_bytes(self.ctx, ctypes.byref(opts) if opts is not None else None,
                                            ctypes.byref(n)))
        return n.value

    def node_coords(self):
        out = np.zeros(self.shape)
        check(self.lib.dgtn_node_coords(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    # --- device -------------------------------------------------------------
    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def bind(self, opts=None):
        import torch
        if not torch.cuda.is_available():
            raise DgtnError("no HIP device visible")
        opts = opts if opts is not None else self.opts
        nbytes = self.workspace_bytes(opts)
        dev = self.device or torch.device("cuda", torch.cuda.current_device())
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        check(self.lib.dgtn_bind(self.ctx, ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                 ctypes.byref(opts) if opts is not None else None, self._stream()))
        self.opts = opts
        return self

    def _ensure(self, opts=None):
        if self.ws is None or (opts is not None and self.opts is None):
            self.bind(opts if opts is not None else self.opts)

    def _check_field(self, t, dtype):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("expected a device tensor")
        if t.dtype != dtype or not t.is_contiguous() or t.numel() != self.n_dof:
            raise ValueError(f"expected a contiguous {dtype} tensor of {self.n_dof} values")

    def empty(self, dtype=None):
        import torch
        self._ensure()
        return torch.empty(self.shape, dtype=dtype or torch.float64, device=self.ws.device)

    def apply(self, u, out=None):
        """A u (SI) in the precision of u (float64 or float32)."""
        import torch
        self._ensure()
        prec = 64 if u.dtype == torch.float64 else 32
        self._check_field(u, u.dtype)
        if out is None:
            out = torch.empty_like(u)
        self._check_field(out, u.dtype)
        check(self.lib.dgtn_apply(self.ctx, prec, ctypes.c_void_p(u.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def apply_stage(self, u, out, stage):
        """One kernel pass of the apply (1 traction, 2 volume-and-flux, 3 both)."""
        import torch
        self._ensure()
        prec = 64 if u.dtype == torch.float64 else 32
        self._check_field(u, u.dtype)
        self._check_field(out, u.dtype)
        check(self.lib.dgtn_apply_stage(self.ctx, prec, stage, ctypes.c_void_p(u.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def residual(self, u, b=None, out=None):
        """b - A u (b defaults to the load vector), with A u evaluated in
        double-double arithmetic and rounded once (dgtn_residual)."""
        import torch
        self._ensure()
        if b is None:
            b = self.rhs()
        self._check_field(u, torch.float64)
        self._check_field(b, torch.float64)
        if out is None:
            out = torch.empty_like(u)
        self._check_field(out, torch.float64)
        check(self.lib.dgtn_residual(self.ctx, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def rhs(self, out=None):
        import torch
        self._ensure()
        if out is None:
            out = self.empty(torch.float64)
        self._check_field(out, torch.float64)
        check(self.lib.dgtn_rhs(self.ctx, ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def energy(self, u, compliance=False):
        """Per-layer elastic energies (numpy, J); with compliance=True also
        1/2 u . b, returned as (U_layers, U_compl)."""
        import torch
        self._ensure()
        self._check_field(u, torch.float64)
        out = np.zeros(self.n_layers)
        comp = ctypes.c_double()
        check(self.lib.dgtn_energy(self.ctx, ctypes.c_void_p(u.data_ptr()),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(comp) if compliance else None, self._stream()))
        return (out, comp.value) if compliance else out

    def jump_indicator(self, u, faces="all", weight="jump"):
        """Face-jump indicator of adaptive refinement: (eta_e^2 per element in the
        element order of u, their per-layer sums), numpy, over the face family
        `faces`: "side", "z" or "all"; weight "jump" (plain squared jumps) or
        "penalty" (each term times the penalty sigma at its node)."""
        import torch
        self._ensure()
        self._check_field(u, torch.float64)
        eta = np.zeros(self.info.n_elem)
        lay = np.zeros(self.n_layers)
        dp = ctypes.POINTER(ctypes.c_double)
        which = {"side": 1, "z": 2, "all": 3}[faces] | {"jump": 0, "penalty": 4}[weight]
        check(self.lib.dgtn_jump_indicator(self.ctx, ctypes.c_void_p(u.data_ptr()), which, eta.ctypes.data_as(dp),
                                           lay.ctypes.data_as(dp), self._stream()))
        return eta, lay

    def energy_parts(self, u):
        """[n_layers, 3] layer energies split by modulus (isotropic: bulk, shear, 0;
        cubic: c11, c12, c44 parts), numpy, J."""
        import torch
        self._ensure()
        self._check_field(u, torch.float64)
        out = np.zeros((self.n_layers, 3))
        check(self.lib.dgtn_energy_parts(self.ctx, ctypes.c_void_p(u.data_ptr()),
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self._stream()))
        return out

    def energy_grad(self, u, w_layers=None):
        """g = dJ/du for J = sum_k w_k U_k (device float64, the adjoint right-hand side)."""
        import torch
        self._ensure()
        self._check_field(u, torch.float64)
        g = torch.empty_like(u)
        w = self._weights(w_layers)
        check(self.lib.dgtn_energy_grad(self.ctx, ctypes.c_void_p(u.data_ptr()),
                                        w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        ctypes.c_void_p(g.data_ptr()), self._stream()))
        return g

    def grad(self, u, lam, params, w_layers=None):
        """dJ/dtheta (numpy) for params = [(kind, index)], given the solution u
        and the adjoint solution lam of A lam = energy_grad(u, w_layers)."""
        import torch
        self._ensure()
        self._check_field(u, torch.float64)
        self._check_field(lam, torch.float64)
        arr = (_lib.Param * max(1, len(params)))()
        for i, (kind, index) in enumerate(params):
            if kind not in PARAM_KINDS:
                raise ValueError(f"unknown parameter kind {kind!r}")
            arr[i] = _lib.Param(PARAM_KINDS[kind], index)
        w = self._weights(w_layers)
        out = np.zeros(max(1, len(params)))
        check(self.lib.dgtn_grad(self.ctx, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                 w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(params), arr,
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self._stream()))
        return out[:len(params)]

    def _weights(self, w_layers):
        w = np.ones(self.n_layers) if w_layers is None else np.ascontiguousarray(w_layers, dtype=np.float64)
        if w.shape != (self.n_layers,):
            raise ValueError(f"expected {self.n_layers} layer weights")
        return w

    def solve(self, b=None, u0=None, opts=None, raise_on_noconv=True):
        """Solves A u = b (b defaults to the load vector); returns (u, stats)."""
        import torch
        opts = opts if opts is not None else (self.opts or default_opts())
        if self.ws is None or self.opts is None or self.workspace_bytes(opts) > self.ws.numel():
            self.bind(opts)
        if b is None:
            b = self.rhs()
        self._check_field(b, torch.float64)
        u = torch.zeros_like(b) if u0 is None else u0.clone()
        stats = _lib.SolveStats()
        st = self.lib.dgtn_solve(self.ctx, ctypes.byref(opts), ctypes.c_void_p(b.data_ptr()),
                                 ctypes.c_void_p(u.data_ptr()), ctypes.byref(stats), self._stream())
        if st == -4 and not raise_on_noconv:   # DGTN_ENOCONV: u holds the last iterate
            stats.converged = False
            return u, stats
        check(st)
        stats.converged = True
        return u, stats

    def precondition(self, v, opts=None):
        """One V-cycle z = M^{-1} v (for the operator divided by y_ref)."""
        import torch
        opts = opts if opts is not None else self.opts
        if self.ws is None or self.opts is None or self.workspace_bytes(opts) > self.ws.numel():
            self.bind(opts)
        self._check_field(v, torch.float64)
        z = torch.empty_like(v)
        check(self.lib.dgtn_precondition(self.ctx, ctypes.byref(opts), ctypes.c_void_p(v.data_ptr()),
                                         ctypes.c_void_p(z.data_ptr()), self._stream()))
        return z

    def level_info(self, opts, level):
        N, E, C = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(self.lib.dgtn_level_info(self.ctx, ctypes.byref(opts), level, ctypes.byref(N), ctypes.byref(E),
                                       ctypes.byref(C)))
        return N.value, E.value, C.value

    def smoother_block(self, opts, level, elem):
        """Schwarz subdomain data of one element: arrays S[c][d] (N x N) and lam[c][d] (N)."""
        N, _, _ = self.level_info(opts, level)
        out = np.zeros(9 * (N * N + N))
        check(self.lib.dgtn_smoother_block(self.ctx, ctypes.byref(opts), level, elem,
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        out = out.reshape(3, 3, N * N + N)
        return out[:, :, :N * N].reshape(3, 3, N, N), out[:, :, N * N:]

    def patch_table(self, opts, level=0):
        """Gather table of the overlapping column patches: array [n_cols, P, P]
        of 2D-grid nodes col * N^2 + j * N + i (or -1), indexed [col, b, a]."""
        Pw = ctypes.c_int()
        check(self.lib.dgtn_patch_table(self.ctx, ctypes.byref(opts), level, ctypes.byref(Pw), None))
        _, _, n_cols = self.level_info(opts, level)
        tab = np.zeros(n_cols * Pw.value ** 2, dtype=np.int32)
        check(self.lib.dgtn_patch_table(self.ctx, ctypes.byref(opts), level, ctypes.byref(Pw),
                                        tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return tab.reshape(n_cols, Pw.value, Pw.value)

    def noise(self, U_layers, phi, T, f):
        return noise_psd(U_layers, phi, T, f, self.spec["load"]["F0"])

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.dgtn_destroy(self.ctx)
            self.ctx = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _energy_fn():
    import torch

    class EnergyFn(torch.autograd.Function):
        """theta -> per-layer elastic energies U_k (float64, on the host).

        forward(theta, spec, params, opts): theta holds the values of
        params = [(kind, index)] (see PARAM_KINDS) substituted into spec; the
        problem is solved on the current device.  backward: with the incoming
        gradient as layer weights w, one adjoint solve A lam = dJ/du and the
        parameter derivatives of dgtn_grad give w . dU/dtheta.
        """

        @staticmethod
        def forward(ctx, theta, spec, params, opts=None):
            params = [tuple(p) for p in params]
            prob = Problem(with_params(spec, params, theta.detach().cpu().tolist()))
            o = opts if opts is not None else default_opts()
            u, _ = prob.solve(opts=o)
            ctx.state = (prob, u, params, o)
            return torch.as_tensor(prob.energy(u), dtype=torch.float64)

        @staticmethod
        def backward(ctx, gU):
            prob, u, params, o = ctx.state
            w = gU.detach().cpu().to(torch.float64).numpy()
            lam, _ = prob.solve(b=prob.energy_grad(u, w), opts=o)
            dJ = prob.grad(u, lam, params, w)
            return torch.as_tensor(dJ, dtype=torch.float64), None, None, None

    return EnergyFn


def __getattr__(name):
    # torch is imported on first use only, so host-only users of the library need not load it
    if name == "EnergyFn":
        fn = _energy_fn()
        globals()["EnergyFn"] = fn
        return fn
    raise AttributeError(name)


def layer_energies(theta, spec, params, opts=None):
    """Differentiable per-layer energies U_k(theta) (see EnergyFn)."""
    fn = globals().get("EnergyFn") or __getattr__("EnergyFn")
    return fn.apply(theta, spec, params, opts)
