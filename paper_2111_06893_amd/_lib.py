"""ctypes declarations of the C ABI in include/dgtn.h."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build, or another build of the same sources named by DGTN_LIBRARY
LIB_PATH = os.environ.get("DGTN_LIBRARY") or os.path.join(HERE, "libdgtn.so")
HEADER = os.path.join(HERE, "..", "include", "dgtn.h")

c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class Material(ctypes.Structure):
    _fields_ = [("kind", c_int), ("youngs", c_double), ("poisson", c_double),
                ("c11", c_double), ("c12", c_double), ("c44", c_double)]


class Layer(ctypes.Structure):
    _fields_ = [("thickness", c_double), ("n_elem", c_int), ("ratio", c_double), ("material", c_int)]


class ProblemC(ctypes.Structure):
    _fields_ = [("domain", c_int), ("R", c_double), ("refine", c_int), ("Lx", c_double), ("Ly", c_double),
                ("nx", c_int), ("ny", c_int), ("p", c_int), ("n_layers", c_int),
                ("layers", ctypes.POINTER(Layer)), ("n_materials", c_int),
                ("materials", ctypes.POINTER(Material)), ("F0", c_double), ("r0", c_double),
                ("xc", c_double), ("yc", c_double), ("bc_top", c_int), ("bc_bottom", c_int),
                ("bc_side", c_int), ("penalty", c_double), ("n_columns", c_int), ("map_order", c_int),
                ("columns_xy", ctypes.POINTER(c_double))]


class Info(ctypes.Structure):
    _fields_ = [("n_elem", c_int), ("N", c_int), ("n_cols", c_int), ("n_zelem", c_int),
                ("n_layers", c_int), ("n_dof", ctypes.c_longlong), ("y_ref", c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("precond_precision", c_int), ("restart", c_int), ("max_iter", c_int), ("rtol", c_double),
                ("mg_levels", c_int), ("smooth_steps", c_int), ("smooth_damping", c_double),
                ("smoother", c_int), ("krylov", c_int), ("overlap", c_int), ("residual_precision", c_int)]


class Param(ctypes.Structure):
    _fields_ = [("kind", c_int), ("index", c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", c_int), ("restarts", c_int), ("rel_res", c_double), ("t_solve_s", c_double)]


P = ctypes.POINTER
_SIGS = {
    "dgtn_create": (c_int, [P(ProblemC), P(c_void_p)]),
    "dgtn_get_info": (c_int, [c_void_p, P(Info)]),
    "dgtn_workspace_bytes": (c_int, [c_void_p, P(SolveOpts), P(c_size_t)]),
    "dgtn_bind": (c_int, [c_void_p, c_void_p, c_size_t, P(SolveOpts), c_void_p]),
    "dgtn_apply": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "dgtn_apply_stage": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "dgtn_rhs": (c_int, [c_void_p, c_void_p, c_void_p]),
    "dgtn_residual": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "dgtn_solve": (c_int, [c_void_p, P(SolveOpts), c_void_p, c_void_p, P(SolveStats), c_void_p]),
    "dgtn_precondition": (c_int, [c_void_p, P(SolveOpts), c_void_p, c_void_p, c_void_p]),
    "dgtn_energy": (c_int, [c_void_p, c_void_p, P(c_double), P(c_double), c_void_p]),
    "dgtn_material_constants": (c_int, [P(Material), P(c_double)]),
    "dgtn_energy_noalloc": (c_int, [c_void_p, c_void_p, P(c_double), P(c_double), c_void_p]),
    "dgtn_energy_grad": (c_int, [c_void_p, c_void_p, P(c_double), c_void_p, c_void_p]),
    "dgtn_grad": (c_int, [c_void_p, c_void_p, c_void_p, P(c_double), c_int, P(Param), P(c_double), c_void_p]),
    "dgtn_noise_psd": (c_int, [P(c_double), P(c_double), c_int, c_double, c_double, c_double, P(c_double)]),
    "dgtn_energy_parts": (c_int, [c_void_p, c_void_p, P(c_double), c_void_p]),
    "dgtn_jump_indicator": (c_int, [c_void_p, c_void_p, c_int, P(c_double), P(c_double), c_void_p]),
    "dgtn_noise_psd_parts": (c_int, [P(c_double), P(c_double), c_int, c_double, c_double, c_double,
                                     P(c_double)]),
    "dgtn_node_coords": (c_int, [c_void_p, P(c_double)]),
    "dgtn_level_info": (c_int, [c_void_p, P(SolveOpts), c_int, P(c_int), P(c_int), P(c_int)]),
    "dgtn_smoother_block": (c_int, [c_void_p, P(SolveOpts), c_int, c_int, P(c_double)]),
    "dgtn_patch_table": (c_int, [c_void_p, P(SolveOpts), c_int, P(c_int), P(c_int)]),
    "dgtn_destroy": (None, [c_void_p]),
    "dgtn_last_error": (ctypes.c_char_p, []),
}

_lib = None


def header_symbols():
    """Function names declared in include/dgtn.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:dgtn_status|void|const char\*)\s+(dgtn_\w+)\s*\(", txt, re.M)))


def load():
    """The HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                           "(python paper_2111_06893_amd/build.py)")
    # torch first: it ships its own HIP runtime under the same soname as the
    # system one the library links, so whichever is loaded first serves both.
    # Loaded the other way round, torch runs on the system runtime, and the
    # library's calls then found no device.  Torch's is the one the device
    # memory and streams come from.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DgtnError(RuntimeError):
    pass


STATUS = {0: "DGTN_OK", -1: "DGTN_EINVAL", -2: "DGTN_EMESH", -3: "DGTN_EHIP", -4: "DGTN_ENOCONV",
          -5: "DGTN_ENOMEM", -6: "DGTN_ENAN"}


def check(st):
    if st != 0:
        msg = load().dgtn_last_error().decode()
        raise DgtnError(f"{STATUS.get(st, st)}: {msg}")
