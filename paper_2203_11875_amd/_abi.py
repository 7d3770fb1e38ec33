"""ctypes declarations of the C ABI in include/rhipm.h (argument marshalling only).

The library is loaded from this package directory; there is no fallback: if
librhipm.so is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# RHIPM_LIB selects another build of the library (the host-sanitised one)
LIB_PATH = os.environ.get("RHIPM_LIB") or os.path.join(HERE, "librhipm.so")

RH_OK, RH_NOT_POSDEF, RH_SMALL_PIVOT, RH_NOT_CONVERGED = 0, 1, 2, 3
RH_ERR_ARG, RH_ERR_HIP, RH_ERR_OOM, RH_ERR_SINGULAR, RH_ERR_STATE = -1, -2, -3, -4, -5

i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)
vp = C.c_void_p


class rh_network_desc(C.Structure):
    _fields_ = [("nb", C.c_int32), ("nl", C.c_int32), ("ng", C.c_int32),
                ("base_mva", C.c_double),
                ("bus_type", i32p), ("pd", f64p), ("qd", f64p), ("vmin", f64p),
                ("vmax", f64p), ("from_", i32p), ("to", i32p), ("r", f64p), ("x", f64p),
                ("b", f64p), ("rate", f64p), ("gen_bus", i32p), ("c2", f64p), ("c1", f64p),
                ("c0", f64p), ("pmin", f64p), ("pmax", f64p), ("qmin", f64p), ("qmax", f64p)]


class rh_options(C.Structure):
    _fields_ = [("panel_width", C.c_int32), ("ordering", C.c_int32),
                ("lds_panel", C.c_int32), ("refactor", C.c_int32), ("cond_waves", C.c_int32),
                ("sweep_grouping", C.c_int32)]


class rh_info(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "nx", "nu", "m", "nb", "nl", "ng", "nnz_gx", "nnz_lu", "nnz_gu", "nnz_a", "nnz_k",
        "levels_lower", "levels_upper", "refactor_ops", "max_lu_row", "panel_width",
        "lds_panel", "max_row_ops", "refactor_kernel", "steps_lower", "sweep_steps",
        "refactor_split", "cond_waves", "steps_l", "steps_u", "steps_ut", "steps_lt",
        "groups_l", "groups_u", "groups_ut", "groups_lt", "sweep_grouped")]


class rh_ipm_options(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("reserved0", C.c_int32),
                ("mu_init", C.c_double), ("obj_scale", C.c_double),
                ("reserved", C.c_int64 * 4)]


class rh_ipm_info(C.Structure):
    _fields_ = [("iter", C.c_int64), ("obj", C.c_double), ("inf_pr", C.c_double),
                ("err", C.c_double), ("mu", C.c_double), ("alpha_pr", C.c_double),
                ("alpha_du", C.c_double), ("delta_w", C.c_double), ("ls_trials", C.c_int64),
                ("obj_scale", C.c_double), ("converged", C.c_int32), ("pf_iters", C.c_int32)]


class rh_batch_condense_item(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("x", "u", "lam", "y", "sig_x", "sig_u", "sig_s", "r",
                                          "K")] + [("ldk", C.c_int64), ("rhs", C.c_void_p)]


class rh_batch_solve_item(C.Structure):
    _fields_ = [("K", C.c_void_p), ("ldk", C.c_int64), ("delta_w", C.c_double),
                ("rhs", C.c_void_p), ("r", C.c_void_p), ("p", C.c_void_p)]


# name -> (restype, argtypes); every symbol declared in include/rhipm.h
SIGNATURES = {
    "rh_status_str": (C.c_char_p, [C.c_int]),
    "rh_analyze_network": (C.c_int, [C.POINTER(rh_network_desc), C.POINTER(rh_options),
                                     C.POINTER(vp)]),
    "rh_destroy_symbolic": (None, [vp]),
    "rh_symbolic_info": (C.c_int, [vp, C.POINTER(rh_info)]),
    "rh_symbolic_index_maps": (C.c_int, [vp, i32p, i32p, i32p, i32p]),
    "rh_symbolic_gx_pattern": (C.c_int, [vp, i32p, i32p, i32p]),
    "rh_symbolic_host_solve": (C.c_int, [vp, f64p, f64p, f64p, C.c_int32]),
    "rh_symbolic_check_levels": (C.c_int, [vp]),
    "rh_symbolic_check_condense": (C.c_int, [vp, C.c_int32, C.c_uint64, C.POINTER(C.c_double)]),
    "rh_init_network": (C.c_int, [C.POINTER(rh_network_desc), C.POINTER(rh_options), vp,
                                  C.POINTER(vp)]),
    "rh_destroy_network": (None, [vp]),
    "rh_get_info": (C.c_int, [vp, C.POINTER(rh_info)]),
    "rh_get_dims": (C.c_int, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                              C.POINTER(C.c_int64)]),
    "rh_get_index_maps": (C.c_int, [vp, i32p, i32p, i32p, i32p]),
    "rh_set_loads": (C.c_int, [vp, vp, vp]),
    "rh_eval_residual": (C.c_int, [vp, vp, vp, vp, vp, vp]),
    "rh_condense_reduced_hessian": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                              C.c_int64, vp]),
    "rh_solve_condensed_kkt": (C.c_int, [vp, vp, C.c_int64, C.c_double, vp, vp, vp, vp]),
    "rh_cholesky_solve_noalloc": (C.c_int, [vp, C.c_int64, C.c_int32, C.c_double, vp, vp, vp,
                                            vp]),
    "rh_profile_enable": (C.c_int, [vp, C.c_int32]),
    "rh_profile_read": (C.c_int, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "rh_profile_kernel_trace": (C.c_int, [vp, C.POINTER(C.c_int64)]),
    "rh_set_objective_scale": (C.c_int, [vp, C.c_double]),
    "rh_ipm_default_options": (C.c_int, [C.POINTER(rh_ipm_options)]),
    "rh_ipm_create": (C.c_int, [vp, C.POINTER(rh_ipm_options), vp, vp, C.POINTER(vp)]),
    "rh_ipm_step": (C.c_int, [vp, C.POINTER(rh_ipm_info)]),
    "rh_ipm_solve": (C.c_int, [vp, C.POINTER(rh_ipm_info)]),
    "rh_ipm_get_state": (C.c_int, [vp, vp, vp, vp, vp, vp]),
    "rh_ipm_destroy": (None, [vp]),
    "rh_ipm_outputs": (C.c_int, [vp, vp, vp, vp]),
    "rh_ipm_backward": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
    "rh_ipm_batch_step": (C.c_int, [vp, vp, vp, vp]),
    "rh_ipm_batch_backward": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, vp]),
    "rh_power_flow": (C.c_int, [vp, vp, vp, C.c_double, C.c_int32, C.POINTER(C.c_int32),
                                C.POINTER(C.c_double)]),
    "rh_redlin_create": (C.c_int, [vp, C.POINTER(rh_ipm_options), vp, vp, C.POINTER(vp)]),
    "rh_redlin_step": (C.c_int, [vp, C.POINTER(rh_ipm_info)]),
    "rh_redlin_solve": (C.c_int, [vp, C.POINTER(rh_ipm_info)]),
    "rh_redlin_get_state": (C.c_int, [vp, vp, vp, vp, vp, vp]),
    "rh_redlin_dims": (C.c_int, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "rh_redlin_destroy": (None, [vp]),
    "rh_batch_create": (C.c_int, [C.POINTER(vp), C.c_int32, vp, C.POINTER(vp)]),
    "rh_batch_destroy": (None, [vp]),
    "rh_batch_condense": (C.c_int, [vp, C.POINTER(rh_batch_condense_item)]),
    "rh_batch_solve": (C.c_int, [vp, C.POINTER(rh_batch_solve_item), i32p]),
    "rh_batch_capture": (C.c_int, [vp, C.POINTER(rh_batch_condense_item),
                                   C.POINTER(rh_batch_solve_item)]),
    "rh_batch_replay": (C.c_int, [vp, C.POINTER(rh_batch_condense_item),
                                  C.POINTER(rh_batch_solve_item), i32p]),
}

PHASES = ["eval", "refactor", "condense", "symmetrize", "cholesky", "recover", "project"]


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2203_11875_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class RhError(RuntimeError):
    def __init__(self, code: int, where: str, lib=None):
        msg = lib.rh_status_str(code).decode() if lib is not None else str(code)
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code
