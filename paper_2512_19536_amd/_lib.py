"""ctypes binding of libpdg's C-ABI (include/pdg.h).  Argument marshalling only.

Every function here forwards to the C entry point of the same name; non-OK
statuses raise :class:`PdgError`.  The library must have been built in-tree
(``paper_2512_19536_amd/libpdg.so``); importing this module without it fails
loudly -- there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdg.so")

PDG_OK, PDG_EINVAL, PDG_ENOMEM, PDG_EHIP, PDG_ENOTSPD, PDG_ENOCONV, PDG_EBREAKDOWN, PDG_ENONFINITE, PDG_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
PDG_F64, PDG_F32, PDG_BF16 = 0, 1, 2
PDG_OPT_TRUE_RESIDUAL, PDG_OPT_CHUNK, PDG_OPT_KERNEL_TIMING, PDG_OPT_SCHWARZ_ITEM_KB = 1, 2, 3, 4
PDG_OPT_GRAPH, PDG_OPT_SPMV_WAVES, PDG_OPT_PRECONDITIONER, PDG_OPT_LANCZOS_CAP = 5, 6, 7, 8
PDG_OPT_ION_EXTRAPOLATION, PDG_OPT_PRESUM, PDG_OPT_BF16_MARGIN = 9, 10, 11
PRECISIONS = {"f64": PDG_F64, "f32": PDG_F32, "bf16": PDG_BF16}

#: every symbol declared in include/pdg.h
EXPORTS = (
    "pdg_create", "pdg_destroy", "pdg_last_error", "pdg_status_string", "pdg_set_mesh", "pdg_set_systems",
    "pdg_get_sizes",
    "pdg_assemble", "pdg_get_matrix", "pdg_set_ionic", "pdg_setup_preconditioner", "pdg_get_precond_sizes",
    "pdg_get_local_inverse", "pdg_get_coarse", "pdg_workspace_query", "pdg_bind_workspace", "pdg_set_option",
    "pdg_kernel_timing", "pdg_project_p0", "pdg_spmv", "pdg_precond_apply", "pdg_precond_apply_noalloc", "pdg_ionic", "pdg_rhs",
    "pdg_solve", "pdg_step", "pdg_get_system_info", "pdg_step_batch", "pdg_autotune", "pdg_step_guess", "pdg_lanczos",
    "pdg_get_pcg_coefficients",
    "pdg_guess_extrapolate", "pdg_mlp_create", "pdg_mlp_destroy", "pdg_mlp_last_error", "pdg_mlp_get_sizes",
    "pdg_mlp_bind_workspace", "pdg_mlp_set_params", "pdg_mlp_get_params", "pdg_mlp_set_normalisation",
    "pdg_mlp_set_batch", "pdg_mlp_features", "pdg_mlp_targets", "pdg_mlp_forward", "pdg_mlp_guess",
    "pdg_mlp_gradients", "pdg_mlp_train_step",
)


class PdgMesh(ctypes.Structure):
    _fields_ = [("dim", c_int32), ("n_elem", c_int64), ("cell_ptr", c_void_p), ("cell_geom", c_void_p),
                ("n_facet", c_int64), ("facet_elem", c_void_p), ("facet_geom", c_void_p),
                ("facet_normal", c_void_p), ("sigma", c_void_p)]


class PdgPrecondDesc(ctypes.Structure):
    _fields_ = [("n_sub", c_int32), ("elem_sub", c_void_p), ("n_coarse", c_int32), ("elem_coarse", c_void_p),
                ("coarse_q", c_int32), ("local_prec", c_int32), ("coarse_prec", c_int32)]


class PdgSolveInfo(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("relres", c_double), ("true_relres", c_double), ("bnorm", c_double),
                ("guess_used", c_int32), ("local_fp32", c_int32)]

    def as_dict(self):
        return {"iters": self.iters, "relres": self.relres, "true_relres": self.true_relres, "bnorm": self.bnorm,
                "guess_used": self.guess_used, "local_fp32": self.local_fp32}


class PdgMlpDesc(ctypes.Structure):
    _fields_ = [("n_in", c_int32), ("width", c_int32), ("n_out", c_int32), ("n_out_valid", c_int32),
                ("max_rows", c_int64)]


class PdgTuneResult(ctypes.Structure):
    _fields_ = [("item_kb", c_int32), ("spmv_waves", c_int32), ("coarse_split", c_int32),
                ("candidates", c_int32), ("iter_us_before", c_double), ("iter_us", c_double)]

    def as_dict(self):
        return {"item_kb": self.item_kb, "spmv_waves": self.spmv_waves, "coarse_split": self.coarse_split,
                "candidates": self.candidates,
                "iter_us_before": self.iter_us_before, "iter_us": self.iter_us}


class PdgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpdg.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_2512_19536_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    V, I32, I64, D, P = c_void_p, c_int32, c_int64, c_double, c_void_p
    sig = {
        "pdg_create": (I32, [POINTER(c_void_p), I32, V]),
        "pdg_destroy": (None, [V]),
        "pdg_last_error": (c_char_p, [V]),
        "pdg_status_string": (c_char_p, [I32]),
        "pdg_set_mesh": (I32, [V, POINTER(PdgMesh), I32]),
        "pdg_set_systems": (I32, [V, I32, P]),
        "pdg_get_sizes": (I32, [V, P, P, P, P]),
        "pdg_assemble": (I32, [V, D, D, D, D]),
        "pdg_get_matrix": (I32, [V, P, P, P, P]),
        "pdg_set_ionic": (I32, [V, P, I32]),
        "pdg_setup_preconditioner": (I32, [V, POINTER(PdgPrecondDesc)]),
        "pdg_get_precond_sizes": (I32, [V, I32, P, P, P]),
        "pdg_get_local_inverse": (I32, [V, I32, P]),
        "pdg_get_coarse": (I32, [V, P, P]),
        "pdg_workspace_query": (I32, [V, POINTER(c_size_t)]),
        "pdg_bind_workspace": (I32, [V, P, c_size_t]),
        "pdg_set_option": (I32, [V, I32, I64]),
        "pdg_kernel_timing": (I32, [V, POINTER(I64), POINTER(D), POINTER(D)]),
        "pdg_project_p0": (I32, [V, P, I32, P]),
        "pdg_spmv": (I32, [V, P, P]),
        "pdg_precond_apply": (I32, [V, P, P]),
        "pdg_precond_apply_noalloc": (I32, [V, P, P]),
        "pdg_ionic": (I32, [V, P, P, P, P]),
        "pdg_rhs": (I32, [V, P, P, P, P]),
        "pdg_solve": (I32, [V, P, P, D, I32, POINTER(PdgSolveInfo)]),
        "pdg_step": (I32, [V, P, P, P, P, D, I32, POINTER(PdgSolveInfo)]),
        "pdg_get_system_info": (I32, [V, I32, POINTER(PdgSolveInfo), POINTER(I32)]),
        "pdg_step_batch": (I32, [P, I32, P, P, P, P, D, I32, P]),
        "pdg_autotune": (I32, [V, I32, POINTER(PdgTuneResult)]),
        "pdg_lanczos": (I32, [V, I32, POINTER(D), POINTER(D), POINTER(D)]),
        "pdg_get_pcg_coefficients": (I32, [V, I32, P, P, I32]),
        "pdg_step_guess": (I32, [V, P, P, P, P, P, D, I32, POINTER(PdgSolveInfo)]),
        "pdg_guess_extrapolate": (I32, [V, P, P, P, I32, P]),
        "pdg_mlp_create": (I32, [POINTER(c_void_p), I32, V, POINTER(PdgMlpDesc)]),
        "pdg_mlp_destroy": (None, [V]),
        "pdg_mlp_last_error": (c_char_p, [V]),
        "pdg_mlp_get_sizes": (I32, [V, POINTER(I64), POINTER(c_size_t)]),
        "pdg_mlp_bind_workspace": (I32, [V, P, c_size_t]),
        "pdg_mlp_set_params": (I32, [V, P, I64]),
        "pdg_mlp_get_params": (I32, [V, P, I64]),
        "pdg_mlp_set_normalisation": (I32, [V, P, P, P, P]),
        "pdg_mlp_set_batch": (I32, [V, I64, P, P, P]),
        "pdg_mlp_features": (I32, [V, I64, I64, I64, I32, P, P, P, P, P, P]),
        "pdg_mlp_targets": (I32, [V, I64, I64, I64, I32, P, P, P]),
        "pdg_mlp_forward": (I32, [V, I64, P]),
        "pdg_mlp_guess": (I32, [V, I64, I64, I32, P, P]),
        "pdg_mlp_gradients": (I32, [V, I64, I64, P, POINTER(D)]),
        "pdg_mlp_train_step": (I32, [V, I64, I64, c_float, c_float, c_float, c_float, POINTER(D)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(status):
    return load().pdg_status_string(status).decode()


def check(ctx, status):
    if status != PDG_OK:
        msg = load().pdg_last_error(ctx).decode() if ctx else ""
        raise PdgError(status, msg)


def check_mlp(mlp, status):
    if status != PDG_OK:
        msg = load().pdg_mlp_last_error(mlp).decode() if mlp else ""
        raise PdgError(status, msg)
