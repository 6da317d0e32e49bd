"""ctypes declarations of the C ABI in ``include/fsmt.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsmt.so")

FSMT_OK, FSMT_EINVAL, FSMT_ENOMEM, FSMT_EUNSUPPORTED, FSMT_ELIMIT, FSMT_EHIP, FSMT_EABORTED = (
    0, -1, -2, -3, -4, -5, -6)
FSMT_HOST_ONLY = -2
FSMT_PROJ_UNIT, FSMT_PROJ_BOX = 0, 1
FSMT_MSG_AUTO, FSMT_MSG_LDS, FSMT_MSG_GENERIC = 0, 1, 2
FSMT_ACCUMULATE = 1

EXPORTED = ["fsmt_last_error", "xbdd_compile", "xbdd_free", "xbdd_info", "xbdd_export_diagram",
            "cop_forward", "cop_backward", "pgd_step", "round_and_check", "erwa_update",
            "fsmt_solve_batched", "fsmt_solve_batched_noalloc", "fsmt_solve_status"]


class Problem(ct.Structure):
    _fields_ = [("n_bool", ct.c_int32), ("n_real", ct.c_int32), ("n_atoms", ct.c_int32),
                ("n_cons", ct.c_int32)] + [(k, ct.c_void_p) for k in (
                    "atom_ptr", "atom_var", "atom_coef", "atom_rhs", "atom_op", "con_kind",
                    "con_ptr", "con_lit", "con_param", "expr_ptr", "expr_ops", "real_lo",
                    "real_hi")]


class CompileOpts(ct.Structure):
    _fields_ = [("device", ct.c_int32), ("max_nodes", ct.c_int32), ("projection", ct.c_int32),
                ("messages", ct.c_int32), ("reserved", ct.c_int32 * 4)]


class Stats(ct.Structure):
    _fields_ = [("n_bool", ct.c_int32), ("n_real", ct.c_int32), ("n_atoms", ct.c_int32),
                ("n_cons", ct.c_int32), ("total_nodes", ct.c_int64), ("n_templates", ct.c_int32),
                ("max_nodes", ct.c_int32), ("max_slots", ct.c_int32), ("n_positions", ct.c_int32),
                ("table_bytes", ct.c_int64), ("atom_nnz", ct.c_int64), ("n_box_units", ct.c_int32),
                ("n_halfspaces", ct.c_int32), ("n_big", ct.c_int32),
                ("n_hs_colors", ct.c_int32), ("n_pair", ct.c_int32),
                ("hs_separable", ct.c_int32), ("n_gd", ct.c_int32), ("n_gd_sep", ct.c_int32)]


class View(ct.Structure):
    _fields_ = [("data", ct.c_void_p), ("rows", ct.c_int32), ("cols", ct.c_int32),
                ("stride_r", ct.c_int64), ("stride_v", ct.c_int64)]


class SolveOpts(ct.Structure):
    _fields_ = [("kappas", ct.c_void_p), ("n_levels", ct.c_int32), ("steps_per_level", ct.c_int32),
                ("eta_a", ct.c_float), ("eta_b", ct.c_float), ("eps", ct.c_float),
                ("rho", ct.c_float), ("gamma", ct.c_float), ("tau", ct.c_int32),
                ("normalize", ct.c_int32), ("stop_on_sat", ct.c_int32), ("schedule", ct.c_int32),
                ("cluster", ct.c_int32), ("level_begin", ct.c_int32), ("spin_limit", ct.c_int32),
                ("inst_schedule", ct.c_void_p)]


class SolveState(ct.Structure):
    _fields_ = [("a", View), ("b", View)] + [(k, ct.c_void_p) for k in (
        "w", "hist", "grad_a", "grad_b", "sat_bits", "n_unsat", "verdict", "level_done",
        "steps_done", "obj")]


_lib = None


def load() -> ct.CDLL:
    """Load the HIP library. There is no fallback: a missing library is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_2603_22877_amd/build.py")
    L = ct.CDLL(LIB_PATH)
    vp, i32, f32, f64 = ct.c_void_p, ct.c_int32, ct.c_float, ct.c_double
    L.fsmt_last_error.restype = ct.c_char_p
    L.fsmt_last_error.argtypes = []
    L.xbdd_compile.argtypes = [ct.POINTER(Problem), ct.POINTER(CompileOpts), ct.POINTER(vp)]
    L.xbdd_compile.restype = i32
    L.xbdd_free.argtypes = [vp]
    L.xbdd_free.restype = None
    L.xbdd_info.argtypes = [vp, ct.POINTER(Stats)]
    L.xbdd_info.restype = i32
    L.xbdd_export_diagram.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]
    L.xbdd_export_diagram.restype = i32
    L.cop_forward.argtypes = [vp, View, View, f64, View, vp, View, i32, vp]
    L.cop_forward.restype = i32
    L.cop_backward.argtypes = [vp, View, View, f64, View, vp, View, View, i32, vp]
    L.cop_backward.restype = i32
    L.pgd_step.argtypes = [vp, View, View, View, View, f32, f32, vp, i32, vp]
    L.pgd_step.restype = i32
    L.round_and_check.argtypes = [vp, View, View, vp, vp, vp, vp, vp]
    L.round_and_check.restype = i32
    L.erwa_update.argtypes = [vp, i32, vp, vp, vp, i32, f32, f32, i32, i32, vp]
    L.erwa_update.restype = i32
    L.fsmt_solve_batched.argtypes = [vp, i32, ct.POINTER(SolveOpts), vp, vp]
    L.fsmt_solve_batched.restype = i32
    L.fsmt_solve_batched_noalloc.argtypes = [vp, i32, ct.POINTER(SolveOpts), vp, vp]
    L.fsmt_solve_batched_noalloc.restype = i32
    L.fsmt_solve_status.argtypes = [vp, i32, vp]
    L.fsmt_solve_status.restype = i32
    _lib = L
    return L


class FsmtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fsmt error {code}: {msg}")
        self.code = code


def check(rc: int) -> None:
    if rc != FSMT_OK:
        raise FsmtError(rc, load().fsmt_last_error().decode(errors="replace"))
