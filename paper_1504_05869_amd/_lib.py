"""ctypes declarations of the C ABI in include/lkp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

# torch's HIP runtime must be the one liblkp binds to: load torch first so the
# dynamic linker reuses its libamdhip64 for liblkp's dependency.
import torch  # noqa: F401

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblkp.so")

LATTICES = {"D1Q5": 0, "D1Q9": 1, "D1Q13": 2, "D2Q5": 3, "D2Q9": 4, "D2Q25": 5,
            "D2Q81": 6, "D2Q169": 7, "D3Q111": 8, "D2Q37": 9, "D2Q77": 10, "D3Q107": 11}
PRECISIONS = {"f64": 0, "f32": 1, "f32_ir": 2, "bf16dev_ir": 3}
STATUS = {0: "LKP_OK", 1: "LKP_ERR_ARG", 2: "LKP_ERR_LATTICE_ORDER", 3: "LKP_ERR_UNSTABLE",
          4: "LKP_ERR_SOURCE_MEAN", 5: "LKP_ERR_OOM", 6: "LKP_ERR_HIP",
          7: "LKP_ERR_NOT_CONVERGED", 8: "LKP_ERR_DIVERGED", 9: "LKP_ERR_STATE",
          10: "LKP_ERR_UNSUPPORTED"}
EXPORTS = ["lkp_create", "lkp_destroy", "lkp_footprint_bytes", "lkp_contraction_bound",
           "lkp_solve", "lkp_step",
           "lkp_residual", "lkp_get_phi", "lkp_get_populations", "lkp_set_populations",
           "lkp_lattice_info", "lkp_get_info", "lkp_get_coefficients", "lkp_set_equilibrium",
           "lkp_sync", "lkp_last_error",
           "lkp_group_create", "lkp_group_add", "lkp_group_remove", "lkp_group_step",
           "lkp_group_destroy", "lkp_group_graph_stats", "lkp_group_split",
           "lkp_residual_noalloc"]
MEMBER_STATES = {0: "running", 1: "converged", 2: "failed"}
FLAG_POPULATION_SWEEP = 1
FLAG_IN_PLACE = 2


class ProblemDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("lattice", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3), ("order", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tau_lb", ctypes.c_double),
                ("knudsen", ctypes.c_double), ("source", ctypes.c_void_p),
                ("source_on_device", ctypes.c_int32), ("subtract_mean", ctypes.c_int32),
                ("allow_unstable", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("drift", ctypes.c_double * 3),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_int64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol_rel_l2", ctypes.c_double), ("tol_maxchange", ctypes.c_double),
                ("max_sweeps", ctypes.c_int64), ("check_every", ctypes.c_int32),
                ("max_outer", ctypes.c_int32), ("ir_inner_tol", ctypes.c_double),
                ("use_graph", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SolveReport(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("total_sweeps", ctypes.c_int64),
                ("outer", ctypes.c_int32), ("status", ctypes.c_int32),
                ("max_change", ctypes.c_double), ("l2_change", ctypes.c_double),
                ("phi_l2", ctypes.c_double), ("mass", ctypes.c_double),
                ("est_rel_err", ctypes.c_double), ("rate", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("glups", ctypes.c_double)]


class ResidualReport(ctypes.Structure):
    _fields_ = [("max_change", ctypes.c_double), ("l2_change", ctypes.c_double),
                ("pop_residual_l2", ctypes.c_double), ("phi_l2", ctypes.c_double),
                ("mass", ctypes.c_double), ("sweeps", ctypes.c_int64)]


class HandleInfo(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("order", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("Q", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("velocity_groups", ctypes.c_int32), ("scalar_stencil", ctypes.c_int32),
                ("in_place", ctypes.c_int32), ("stencil_tile", ctypes.c_int32),
                ("stencil_remap", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
                ("tau_lb", ctypes.c_double), ("omega", ctypes.c_double),
                ("cs2", ctypes.c_double), ("total_sweeps", ctypes.c_int64),
                ("footprint_bytes", ctypes.c_int64)]


class MemberReport(ctypes.Structure):
    _fields_ = [("handle", ctypes.c_void_p), ("state", ctypes.c_int32), ("status", ctypes.c_int32),
                ("sweeps", ctypes.c_int64), ("outer", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("est_rel_err", ctypes.c_double), ("max_change", ctypes.c_double),
                ("phi_l2", ctypes.c_double)]


_LIB = None


def load() -> ctypes.CDLL:
    """Load liblkp.so (built in-tree); fails loudly when it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1504_05869_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    P = ctypes.POINTER
    sig = {
        "lkp_create": (ctypes.c_int, [P(ProblemDesc), P(H)]),
        "lkp_destroy": (ctypes.c_int, [H]),
        "lkp_footprint_bytes": (ctypes.c_int64, [P(ProblemDesc)]),
        "lkp_contraction_bound": (ctypes.c_int, [P(ProblemDesc), P(ctypes.c_double)]),
        "lkp_solve": (ctypes.c_int, [H, P(SolveOpts), P(SolveReport)]),
        "lkp_step": (ctypes.c_int, [H, ctypes.c_int64]),
        "lkp_residual": (ctypes.c_int, [H, P(ResidualReport)]),
        "lkp_get_phi": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_int32]),
        "lkp_get_populations": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_int32]),
        "lkp_set_populations": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_int32]),
        "lkp_lattice_info": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32,
                                            P(ctypes.c_int32), P(ctypes.c_int32),
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, P(ctypes.c_double)]),
        "lkp_get_info": (ctypes.c_int, [H, P(HandleInfo)]),
        "lkp_get_coefficients": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_void_p]),
        "lkp_set_equilibrium": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_int32]),
        "lkp_sync": (ctypes.c_int, [H]),
        "lkp_residual_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int64),
                                                ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p]),
        "lkp_last_error": (ctypes.c_char_p, []),
        "lkp_group_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_void_p, P(H)]),
        "lkp_group_add": (ctypes.c_int, [H, H, P(SolveOpts)]),
        "lkp_group_remove": (ctypes.c_int, [H, H]),
        "lkp_group_step": (ctypes.c_int, [H, ctypes.c_int32, P(MemberReport), ctypes.c_int32,
                                          P(ctypes.c_int32)]),
        "lkp_group_destroy": (ctypes.c_int, [H]),
        "lkp_group_graph_stats": (ctypes.c_int, [H, P(ctypes.c_int64), P(ctypes.c_int64)]),
        "lkp_group_split": (ctypes.c_int, [H, P(ctypes.c_int32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class LkpError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().lkp_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


def check(status: int, where: str):
    if status != 0:
        raise LkpError(status, where)
