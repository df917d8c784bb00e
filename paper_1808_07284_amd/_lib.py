"""ctypes declarations of the C ABI in include/emd_mi355x.h.

Loading fails loudly (RuntimeError) when the built library is missing: there is no
fallback implementation of any step.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# EMD_MI355X_LIB selects another build of the same sources (e.g. one with host-side
# sanitizers); by default the in-tree build is loaded
LIB_PATH = os.environ.get("EMD_MI355X_LIB") or os.path.join(PKG, "libemd_mi355x.so")

# call status
EMD_SUCCESS = 0
STATUS_NAMES = {0: "EMD_SUCCESS", 1: "EMD_ERR_INVALID_ARGUMENT", 2: "EMD_ERR_NULL_POINTER",
                3: "EMD_ERR_DEVICE", 4: "EMD_ERR_HIP", 5: "EMD_ERR_OUT_OF_MEMORY",
                6: "EMD_ERR_UNSUPPORTED"}
# per-gather status
GATHER_STATUS = ["RUNNING", "CONVERGED", "MAX_ITER", "ZERO_SOURCE", "NONFINITE", "LS_FAIL",
                 "MASS_IMBALANCE"]
MASS_BALANCE, MASS_UNIT, MASS_NONE = 0, 1, 2
LS_L2, LS_L1, LS_FIXED = 0, 1, 2
F32, F64 = 0, 1

# every symbol the public header declares
EXPORTED = ["emd_params_default", "emd_plan_create", "emd_plan_destroy", "emd_plan_set_params",
            "emd_plan_set_tiling", "emd_plan_set_gather_tiling", "emd_plan_get_gather_tiling",
            "emd_plan_autotune", "emd_plan_set_history", "emd_plan_query", "emd_decompose", "emd_pdhg_solve",
            "emd_pdhg_solve_replay", "emd_solver_state", "emd_pdhg_solve_resume",
            "emd_adjoint_source", "emd_lsd_misfit", "emd_restrict", "emd_prolong",
            "emd_decompose_noalloc", "emd_status_string", "emd_last_error"]


class GatherDesc(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nt", C.c_int32), ("dx", C.c_double), ("dt", C.c_double),
                ("offset", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("eps", C.c_double), ("xi", C.c_double), ("zeta", C.c_double),
                ("delta", C.c_double), ("alpha1", C.c_double), ("alpha_max_factor", C.c_double),
                ("tol_res", C.c_double), ("mass_tol", C.c_double), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("max_ls_trials", C.c_int32), ("ls_mode", C.c_int32),
                ("mass_mode", C.c_int32), ("precision", C.c_int32),
                ("sweeps_per_sync", C.c_int32), ("iters_per_sweep", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("ls_trials", C.c_int32),
                ("pad", C.c_int32), ("rel_res", C.c_double), ("emd", C.c_double),
                ("transport", C.c_double), ("alpha", C.c_double), ("primal", C.c_double)]


class GatherState(C.Structure):
    _fields_ = [("alpha", C.c_double), ("theta", C.c_double), ("iters", C.c_int32),
                ("ls_trials", C.c_int32), ("status", C.c_int32), ("pad", C.c_int32),
                ("rel_res", C.c_double), ("primal", C.c_double), ("transport", C.c_double)]


class PlanStats(C.Structure):
    _fields_ = [("ngather", C.c_int32), ("tiles", C.c_int32), ("rows_per_tile", C.c_int32),
                ("samples_per_tile", C.c_int32), ("batch_len", C.c_int64), ("cells", C.c_int64),
                ("workspace_bytes", C.c_int64), ("last_sweeps", C.c_int64),
                ("last_cell_updates", C.c_int64), ("last_sweep_ms", C.c_double),
                ("last_table_rebuilds", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises RuntimeError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1808_07284_amd.build` "
                           "(there is no non-HIP implementation)")
    lib = C.CDLL(path)
    vp = C.c_void_p
    st = C.c_int32
    lib.emd_params_default.argtypes = [C.POINTER(Params)]
    lib.emd_plan_create.argtypes = [C.POINTER(GatherDesc), C.c_int32, C.c_int64,
                                    C.POINTER(Params), C.POINTER(vp)]
    lib.emd_plan_destroy.argtypes = [vp]
    lib.emd_plan_set_params.argtypes = [vp, C.POINTER(Params)]
    lib.emd_plan_set_tiling.argtypes = [vp, C.c_int32]
    lib.emd_plan_set_gather_tiling.argtypes = [vp, C.POINTER(C.c_int32)]
    lib.emd_plan_get_gather_tiling.argtypes = [vp, C.POINTER(C.c_int32)]
    lib.emd_plan_autotune.argtypes = [vp, vp, C.c_int32, vp]
    lib.emd_plan_set_history.argtypes = [vp, vp, C.c_int32]
    lib.emd_plan_query.argtypes = [vp, C.POINTER(PlanStats)]
    lib.emd_decompose.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.emd_pdhg_solve.argtypes = [vp, vp, vp, vp, C.c_int32, vp, vp, vp, vp]
    lib.emd_pdhg_solve_replay.argtypes = [vp, vp, vp, vp, C.c_int32, vp, C.c_int32, vp, vp, vp]
    lib.emd_adjoint_source.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.emd_solver_state.argtypes = [vp, C.POINTER(GatherState)]
    lib.emd_pdhg_solve_resume.argtypes = [vp, vp, vp, vp, C.POINTER(GatherState), vp, vp, vp, vp]
    lib.emd_lsd_misfit.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.emd_restrict.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, vp, vp]
    lib.emd_prolong.argtypes = [vp, vp, C.c_int32, C.c_int32, vp, vp, vp, vp, vp]
    lib.emd_decompose_noalloc.argtypes = [C.POINTER(GatherDesc), C.c_int32, C.c_int32, C.c_int32,
                                          vp, vp, vp, vp, vp, vp, vp]
    for name in EXPORTED:
        if name not in ("emd_status_string", "emd_last_error"):
            getattr(lib, name).restype = st
    lib.emd_status_string.argtypes = [st]
    lib.emd_status_string.restype = C.c_char_p
    lib.emd_last_error.argtypes = []
    lib.emd_last_error.restype = C.c_char_p
    _lib = lib
    return lib


class EMDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int):
    if status != EMD_SUCCESS:
        raise EMDError(status, load().emd_last_error().decode())
