"""ctypes binding of libmonox.so (include/monox.h): argument marshalling only.

Every function of the C ABI is exposed under its own name.  Loading fails
loudly (``RuntimeError``) if the library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmonox.so")

# status codes
MDX_OK = 0
MDX_WARN_NOT_CONVERGED = 1
MDX_ERR_INVALID_ARG = -1
MDX_ERR_BAD_MESH = -2
MDX_ERR_DEVICE = -3
MDX_ERR_NO_WORKSPACE = -4
MDX_ERR_NONFINITE = -5
MDX_ERR_STATE = -6
MDX_ERR_UNSUPPORTED = -7

MDX_IONIC_NONE, MDX_IONIC_MS, MDX_IONIC_TT, MDX_IONIC_CRN = 0, 1, 2, 3
MDX_WS_PREV, MDX_WS_EXTRAP, MDX_WS_MLP = 0, 1, 2
MDX_REL_INITIAL, MDX_REL_RHS = 0, 1
MDX_PREC_FP64, MDX_PREC_MIXED, MDX_PREC_MIXED_GATES32 = 0, 1, 2
MDX_MAT_M, MDX_MAT_K, MDX_MAT_A = 0, 1, 2
MDX_TUNE_MAX_GROUPS, MDX_TUNE_ITER_SCHEME = 1, 2
MDX_TUNE_LANES_PER_ROW, MDX_TUNE_TILES_PER_GROUP, MDX_TUNE_GRAPH, MDX_TUNE_FORMAT = 3, 4, 5, 6
MDX_TUNE_NONTEMPORAL = 7
MDX_TUNE_COMPACT_COLUMNS = 8
MDX_TUNE_SPMV_MAX_GROUPS = 9
MDX_TUNE_PERSISTENT = 10
MDX_TUNE_MAX_CANDIDATES = 32


class SolverOpts(C.Structure):
    _fields_ = [("atol", C.c_double), ("rtol", C.c_double), ("rel_mode", C.c_int32),
                ("max_iter", C.c_int32), ("warm_start", C.c_int32), ("precision", C.c_int32),
                ("rr_interval", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("cg_iters_total", C.c_int64),
                ("cg_iters_max", C.c_int64), ("not_converged", C.c_int64),
                ("n_nodes", C.c_int64), ("nnz", C.c_int64), ("n_sell_slots", C.c_int64),
                ("bandwidth", C.c_int64), ("step_loop_seconds", C.c_double),
                ("spmv_timed", C.c_int64), ("spmv_seconds", C.c_double),
                ("spmv_work", C.c_int64), ("spmv_bytes", C.c_double),
                ("host_wait_seconds", C.c_double), ("fallbacks", C.c_int64),
                ("col_index_bytes", C.c_int64)]


class TuneReport(C.Structure):
    _fields_ = [("format", C.c_int32), ("lanes_per_row", C.c_int32),
                ("tiles_per_group", C.c_int32), ("n_candidates", C.c_int32),
                ("seconds", C.c_double), ("bytes", C.c_double),
                ("cand_format", C.c_int32 * MDX_TUNE_MAX_CANDIDATES),
                ("cand_lanes_per_row", C.c_int32 * MDX_TUNE_MAX_CANDIDATES),
                ("cand_tiles_per_group", C.c_int32 * MDX_TUNE_MAX_CANDIDATES),
                ("cand_seconds", C.c_double * MDX_TUNE_MAX_CANDIDATES)]


class MdxError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"mdx status {status}: {message}")
        self.status = status


P = C.c_void_p
_SIGS = {
    "mdx_version": (C.c_int, []),
    "mdx_ionic_nstates": (C.c_int32, [C.c_int32]),
    "mdx_ionic_nparams": (C.c_int32, [C.c_int32]),
    "mdx_create": (C.c_int, [C.POINTER(P), C.c_int, P]),
    "mdx_destroy": (None, [P]),
    "mdx_last_error": (C.c_char_p, [P]),
    "mdx_set_mesh": (C.c_int, [P, C.c_int64, P, C.c_double, C.c_int64, P, P, P]),
    "mdx_set_surface_mesh": (C.c_int, [P, C.c_int64, P, C.c_double, C.c_int64, P, P, P]),
    "mdx_set_surface_mesh_batch": (C.c_int, [P, C.c_int32, P, C.c_int64, P, C.c_double,
                                             C.c_int64, P, P, P]),
    "mdx_set_mesh_batch": (C.c_int, [P, C.c_int32, P, C.c_int64, P, C.c_double, C.c_int64, P, P,
                                     P]),
    "mdx_get_instance_iterations": (C.c_int, [P, C.c_int64, P]),
    "mdx_autotune": (C.c_int, [P, C.c_int32, C.POINTER(TuneReport)]),
    "mdx_add_conductivity": (C.c_int, [P, C.c_int32, P, C.c_double, C.c_double]),
    "mdx_add_conductivity_ie": (C.c_int, [P, C.c_int32, P, C.c_double, C.c_double, C.c_double,
                                          C.c_double]),
    "mdx_set_mass_lumping": (C.c_int, [P, C.c_int32]),
    "mdx_set_tissue": (C.c_int, [P, C.c_double, C.c_double, C.c_double]),
    "mdx_set_ionic": (C.c_int, [P, C.c_int32, C.c_int32, P]),
    "mdx_add_stimulus": (C.c_int, [P, C.c_int64, P, C.c_double, C.c_double, C.c_double]),
    "mdx_set_solver": (C.c_int, [P, C.POINTER(SolverOpts)]),
    "mdx_workspace_size": (C.c_int, [P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "mdx_bind_workspace": (C.c_int, [P, P, C.c_size_t]),
    "mdx_prepare": (C.c_int, [P, C.c_double, P, C.c_size_t]),
    "mdx_run": (C.c_int, [P, C.c_int64, C.c_int64, P]),
    "mdx_get_times": (C.c_int, [P, P, P]),
    "mdx_get_apd": (C.c_int, [P, P]),
    "mdx_get_iterations": (C.c_int, [P, C.c_int64, P]),
    "mdx_get_stats": (C.c_int, [P, C.POINTER(Stats)]),
    "mdx_set_profiling": (C.c_int, [P, C.c_int32]),
    "mdx_set_tuning": (C.c_int, [P, C.c_int32, C.c_int64]),
    "mdx_get_state": (C.c_int, [P, P, P, P, P, P, C.POINTER(C.c_int64)]),
    "mdx_set_state": (C.c_int, [P, P, P, P, P, P, C.c_int64]),
    "mdx_get_matrix": (C.c_int, [P, C.c_int32, C.POINTER(C.c_int64), P, P, P]),
    "mdx_solve": (C.c_int, [P, P, P, P, C.POINTER(C.c_int32)]),
    "mdx_spmv": (C.c_int, [P, C.c_int32, P, P]),
    "mdx_ionic_step": (C.c_int, [P, C.c_double, C.c_int64, P, P, P]),
    "mdx_mlp_nparams": (C.c_int32, []),
    "mdx_set_mlp": (C.c_int, [P, P, P]),
    "mdx_set_recorder": (C.c_int, [P, P, P, P]),
    "mdx_get_node_order": (C.c_int, [P, P]),
    "mdx_mlp_forward": (C.c_int, [P, P, C.c_int64, P, P]),
    "mdx_mlp_grad_scratch": (C.c_size_t, [C.c_int64]),
    "mdx_mlp_grad": (C.c_int, [P, P, C.c_int64, P, P, P, P, P, C.c_size_t]),
    "mdx_mlp_grad_noalloc": (C.c_int, [P, P, C.c_int64, P, P, P, P]),
    "mdx_mlp_adam": (C.c_int, [P, P, P, P, P, C.c_int32, C.c_double, C.c_double, C.c_double,
                               C.c_double]),
    "mdx_mlp_samples": (C.c_int, [P, C.c_int64, P, C.c_int64, P, P, P, P, P]),
}

_lib = None


def lib():
    """The loaded library; raises RuntimeError if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2510_12011_amd.build` "
                "(the HIP library is the only implementation; there is no fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)
