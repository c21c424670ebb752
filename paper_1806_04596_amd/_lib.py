"""ctypes binding of libhypersara.so (argument marshalling only).

Every entry point of ``include/hypersara.h`` is exposed under the same name.
Device buffers are torch tensors on the HIP device; their ``data_ptr()`` is
passed through.  No computation happens here.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhypersara.so")
TUNING_CACHE = os.path.join(HERE, "tuning_cache.jsonl")

HS_OK = 0
HS_F32, HS_F64 = 0, 1
HS_NORM_PHI_PRECOND, HS_NORM_PSI = 0, 1
PRIORS = {"lrjas": 0, "lr": 1, "jas": 2, "sara": 3}
GRAM_MODES = {"f64": 0, "f32": 1, "bf16_split": 2}

STATUS = {0: "HS_OK", -1: "HS_ERR_INVALID_ARG", -2: "HS_ERR_SHAPE", -3: "HS_ERR_DTYPE", -4: "HS_ERR_NOT_PLANNED",
          -5: "HS_ERR_NO_WORKSPACE", -6: "HS_ERR_NONFINITE", -7: "HS_ERR_HIP", -8: "HS_ERR_NOT_CONVERGED"}


class ProblemDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("L", C.c_int32), ("oversamp", C.c_int32), ("J", C.c_int32),
                ("levels", C.c_int32), ("n_db", C.c_int32), ("dtype", C.c_int32), ("tile", C.c_int32),
                ("device", C.c_int32), ("stream", C.c_void_p), ("gram_mode", C.c_int32), ("per_channel", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n_vis", C.c_int64), ("n_blocks", C.c_int64), ("n_bins", C.c_int64), ("n_runs", C.c_int64),
                ("n_degrid_units", C.c_int64), ("n_grid_units", C.c_int64), ("tile", C.c_int32),
                ("kb_terms", C.c_int32), ("workspace_bytes", C.c_size_t)]


class Tuning(C.Structure):
    _fields_ = [("tile", C.c_int32), ("grid_split", C.c_int32), ("degrid_batches", C.c_int32),
                ("fft_col_tile", C.c_int32), ("grid_xcd_group", C.c_int32), ("degrid_xcd_group", C.c_int32),
                ("ms", C.c_double)]


class PDParams(C.Structure):
    _fields_ = [("mu", C.c_double), ("tau", C.c_double), ("kappa1", C.c_double), ("kappa2", C.c_double),
                ("kappa3", C.c_double), ("wbar", C.c_void_p), ("w", C.POINTER(C.c_double)),
                ("adaptive_eps", C.c_int32), ("lam1", C.c_double), ("lam2", C.c_double), ("lam3", C.c_double),
                ("vartheta_bar", C.c_int32), ("prior", C.c_int32)]


class StatePtrs(C.Structure):
    _fields_ = [("X", C.c_void_p), ("Xt", C.c_void_p), ("P", C.c_void_p), ("A", C.c_void_p), ("v", C.c_void_p),
                ("eps", C.POINTER(C.c_double)), ("vartheta", C.POINTER(C.c_int32)),
                ("scalars", C.POINTER(C.c_double)), ("wbar", C.c_void_p), ("w", C.POINTER(C.c_double))]


class SolveParams(C.Structure):
    _fields_ = [("n_reweights", C.c_int32), ("iters_per_reweight", C.c_int32), ("gamma_factor", C.c_double),
                ("beta_tol", C.c_double), ("check_every", C.c_int32), ("gamma0", C.c_double),
                ("gamma_bar0", C.c_double), ("reweight_first", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("reweights", C.c_int32), ("final_beta", C.c_double),
                ("gamma", C.c_double), ("gamma_bar", C.c_double)]


P = C.c_void_p
dptr = C.POINTER(C.c_double)
i64p = C.POINTER(C.c_int64)
ctxp = C.c_void_p

SIGNATURES = {
    "hs_status_string": (C.c_char_p, [C.c_int32]),
    "hs_last_error": (C.c_char_p, [ctxp]),
    "hs_create": (C.c_int32, [C.POINTER(ProblemDesc), C.POINTER(C.c_void_p)]),
    "hs_destroy": (C.c_int32, [ctxp]),
    "hs_set_channel": (C.c_int32, [ctxp, C.c_int32, C.c_int64, C.c_int32, i64p, dptr, dptr, dptr, dptr, dptr]),
    "hs_set_data": (C.c_int32, [ctxp, C.c_int32, dptr, dptr, dptr]),
    "hs_plan": (C.c_int32, [ctxp, C.POINTER(C.c_size_t)]),
    "hs_bind_workspace": (C.c_int32, [ctxp, P, C.c_size_t]),
    "hs_get_info": (C.c_int32, [ctxp, C.POINTER(Info)]),
    "hs_get_tuning": (C.c_int32, [ctxp, C.POINTER(Tuning)]),
    "hs_set_tuning": (C.c_int32, [ctxp, C.POINTER(Tuning)]),
    "hs_autotune_bytes": (C.c_int32, [ctxp, C.POINTER(C.c_size_t)]),
    "hs_autotune": (C.c_int32, [ctxp, P, C.c_size_t, C.c_char_p, C.POINTER(Tuning)]),
    "hs_density_precond": (C.c_int32, [C.c_int64, dptr, C.c_int32, C.c_int32, dptr]),
    "hs_visibility_order": (C.c_int32, [C.c_int64, dptr, dptr, C.c_int32, i64p, C.c_int32, C.c_int32, C.c_int32,
                                        i64p, i64p]),
    "hs_daubechies_filter": (C.c_int32, [C.c_int32, dptr]),
    "hs_phi": (C.c_int32, [ctxp, P, P]),
    "hs_phi_adj": (C.c_int32, [ctxp, P, P]),
    "hs_psi_adj": (C.c_int32, [ctxp, P, P]),
    "hs_psi": (C.c_int32, [ctxp, P, P]),
    "hs_psi_adj_n": (C.c_int32, [ctxp, P, P, C.c_int32]),
    "hs_psi_n": (C.c_int32, [ctxp, P, P, C.c_int32]),
    "hs_l21_rowsq": (C.c_int32, [ctxp, P, C.c_int32, P, C.c_int32]),
    "hs_l21_rowscale": (C.c_int32, [ctxp, P, C.c_int32, P, P, C.c_double]),
    "hs_l21_from_rowsq": (C.c_int32, [ctxp, P, P, C.POINTER(C.c_double)]),
    "hs_prox_l21": (C.c_int32, [ctxp, P, P, C.c_double]),
    "hs_dual_l21": (C.c_int32, [ctxp, P, P, P, C.c_double, P]),
    "hs_prox_nuclear": (C.c_int32, [ctxp, P, dptr, dptr]),
    "hs_dual_nuclear": (C.c_int32, [ctxp, P, P, dptr]),
    "hs_prox_nuclear_noalloc": (C.c_int32, [P, C.c_int32, C.c_int64, C.c_int32, dptr, dptr, P, C.c_int32]),
    "hs_dual_data": (C.c_int32, [ctxp, P, P, P]),
    "hs_proj_ellipsoid": (C.c_int32, [ctxp, C.c_int32, C.c_int32, P]),
    "hs_op_norm": (C.c_int32, [ctxp, C.c_int32, C.c_int32, C.c_double, P, dptr, dptr, C.POINTER(C.c_int32)]),
    "hs_dirty_mu": (C.c_int32, [ctxp, P, dptr]),
    "hs_pd_init": (C.c_int32, [ctxp, C.POINTER(PDParams)]),
    "hs_pd_set_state": (C.c_int32, [ctxp, C.POINTER(StatePtrs)]),
    "hs_pd_get_state": (C.c_int32, [ctxp, C.POINTER(StatePtrs)]),
    "hs_pd_iterate": (C.c_int32, [ctxp, C.c_int32]),
    "hs_pd_stats": (C.c_int32, [ctxp, dptr, dptr, dptr]),
    "hs_solve": (C.c_int32, [ctxp, C.POINTER(SolveParams), P, C.POINTER(Report)]),
    "hs_profile_phases": (C.c_int32, [ctxp, C.c_int32, dptr]),
    "hs_get_diag": (C.c_int32, [ctxp, dptr, C.c_int32]),
}

PHASES = ["fft_fwd", "degrid", "roots", "dual_apply", "grid", "fft_adj", "gram", "eig", "backproject", "psi_adj",
          "l21", "psi", "primal"]

_lib = None


class HSError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HSError(f"{path} not found: build it with paper_1806_04596_amd.build.build()")
    # Load torch first: it brings its own HIP runtime (same soname), which the
    # library must share; loading the library first would pull in a second
    # runtime instance next to torch's.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, ctx=None, what: str = ""):
    if status != HS_OK:
        lib = load()
        msg = lib.hs_last_error(ctx)
        msg = msg.decode() if msg else ""
        raise HSError(f"{what}: {STATUS.get(status, status)} {msg}")


def as_dptr(a):
    """numpy float64 array -> POINTER(c_double) (or None)."""
    if a is None:
        return None
    return a.ctypes.data_as(dptr)


def as_i64p(a):
    return a.ctypes.data_as(i64p)
