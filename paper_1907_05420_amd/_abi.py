"""ctypes declarations mirroring include/kkt.h (argument marshalling only)."""
import ctypes as C

KKT_OK = 0
KKT_ERR_ARG = -1
KKT_ERR_NOMEM = -2
KKT_ERR_ORDER = -3
KKT_ERR_STRUCT = -4
KKT_ERR_HIP = -5
KKT_ERR_NONFINITE = -6
KKT_ERR_TOOBIG = -7
KKT_WARN_PERTURBED = 1
KKT_WARN_INERTIA = 2
KKT_WARN_REFINE = 3
KKT_FP64 = 0
KKT_MIXED = 1
KKT_REFINE_FGMRES = 0
KKT_REFINE_CLASSIC = 1
KKT_SCHUR_DENSE = 0
KKT_SCHUR_STRUCTURED = 1


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("pivot_eps", C.c_double), ("refine_tol", C.c_double),
                ("refine_max", C.c_int), ("verbose", C.c_int), ("refine_method", C.c_int),
                ("big_tile_rows", C.c_int),
                ("schur_mode", C.c_int), ("recompute_periods", C.c_int), ("dual_wait", C.c_int)]


class Structure(C.Structure):
    _fields_ = [("nA", C.c_int64), ("n_primal", C.c_int64), ("N", C.c_int64), ("Ns", C.c_int64),
                ("A_colptr", C.c_void_p), ("A_rowind", C.c_void_p),
                ("C0_rowptr", C.c_void_p), ("C0_colind", C.c_void_p),
                ("C1_rowptr", C.c_void_p), ("C1_colind", C.c_void_p)]


class Inertia(C.Structure):
    _fields_ = [("n_pos", C.c_int64), ("n_neg", C.c_int64), ("n_zero", C.c_int64),
                ("n_perturbed", C.c_int64), ("inertia_ok", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("refine_iters", C.c_int), ("rel_res", C.c_double), ("omega", C.c_double),
                ("fallback_used", C.c_int), ("rel_floor", C.c_double)]


class SymbolicStats(C.Structure):
    _fields_ = [("n_supernodes", C.c_int64), ("n_levels", C.c_int64), ("nnz_L", C.c_int64),
                ("u_entries", C.c_int64), ("max_front", C.c_int64), ("max_pivots", C.c_int64),
                ("flops_factor", C.c_double), ("device_bytes", C.c_int64)]


class KernelStat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


# name -> (restype, argtypes); every symbol include/kkt.h declares
SIGNATURES = {
    "kkt_default_options": (None, [C.POINTER(Options)]),
    "kkt_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_void_p, C.POINTER(Options)]),
    "kkt_analyze": (C.c_int, [C.c_void_p, C.POINTER(Structure)]),
    "kkt_footprint": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "kkt_plan": (C.c_int, [C.POINTER(Structure), C.POINTER(Options), C.c_int64,
                           C.POINTER(SymbolicStats), C.c_void_p]),
    "kkt_factor": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_double, C.c_double, C.POINTER(Inertia)]),
    "kkt_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(SolveInfo)]),
    "kkt_schur": (C.c_int, [C.c_void_p, C.c_void_p]),
    "kkt_schur_blocks": (C.c_int, [C.c_void_p, C.c_void_p]),
    "kkt_stats": (C.c_int, [C.c_void_p, C.POINTER(SymbolicStats)]),
    "kkt_enable_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "kkt_phase_times": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "kkt_dominant_kernel": (C.c_int, [C.c_void_p, C.POINTER(KernelStat)]),
    "kkt_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "kkt_factor_async": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_double, C.c_double]),
    "kkt_factor_status": (C.c_int, [C.c_void_p, C.POINTER(Inertia)]),
    "kkt_solve_async": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int]),
    "kkt_solve_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int]),
    "kkt_set_slacks": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
    "kkt_slack_reduce": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_int64]),
    "kkt_slack_recover": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "kkt_solve_status": (C.c_int, [C.c_void_p, C.POINTER(SolveInfo)]),
    "kkt_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "kkt_batch_add": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_int64]),
    "kkt_batch_run": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "kkt_batch_wait": (C.c_int, [C.c_void_p]),
    "kkt_batch_stream_of": (C.c_int, [C.c_void_p, C.c_int64]),
    "kkt_batch_destroy": (None, [C.c_void_p]),
    "kkt_destroy": (None, [C.c_void_p]),
    "kkt_strerror": (C.c_char_p, [C.c_int]),
}


def bind(lib):
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib
