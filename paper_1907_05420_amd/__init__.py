"""MI355X solver for the block-bordered (arrowhead) KKT system of multiperiod
AC-OPF with storage (Kardos, Kourounis, Schenk, arXiv 1907.05420, sections
4.1-4.3).

Thin binding over the C-ABI library libkkt.so (include/kkt.h). Every step of
the factorisation and solve runs in the library's HIP kernels; this module only
marshals arguments: numpy arrays for the host-side pattern, torch tensors on
the GPU for values, right-hand sides and solutions, and torch's current HIP
stream. There is no CPU fallback: loading fails loudly when libkkt.so is
missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _abi
from ._abi import (KKT_OK, KKT_ERR_ARG, KKT_ERR_NOMEM, KKT_ERR_ORDER, KKT_ERR_STRUCT, KKT_ERR_HIP,
                   KKT_ERR_NONFINITE, KKT_ERR_TOOBIG, KKT_WARN_PERTURBED, KKT_WARN_INERTIA, KKT_WARN_REFINE, KKT_FP64,
                   KKT_MIXED, KKT_REFINE_FGMRES, KKT_REFINE_CLASSIC, KKT_SCHUR_DENSE, KKT_SCHUR_STRUCTURED)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkkt.so")
_lib = None


class KKTError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {code} ({strerror(code) if _lib else code})")
        self.code = code


def load_library(path: str = LIB_PATH):
    """Load libkkt.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_1907_05420_amd.build`")
        _lib = _abi.bind(C.CDLL(path))
    return _lib


def strerror(code: int) -> str:
    return load_library().kkt_strerror(int(code)).decode()


def _check(rc, what, allow_warn=True):
    if rc < 0 or (rc > 0 and not allow_warn):
        raise KKTError(rc, what)
    return rc


# ---- same names as the C-ABI ----------------------------------------------------

def kkt_default_options():
    o = _abi.Options()
    load_library().kkt_default_options(C.byref(o))
    return o


def _structure(nA, n_primal, N, Ns, colptr, rowind, C0p, C0i, C1p, C1i):
    keep = [np.ascontiguousarray(colptr, dtype=np.int64), np.ascontiguousarray(rowind, dtype=np.int32)]
    if Ns > 0:
        keep += [np.ascontiguousarray(C0p, dtype=np.int64), np.ascontiguousarray(C0i, dtype=np.int32),
                 np.ascontiguousarray(C1p, dtype=np.int64), np.ascontiguousarray(C1i, dtype=np.int32)]
        ptrs = [a.ctypes.data for a in keep]
    else:
        ptrs = [keep[0].ctypes.data, keep[1].ctypes.data, None, None, None, None]
    s = _abi.Structure(int(nA), int(n_primal), int(N), int(Ns), *ptrs)
    return s, keep


def kkt_plan(nA, n_primal, N, Ns, colptr, rowind, C0p=None, C0i=None, C1p=None, C1i=None, precision=KKT_FP64,
             nrhs_max=1, want_perm=False, schur_mode=KKT_SCHUR_DENSE, dual_wait=0, recompute_periods=0):
    """Host-only symbolic analysis; returns (stats dict, perm or None)."""
    lib = load_library()
    s, keep = _structure(nA, n_primal, N, Ns, colptr, rowind, C0p, C0i, C1p, C1i)
    o = kkt_default_options()
    o.precision = precision
    o.schur_mode = schur_mode
    o.dual_wait = dual_wait
    o.recompute_periods = recompute_periods
    st = _abi.SymbolicStats()
    perm = np.zeros(nA, np.int32) if want_perm else None
    rc = lib.kkt_plan(C.byref(s), C.byref(o), int(nrhs_max), C.byref(st),
                      perm.ctypes.data if want_perm else None)
    _check(rc, "kkt_plan")
    return {f: getattr(st, f) for f, _ in st._fields_}, perm


def kkt_create(stream=None, precision=KKT_FP64, refine_tol=1e-10, refine_max=20, pivot_eps=0.0, verbose=0,
               refine_method=KKT_REFINE_FGMRES, big_tile_rows=0, schur_mode=0, dual_wait=0, recompute_periods=0):
    lib = load_library()
    o = kkt_default_options()
    o.precision, o.refine_tol, o.refine_max, o.pivot_eps, o.verbose = precision, refine_tol, refine_max, pivot_eps, verbose
    o.refine_method = refine_method
    o.big_tile_rows = big_tile_rows
    o.schur_mode = schur_mode
    o.dual_wait = dual_wait
    o.recompute_periods = recompute_periods
    h = C.c_void_p()
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    _check(lib.kkt_create(C.byref(h), C.c_void_p(stream), C.byref(o)), "kkt_create")
    return h


def kkt_analyze(ctx, nA, n_primal, N, Ns, colptr, rowind, C0p=None, C0i=None, C1p=None, C1i=None):
    s, keep = _structure(nA, n_primal, N, Ns, colptr, rowind, C0p, C0i, C1p, C1i)
    return _check(load_library().kkt_analyze(ctx, C.byref(s)), "kkt_analyze")


def kkt_footprint(ctx):
    b = C.c_size_t()
    _check(load_library().kkt_footprint(ctx, C.byref(b)), "kkt_footprint")
    return int(b.value)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or t.dtype.itemsize != 8 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def kkt_factor(ctx, A_vals, C0_vals=None, C1_vals=None, corner_diag=None, delta_w=0.0, delta_c=0.0,
               want_inertia=True):
    """Returns (status, inertia dict or None)."""
    inn = _abi.Inertia() if want_inertia else None
    rc = load_library().kkt_factor(ctx, _ptr(A_vals), _ptr(C0_vals), _ptr(C1_vals), _ptr(corner_diag),
                                   float(delta_w), float(delta_c), C.byref(inn) if want_inertia else None)
    _check(rc, "kkt_factor")
    return rc, ({f: getattr(inn, f) for f, _ in inn._fields_} if want_inertia else None)


def kkt_solve(ctx, b, x, nrhs, want_info=True):
    info = _abi.SolveInfo() if want_info else None
    rc = load_library().kkt_solve(ctx, _ptr(b), _ptr(x), int(nrhs), C.byref(info) if want_info else None)
    _check(rc, "kkt_solve")
    return rc, ({f: getattr(info, f) for f, _ in info._fields_} if want_info else None)


def kkt_schur(ctx, S_out):
    return _check(load_library().kkt_schur(ctx, _ptr(S_out)), "kkt_schur")


def kkt_schur_blocks(ctx, out):
    return _check(load_library().kkt_schur_blocks(ctx, _ptr(out)), "kkt_schur_blocks")


def kkt_stats(ctx):
    st = _abi.SymbolicStats()
    _check(load_library().kkt_stats(ctx, C.byref(st)), "kkt_stats")
    return {f: getattr(st, f) for f, _ in st._fields_}


def kkt_enable_timing(ctx, on=True):
    return _check(load_library().kkt_enable_timing(ctx, int(bool(on))), "kkt_enable_timing")


def kkt_phase_times(ctx):
    t = (C.c_double * 5)()
    _check(load_library().kkt_phase_times(ctx, t), "kkt_phase_times")
    return list(t)


def kkt_dominant_kernel(ctx):
    st = _abi.KernelStat()
    _check(load_library().kkt_dominant_kernel(ctx, C.byref(st)), "kkt_dominant_kernel")
    return {f: getattr(st, f) for f, _ in st._fields_}


def kkt_set_stream(ctx, stream):
    return _check(load_library().kkt_set_stream(ctx, C.c_void_p(stream)), "kkt_set_stream")


def kkt_factor_async(ctx, A_vals, C0_vals=None, C1_vals=None, corner_diag=None, delta_w=0.0, delta_c=0.0):
    return _check(load_library().kkt_factor_async(ctx, _ptr(A_vals), _ptr(C0_vals), _ptr(C1_vals), _ptr(corner_diag),
                                                  float(delta_w), float(delta_c)), "kkt_factor_async")


def kkt_factor_status(ctx):
    inn = _abi.Inertia()
    rc = _check(load_library().kkt_factor_status(ctx, C.byref(inn)), "kkt_factor_status")
    return rc, {f: getattr(inn, f) for f, _ in inn._fields_}


def kkt_solve_async(ctx, b, x, nrhs, steps):
    return _check(load_library().kkt_solve_async(ctx, _ptr(b), _ptr(x), int(nrhs), int(steps)), "kkt_solve_async")


def kkt_solve_noalloc(ctx, b, x, nrhs, steps):
    """kkt_solve_async with its workspace in the library's fixed device array
    (allocates nothing)."""
    return _check(load_library().kkt_solve_noalloc(ctx, _ptr(b), _ptr(x), int(nrhs), int(steps)), "kkt_solve_noalloc")


def kkt_set_slacks(ctx, lam_row):
    """The multiplier row of A_n each eliminated slack is linked to (host)."""
    lam_row = np.ascontiguousarray(lam_row, dtype=np.int32)
    return _check(load_library().kkt_set_slacks(ctx, int(lam_row.size), lam_row.ctypes.data if lam_row.size else None),
                  "kkt_set_slacks")


def kkt_slack_reduce(ctx, A_vals, Ls, b, rs, A_out, b_out, nrhs):
    """Eq. SCOPFhessianReduced on device arrays (see include/kkt.h)."""
    return _check(load_library().kkt_slack_reduce(ctx, _ptr(A_vals), _ptr(Ls), _ptr(b), _ptr(rs), _ptr(A_out),
                                                  _ptr(b_out), int(nrhs)), "kkt_slack_reduce")


def kkt_slack_recover(ctx, Ls, rs, x, s_out, nrhs):
    """Eq. SCOPFslackReduction on device arrays (see include/kkt.h)."""
    return _check(load_library().kkt_slack_recover(ctx, _ptr(Ls), _ptr(rs), _ptr(x), _ptr(s_out), int(nrhs)),
                  "kkt_slack_recover")


def kkt_solve_status(ctx):
    info = _abi.SolveInfo()
    rc = _check(load_library().kkt_solve_status(ctx, C.byref(info)), "kkt_solve_status")
    return rc, {f: getattr(info, f) for f, _ in info._fields_}


def kkt_batch_create(nstreams):
    h = C.c_void_p()
    _check(load_library().kkt_batch_create(C.byref(h), int(nstreams)), "kkt_batch_create")
    return h


def kkt_batch_add(batch, ctx, A_vals, C0_vals, C1_vals, corner_diag, rhs, x, nrhs):
    return _check(load_library().kkt_batch_add(batch, ctx, _ptr(A_vals), _ptr(C0_vals), _ptr(C1_vals),
                                               _ptr(corner_diag), _ptr(rhs), _ptr(x), int(nrhs)), "kkt_batch_add")


def kkt_batch_run(batch, refine_steps, use_graph):
    return _check(load_library().kkt_batch_run(batch, int(refine_steps), int(bool(use_graph))), "kkt_batch_run")


def kkt_batch_wait(batch):
    return _check(load_library().kkt_batch_wait(batch), "kkt_batch_wait")


def kkt_batch_stream_of(batch, i):
    return int(load_library().kkt_batch_stream_of(batch, int(i)))


def kkt_batch_destroy(batch):
    if batch:
        load_library().kkt_batch_destroy(batch)


def kkt_destroy(ctx):
    if ctx:
        load_library().kkt_destroy(ctx)


# ---- convenience wrapper ---------------------------------------------------------

class Solver:
    """One analysed pattern on the current device and stream.

    `inst` is any object with the fields of kktgen.Instance's pattern (n_A,
    n_primal, N, ns, colptr, rowind, C0_/C1_rowptr/colind)."""

    def __init__(self, inst, precision=KKT_FP64, stream=None, refine_tol=1e-10, refine_max=20, pivot_eps=0.0,
                 verbose=0, refine_method=KKT_REFINE_FGMRES, big_tile_rows=0, schur_mode=0, dual_wait=0,
                 recompute_periods=0):
        self.inst = inst
        self.ctx = kkt_create(stream, precision, refine_tol, refine_max, pivot_eps, verbose, refine_method,
                              big_tile_rows, schur_mode, dual_wait, recompute_periods)
        kkt_analyze(self.ctx, inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, inst.rowind,
                    inst.C0_rowptr, inst.C0_colind, inst.C1_rowptr, inst.C1_colind)

    def factor(self, vals, C0, C1, corner=None, delta_w=0.0, delta_c=0.0, want_inertia=True):
        return kkt_factor(self.ctx, vals, C0, C1, corner, delta_w, delta_c, want_inertia)

    def solve(self, b, x=None, want_info=True):
        import torch
        nrhs = b.shape[0] if b.dim() == 2 else 1
        if x is None:
            x = torch.empty_like(b)
        rc, info = kkt_solve(self.ctx, b, x, nrhs, want_info)
        return x, rc, info

    def schur(self):
        import torch
        ng = self.inst.N * self.inst.ns
        S = torch.empty((ng, ng), dtype=torch.float64, device="cuda")
        kkt_schur(self.ctx, S)
        return S

    def schur_blocks(self):
        import torch
        nb = 2 * self.inst.ns
        out = torch.empty((self.inst.N, nb, nb), dtype=torch.float64, device="cuda")
        kkt_schur_blocks(self.ctx, out)
        return out

    def footprint(self):
        return kkt_footprint(self.ctx)

    def stats(self):
        return kkt_stats(self.ctx)

    def close(self):
        if self.ctx:
            kkt_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent instances factored and solved together on several
    streams, optionally through a captured HIP graph (kkt_batch_*). Each
    instance keeps its own Solver (context); its device buffers (values,
    right-hand sides, solutions) are fixed for the life of the batch."""

    def __init__(self, instances, nstreams=4, precision=KKT_FP64, big_tile_rows=None):
        import torch
        rows = big_tile_rows if big_tile_rows is not None else [0] * len(instances)
        self.solvers = [Solver(inst, precision=precision, big_tile_rows=r) for inst, r in zip(instances, rows)]
        self.inputs = [device_inputs(inst) for inst in instances]
        self.x = [torch.empty_like(d["b"]) for d in self.inputs]
        self.h = None
        self.restream(nstreams)

    def restream(self, nstreams):
        """Spread the same instances over a new set of nstreams streams."""
        if self.h:
            kkt_batch_destroy(self.h)
        self.h = kkt_batch_create(nstreams)
        self.nstreams = nstreams
        for s, d, x in zip(self.solvers, self.inputs, self.x):
            kkt_batch_add(self.h, s.ctx, d["vals"], d["C0"], d["C1"], d["corner"], d["b"], x, d["b"].shape[0])
        self.ran_eager = False

    def run(self, refine_steps=3, use_graph=False):
        kkt_batch_run(self.h, refine_steps, use_graph and self.ran_eager)
        self.ran_eager = True

    def wait(self):
        kkt_batch_wait(self.h)

    def status(self):
        out = []
        for s in self.solvers:
            rc_f, inn = kkt_factor_status(s.ctx)
            rc_s, info = kkt_solve_status(s.ctx)
            out.append(dict(rc_factor=rc_f, inertia=inn, rc_solve=rc_s, info=info))
        return out

    def close(self):
        if self.h:
            kkt_batch_destroy(self.h)
            self.h = None
        for s in self.solvers:
            s.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_inputs(inst, device="cuda"):
    """Upload an instance's values, coupling, corner and right-hand sides."""
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(device)
    return dict(vals=t(inst.vals), C0=t(inst.C0_vals), C1=t(inst.C1_vals), corner=t(inst.corner_diag), b=t(inst.b))
