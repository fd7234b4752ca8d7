"""Serving loop for KKT solve requests (continuous batching).

A request is one interior-point solve: an analysed pattern (grid and horizon)
and a number of IPM-like iterations, each a factorisation with new barrier
diagonals and a solve. The server keeps a request's symbolic analysis,
factors and workspace resident on the device for all its iterations, admits
waiting requests in arrival order whenever a slot and enough HBM are free
(the footprint comes from the host-only planning query kkt_plan), and runs
the admitted requests side by side on their own streams. Two ways to run an
admitted request:

* "fixed": the enqueue-only entry points (kkt_factor_async, kkt_solve_async)
  with a fixed number of FP64 refinement steps; one host loop enqueues work
  and polls completion events.
* "tolerance": kkt_factor and kkt_solve, which refine until the relative
  residual reaches the context's tolerance (reading norms back between
  steps); each admitted request runs in a host thread of its own (the calls
  release the interpreter lock), so the requests still overlap on the device.

All arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import (KKT_FP64, Solver, device_inputs, kkt_factor, kkt_factor_async, kkt_factor_status, kkt_plan,
               kkt_set_stream, kkt_solve, kkt_solve_async, kkt_solve_status)


@dataclass
class Request:
    rid: int
    inst: object                  # kktgen.Instance-like pattern + values
    arrival: float                # seconds after the start of the run
    iterations: int = 30
    values: list = None           # per-iteration value arrays [N][nnz] (host); None keeps inst.vals
    redraw: object = None         # or redraw(it, vals): writes iteration it's values into the device
                                  # tensor vals on the current stream
    # filled in by the server
    footprint: int = 0
    admitted: float = None
    finished: float = None
    rel_res: list = field(default_factory=list)
    inertia_ok: list = field(default_factory=list)
    solve_s: list = field(default_factory=list)   # per iteration: enqueue -> completion seen by the host
    x: np.ndarray = None          # solution of the last iteration


class _Active:
    def __init__(self, req, slot, precision, refine_steps, keep_x):
        import torch
        self.req, self.slot = req, slot
        self.stream = torch.cuda.Stream()
        self.solver = Solver(req.inst, precision=precision)
        kkt_set_stream(self.solver.ctx, self.stream.cuda_stream)
        with torch.cuda.stream(self.stream):
            self.d = device_inputs(req.inst)
            self.x = torch.empty_like(self.d["b"])
        self.it = 0
        self.event = None
        self.refine_steps = refine_steps
        self.keep_x = keep_x

    def enqueue(self):
        import torch
        r = self.req
        self.t_enq = time.perf_counter()
        with torch.cuda.stream(self.stream):
            if r.redraw is not None:
                r.redraw(self.it, self.d["vals"])
            elif r.values is not None:
                self.d["vals"].copy_(torch.as_tensor(r.values[self.it]), non_blocking=False)
            kkt_factor_async(self.solver.ctx, self.d["vals"], self.d["C0"], self.d["C1"], self.d["corner"])
            kkt_solve_async(self.solver.ctx, self.d["b"], self.x, self.d["b"].shape[0], self.refine_steps)
            self.event = torch.cuda.Event()
            self.event.record(self.stream)

    def done(self):
        return self.event is not None and self.event.query()

    def collect(self):
        self.req.solve_s.append(time.perf_counter() - self.t_enq)
        rc_f, inn = kkt_factor_status(self.solver.ctx)
        rc_s, info = kkt_solve_status(self.solver.ctx)
        self.req.rel_res.append(info["rel_res"])
        self.req.inertia_ok.append(inn["inertia_ok"])
        self.it += 1
        if self.it == self.req.iterations and self.keep_x:
            self.req.x = self.x.cpu().numpy()

    def close(self):
        self.solver.close()


def _run_to_tolerance(req, precision, keep_x):
    """All iterations of one request on a stream of its own (host thread)."""
    import torch
    stream = torch.cuda.Stream()
    solver = Solver(req.inst, precision=precision)
    try:
        kkt_set_stream(solver.ctx, stream.cuda_stream)
        with torch.cuda.stream(stream):
            d = device_inputs(req.inst)
            x = torch.empty_like(d["b"])
            for it in range(req.iterations):
                t = time.perf_counter()
                if req.redraw is not None:
                    req.redraw(it, d["vals"])
                elif req.values is not None:
                    d["vals"].copy_(torch.as_tensor(req.values[it]), non_blocking=False)
                _, inn = kkt_factor(solver.ctx, d["vals"], d["C0"], d["C1"], d["corner"])
                _, info = kkt_solve(solver.ctx, d["b"], x, d["b"].shape[0])
                req.solve_s.append(time.perf_counter() - t)
                req.rel_res.append(info["rel_res"])
                req.inertia_ok.append(inn["inertia_ok"])
            if keep_x:
                req.x = x.cpu().numpy()
            stream.synchronize()
    finally:
        solver.close()


def footprint_bytes(inst, precision=KKT_FP64, nrhs=1):
    """Device bytes a context of this pattern will hold (kkt_plan)."""
    st, _ = kkt_plan(inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, inst.rowind, inst.C0_rowptr,
                     inst.C0_colind, inst.C1_rowptr, inst.C1_colind, precision=precision, nrhs_max=nrhs)
    return int(st["device_bytes"])


def serve(requests, slots=4, hbm_budget=200 << 30, precision=KKT_FP64, refine_steps=3, keep_x=False,
          poll_sleep=0.0005, log=None, refine="fixed"):
    """Run `requests` (sorted by arrival) to completion. Returns the requests
    (with their admission/finish times, per-iteration residuals and inertia
    flags, and the last solution when keep_x) and a dict with the largest
    footprint in use and the most requests in flight at any time. `refine`:
    "fixed" (refine_steps FP64 steps per solve) or "tolerance" (refine to the
    residual tolerance)."""
    if refine not in ("fixed", "tolerance"):
        raise ValueError(f"refine must be 'fixed' or 'tolerance', not {refine!r}")
    if refine == "tolerance":
        return _serve_threads(requests, slots, hbm_budget, precision, keep_x, poll_sleep, log)
    import torch
    pending = sorted(requests, key=lambda r: r.arrival)
    for r in pending:
        r.footprint = footprint_bytes(r.inst, precision, r.inst.b.shape[0])
        if r.footprint > hbm_budget:
            raise ValueError(f"request {r.rid} needs {r.footprint} B, more than the budget {hbm_budget} B")
    active, used, t0 = [], 0, time.perf_counter()
    free_slots = list(range(slots))
    stats = dict(max_used=0, max_active=0, iterations=0)
    while pending or active:
        now = time.perf_counter() - t0
        # admission in arrival order: a slot and the footprint must be free
        while pending and pending[0].arrival <= now and free_slots and used + pending[0].footprint <= hbm_budget:
            r = pending.pop(0)
            r.admitted = now
            a = _Active(r, free_slots.pop(0), precision, refine_steps, keep_x)
            used += r.footprint
            a.enqueue()
            active.append(a)
            stats["max_used"] = max(stats["max_used"], used)
            stats["max_active"] = max(stats["max_active"], len(active))
            if log:
                log(f"t={now:.3f}s admit request {r.rid} (slot {a.slot}, {r.footprint / 2**30:.2f} GiB in use "
                    f"{used / 2**30:.2f})")
        progressed = False
        for a in list(active):
            if a.done():
                progressed = True
                a.collect()
                stats["iterations"] += 1
                if a.it < a.req.iterations:
                    a.enqueue()
                else:
                    a.req.finished = time.perf_counter() - t0
                    active.remove(a)
                    free_slots.append(a.slot)
                    used -= a.req.footprint
                    a.close()
        if not progressed:
            if not active and pending:
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            elif poll_sleep:
                time.sleep(poll_sleep)
    torch.cuda.synchronize()
    stats["wall_s"] = time.perf_counter() - t0
    return requests, stats


def _serve_threads(requests, slots, hbm_budget, precision, keep_x, poll_sleep, log):
    import torch
    pending = sorted(requests, key=lambda r: r.arrival)
    for r in pending:
        r.footprint = footprint_bytes(r.inst, precision, r.inst.b.shape[0])
        if r.footprint > hbm_budget:
            raise ValueError(f"request {r.rid} needs {r.footprint} B, more than the budget {hbm_budget} B")
    active, used, t0 = [], 0, time.perf_counter()
    stats = dict(max_used=0, max_active=0, iterations=0)
    with ThreadPoolExecutor(max_workers=slots) as pool:
        while pending or active:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now and len(active) < slots and \
                    used + pending[0].footprint <= hbm_budget:
                r = pending.pop(0)
                r.admitted = now
                used += r.footprint
                active.append((r, pool.submit(_run_to_tolerance, r, precision, keep_x)))
                stats["max_used"] = max(stats["max_used"], used)
                stats["max_active"] = max(stats["max_active"], len(active))
                if log:
                    log(f"t={now:.3f}s admit request {r.rid} ({r.footprint / 2**30:.2f} GiB, in use "
                        f"{used / 2**30:.2f} GiB)")
            progressed = False
            for item in list(active):
                r, fut = item
                if fut.done():
                    fut.result()  # re-raises a failure of the request
                    progressed = True
                    r.finished = time.perf_counter() - t0
                    stats["iterations"] += len(r.rel_res)
                    active.remove(item)
                    used -= r.footprint
            if not progressed:
                if not active and pending:
                    wait = pending[0].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                elif poll_sleep:
                    time.sleep(poll_sleep)
    torch.cuda.synchronize()
    stats["wall_s"] = time.perf_counter() - t0
    return requests, stats


def poisson_arrivals(count, rate, rng):
    """Arrival times (seconds) of a Poisson process with the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
