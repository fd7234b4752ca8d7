"""Autotuning of tile shapes and stream counts for batches of KKT systems.

Host-side timing loops over the C-ABI: every candidate runs the library's own
kernels on the device, and the fastest is kept. Three knobs:

* big_tile_rows (kkt_options): the trailing-update size from which the
  128x128 MFMA tile kernel replaces the 64x64 one. Tuned per size class (the
  instance's largest front and Schur dimension, rounded to powers of two) on
  the class's largest member, by the measured factorisation time.
* the number of streams a batch spreads its instances over, by the measured
  time of runs of the whole batch.
* dual_wait (kkt_options): how many primal neighbours a dual waits for in the
  elimination order. Fewer give fronts with fewer update entries (less
  extend-add traffic) but more factor flops on some networks; the measured
  factorisation plus refined solve of the instance decides. The pattern is
  the same in every interior-point iteration, so this is tuned once per
  network.
"""
from __future__ import annotations

import json
import math
import os
import time

CANDIDATE_ROWS = (256, 512, 1024, 2048)
CANDIDATE_STREAMS = (2, 4, 8)
CANDIDATE_DUAL_WAIT = (2, 4)


def size_class(inst, stats):
    """(log2 of the largest front, log2 of the Schur dimension), rounded."""
    f = max(int(stats["max_front"]), 1)
    g = max(int(inst.n_g), 1)
    return (int(round(math.log2(f))), int(round(math.log2(g))))


def _factor_ms(inst, precision, rows, reps):
    import torch
    from . import Solver, device_inputs, kkt_enable_timing, kkt_phase_times
    s = Solver(inst, precision=precision, big_tile_rows=rows)
    d = device_inputs(inst)
    kkt_enable_timing(s.ctx, True)
    best = float("inf")
    for _ in range(reps + 1):
        s.factor(d["vals"], d["C0"], d["C1"], d["corner"], want_inertia=False)
        t = kkt_phase_times(s.ctx)
        best = min(best, t[0] + t[1] + t[2])
    torch.cuda.synchronize()
    s.close()
    return best


def tune_tiles(instances, precision=0, reps=1, cache_path=None, log=None):
    """big_tile_rows for every instance (one timing sweep per size class)."""
    from . import kkt_plan
    cache = {}
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
    classes, stats = {}, []
    for i, inst in enumerate(instances):
        st, _ = kkt_plan(inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, inst.rowind, inst.C0_rowptr,
                         inst.C0_colind, inst.C1_rowptr, inst.C1_colind, precision=precision)
        stats.append(st)
        key = "%d_%d_p%d" % (size_class(inst, st) + (precision,))
        classes.setdefault(key, []).append(i)
    choice = {}
    for key, members in classes.items():
        if key in cache:
            choice[key] = cache[key]
            continue
        rep = max(members, key=lambda i: stats[i]["flops_factor"] * instances[i].N + instances[i].n_g ** 3)
        times = {r: _factor_ms(instances[rep], precision, r, reps) for r in CANDIDATE_ROWS}
        choice[key] = min(times, key=times.get)
        if log:
            log(f"tiles {key}: {', '.join(f'{r}:{t:.2f}ms' for r, t in times.items())} -> {choice[key]}")
    if cache_path:
        cache.update(choice)
        json.dump(cache, open(cache_path, "w"), indent=1, sort_keys=True)
    keys = {i: k for k, ms in classes.items() for i in ms}
    return [choice[keys[i]] for i in range(len(instances))], choice


def tune_streams(batch, refine_steps, candidates=CANDIDATE_STREAMS, reps=2, log=None):
    """Fastest stream count for runs of `batch` (a Batch); leaves the batch
    on that count."""
    import torch
    best, best_t = None, float("inf")
    for ns in candidates:
        batch.restream(ns)
        batch.run(refine_steps)
        batch.wait()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            batch.run(refine_steps)
        batch.wait()
        t = (time.perf_counter() - t0) / reps
        if log:
            log(f"streams {ns}: {t*1e3:.1f} ms per batch")
        if t < best_t:
            best, best_t = ns, t
    batch.restream(best)
    return best


def tune_order(inst, precision=0, candidates=CANDIDATE_DUAL_WAIT, reps=1, schur_mode=0, log=None):
    """dual_wait with the shortest measured factorisation + refined solve of
    `inst` (best of reps + 1 runs each). Returns (choice, {dual_wait: ms})."""
    import torch
    from . import Solver, device_inputs
    d = device_inputs(inst)
    x = torch.empty_like(d["b"])
    times = {}
    for dw in candidates:
        s = Solver(inst, precision=precision, dual_wait=dw, schur_mode=schur_mode)
        best = float("inf")
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.factor(d["vals"], d["C0"], d["C1"], d["corner"], want_inertia=False)
            s.solve(d["b"], x)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        s.close()
        times[dw] = best * 1e3
        if log:
            log(f"order dual_wait {dw}: {times[dw]:.2f} ms per factor + solve")
    return min(times, key=times.get), times
