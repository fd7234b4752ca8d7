"""Benchmark: KKT solves per second on one MI355X.

One step = kkt_factor with new values (all 96 period blocks, the Schur
complement of dimension 19200 and its dense LDL^T) + kkt_solve with all 4
right-hand sides including FP64 refinement, on the 2000-bus / 3000-line mesh
with 400 generators and 200 storage units over 96 periods (barrier diagonals
log-uniform in [1e-8, 1e8]). Inputs are synthetic, seeded and resident in HBM
before the timed region; two value sets (re-drawn barrier diagonals)
alternate so that every step factors new values. Symbolic analysis is done
once, outside the timed region, and reported separately.

    python bench.py [--steps K] [--warmup W] [--precision fp64|mixed]
    python bench.py --copy-probe      (plain device copy, counter calibration)

Prints one JSON line on stdout.
"""
import argparse
import copy
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KKT solves/sec at rel. residual 1e-10 (mixed vs FP64 GPU); p50/p99 latency"
MI355X_HBM_GBS = 8000.0
MI355X_FP64_TFLOPS = 78.6
MI355X_FP32_TFLOPS = 157.3


def cpu_baseline():
    """Time the FP64 oracle (Algorithm 1 of section 4.2 as oracle/ implements
    it, untuned) on the host's cores, on a bounded sample of the same
    workload, and scale the sample to one full KKT solve (factor + solve to
    the residual target):
      * the per-period steps (factor A_n by SuperLU, the 2 Ns solves of Eq.
        LocalSchurBs3) for the first P periods, spread over a pool of one
        thread per core (Algorithm 1 distributes the blocks; SuperLU releases
        the interpreter lock), scaled by N / P;
      * LAPACK's Cholesky of -S (the oracle's large-size Schur factor) timed at
        the full n_g on a same-size SPD matrix, its BLAS on every core, and
        one solve with it;
      * the solve passes: Algorithm 1's solve on the P-period sample (period
        solves on the pool) scaled by N / P, plus the full-size Schur solve,
        times the passes the oracle's refinement needs on the sample."""
    import numpy as np
    import scipy.linalg as sl
    from concurrent.futures import ThreadPoolExecutor
    import threadpoolctl
    import kktgen
    from oracle import schur as sc
    from oracle import arrowhead as ah
    cores = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    model = next((l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")), "?")
    blas = max((i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()), default=1)
    inst = kktgen.make_workload(2)
    P = min(inst.N, 2 * cores)
    short = copy.copy(inst)
    short.N = P
    short.vals = inst.vals[:P]
    short.corner_diag = inst.corner_diag[: P * inst.ns]
    nA = inst.n_A
    short.b = np.concatenate([inst.b[:, : P * nA], inst.b[:, inst.N * nA: inst.N * nA + P * inst.ns]], 1)
    t_begin = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        t0 = time.perf_counter()
        factors = list(ex.map(lambda n: sc.BlockFactor(ah.block(short, n), short.n_primal, dense_limit=0),
                              range(P)))
        Sbar = list(ex.map(lambda F: sc.local_schur_bar(short, F), factors))
        t_periods = time.perf_counter() - t0
        # one solve pass on the sample (Schur factor of the sample's S)
        out = sc.algorithm1(short, factors=factors, assembly="prefix", schur_factor="cholesky")
        fac = out["schur_fac"]
        t0 = time.perf_counter()
        bparts, _ = ah.split(short, short.b)
        list(ex.map(lambda n: factors[n].solve(bparts[:, n, :].T), range(P)))
        list(ex.map(lambda n: factors[n].solve(bparts[:, n, :].T), range(P)))
        t_pass_periods = time.perf_counter() - t0
    # refinement passes the oracle needs on the sample (FP64 residuals)
    K = ah.assemble(short)
    solve = lambda r: sc.algorithm1(short, b=r, factors=factors, schur=fac)["x"]
    _, hist = sc.refine(short, out["x"], short.b, solve, tol=1e-10, maxit=10, K=K)
    passes = len(hist)
    # dense Cholesky of an n_g x n_g SPD matrix and one solve with it
    ng = inst.n_g
    M = np.full((ng, ng), 0.5)
    np.fill_diagonal(M, float(ng))
    t0 = time.perf_counter()
    cf = sl.cho_factor(M, lower=True, overwrite_a=True, check_finite=False)
    t_chol = time.perf_counter() - t0
    t0 = time.perf_counter()
    sl.cho_solve(cf, np.ones((ng, inst.nrhs)), check_finite=False)
    t_ssolve = time.perf_counter() - t0
    del M, cf
    measured = time.perf_counter() - t_begin
    scale = inst.N / P
    est = t_periods * scale + t_chol + passes * (t_pass_periods * scale + t_ssolve)
    return dict(value=1.0 / est, unit="solves/s", cores=cores, kind="oracle",
                sample=(f"Algorithm 1 on the first {P} of {inst.N} periods ({cores} threads, {t_periods:.1f}s for "
                        f"the period factors and local Schur blocks, x{inst.N}/{P}); LAPACK Cholesky of an "
                        f"{ng}x{ng} SPD matrix ({t_chol:.1f}s, BLAS threads {blas}); {passes} solve passes "
                        f"({t_pass_periods:.2f}s periods x{inst.N}/{P} + {t_ssolve:.2f}s Schur solve each); "
                        f"est. {est:.1f}s per solve, {measured:.1f}s measured"),
                cpu_model=model, blas_threads=blas, seconds_measured=measured)


PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "k_update_big_mesh2000_N96_counters.txt")
# the dominant kernel's source: the kernel file and its tile-order header
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1907_05420_amd", "csrc", f) for f in ("k_factor.hip", "tile_order.hpp", "device.hpp", "step_plan.hpp")]


def git_blob_sha1(path):
    """git's blob hash of a file (what `git hash-object` prints)."""
    import hashlib
    data = open(path, "rb").read()
    return hashlib.sha1(b"blob %d\0" % len(data) + data).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when the kernel source changed after the counters were
    taken (the summary records the blob hashes of its source files)."""
    if not os.path.exists(PROFILE_COUNTERS):
        return None
    vals = {}
    for line in open(PROFILE_COUNTERS):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha1") != " ".join(git_blob_sha1(p) for p in KERNEL_SOURCES):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(nbytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}))


def measure(args, inst, vals2, prec, log, schur_mode=0, steps=None, warmup=None):
    """Warm up, then time exactly `steps` (default args.steps) factor+solve steps."""
    import numpy as np
    import torch
    import paper_1907_05420_amd as pk
    d = pk.device_inputs(inst)
    vsets = [d["vals"], torch.as_tensor(vals2).cuda()]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    s = pk.Solver(inst, precision=prec, schur_mode=schur_mode, dual_wait=args.dual_wait,
                  recompute_periods=args.recompute_periods,
                  refine_method=pk.KKT_REFINE_CLASSIC if args.refine == "classic" else pk.KKT_REFINE_FGMRES)
    t_analyze = time.perf_counter() - t0
    st = s.stats()
    st["footprint"] = s.footprint()
    log(f"analyze {t_analyze*1e3:.1f} ms; stats {st}")
    pk.kkt_enable_timing(s.ctx, True)
    x = torch.empty_like(d["b"])
    for i in range(warmup):
        s.factor(vsets[i % 2], d["C0"], d["C1"], d["corner"], want_inertia=False)
        _, rc, info = s.solve(d["b"], x)
        log(f"warmup {i}: rc {rc} info {info} phases {pk.kkt_phase_times(s.ctx)}")
    torch.cuda.synchronize()
    lat, phases, infos, kstats, rcs = [], [], [], [], []
    t_start = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        s.factor(vsets[i % 2], d["C0"], d["C1"], d["corner"], want_inertia=False)
        _, rc, info = s.solve(d["b"], x)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        phases.append(pk.kkt_phase_times(s.ctx))
        kstats.append(pk.kkt_dominant_kernel(s.ctx))
        infos.append(info)
        rcs.append(rc)
        log(f"step {i}: {lat[-1]*1e3:.2f} ms rc {rc} info {info}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    st["footprint_after"] = s.footprint()
    s.close()
    lat_ms = np.array(lat) * 1e3
    return dict(value=steps / elapsed, elapsed=elapsed, lat_ms=lat_ms, phases=np.array(phases).mean(0).tolist(),
                infos=infos, kstats=kstats, rcs=rcs, analyze_ms=t_analyze * 1e3, stats=st,
                x_last=x.cpu().numpy(), last_set=(steps - 1) % 2)


def bench_batch(args, log):
    """64 independent instances of the uneven mixture (bus counts log-uniform
    in [118, 3000], horizons 12/24/48/96), each factored and solved with a
    fixed number of FP64 refinement steps; the batch runs on several streams,
    tile shapes and stream count autotuned first. A step is one run of the
    whole batch (64 KKT solves)."""
    import numpy as np
    import torch
    import kktgen
    import paper_1907_05420_amd as pk
    from paper_1907_05420_amd import autotune
    prec = pk.KKT_MIXED if args.precision == "mixed" else pk.KKT_FP64
    insts = kktgen.uneven_batch()
    t0 = time.perf_counter()
    rows, choice = autotune.tune_tiles(insts, prec, reps=1, log=log)
    t_tune_tiles = time.perf_counter() - t0
    t0 = time.perf_counter()
    b = pk.Batch(insts, nstreams=4, precision=prec, big_tile_rows=rows)
    t_analyze = time.perf_counter() - t0
    ns = autotune.tune_streams(b, args.refine_steps, log=log)
    for _ in range(max(args.warmup, 1)):
        b.run(args.refine_steps)
    b.wait()
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        b.run(args.refine_steps)
        b.wait()
        lat.append(time.perf_counter() - ts)
    elapsed = time.perf_counter() - t_start
    st = b.status()
    # the same instances one after another on one stream, eagerly
    stream = torch.cuda.current_stream().cuda_stream
    torch.cuda.synchronize()
    t_seq = time.perf_counter()
    for s, d, x in zip(b.solvers, b.inputs, b.x):
        pk.kkt_set_stream(s.ctx, stream)
        pk.kkt_factor_async(s.ctx, d["vals"], d["C0"], d["C1"], d["corner"])
        pk.kkt_solve_async(s.ctx, d["b"], x, d["b"].shape[0], args.refine_steps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t_seq
    n = len(insts)
    rel = [r["info"]["rel_res"] for r in st]
    lat_ms = np.array(lat) * 1e3
    res = {
        "metric": METRIC, "value": n * args.steps / elapsed, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == pk.KKT_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": "uneven64", "instances": n, "buses": [118, 3000], "horizons": [12, 24, 48, 96],
                   "nrhs": 1, "barrier_range": [1e-6, 1e6], "precision": args.precision,
                   "refine_steps": args.refine_steps, "streams": ns, "hip_graph": False},
        "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
        "rel_res_max": float(max(rel)), "rel_res_median": float(np.median(rel)),
        "inertia_ok": int(sum(r["inertia"]["inertia_ok"] for r in st)),
        "sequential_solves_per_s": n / t_seq, "speedup_vs_sequential": (n * args.steps / elapsed) / (n / t_seq),
        "tiles": choice, "tune_tiles_s": t_tune_tiles, "analyze_s": t_analyze,
        "device_gb": sum(s.footprint() for s in b.solvers) / 1e9,
    }
    b.close()
    return res


class DeviceRedraw:
    """Per-iteration barrier re-draw on the device (input synthesis for the
    serving workload, the device form of kktgen.redraw_barrier): Hessian
    diagonals = row sums of |off-diagonal| + a log-uniform barrier, pure
    barrier entries = the barrier; the off-diagonals and Jacobian stay."""

    def __init__(self, inst, seed):
        import numpy as np
        kind = np.asarray(inst.meta["kind"])
        self.inst, self.seed = inst, seed
        cols = np.repeat(np.arange(inst.n_A), np.diff(inst.colptr))
        self.h = np.nonzero(kind == 1)[0]
        self.b = np.nonzero(kind == 2)[0]
        self.off = np.nonzero(kind == 0)[0]
        self.cols, self.rows = cols, np.asarray(inst.rowind, dtype=np.int64)
        self.lo, self.hi = inst.barrier_range
        self.dev = None

    def _setup(self, vals):
        import torch
        t = lambda a: torch.as_tensor(a, dtype=torch.int64, device=vals.device)
        off, h, b = t(self.off), t(self.h), t(self.b)
        rows, cols = t(self.rows), t(self.cols)
        av = vals[:, off].abs()
        rs = torch.zeros(vals.shape[0], self.inst.n_A, dtype=vals.dtype, device=vals.device)
        rs.index_add_(1, rows[off], av)
        rs.index_add_(1, cols[off], av)
        self.dev = dict(h=h, b=b, hcols=cols[h], bcols=cols[b], base=rs[:, cols[h]].contiguous())

    def __call__(self, it, vals):
        import math
        import torch
        if self.dev is None:
            self._setup(vals)
        d = self.dev
        g = torch.Generator(device=vals.device)
        g.manual_seed(self.seed * 1000 + it)
        u = torch.rand(vals.shape[0], self.inst.n_A, generator=g, dtype=vals.dtype, device=vals.device)
        bar = torch.exp(math.log(self.lo) + u * (math.log(self.hi) - math.log(self.lo)))
        vals[:, d["h"]] = d["base"] + bar[:, d["hcols"]]
        vals[:, d["b"]] = bar[:, d["bcols"]]


def bench_serve(args, log):
    """Serving: a Poisson stream of requests drawn from the uneven mixture
    (bus counts log-uniform in [118, 3000], horizons 12/24/48/96), each 30
    IPM-like iterations (barrier re-drawn on the device, then factor + solve
    with fixed refinement steps), admitted by device footprint into a few
    slots and run side by side on their own streams. A step is one solve."""
    import numpy as np
    import torch
    import kktgen
    import paper_1907_05420_amd as pk
    from paper_1907_05420_amd import serve
    prec = pk.KKT_MIXED if args.precision == "mixed" else pk.KKT_FP64
    iters = args.iterations

    def make(count, seed, rate):
        insts = kktgen.uneven_batch(count=count, seed=seed)
        arr = serve.poisson_arrivals(count, rate=rate, rng=np.random.default_rng(seed + 1))
        return [serve.Request(i, inst, float(t), iters, redraw=DeviceRedraw(inst, seed + i))
                for i, (inst, t) in enumerate(zip(insts, arr))]

    # warmup: two small requests (module loading, first launches)
    warm = kktgen.uneven_batch(count=2, seed=kktgen.seed_for(5, 9), nb_range=(118, 300), horizons=(12,))
    serve.serve([serve.Request(i, w, 0.0, 2, redraw=DeviceRedraw(w, 7 + i)) for i, w in enumerate(warm)],
                slots=2, precision=prec, refine_steps=args.refine_steps, refine=args.serve_refine)
    torch.cuda.synchronize()
    reqs = make(args.requests, kktgen.seed_for(5, 0), args.rate)
    done, st = serve.serve(reqs, slots=args.slots, hbm_budget=int(args.hbm_budget_gb * 2**30), precision=prec,
                           refine_steps=args.refine_steps, log=log, refine=args.serve_refine)
    n = sum(len(r.rel_res) for r in done)
    lat_req = np.array([r.finished - r.arrival for r in done]) * 1e3
    lat_it = np.concatenate([np.array(r.solve_s) for r in done]) * 1e3
    rel = np.concatenate([np.array(r.rel_res) for r in done])
    return {
        "metric": METRIC, "value": n / st["wall_s"], "unit": "solves/s", "n_gpus": 1, "steps": int(n),
        "warmup": 2, "ms_per_step": st["wall_s"] / n * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == pk.KKT_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": "serve", "requests": len(done), "iterations": iters, "arrival_rate_per_s": args.rate,
                   "slots": args.slots, "hbm_budget_gb": args.hbm_budget_gb, "buses": [118, 3000],
                   "horizons": [12, 24, 48, 96], "barrier_range": [1e-6, 1e6], "precision": args.precision,
                   "refine": args.serve_refine,
                   "refine_steps": args.refine_steps if args.serve_refine == "fixed" else None},
        "p50_ms": float(np.percentile(lat_it, 50)), "p99_ms": float(np.percentile(lat_it, 99)),
        "request_p50_ms": float(np.percentile(lat_req, 50)), "request_p99_ms": float(np.percentile(lat_req, 99)),
        "rel_res_max": float(rel.max()), "above_1e-10": int((rel > 1e-10).sum()),
        "inertia_ok": int(sum(sum(r.inertia_ok) for r in done)), "max_in_flight": st["max_active"],
        "max_device_gb": st["max_used"] / 1e9, "wall_s": st["wall_s"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--refine", default="fgmres", choices=["fgmres", "classic"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--workload", default="mesh2000_N96",
                    choices=["mesh2000_N96", "mesh9241_N24", "uneven64", "serve"])
    ap.add_argument("--requests", type=int, default=24, help="serve: number of requests")
    ap.add_argument("--iterations", type=int, default=30, help="serve: IPM-like iterations per request")
    ap.add_argument("--rate", type=float, default=50.0, help="serve: Poisson arrival rate (requests/s)")
    ap.add_argument("--slots", type=int, default=4, help="serve: requests in flight at most")
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0, help="serve: device memory for admission")
    ap.add_argument("--serve-refine", default="tolerance", choices=["tolerance", "fixed"],
                    help="serve: refine every solve to 1e-10, or a fixed number of steps (--refine-steps)")
    ap.add_argument("--refine-steps", type=int, default=3, help="fixed refinement steps of a batch")
    ap.add_argument("--no-extra", action="store_true",
                    help="mesh2000_N96: skip the other workloads reported beside the headline")
    ap.add_argument("--recompute-periods", type=int, default=0,
                    help="hold the factors of this many periods only and recompute them in every solve pass "
                         "(0 = keep all)")
    ap.add_argument("--dual-wait", type=int, default=-1,
                    help="elimination order: primal neighbours a dual waits for (0 = library default, "
                         "-1 = autotuned on the workload before the timed steps)")
    ap.add_argument("--schur", default="both", choices=["both", "dense", "structured"],
                    help="mesh2000_N96: factor S densely (the timed value), by structured block elimination, or "
                         "both (dense timed, structured reported beside it)")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline()))
        return 0
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        return 2
    if args.copy_probe:
        copy_probe()
        return 0
    import numpy as np
    import kktgen
    import paper_1907_05420_amd as pk

    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    if args.workload in ("uneven64", "serve"):
        res = bench_batch(args, log) if args.workload == "uneven64" else bench_serve(args, log)
        print(json.dumps(res), flush=True)
        return 0
    cfg = 3 if args.workload == "mesh9241_N24" else 2
    w = kktgen.WORKLOADS[cfg]
    inst = kktgen.make_workload(cfg)
    rng = np.random.default_rng(kktgen.seed_for(cfg, 9))
    vals2 = kktgen.redraw_barrier(inst, rng)
    prec = pk.KKT_MIXED if args.precision == "mixed" else pk.KKT_FP64
    main_mode = pk.KKT_SCHUR_STRUCTURED if args.schur == "structured" else pk.KKT_SCHUR_DENSE
    order_times = None
    if args.dual_wait < 0:
        # elimination order tuned once for the network (untimed, like the analysis)
        from paper_1907_05420_amd import autotune
        args.dual_wait, order_times = autotune.tune_order(inst, prec, schur_mode=main_mode, log=log)
    m = measure(args, inst, vals2, prec, log, schur_mode=main_mode)
    ph = m["phases"]
    ng = inst.n_g
    # dominant kernel: the dense Schur trailing update (FP64 MFMA)
    launches = sum(k["launches"] for k in m["kstats"])
    k_ms = sum(k["total_ms"] for k in m["kstats"])
    k_flops = sum(k["flops"] for k in m["kstats"])
    k_bytes = sum(k["bytes"] for k in m["kstats"])
    achieved = k_flops / (k_ms * 1e-3) / 1e12 if k_ms > 0 else 0.0
    traffic = measured_traffic() if cfg == 2 else None  # the committed counters are of mesh2000_N96
    # the other phases against their own rooflines (algorithmic work only):
    # block factor: N x the period's factorisation flops, N x (entries of A's
    # stored triangle + factor entries) x 8 bytes read/written once;
    # solve: every pass reads each period's factor twice (forward, backward)
    # and the dense Schur factor's two triangles once each; every FGMRES
    # iteration adds one product with K (values 8 B + column index 4 B per
    # stored entry, both triangles)
    st = m["stats"]
    N = w["N"]
    nnz_a = int(inst.colptr[-1])
    bf_flops = N * st["flops_factor"]
    bf_bytes = 8.0 * N * (nnz_a + st["nnz_L"])
    t_bf = max(bf_flops / (MI355X_FP64_TFLOPS * 1e12), bf_bytes / (MI355X_HBM_GBS * 1e9))
    iters = float(np.mean([i["refine_iters"] for i in m["infos"]]))
    pass_bytes = 16.0 * N * st["nnz_L"] + 8.0 * ng * ng
    matvec_bytes = 12.0 * N * (2 * nnz_a - inst.n_A)
    sv_bytes = (iters + 1) * pass_bytes + iters * matvec_bytes
    phase_roofline = {
        "block_factor": {"flops": bf_flops, "bytes": bf_bytes, "ms": ph[0],
                         "tflops": bf_flops / (ph[0] * 1e-3) / 1e12 if ph[0] > 0 else 0.0,
                         "gbs": bf_bytes / (ph[0] * 1e-3) / 1e9 if ph[0] > 0 else 0.0,
                         "attainable_ms": t_bf * 1e3, "frac_attainable": t_bf * 1e3 / ph[0] if ph[0] > 0 else 0.0},
        "solve_refined": {"passes": iters + 1, "pass_bytes": pass_bytes, "matvec_bytes": matvec_bytes,
                          "bytes": sv_bytes, "ms": ph[3],
                          "gbs": sv_bytes / (ph[3] * 1e-3) / 1e9 if ph[3] > 0 else 0.0,
                          "frac_hbm": sv_bytes / (ph[3] * 1e-3) / 1e9 / MI355X_HBM_GBS if ph[3] > 0 else 0.0},
    }
    res = {
        "metric": METRIC,
        "value": m["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == pk.KKT_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "buses": w["nb"], "lines": w["nlines"], "generators": w["ng"],
                   "storage": w["ns"], "periods": w["N"], "block_rows": inst.n_A, "schur_dim": ng,
                   "nrhs": w["nrhs"], "barrier_range": list(w["barrier"]), "precision": args.precision,
                   "refine": args.refine, "recompute_periods": args.recompute_periods,
                   "dual_wait": args.dual_wait,
                   "dual_wait_tuned_ms": ({str(k): round(v, 2) for k, v in order_times.items()}
                                          if order_times else None),
                   "schur": "structured" if main_mode == pk.KKT_SCHUR_STRUCTURED else "dense"},
        "device_bytes": m["stats"]["footprint_after"],
        "p50_ms": float(np.percentile(m["lat_ms"], 50)),
        "p99_ms": float(np.percentile(m["lat_ms"], 99)),
        "rel_res": max(i["rel_res"] for i in m["infos"]),
        "rel_res_steps": [i["rel_res"] for i in m["infos"]],
        "solves_at_tolerance": sum(1 for rc, i in zip(m["rcs"], m["infos"]) if rc == 0 and i["rel_res"] <= 1e-10),
        "rc_steps": m["rcs"],
        "residual_eval": "compensated FP64 (twice-working-precision sums) on the unscaled K",
        "omega": max(i["omega"] for i in m["infos"]),
        "refine_iters": [i["refine_iters"] for i in m["infos"]],
        "phase_ms": {"block_factor": ph[0], "schur_assembly": ph[1], "schur_ldlt": ph[2], "solve_refined": ph[3],
                     "schur_update_kernel": ph[4]},
        "schur_ldlt_tflops": ng ** 3 / 3.0 / (ph[2] * 1e-3) / 1e12 if ph[2] > 0 else 0.0,
        "analyze_ms": m["analyze_ms"],
        "phase_roofline": phase_roofline,
        "roofline": {"bound": "mfma", "kernel": "k_update_big (dense Schur trailing update, FP64 MFMA)",
                     "achieved": achieved, "peak": MI355X_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / MI355X_FP64_TFLOPS,
                     "traffic": traffic,
                     "launches_per_step": launches / max(args.steps, 1),
                     "avg_launch_ms": k_ms / launches if launches else 0.0,
                     "flops_per_launch": k_flops / launches if launches else 0.0,
                     "algorithmic_bytes_per_launch": k_bytes / launches if launches else 0.0},
    }
    if prec == pk.KKT_MIXED:
        # the same workload on the FP64 path: speed-up and forward error
        m64 = measure(args, inst, vals2, pk.KKT_FP64, log, schur_mode=main_mode)
        x64, xm = m64["x_last"], m["x_last"]
        res["mixed"] = {
            "fallback_used": [i["fallback_used"] for i in m["infos"]],
            "fp64_value": m64["value"], "speedup_vs_fp64": m["value"] / m64["value"],
            "forward_error_vs_fp64": float(np.linalg.norm(xm - x64) / np.linalg.norm(x64))
            if m["last_set"] == m64["last_set"] else None,
            "device_bytes": m["stats"]["footprint_after"], "device_bytes_fp64": m64["stats"]["footprint_after"],
            "dual_wait": args.dual_wait}
    if args.schur == "both" and prec == pk.KKT_FP64:
        # the same workload with S factored by structured block elimination
        ms = measure(args, inst, vals2, prec, log, schur_mode=pk.KKT_SCHUR_STRUCTURED)
        ps = ms["phases"]
        res["schur_structured"] = {
            "value": ms["value"], "unit": "solves/s", "ms_per_step": ms["elapsed"] / args.steps * 1e3,
            "speedup_vs_dense": ms["value"] / m["value"],
            "p50_ms": float(np.percentile(ms["lat_ms"], 50)), "p99_ms": float(np.percentile(ms["lat_ms"], 99)),
            "rel_res": max(i["rel_res"] for i in ms["infos"]), "omega": max(i["omega"] for i in ms["infos"]),
            "solves_at_tolerance": sum(1 for rc, i in zip(ms["rcs"], ms["infos"])
                                       if rc == 0 and i["rel_res"] <= 1e-10),
            "refine_iters": [i["refine_iters"] for i in ms["infos"]],
            "phase_ms": {"block_factor": ps[0], "schur_prefix": ps[1], "schur_elimination": ps[2],
                         "solve_refined": ps[3]},
            "device_bytes": ms["stats"]["footprint"], "device_bytes_dense": m["stats"]["footprint"]}
    if cfg == 2 and not args.no_extra and prec == pk.KKT_FP64 and args.recompute_periods == 0:
        # the other workloads, each in a process of its own (device memory
        # released in between), reported beside the headline
        extra = {"serve": ["--workload", "serve", "--requests", "12", "--iterations", "10"],
                 "uneven64": ["--workload", "uneven64", "--steps", "2", "--warmup", "1"],
                 "mesh9241_N24": ["--workload", "mesh9241_N24", "--steps", "3", "--warmup", "1", "--schur", "dense",
                                  "--no-cpu-baseline"]}
        res["other_workloads"] = {}
        for name, argv in extra.items():
            try:
                r = subprocess.run([sys.executable, os.path.abspath(__file__)] + argv, capture_output=True,
                                   text=True, timeout=400)
                line = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
            except (subprocess.TimeoutExpired, ValueError, IndexError) as e:
                log(f"{name}: {e}")
                line = None
            if line is None:
                res["other_workloads"][name] = None
                continue
            keep = ("value", "unit", "ms_per_step", "p50_ms", "p99_ms", "rel_res", "rel_res_max", "above_1e-10",
                    "solves_at_tolerance", "refine_iters", "inertia_ok", "speedup_vs_sequential", "device_gb",
                    "device_bytes", "request_p50_ms", "request_p99_ms", "phase_ms", "config")
            res["other_workloads"][name] = {k: line[k] for k in keep if k in line}
            log(f"{name}: {res['other_workloads'][name].get('value')}")
    if not args.no_cpu_baseline and cfg == 2:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only"],
                           capture_output=True, text=True, timeout=900)
        if r.returncode == 0:
            res["cpu_baseline"] = json.loads(r.stdout.strip().splitlines()[-1])
        else:
            log("cpu baseline failed:", r.stderr[-2000:])
            res["cpu_baseline"] = None
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
