"""Seeded synthetic inputs for the block-bordered (arrowhead) KKT system of
multiperiod AC-OPF with storage.

This module only draws topologies, sparsity patterns, values and right-hand
sides. It performs none of the solver's arithmetic, so both the FP64 oracle and
the GPU library can consume its output without sharing any solver code.

Block layout (one time period, caller order), following the MPOPF variable
grouping u_n = (x_n, lambda_E,n) of the structure-revealing ordering (section
4.1, Eq. orderingMPOPF) restricted to the equality multipliers:

    x_n      = (theta[Nb], V[Nb], Pg[Ng], Qg[Ng], Psd[Ns], Psc[Ns])   primal
    lambda_n = (lamP[Nb], lamQ[Nb])                                  duals

A_n = [[Ht, J^T], [J, -delta_c I]] where Ht couples (theta, V) over closed bus
neighbourhoods (the admittance graph of the AC power-flow model, section 3.1)
and carries a barrier diagonal X^-1 Z; J is the power-balance Jacobian: the P
and Q balance rows of bus k touch (theta_j, V_j) for j in N[k], the bus's
generator P (resp. Q) column, and the storage discharge/charge columns in the
P row (storage power injections p^S = (p^Sd, p^Sc), section 3.2).

The storage coupling follows Eq. B12N: B_n has block rows 0 (m < n), C_1
(m = n) and C_0 (m > n), each C_j an Ns x nA matrix with one row per storage
unit holding its (discharge, charge) columns. C_0 and C_1 are two independent
draws (they must differ for Eq. GlobalSchur's diagonal and sub-diagonal blocks
to differ). The corner block is -1e-8 I (a dual regularisation of the same size
as the block duals) unless asked to be zero.

Values: off-diagonal Hessian and Jacobian entries ~ N(0,1). The (theta,V)
Hessian diagonal is the row's absolute off-diagonal sum plus a barrier term
drawn log-uniformly, so Ht is positive definite and every A_n has the inertia
the IPM requires (section 2.3): (n_primal, n_dual, 0).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SEED_BASE = 1907054200
DUAL_REG = 1e-8


def seed_for(cfg: int, rep: int = 0) -> int:
    """Seed of repetition `rep` of workload `cfg` (1-based workload index)."""
    return SEED_BASE + 10 * cfg + rep


# ----------------------------------------------------------------------------
# topology
# ----------------------------------------------------------------------------

def ring_with_chords(nb: int, nchords: int, rng: np.random.Generator):
    """Ring over nb buses plus `nchords` distinct uniform random chords."""
    edges = {(k, (k + 1) % nb) if k < (k + 1) % nb else ((k + 1) % nb, k) for k in range(nb)}
    want = len(edges) + nchords
    while len(edges) < want:
        a, b = rng.integers(0, nb, size=2)
        if a == b:
            continue
        e = (int(min(a, b)), int(max(a, b)))
        edges.add(e)
    return np.array(sorted(edges), dtype=np.int64)


def tree_with_chords(nb: int, nlines: int, rng: np.random.Generator, deg_cap: int = 6):
    """Random recursive spanning tree (bus k attaches to a uniformly random
    earlier bus whose degree is below the cap) plus uniform random chords
    between buses below the cap, up to `nlines` lines in total."""
    deg = np.zeros(nb, dtype=np.int64)
    edges = set()
    open_buses = [0]  # earlier buses with degree < cap
    pos = {0: 0}
    for k in range(1, nb):
        j = open_buses[int(rng.integers(0, len(open_buses)))]
        edges.add((j, k))
        deg[j] += 1
        deg[k] += 1
        if deg[j] >= deg_cap:
            # remove j from open list (swap-remove)
            p = pos.pop(j)
            last = open_buses.pop()
            if last != j:
                open_buses[p] = last
                pos[last] = p
        pos[k] = len(open_buses)
        open_buses.append(k)
    attempts = 0
    max_attempts = 50 * nlines + 1000
    while len(edges) < nlines and attempts < max_attempts:
        attempts += 1
        a, b = (int(v) for v in rng.integers(0, nb, size=2))
        if a == b or deg[a] >= deg_cap or deg[b] >= deg_cap:
            continue
        e = (min(a, b), max(a, b))
        if e in edges:
            continue
        edges.add(e)
        deg[a] += 1
        deg[b] += 1
    return np.array(sorted(edges), dtype=np.int64)


# ----------------------------------------------------------------------------
# instance
# ----------------------------------------------------------------------------

@dataclass
class Instance:
    nb: int
    ng: int
    ns: int
    N: int
    lines: np.ndarray
    gen_bus: np.ndarray
    sto_bus: np.ndarray
    n_A: int
    n_primal: int
    colptr: np.ndarray      # int64 [n_A+1], lower-triangular CSC pattern of A_n
    rowind: np.ndarray      # int32 [nnz]
    vals: np.ndarray        # float64 [N, nnz]
    C0_rowptr: np.ndarray   # int64 [ns+1]
    C0_colind: np.ndarray   # int32
    C0_vals: np.ndarray     # float64
    C1_rowptr: np.ndarray
    C1_colind: np.ndarray
    C1_vals: np.ndarray
    corner_diag: np.ndarray  # float64 [n_g]  (diagonal of the corner block C)
    b: np.ndarray            # float64 [nrhs, N*n_A + n_g]
    barrier_range: tuple = (1e-6, 1e6)
    meta: dict = field(default_factory=dict)

    @property
    def n_g(self) -> int:
        return self.N * self.ns

    @property
    def nnz(self) -> int:
        return int(self.rowind.shape[0])

    @property
    def n_total(self) -> int:
        return self.N * self.n_A + self.n_g

    @property
    def nrhs(self) -> int:
        return int(self.b.shape[0])


def _var_index(nb, ng, ns, n_flow=0, n_keep=0):
    """Row indices of every variable group of one period block:
    x = (theta, V, Pg, Qg, Psd, Psc), the kept slacks, then the duals
    lambda_E = (lamP, lamQ) and lambda_I (n_flow line-flow rows)."""
    n_x = 2 * nb + 2 * ng + 2 * ns
    n_primal = n_x + n_keep
    idx = dict(
        theta=np.arange(nb),
        V=nb + np.arange(nb),
        Pg=2 * nb + np.arange(ng),
        Qg=2 * nb + ng + np.arange(ng),
        Psd=2 * nb + 2 * ng + np.arange(ns),
        Psc=2 * nb + 2 * ng + ns + np.arange(ns),
        slack=n_x + np.arange(n_keep),
        lamP=n_primal + np.arange(nb),
        lamQ=n_primal + nb + np.arange(nb),
        lamI=n_primal + 2 * nb + np.arange(n_flow),
    )
    return idx, n_primal, n_primal + 2 * nb + n_flow


def block_pattern(nb, lines, gen_bus, sto_bus, line_flow=False, keep=None):
    """Lower-triangular CSC pattern of one period block and the role of every
    entry. Returns (n_A, n_primal, colptr, rowind, kind) where kind[k] is
    0 = Hessian (theta,V) off-diagonal, 1 = Hessian (theta,V) diagonal,
    2 = barrier-only diagonal (gen / storage), 3 = Jacobian, 4 = dual diagonal,
    5 = kept slack diagonal (L_s), 6 = kept slack link (-1).

    With line_flow, every line l = (f, t) has two flow-limit rows in J_I (the
    flow at its f end, then the flow at its t end; all f-end rows first, in
    line order), each touching (theta_f, theta_t, V_f, V_t) (section 3.1's
    line-flow constraints, pattern of Fig. KKTsystemOPF), with a slack each
    (c_I(x) - s = 0, section 2). keep[j] (bool per flow row) keeps slack j as
    a primal row of the block, linked to its flow row by -1 (Eq.
    SCOPFhessianSymmetric); the other slacks are eliminated (Eq.
    SCOPFhessianReduced) and only their flow row's diagonal stays."""
    ng, ns = len(gen_bus), len(sto_bus)
    n_flow = 2 * len(lines) if line_flow else 0
    keep = np.zeros(n_flow, bool) if keep is None else np.asarray(keep, bool)
    assert keep.shape == (n_flow,)
    kept = np.nonzero(keep)[0]
    idx, n_primal, n_A = _var_index(nb, ng, ns, n_flow, len(kept))
    th, V = idx["theta"], idx["V"]
    ents = {}

    def put(i, j, kind):
        i, j = int(i), int(j)
        if i < j:
            i, j = j, i
        ents[(i, j)] = kind

    nbr = [[k] for k in range(nb)]
    for a, b in lines:
        nbr[a].append(int(b))
        nbr[b].append(int(a))
    # Hessian over closed neighbourhoods (theta, V) x (theta, V)
    for k in range(nb):
        put(th[k], th[k], 1)
        put(V[k], V[k], 1)
        put(V[k], th[k], 0)
    for a, b in lines:
        for u in (th[a], V[a]):
            for w in (th[b], V[b]):
                put(u, w, 0)
    for g in range(ng):
        put(idx["Pg"][g], idx["Pg"][g], 2)
        put(idx["Qg"][g], idx["Qg"][g], 2)
    for s in range(ns):
        put(idx["Psd"][s], idx["Psd"][s], 2)
        put(idx["Psc"][s], idx["Psc"][s], 2)
    # power-balance Jacobian
    for k in range(nb):
        for j in nbr[k]:
            for u in (th[j], V[j]):
                put(idx["lamP"][k], u, 3)
                put(idx["lamQ"][k], u, 3)
        put(idx["lamP"][k], idx["lamP"][k], 4)
        put(idx["lamQ"][k], idx["lamQ"][k], 4)
    for g, k in enumerate(gen_bus):
        put(idx["lamP"][k], idx["Pg"][g], 3)
        put(idx["lamQ"][k], idx["Qg"][g], 3)
    for s, k in enumerate(sto_bus):
        put(idx["lamP"][k], idx["Psd"][s], 3)
        put(idx["lamP"][k], idx["Psc"][s], 3)
    if line_flow:
        nl = len(lines)
        for end in range(2):
            for l, (f, t) in enumerate(lines):
                r = idx["lamI"][end * nl + l]
                for u in (th[f], th[t], V[f], V[t]):
                    put(r, u, 3)
                put(r, r, 4)
        for q, j in enumerate(kept):
            put(idx["slack"][q], idx["slack"][q], 5)
            put(idx["lamI"][j], idx["slack"][q], 6)
    keys = sorted(ents.keys(), key=lambda ij: (ij[1], ij[0]))
    rows = np.array([ij[0] for ij in keys], dtype=np.int32)
    cols = np.array([ij[1] for ij in keys], dtype=np.int64)
    kind = np.array([ents[ij] for ij in keys], dtype=np.int8)
    colptr = np.zeros(n_A + 1, dtype=np.int64)
    np.add.at(colptr, cols + 1, 1)
    colptr = np.cumsum(colptr)
    return n_A, n_primal, colptr, rows, kind


def draw_values(n_A, colptr, rowind, kind, N, rng, barrier_range, dual_reg=DUAL_REG):
    """Values [N, nnz] for the given pattern (see module docstring)."""
    nnz = rowind.shape[0]
    cols = np.repeat(np.arange(n_A), np.diff(colptr))
    lo, hi = barrier_range
    vals = np.empty((N, nnz), dtype=np.float64)
    off = kind == 0
    jac = kind == 3
    hdiag = kind == 1
    bdiag = kind == 2
    ddiag = kind == 4
    for n in range(N):
        v = np.zeros(nnz)
        v[off] = rng.standard_normal(int(off.sum()))
        v[jac] = rng.standard_normal(int(jac.sum()))
        barrier = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_A))
        # absolute off-diagonal Hessian row sums (symmetric pattern, lower stored)
        rs = np.zeros(n_A)
        np.add.at(rs, rowind[off], np.abs(v[off]))
        np.add.at(rs, cols[off], np.abs(v[off]))
        d = cols[hdiag]
        v[hdiag] = rs[d] + barrier[d]
        d = cols[bdiag]
        v[bdiag] = barrier[d]
        v[ddiag] = -dual_reg
        vals[n] = v
    return vals


def draw_slacks(n_flow, N, rng, ls_range, keep_below):
    """L_s = S^-1 Y of every line-flow slack and period, log-uniform in
    ls_range; a slack whose L_s falls below keep_below in any period is kept
    in the block (the reduction needs L_s away from zero, section 2.1)."""
    lo, hi = ls_range
    Ls = np.exp(rng.uniform(math.log(lo), math.log(hi), size=(N, n_flow)))
    keep = (Ls < keep_below).any(axis=0)
    return Ls, keep


def redraw_barrier(inst: "Instance", rng: np.random.Generator, barrier_range=None) -> np.ndarray:
    """New values with only the barrier diagonal re-drawn (an IPM-like
    iteration that keeps the pattern, the Hessian off-diagonals and Jacobian)."""
    kind = inst.meta["kind"]
    lo, hi = barrier_range or inst.barrier_range
    cols = np.repeat(np.arange(inst.n_A), np.diff(inst.colptr))
    off = kind == 0
    vals = inst.vals.copy()
    for n in range(inst.N):
        v = vals[n]
        barrier = np.exp(rng.uniform(math.log(lo), math.log(hi), size=inst.n_A))
        rs = np.zeros(inst.n_A)
        np.add.at(rs, inst.rowind[off], np.abs(v[off]))
        np.add.at(rs, cols[off], np.abs(v[off]))
        h = kind == 1
        v[h] = rs[cols[h]] + barrier[cols[h]]
        bmask = kind == 2
        v[bmask] = barrier[cols[bmask]]
    return vals


def storage_coupling(nb, ng, ns, rng):
    """C_0, C_1 as CSR (ns x n_A): row s holds unit s's (discharge, charge)."""
    idx, _, _ = _var_index(nb, ng, ns)
    rowptr = np.arange(0, 2 * ns + 1, 2, dtype=np.int64)
    colind = np.empty(2 * ns, dtype=np.int32)
    colind[0::2] = idx["Psd"]
    colind[1::2] = idx["Psc"]
    C0 = rng.standard_normal(2 * ns)
    C1 = rng.standard_normal(2 * ns)
    return rowptr, colind, C0, rowptr.copy(), colind.copy(), C1


def make_instance(nb, lines, ng, ns, N, nrhs, seed, barrier_range=(1e-6, 1e6),
                  corner="diag", rng=None, gen_bus=None, sto_bus=None, line_flow=False, ls_range=None,
                  keep_below=1e-3) -> Instance:
    """One instance. With line_flow the blocks carry the line-flow rows and
    their slacks (block_pattern): slacks whose L_s falls below keep_below in
    some period stay in the block, the others are eliminated and described
    by inst.slack: lam_row (the flow row of A_n each one is linked to by
    -1), Ls [N, n_elim] and rs [nrhs, N * n_elim] (their right-hand sides,
    period-major)."""
    rng = rng if rng is not None else np.random.default_rng(seed)
    if gen_bus is None:
        gen_bus = np.sort(rng.choice(nb, size=ng, replace=False)).astype(np.int64)
    if sto_bus is None:
        sto_bus = np.sort(rng.choice(nb, size=ns, replace=False)).astype(np.int64)
    keep = Ls = None
    if line_flow:
        Ls, keep = draw_slacks(2 * len(lines), N, rng, ls_range or barrier_range, keep_below)
    n_A, n_primal, colptr, rowind, kind = block_pattern(nb, lines, gen_bus, sto_bus, line_flow, keep)
    vals = draw_values(n_A, colptr, rowind, kind, N, rng, barrier_range)
    slack = None
    if line_flow:
        idx, _, _ = _var_index(nb, ng, ns, 2 * len(lines), int(keep.sum()))
        cols = np.repeat(np.arange(n_A), np.diff(colptr))
        kept = np.nonzero(keep)[0]
        for q, j in enumerate(kept):      # kept slack q: diagonal L_s, link -1
            d = np.nonzero((kind == 5) & (cols == idx["slack"][q]))[0]
            vals[:, d] = Ls[:, j][:, None]
        vals[:, kind == 6] = -1.0
        elim = np.nonzero(~keep)[0]
        slack = dict(lam_row=idx["lamI"][elim].astype(np.int32), Ls=np.ascontiguousarray(Ls[:, elim]),
                     keep=keep)
    c0p, c0i, c0v, c1p, c1i, c1v = storage_coupling(nb, ng, ns, rng)
    n_g = N * ns
    if corner == "diag":
        corner_diag = np.full(n_g, -DUAL_REG)
    elif corner == "zero":
        corner_diag = np.zeros(n_g)
    else:
        raise ValueError(corner)
    b = rng.standard_normal((nrhs, N * n_A + n_g))
    if slack is not None:
        slack["rs"] = rng.standard_normal((nrhs, N * len(slack["lam_row"])))
    return Instance(nb=nb, ng=ng, ns=ns, N=N, lines=lines, gen_bus=gen_bus, sto_bus=sto_bus,
                    n_A=n_A, n_primal=n_primal, colptr=colptr, rowind=rowind, vals=vals,
                    C0_rowptr=c0p, C0_colind=c0i, C0_vals=c0v,
                    C1_rowptr=c1p, C1_colind=c1i, C1_vals=c1v,
                    corner_diag=corner_diag, b=b, barrier_range=barrier_range,
                    meta=dict(kind=kind, seed=seed, slack=slack))


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

WORKLOADS = {
    1: dict(name="ring30_N8", nb=30, topo="ring", nchords=11, ng=6, ns=2, N=8, nrhs=1,
            barrier=(1e-6, 1e6)),
    2: dict(name="mesh2000_N96", nb=2000, topo="tree", nlines=3000, ng=400, ns=200, N=96, nrhs=4,
            barrier=(1e-8, 1e8)),
    3: dict(name="mesh9241_N24", nb=9241, topo="tree", nlines=16000, ng=1400, ns=500, N=24, nrhs=1,
            barrier=(1e-6, 1e6)),
}


def make_workload(cfg: int, rep: int = 0, N=None, nrhs=None, corner="diag", barrier=None) -> Instance:
    """Instance of workload `cfg` (1, 2 or 3); N / nrhs / barrier may be
    overridden for reduced test cases (topology and values stay seeded)."""
    w = WORKLOADS[cfg]
    seed = seed_for(cfg, rep)
    rng = np.random.default_rng(seed)
    if w["topo"] == "ring":
        lines = ring_with_chords(w["nb"], w["nchords"], rng)
    else:
        lines = tree_with_chords(w["nb"], w["nlines"], rng)
    inst = make_instance(w["nb"], lines, w["ng"], w["ns"], N or w["N"], nrhs or w["nrhs"], seed,
                         barrier_range=barrier or w["barrier"], corner=corner, rng=rng)
    inst.meta["workload"] = w["name"]
    return inst


def make_small(nb=12, nextra=6, ng=3, ns=2, N=3, nrhs=1, seed=0, barrier_range=(1e-6, 1e6),
               corner="diag", topo="tree", line_flow=False, ls_range=None, keep_below=1e-3) -> Instance:
    """A tiny instance for brute-force checks."""
    rng = np.random.default_rng(seed)
    if topo == "ring":
        lines = ring_with_chords(nb, nextra, rng)
    else:
        lines = tree_with_chords(nb, nb - 1 + nextra, rng)
    return make_instance(nb, lines, ng, ns, N, nrhs, seed, barrier_range=barrier_range,
                         corner=corner, rng=rng, line_flow=line_flow, ls_range=ls_range, keep_below=keep_below)


def uneven_batch(count=64, seed=None, nb_range=(118, 3000), horizons=(12, 24, 48, 96), nrhs=1,
                 barrier=(1e-6, 1e6), max_instances=None):
    """The uneven mixture: bus counts log-uniform in nb_range, lines ~1.5 Nb,
    generators ~0.2 Nb, storage ~0.1 Nb (at least 1), horizon uniform over
    `horizons`. Returns a list of Instances."""
    seed = seed_for(4, 0) if seed is None else seed
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count if max_instances is None else min(count, max_instances)):
        nb = int(round(math.exp(rng.uniform(math.log(nb_range[0]), math.log(nb_range[1])))))
        nl = int(round(1.5 * nb))
        ng = max(1, int(round(0.2 * nb)))
        ns = max(1, int(round(0.1 * nb)))
        N = int(rng.choice(np.array(horizons)))
        sub = int(rng.integers(0, 2**31 - 1))
        r2 = np.random.default_rng(sub)
        lines = tree_with_chords(nb, nl, r2)
        inst = make_instance(nb, lines, ng, ns, N, nrhs, sub, barrier_range=barrier, rng=r2)
        inst.meta["workload"] = f"uneven[{i}]"
        out.append(inst)
    return out
