"""GPU parity: the HIP path (called through the C-ABI) against the FP64 oracle.

Tolerances (FP64 path): the relative residual max_k ||b_k - K x_k||_2/||b_k||_2,
computed on the CPU from the oracle's assembled K in extended precision, must
be <= 1e-10 (the target of the workload definition), or twice the best the
oracle's refined FP64 solution reaches where that is more (flagged). On the
well-conditioned inputs (barrier range [1e-2, 1e2]) x is compared with the
oracle's element by element (1e-10 ||x||_inf + 1e-7 |x_i|), both unrefined
(refine_max = 0, against the oracle's unrefined Algorithm 1) and refined (at
most one refinement step); on the wide barrier ranges normwise at 1e-6.
Schur complements are unique and are compared elementwise relative to max|S|
(1e-9 well-conditioned). Inertia is exact."""
import numpy as np
import pytest

import kktgen
from oracle import arrowhead as ah
from oracle import schur as sc

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_gpu(inst, precision=0, want_schur=True, delta_w=0.0, delta_c=0.0, vals=None, refine_max=20, dual_wait=0):
    torch = _torch()
    import paper_1907_05420_amd as pk
    d = pk.device_inputs(inst)
    if vals is not None:
        d["vals"] = torch.as_tensor(vals).cuda()
    s = pk.Solver(inst, precision=precision, refine_max=refine_max, dual_wait=dual_wait)
    rc_f, inertia = s.factor(d["vals"], d["C0"], d["C1"], d["corner"], delta_w, delta_c)
    x, rc_s, info = s.solve(d["b"])
    out = dict(x=x.cpu().numpy(), rc_factor=rc_f, rc_solve=rc_s, inertia=inertia, info=info,
               footprint=s.footprint())
    if want_schur and inst.n_g:
        out["S"] = s.schur().cpu().numpy()
        out["Sbar"] = s.schur_blocks().cpu().numpy()
    torch.cuda.synchronize()
    s.close()
    return out


def reference(inst):
    """The oracle's Algorithm 1, refined with extended-precision residuals
    (section 2.1) until they stop improving; best_rel is the smallest
    relative residual along the way (what an FP64 solution can reach)."""
    out = sc.algorithm1(inst)
    K = ah.assemble(inst)
    solve = lambda r: sc.algorithm1(inst, b=r, factors=out["factors"], schur=out["schur_fac"])["x"]
    x, hist = sc.refine(inst, out["x"], inst.b, solve, tol=1e-16, K=K, extended=True)
    out["best_rel"] = min(hist)
    return out, x, K


def residual_bar(ref):
    """1e-10, or twice what the FP64 oracle itself reaches when that is more
    (an instance whose conditioning puts 1e-10 out of FP64's reach; flagged)."""
    bar = max(1e-10, 2.0 * ref["best_rel"])
    if bar > 1e-10:
        print(f"[flagged] FP64 oracle reaches only {ref['best_rel']:.2e}; bar {bar:.2e}")
    return bar


SMALL = [
    dict(nb=8, nextra=3, ng=2, ns=2, N=3, nrhs=1, seed=0),
    dict(nb=12, nextra=6, ng=3, ns=3, N=4, nrhs=4, seed=1),
    dict(nb=10, nextra=4, ng=2, ns=1, N=1, nrhs=2, seed=2),          # N = 1
    dict(nb=9, nextra=5, ng=3, ns=0, N=3, nrhs=1, seed=3),           # Ns = 0: independent blocks
    dict(nb=15, nextra=8, ng=4, ns=2, N=5, nrhs=1, seed=4, corner="zero"),
    dict(nb=70, nextra=40, ng=12, ns=9, N=9, nrhs=3, seed=6),        # n_g = 81: two Schur steps, ragged
    dict(nb=160, nextra=90, ng=30, ns=12, N=7, nrhs=2, seed=8),      # several large fronts
    # Schur dimensions around the 256-wide blocks of the dense solves
    dict(nb=60, nextra=30, ng=8, ns=26, N=12, nrhs=2, seed=10),      # n_g = 312: last block 56 wide
    dict(nb=70, nextra=30, ng=8, ns=43, N=12, nrhs=1, seed=12),      # n_g = 516: last block 4 wide
    dict(nb=40, nextra=20, ng=6, ns=16, N=32, nrhs=1, seed=11),      # n_g = 512: two whole blocks
    dict(nb=50, nextra=25, ng=8, ns=24, N=20, nrhs=3, seed=13),      # n_g = 480: last block 224 wide
    dict(nb=80, nextra=40, ng=10, ns=50, N=16, nrhs=2, seed=14),     # n_g = 800: a second 512-panel with two halves
]


def assert_x_close(x, xref, atol_inf, rtol):
    """Element by element: |x_i - xref_i| <= atol_inf ||xref||_inf + rtol |xref_i|
    (per right-hand side)."""
    xinf = np.max(np.abs(xref), axis=-1, keepdims=True)
    err = np.abs(x - xref)
    tol = atol_inf * xinf + rtol * np.abs(xref)
    worst = np.unravel_index(np.argmax(err / tol), err.shape)
    assert np.all(err <= tol), (worst, x[worst], xref[worst], err[worst] / xinf[worst[0], 0])


GROWTH_FREE = 1 << 30   # dual_wait: every dual waits for all its primal neighbours


class _OrderedFactor:
    """The oracle's dense LDL^T of one block in a given elimination order
    (natural order on P A P^T), in the form oracle.schur.algorithm1 takes."""

    def __init__(self, A, n_primal, perm):
        from oracle.ldlt import ldlt
        self.p = perm
        signs = np.where(perm < n_primal, 1.0, -1.0)
        self.L, self.d, self.n_perturbed, _ = ldlt(A.toarray()[np.ix_(perm, perm)], signs=signs, eps=1e-20,
                                                   return_raw=True)
        self.inertia = None
        self.kind = "dense"

    def solve(self, y):
        from oracle.ldlt import ldlt_solve
        y = np.asarray(y, dtype=np.float64)
        out = np.empty_like(y)
        out[self.p] = ldlt_solve(self.L, self.d, y[self.p])
        return out


def oracle_in_order(inst, dual_wait=0):
    """The oracle's unrefined Algorithm 1 with every period block eliminated
    in the order the library's symbolic analysis chooses (host-only plan)."""
    import paper_1907_05420_amd as pk
    _, perm = pk.kkt_plan(inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, inst.rowind, inst.C0_rowptr,
                          inst.C0_colind, inst.C1_rowptr, inst.C1_colind, want_perm=True, dual_wait=dual_wait)
    facs = [_OrderedFactor(ah.block(inst, n), inst.n_primal, perm) for n in range(inst.N)]
    return sc.algorithm1(inst, factors=facs)


@pytest.mark.parametrize("case", SMALL)
def test_parity_small_unrefined(case):
    """refine_max = 0: the factorisation's own solution (Algorithm 1 with no
    refinement step), so refinement cannot hide a wrong factor.

    In the elimination order where every dual waits for all its primal
    neighbours (no pivot growth on these blocks; the same kernels as every
    other order) the unrefined solution meets the oracle pin's 1e-11
    residual bar, or 3 x what the oracle's unrefined Algorithm 1 reaches in
    that same order where that is more, and matches the oracle's unrefined
    Algorithm 1 element by element: two FP64 solves of these
    well-conditioned systems in different elimination orders differ by at
    most 2e-12 ||x||_inf and 1e-8 of an entry (oracle against the LAPACK
    solve of the assembled K), checked at 1e-10 ||x||_inf + 1e-7 |x_i|.

    In the default order (dual wait 4 with pairing) these blocks show pivot
    growth up to 3e5, so the unrefined residual there is held to
    max(1e-9, 30 x the oracle's unrefined Algorithm 1 in the same elimination
    order): the same arithmetic up to its grouping, except that the kernels
    apply explicit inverses of the 64-column pivot blocks and of the dense
    factor's 1024-wide diagonal blocks where the oracle substitutes column by
    column, which multiplies rounding errors by up to the condition numbers
    of those unit triangular blocks (measured: 0.3 to 10.4 x the oracle's
    residual on these cases). A wrong factor lands orders of magnitude
    above."""
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    ora = sc.algorithm1(inst)
    K = ah.assemble(inst)
    assert ah.rel_residual_ld(inst, ora["x"], inst.b, K) <= 1e-11
    g = run_gpu(inst, want_schur=False, refine_max=0, dual_wait=GROWTH_FREE)
    rel = ah.rel_residual_ld(inst, g["x"], inst.b, K)
    rel_g = ah.rel_residual_ld(inst, oracle_in_order(inst, GROWTH_FREE)["x"], inst.b, K)
    assert rel <= max(1e-11, 3.0 * rel_g), (rel, rel_g)
    assert g["info"]["refine_iters"] == 0
    assert g["rc_solve"] == 0
    assert abs(g["info"]["rel_res"] - rel) <= 1e-2 * rel + 1e-17
    assert_x_close(g["x"], ora["x"], 1e-10, 1e-7)
    inn = g["inertia"]
    assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == ora["inertia"] and inn["n_perturbed"] == 0
    d = run_gpu(inst, want_schur=False, refine_max=0)
    rel_d = ah.rel_residual_ld(inst, d["x"], inst.b, K)
    rel_o = ah.rel_residual_ld(inst, oracle_in_order(inst)["x"], inst.b, K)
    assert rel_d <= max(1e-9, 30.0 * rel_o), (rel_d, rel_o)
    assert d["info"]["refine_iters"] == 0


@pytest.mark.parametrize("case", SMALL)
def test_parity_small(case):
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    ref, xref, K = reference(inst)
    g = run_gpu(inst)
    rel = ah.rel_residual_ld(inst, g["x"], inst.b, K)
    assert rel <= 1e-10, rel
    assert_x_close(g["x"], xref, 1e-10, 1e-7)
    assert g["info"]["rel_res"] <= 1e-10
    assert g["info"]["refine_iters"] <= 1
    expect = (inst.N * inst.n_primal, inst.N * (inst.n_A - inst.n_primal) + inst.n_g, 0)
    inn = g["inertia"]
    assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == expect == ref["inertia"]
    assert inn["inertia_ok"] == 1 and inn["n_perturbed"] == 0
    if inst.n_g:
        scale = np.max(np.abs(ref["S"]))
        assert np.max(np.abs(np.tril(g["S"]) - np.tril(ref["S"]))) <= 1e-9 * scale
        assert np.allclose(g["S"], g["S"].T, rtol=0, atol=0)
        sb = ref["Sbar"]
        assert np.max(np.abs(g["Sbar"] - sb)) <= 1e-9 * np.max(np.abs(sb))


# Schur sizes around the 1024-wide inverted diagonal blocks that the dense
# solves use: a second block 16 wide, a second block of exactly half width
# (built from two 256-wide inverses, no second half to combine), and three
# blocks with a 52-wide tail
def test_parity_wide_fronts_unrefined():
    """A front with more pivots than two of the solves' 256-pivot windows
    (526 pivots in the growth-free order: windows of 256, 256 and 14, each
    window solved by one workgroup per period and its products with the
    rest of the pivot part spread over many): with refine_max = 0 the
    solution meets the small cases' bar (1e-11, or 3 x the oracle's
    unrefined Algorithm 1 in the same order) and matches the oracle's
    unrefined Algorithm 1 element by element, for 3 right-hand sides (one
    pass of four with a padded one) and for 1."""
    import paper_1907_05420_amd as pk
    for nrhs in (3, 1):
        inst = kktgen.make_small(nb=400, nextra=200, ng=50, ns=20, N=2, nrhs=nrhs, seed=21,
                                 barrier_range=(1e-2, 1e2))
        st, _ = pk.kkt_plan(inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, inst.rowind, inst.C0_rowptr,
                            inst.C0_colind, inst.C1_rowptr, inst.C1_colind, dual_wait=GROWTH_FREE)
        assert st["max_pivots"] > 2 * 256
        K = ah.assemble(inst)
        ora = sc.algorithm1(inst)
        g = run_gpu(inst, want_schur=False, refine_max=0, dual_wait=GROWTH_FREE)
        rel = ah.rel_residual_ld(inst, g["x"], inst.b, K)
        rel_g = ah.rel_residual_ld(inst, oracle_in_order(inst, GROWTH_FREE)["x"], inst.b, K)
        assert rel <= max(1e-11, 3.0 * rel_g), (nrhs, rel, rel_g)
        assert g["info"]["refine_iters"] == 0 and g["rc_solve"] == 0
        assert_x_close(g["x"], ora["x"], 1e-10, 1e-7)
        inn = g["inertia"]
        assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == ora["inertia"] and inn["n_perturbed"] == 0


DENSE_BLOCKS = [
    dict(nb=40, nextra=20, ng=6, ns=40, N=26, nrhs=2, seed=15),    # n_g = 1040
    dict(nb=60, nextra=30, ng=6, ns=48, N=32, nrhs=1, seed=16),    # n_g = 1536
    dict(nb=40, nextra=20, ng=5, ns=35, N=60, nrhs=1, seed=17),    # n_g = 2100
]


@pytest.mark.parametrize("case", DENSE_BLOCKS)
def test_parity_dense_solve_blocks(case):
    """refine_max = 0 in the growth-free order at Schur sizes that end
    inside, at half of and past several of the dense factor's inverted
    diagonal blocks: the unrefined solution meets the bars of the small
    cases (1e-11, or 3 x the oracle's unrefined Algorithm 1 in the same
    order: 1.7e-11 at n_g = 1040) and matches the oracle's unrefined
    Algorithm 1 element by element; with refinement, at most one step to
    1e-10."""
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    assert inst.n_g in (1040, 1536, 2100)
    ora = sc.algorithm1(inst)
    K = ah.assemble(inst)
    g = run_gpu(inst, want_schur=False, refine_max=0, dual_wait=GROWTH_FREE)
    rel = ah.rel_residual_ld(inst, g["x"], inst.b, K)
    rel_g = ah.rel_residual_ld(inst, oracle_in_order(inst, GROWTH_FREE)["x"], inst.b, K)
    assert rel <= max(1e-11, 3.0 * rel_g), (rel, rel_g)
    assert_x_close(g["x"], ora["x"], 1e-10, 1e-7)
    inn = g["inertia"]
    assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == ora["inertia"] and inn["n_perturbed"] == 0
    r = run_gpu(inst, want_schur=False)
    assert ah.rel_residual_ld(inst, r["x"], inst.b, K) <= 1e-10
    assert r["info"]["refine_iters"] <= 1 and r["rc_solve"] == 0


def test_parity_ring30():
    """30-bus ring with 11 chords, 8 periods, 2 storage units (n_g = 16)."""
    inst = kktgen.make_workload(1)
    ref, xref, K = reference(inst)
    g = run_gpu(inst)
    rel = ah.rel_residual_ld(inst, g["x"], inst.b, K)
    assert rel <= residual_bar(ref), rel
    assert _rel(g["x"], xref) <= 1e-6
    inn = g["inertia"]
    assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == (8 * 76, 8 * 60 + 16, 0)
    assert np.max(np.abs(np.tril(g["S"]) - np.tril(ref["S"]))) <= 1e-8 * np.max(np.abs(ref["S"]))


def test_parity_ring30_wide_barrier():
    inst = kktgen.make_workload(1, rep=1, barrier=(1e-8, 1e8), nrhs=4)
    ref, xref, K = reference(inst)
    g = run_gpu(inst, want_schur=False)
    rel = ah.rel_residual_ld(inst, g["x"], inst.b, K)
    assert rel <= residual_bar(ref), rel
    assert abs(g["info"]["rel_res"] - rel) <= 1e-2 * rel
    assert ah.backward_error(inst, g["x"], inst.b, K) <= 1e-14
    assert _rel(g["x"], xref) <= 1e-6


def test_deterministic_bitwise():
    inst = kktgen.make_small(nb=70, nextra=40, ng=12, ns=9, N=9, nrhs=3, seed=6)
    a = run_gpu(inst)
    b = run_gpu(inst)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["S"], b["S"])


def test_schur_structure_invariants():
    """Eq. GlobalSchur on the GPU's S: equal sub-diagonal blocks per block column."""
    inst = kktgen.make_small(nb=40, nextra=20, ng=8, ns=3, N=6, seed=9, barrier_range=(1e-2, 1e2))
    g = run_gpu(inst)
    S, ns = g["S"], inst.ns
    blk = lambda m: slice(m * ns, (m + 1) * ns)
    for mp in range(inst.N):
        for m in range(mp + 2, inst.N):
            assert np.array_equal(S[blk(m), blk(mp)], S[blk(mp + 1), blk(mp)])
    assert np.all(np.linalg.eigvalsh(S) < 0)


# ----------------------------------------------------------------------------
# error paths through the C-ABI
# ----------------------------------------------------------------------------

def test_call_order_and_nonfinite():
    torch = _torch()
    import paper_1907_05420_amd as pk
    inst = kktgen.make_small(nb=8, nextra=3, ng=2, ns=2, N=2, seed=0)
    d = pk.device_inputs(inst)
    ctx = pk.kkt_create()
    try:
        with pytest.raises(pk.KKTError) as e:
            pk.kkt_factor(ctx, d["vals"], d["C0"], d["C1"], d["corner"])
        assert e.value.code == pk.KKT_ERR_ORDER
        pk.kkt_analyze(ctx, inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, inst.rowind,
                       inst.C0_rowptr, inst.C0_colind, inst.C1_rowptr, inst.C1_colind)
        x = torch.empty_like(d["b"])
        with pytest.raises(pk.KKTError) as e:
            pk.kkt_solve(ctx, d["b"], x, 1)
        assert e.value.code == pk.KKT_ERR_ORDER
        bad = d["vals"].clone()
        bad[1, 3] = float("nan")
        with pytest.raises(pk.KKTError) as e:
            pk.kkt_factor(ctx, bad, d["C0"], d["C1"], d["corner"])
        assert e.value.code == pk.KKT_ERR_NONFINITE
        # the context is still unfactored: solve keeps refusing
        with pytest.raises(pk.KKTError) as e:
            pk.kkt_solve(ctx, d["b"], x, 1)
        assert e.value.code == pk.KKT_ERR_ORDER
        rc, inn = pk.kkt_factor(ctx, d["vals"], d["C0"], d["C1"], d["corner"])
        assert rc == 0 and inn["inertia_ok"] == 1
        with pytest.raises(pk.KKTError) as e:
            pk.kkt_solve(ctx, d["b"], d["b"], 1)        # b == x
        assert e.value.code == pk.KKT_ERR_ARG
    finally:
        pk.kkt_destroy(ctx)


def test_wrong_sign_barrier_reports_inertia():
    """A negative Hessian diagonal (wrong-sign barrier) leaves a wrong-sign pivot:
    the factor reports the inertia warning instead of hiding it (section 2.3)."""
    inst = kktgen.make_small(nb=8, nextra=3, ng=2, ns=2, N=2, seed=0)
    vals = inst.vals.copy()
    kind = inst.meta["kind"]
    cols = np.repeat(np.arange(inst.n_A), np.diff(inst.colptr))
    k = np.nonzero((kind == 2) & (cols == 2 * inst.nb))[0][0]   # Pg_0 diagonal of period 0
    vals[0, k] = -50.0
    g = run_gpu(inst, want_schur=False, vals=vals)
    import paper_1907_05420_amd as pk
    assert g["rc_factor"] == pk.KKT_WARN_INERTIA
    assert g["inertia"]["inertia_ok"] == 0
    K = ah.assemble(inst)
    from oracle.ldlt import inertia_eig
    import copy
    i2 = copy.copy(inst)
    i2.vals = vals
    w = inertia_eig(ah.assemble(i2).toarray())
    assert (g["inertia"]["n_pos"], g["inertia"]["n_neg"], g["inertia"]["n_zero"]) == w


def test_inertia_correction_shifts():
    """delta_w / delta_c (section 2.3) match the oracle on the shifted matrix."""
    inst = kktgen.make_small(nb=12, nextra=6, ng=3, ns=3, N=4, nrhs=1, seed=1, barrier_range=(1e-2, 1e2))
    dw, dc = 0.25, 1e-4
    g = run_gpu(inst, delta_w=dw, delta_c=dc)
    import copy
    i2 = copy.copy(inst)
    v = inst.vals.copy()
    kind = inst.meta["kind"]
    cols = np.repeat(np.arange(inst.n_A), np.diff(inst.colptr))
    diag = inst.rowind == cols
    v[:, diag & (cols < inst.n_primal)] += dw
    v[:, diag & (cols >= inst.n_primal)] -= dc
    i2.vals = v
    x, K = sc.solve_mono(i2)
    assert _rel(g["x"], x) <= 1e-9


@pytest.mark.parametrize("case", [SMALL[1], SMALL[3], SMALL[5], SMALL[8]])
@pytest.mark.parametrize("precision,schur_mode", [(0, 0), (1, 0), (0, 1)])
def test_plan_equals_footprint(case, precision, schur_mode):
    """The host-only planning query (used for admission) names exactly the
    device bytes the context holds after analysis and a solve."""
    import paper_1907_05420_amd as pk
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    nrhs = inst.b.shape[0]
    st, _ = pk.kkt_plan(inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, inst.rowind, inst.C0_rowptr,
                        inst.C0_colind, inst.C1_rowptr, inst.C1_colind, precision=precision, nrhs_max=nrhs,
                        schur_mode=schur_mode)
    s = pk.Solver(inst, precision=precision, schur_mode=schur_mode)
    d = pk.device_inputs(inst)
    s.factor(d["vals"], d["C0"], d["C1"], d["corner"])
    s.solve(d["b"])
    assert s.footprint() == st["device_bytes"]
    s.close()


@pytest.mark.parametrize("case", SMALL)
def test_parity_structured_schur(case):
    """The structured Schur elimination (section 4.3) gives the oracle's
    solution and inertia, like the dense path."""
    import paper_1907_05420_amd as pk
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    ref, xref, K = reference(inst)
    d = pk.device_inputs(inst)
    s = pk.Solver(inst, schur_mode=pk.KKT_SCHUR_STRUCTURED)
    rc_f, inn = s.factor(d["vals"], d["C0"], d["C1"], d["corner"])
    x, rc_s, info = s.solve(d["b"])
    x = x.cpu().numpy()
    s.close()
    rel = ah.rel_residual_ld(inst, x, inst.b, K)
    assert rel <= 1e-10, rel
    assert _rel(x, xref) <= 1e-9, _rel(x, xref)
    assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == ref["inertia"]
    assert inn["inertia_ok"] == 1 and inn["n_perturbed"] == 0


def test_parity_structured_ring30_wide_barrier():
    import paper_1907_05420_amd as pk
    inst = kktgen.make_workload(1, rep=1, barrier=(1e-8, 1e8), nrhs=4)
    ref, xref, K = reference(inst)
    d = pk.device_inputs(inst)
    out = {}
    for mode in (pk.KKT_SCHUR_DENSE, pk.KKT_SCHUR_STRUCTURED):
        s = pk.Solver(inst, schur_mode=mode)
        _, inn = s.factor(d["vals"], d["C0"], d["C1"], d["corner"])
        x, _, info = s.solve(d["b"])
        out[mode] = (x.cpu().numpy(), inn, info)
        s.close()
    xs, inn, info = out[pk.KKT_SCHUR_STRUCTURED]
    rel = ah.rel_residual_ld(inst, xs, inst.b, K)
    assert rel <= residual_bar(ref), rel
    assert inn["inertia_ok"] == 1
    assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == \
        (out[pk.KKT_SCHUR_DENSE][1]["n_pos"], out[pk.KKT_SCHUR_DENSE][1]["n_neg"], 0)
    assert _rel(xs, out[pk.KKT_SCHUR_DENSE][0]) <= 1e-6


def test_residual_floor_reported():
    """rel_floor = eps || |K||x| + |b| ||_2 / ||b||_2 of the returned x. The
    library evaluates the border coupling of the period rows through the
    suffix sums of Eq. B12N, so its scale holds |C_0^T| |sum_{m>n} x_g[m]|
    where the assembled K has sum_{m>n} |C_0^T x_g[m]|: by the triangle
    inequality it is at most the oracle's value, and close to it."""
    import paper_1907_05420_amd as pk
    inst = kktgen.make_workload(1, rep=1, barrier=(1e-8, 1e8), nrhs=4)
    K = ah.assemble(inst)
    d = pk.device_inputs(inst)
    s = pk.Solver(inst)
    s.factor(d["vals"], d["C0"], d["C1"], d["corner"])
    x, _, info = s.solve(d["b"])
    x = x.cpu().numpy()
    s.close()
    scale = np.abs(K) @ np.abs(x).T + np.abs(inst.b).T
    ref = max(2.220446049250313e-16 * np.linalg.norm(scale[:, k]) / np.linalg.norm(inst.b[k])
              for k in range(inst.b.shape[0]))
    assert 0.9 * ref <= info["rel_floor"] <= ref * (1 + 1e-9), (info["rel_floor"], ref)


def test_parity_structured_wide_border():
    """N_s = 260 > 256: the structured elimination inverts each pivot block
    in two 256-wide halves and combines them, and the solve chains take
    their products in several load batches. Checked by properties that hold
    at any size (the full oracle solve takes half a minute here): residual
    from the oracle's assembled K, exact inertia, and the dense path's
    solution (which the small cases pin to the oracle)."""
    import paper_1907_05420_amd as pk
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), nb=300, nextra=150, ng=10, ns=260, N=3, nrhs=2, seed=15)
    K = ah.assemble(inst)
    d = pk.device_inputs(inst)
    expect = (inst.N * inst.n_primal, inst.N * (inst.n_A - inst.n_primal) + inst.n_g, 0)
    xs = {}
    for mode in (pk.KKT_SCHUR_DENSE, pk.KKT_SCHUR_STRUCTURED):
        s = pk.Solver(inst, schur_mode=mode)
        _, inn = s.factor(d["vals"], d["C0"], d["C1"], d["corner"])
        x, _, info = s.solve(d["b"])
        xs[mode] = x.cpu().numpy()
        s.close()
        rel = ah.rel_residual_ld(inst, xs[mode], inst.b, K)
        assert rel <= 1e-10, (mode, rel)
        assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == expect, (mode, inn)
        assert inn["n_perturbed"] == 0
    assert _rel(xs[pk.KKT_SCHUR_STRUCTURED], xs[pk.KKT_SCHUR_DENSE]) <= 1e-9


@pytest.mark.parametrize("case", [SMALL[1], SMALL[5], SMALL[6], SMALL[11]])
@pytest.mark.parametrize("schur_mode", [0, 1])
def test_recompute_periods_equals_stored(case, schur_mode):
    """The memory-saving variant (section 4.3): with the factors of only P
    periods held and recomputed in every solve pass, the solution, the
    inertia, S and the local Schur blocks equal those of the stored-factor
    path bit for bit (each period's arithmetic is the same), and the
    context holds less device memory; the planning query agrees."""
    import paper_1907_05420_amd as pk
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    d = pk.device_inputs(inst)
    out = {}
    for P in (0, 1, 2):
        s = pk.Solver(inst, schur_mode=schur_mode, recompute_periods=P)
        _, inn = s.factor(d["vals"], d["C0"], d["C1"], d["corner"])
        x, rc, info = s.solve(d["b"])
        sb = s.schur_blocks().cpu().numpy() if inst.n_g else None
        st, _ = pk.kkt_plan(inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, inst.rowind, inst.C0_rowptr,
                            inst.C0_colind, inst.C1_rowptr, inst.C1_colind, nrhs_max=inst.b.shape[0],
                            schur_mode=schur_mode, recompute_periods=P)
        out[P] = (x.cpu().numpy(), inn, info, sb, s.footprint(), st["device_bytes"])
        s.close()
    x0, inn0, info0, sb0, f0, _ = out[0]
    for P in (1, 2):
        x, inn, info, sb, f, fplan = out[P]
        assert np.array_equal(x, x0), P
        assert inn == inn0 and info["refine_iters"] == info0["refine_iters"]
        if sb0 is not None:
            assert np.array_equal(sb, sb0)
        assert f == fplan and f < f0, (P, f, f0)
    K = ah.assemble(inst)
    assert ah.rel_residual_ld(inst, out[1][0], inst.b, K) <= 1e-10
