"""Pins of the FP64 oracle against what the paper and the mathematics fix:
brute-force dense solves (LAPACK), eigenvalue inertia, the exact identity
decomposed == monolithic (Eqs. SCform, SCsolve, SCsolve1), Haynsworth inertia
additivity, the MPOPF Schur structure (Eqs. LocalSchurBs, GlobalSchur) and the
special cases Ns = 0 and N = 1. The mutant tests plant plausible mistakes in
the oracle and check that a pin catches each one."""
import numpy as np
import pytest

import kktgen
from oracle import arrowhead as ah
from oracle import schur as sc
from oracle.ldlt import ldlt, ldlt_solve, inertia_from_d, inertia_eig


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# --------------------------------------------------------------------------
# dense LDL^T
# --------------------------------------------------------------------------

def _quasi_definite(n1, n2, seed):
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((n1, n1))
    H = H @ H.T + n1 * np.eye(n1)
    J = rng.standard_normal((n2, n1))
    D = np.diag(rng.uniform(0.1, 1.0, n2))
    return np.block([[H, J.T], [J, -D]])


@pytest.mark.parametrize("n1,n2,seed", [(5, 3, 0), (20, 12, 1), (60, 40, 2)])
def test_ldlt_reconstructs_and_solves(n1, n2, seed):
    A = _quasi_definite(n1, n2, seed)
    signs = np.r_[np.ones(n1), -np.ones(n2)]
    L, d, npert = ldlt(A, signs=signs)
    assert npert == 0
    assert np.allclose(np.tril(L), L) and np.allclose(np.diag(L), 1.0)
    assert _rel(L @ np.diag(d) @ L.T, A) < 1e-13
    b = np.random.default_rng(seed).standard_normal((n1 + n2, 3))
    assert _rel(ldlt_solve(L, d, b), np.linalg.solve(A, b)) < 1e-11
    assert inertia_from_d(d) == inertia_eig(A) == (n1, n2, 0)


def test_ldlt_perturbs_vanishing_pivot_and_reports_wrong_sign():
    A = _quasi_definite(6, 4, 3)
    # column 2 made a copy of column 1 (and row likewise): pivot 2 vanishes
    # after pivot 1 is eliminated, up to rounding
    A[:, 2] = A[:, 1]
    A[2, :] = A[1, :]
    L, d, npert, raw = ldlt(A, signs=np.r_[np.ones(6), -np.ones(4)], eps=1e-14, return_raw=True)
    assert npert == 1 and abs(raw[2]) <= 1e-14 * abs(A[2, 2])
    assert np.isfinite(L).all()
    # a wrong-sign (not vanishing) pivot is kept and shows in the inertia
    B = _quasi_definite(6, 4, 4)
    B[3, 3] = -1e3
    L, d, npert, raw = ldlt(B, signs=np.r_[np.ones(6), -np.ones(4)], return_raw=True)
    assert npert == 0 and inertia_from_d(raw) == inertia_eig(B) != (6, 4, 0)


# --------------------------------------------------------------------------
# Algorithm 1 vs the monolithic solve
# --------------------------------------------------------------------------

CASES = [
    dict(nb=8, nextra=3, ng=2, ns=2, N=3, nrhs=1, seed=0),
    dict(nb=12, nextra=6, ng=3, ns=3, N=4, nrhs=4, seed=1),
    dict(nb=10, nextra=4, ng=2, ns=1, N=1, nrhs=2, seed=2),       # N = 1
    dict(nb=9, nextra=5, ng=3, ns=0, N=3, nrhs=1, seed=3),        # Ns = 0
    dict(nb=15, nextra=8, ng=4, ns=2, N=5, nrhs=1, seed=4, corner="zero"),
]


def pin_decomposed_equals_monolithic(inst, tol=1e-8, tol_unrefined=1e-11):
    """Algorithm 1 (refined in FP64 with its own factors, section 2.1) and the
    LAPACK solve of the assembled K agree; the unrefined Algorithm 1 residual
    is already small (refinement cannot hide a wrong step)."""
    out = sc.algorithm1(inst)
    x_mono, K = sc.solve_mono(inst)
    rel0, _ = ah.rel_residual(inst, out["x"], inst.b, K)
    assert rel0 < tol_unrefined, rel0
    solve = lambda r: sc.algorithm1(inst, b=r, factors=out["factors"])["x"]
    x_dec, hist = sc.refine(inst, out["x"], inst.b, solve, tol=1e-13, K=K)
    rel_mono, _ = ah.rel_residual(inst, x_mono, inst.b, K)
    assert hist[-1] < 1e-10 and rel_mono < 1e-10, (hist, rel_mono)
    assert _rel(x_dec, x_mono) < tol, _rel(x_dec, x_mono)
    return out, x_mono, K


@pytest.mark.parametrize("case", CASES)
def test_decomposed_equals_monolithic(case):
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    pin_decomposed_equals_monolithic(inst)


def test_decomposed_equals_monolithic_ring30():
    inst = kktgen.make_workload(1)
    out, x_mono, K = pin_decomposed_equals_monolithic(inst, tol=1e-6, tol_unrefined=1e-6)


def pin_plain_equals_structured(inst):
    a = sc.algorithm1(inst, structured=True)
    b = sc.algorithm1(inst, structured=False)
    assert _rel(a["S"], b["S"]) < 1e-11, _rel(a["S"], b["S"])


@pytest.mark.parametrize("case", CASES[:3])
def test_structured_schur_equals_plain(case):
    """Eq. LocalSchurBs placement of S_bar_n == C - sum_n B_n A_n^-1 B_n^T."""
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    pin_plain_equals_structured(inst)


@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[4]])
def test_prefix_assembly_and_cholesky_path(case):
    """The large-size route of the oracle: S summed per block position
    (Eq. LocalSchurBs, prefix sums of the S_00 blocks) equals the sum of the
    placed S_n; LAPACK's Cholesky of -S gives Algorithm 1 the same solution
    as the oracle's own LDL^T of S; and the refinement with extended-precision
    residuals reaches below 1e-14 like the FP64 one."""
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    a = sc.algorithm1(inst)
    b = sc.algorithm1(inst, assembly="prefix", schur_factor="cholesky")
    c = sc.algorithm1(inst, assembly="prefix")
    assert np.max(np.abs(c["S"] - a["S"])) <= 1e-13 * np.max(np.abs(a["S"]))
    assert _rel(b["x"], a["x"]) < 1e-11
    K = ah.assemble(inst)
    solve = lambda r: sc.algorithm1(inst, b=r, factors=b["factors"], schur=b["schur_fac"])["x"]
    x, hist = sc.refine(inst, b["x"], inst.b, solve, tol=1e-15, K=K, extended=True)
    assert hist[-1] < 1e-14 and _rel(x, sc.solve_mono(inst)[0]) < 1e-10


def pin_structured_elimination(inst):
    """Section 4.3's block elimination of S (reading R21) solves S x = r like
    LAPACK on the assembled S, finds its inertia (all negative: S is negative
    definite here), and carries U_j = sum of the eliminated B A^-1 B^T: U_1
    is B_0 A_0^-1 B_0^T computed directly."""
    out = sc.algorithm1(inst)
    S, N, ns = out["S"], inst.N, inst.ns
    rhs = np.random.default_rng(7).standard_normal((3, inst.n_g))
    x, inertia, Us = sc.structured_schur_solve(S, N, ns, rhs)
    xref = np.linalg.solve(S, rhs.T).T
    # two backward-stable solves differ by at most ~ eps cond(S) each
    tol = 100 * np.finfo(float).eps * np.linalg.cond(S)
    assert _rel(x, xref) < tol, (_rel(x, xref), tol)
    assert inertia == (0, inst.n_g, 0) == inertia_eig(S)
    if N > 1:
        A0, B0 = S[:ns, :ns], S[ns:2 * ns, :ns]
        U1 = B0 @ np.linalg.solve(A0, B0.T)
        assert np.max(np.abs(Us[1] - U1)) <= 1e-10 * np.max(np.abs(U1))


@pytest.mark.parametrize("case", [c for c in CASES if c["ns"] > 0])
def test_structured_elimination_of_schur(case):
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    pin_structured_elimination(inst)


def test_structured_elimination_of_schur_ring30():
    pin_structured_elimination(kktgen.make_workload(1))


def test_structured_elimination_needs_the_common_update():
    """Dropping U_j (eliminating each diagonal block alone) is a plausible
    mistake; it gives another solution."""
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **CASES[1])
    S = sc.algorithm1(inst)["S"]
    rhs = np.ones((1, inst.n_g))
    ns = inst.ns
    Sdrop = S.copy()
    for j in range(inst.N):
        for i in range(j + 2, inst.N):
            # a matrix without the repeated blocks below the first sub-diagonal
            Sdrop[i * ns:(i + 1) * ns, j * ns:(j + 1) * ns] = 0.0
            Sdrop[j * ns:(j + 1) * ns, i * ns:(i + 1) * ns] = 0.0
    x, _, _ = sc.structured_schur_solve(S, inst.N, ns, rhs)
    assert _rel(x, np.linalg.solve(Sdrop, rhs.T).T) > 1e-6


def pin_inertia_additivity(inst):
    out = sc.algorithm1(inst)
    K = ah.assemble(inst).toarray()
    expect = (inst.N * inst.n_primal, inst.N * (inst.n_A - inst.n_primal) + inst.n_g, 0)
    assert inertia_eig(K) == expect
    assert out["inertia"] == expect
    # S is negative definite when every A_n and K have the correct inertia
    if inst.n_g:
        np.linalg.cholesky(-out["S"])


@pytest.mark.parametrize("case", CASES)
def test_haynsworth_inertia(case):
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    pin_inertia_additivity(inst)


def test_haynsworth_inertia_ring30():
    pin_inertia_additivity(kktgen.make_workload(1))


def pin_local_schur_blocks(inst):
    """S_ij,n = -C_i A_n^-1 C_j^T (Eq. LocalSchurBs) with a LAPACK solve, and
    the placement of Eq. LocalSchurBs: S_11 at the diagonal block (n, n), S_10
    below it, S_00 further down and right, zero before period n."""
    out = sc.algorithm1(inst, structured=False)    # S from the full B_n of Eq. B12N
    # C_0, C_1 straight from the instance's CSR arrays, not via the oracle
    C0 = np.zeros((inst.ns, inst.n_A))
    C1 = np.zeros((inst.ns, inst.n_A))
    for s_ in range(inst.ns):
        for k in range(inst.C0_rowptr[s_], inst.C0_rowptr[s_ + 1]):
            C0[s_, inst.C0_colind[k]] += inst.C0_vals[k]
        for k in range(inst.C1_rowptr[s_], inst.C1_rowptr[s_ + 1]):
            C1[s_, inst.C1_colind[k]] += inst.C1_vals[k]
    ns, N = inst.ns, inst.N
    blk = lambda m: slice(m * ns, (m + 1) * ns)
    P = np.zeros((ns, ns))            # running sum of S_00,n, n < m'
    S = out["S"]
    Cc = np.diag(inst.corner_diag)
    for mp in range(N):
        A = ah.block(inst, mp).toarray()
        S11 = -C1 @ np.linalg.solve(A, C1.T)
        S10 = -C0 @ np.linalg.solve(A, C1.T)
        S00 = -C0 @ np.linalg.solve(A, C0.T)
        assert _rel(S[blk(mp), blk(mp)], Cc[blk(mp), blk(mp)] + P + S11) < 1e-9
        for m in range(mp + 1, N):
            assert _rel(S[blk(m), blk(mp)], P + S10) < 1e-9
        P = P + S00


@pytest.mark.parametrize("case", CASES[:2] + CASES[4:])
def test_local_schur_blocks(case):
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    pin_local_schur_blocks(inst)


def test_schur_subdiagonal_blocks_equal_and_independent_of_horizon():
    """Eq. GlobalSchur: below the diagonal every block of a block column is the
    same matrix; S_bar_n does not depend on N (section 4.3)."""
    inst = kktgen.make_small(nb=10, nextra=4, ng=2, ns=2, N=5, seed=7, barrier_range=(1e-2, 1e2))
    out = sc.algorithm1(inst)
    ns, S = inst.ns, out["S"]
    blk = lambda m: slice(m * ns, (m + 1) * ns)
    for mp in range(inst.N):
        for m in range(mp + 2, inst.N):
            assert np.array_equal(S[blk(m), blk(mp)], S[blk(mp + 1), blk(mp)])
    # truncate the horizon to the first 3 periods
    import copy
    short = copy.copy(inst)
    short.N = 3
    short.vals = inst.vals[:3]
    short.corner_diag = inst.corner_diag[: 3 * ns]
    short.b = np.concatenate([inst.b[:, : 3 * inst.n_A], inst.b[:, inst.N * inst.n_A: inst.N * inst.n_A + 3 * ns]], 1)
    out2 = sc.algorithm1(short)
    assert np.allclose(out2["Sbar"], out["Sbar"][:3], rtol=1e-13, atol=0)


def test_ns0_is_independent_block_solves():
    inst = kktgen.make_small(nb=9, nextra=5, ng=3, ns=0, N=3, seed=3, barrier_range=(1e-2, 1e2))
    out = sc.algorithm1(inst)
    for n in range(inst.N):
        A = ah.block(inst, n).toarray()
        xn = np.linalg.solve(A, inst.b[0, n * inst.n_A:(n + 1) * inst.n_A])
        assert _rel(out["x"][0, n * inst.n_A:(n + 1) * inst.n_A], xn) < 1e-10


def test_refinement_reaches_tolerance_wide_barrier():
    """[1e-8, 1e8] barrier range: FP64 Algorithm 1 + refinement reaches the
    1e-10 relative residual on the 30-bus grid."""
    inst = kktgen.make_workload(1, barrier=(1e-8, 1e8))
    out = sc.algorithm1(inst)
    K = ah.assemble(inst)
    solve = lambda r: sc.algorithm1(inst, b=r, factors=out["factors"])["x"]
    x, hist = sc.refine(inst, out["x"], inst.b, solve, tol=1e-12, K=K)
    assert hist[-1] < 1e-10, hist


# --------------------------------------------------------------------------
# assembly, residuals and backward error
# --------------------------------------------------------------------------

def _dense_from_raw(inst):
    """K built entry by entry from the instance's raw arrays, with none of the
    oracle's code: every stored lower entry of A_n at (i, j) and (j, i), the
    rows of C_1 in block row m = n of B_n and those of C_0 in every block row
    m > n (Eq. B12N), the corner diagonal."""
    nA, N, ns = inst.n_A, inst.N, inst.ns
    K = np.zeros((inst.n_total, inst.n_total))
    for p in range(N):
        o = p * nA
        for j in range(nA):
            for q in range(inst.colptr[j], inst.colptr[j + 1]):
                i = int(inst.rowind[q])
                K[o + i, o + j] = inst.vals[p, q]
                K[o + j, o + i] = inst.vals[p, q]
    g0 = N * nA
    for p in range(N):
        for m in range(p, N):
            rp, ci, cv = ((inst.C1_rowptr, inst.C1_colind, inst.C1_vals) if m == p
                          else (inst.C0_rowptr, inst.C0_colind, inst.C0_vals))
            for s_ in range(ns):
                for q in range(rp[s_], rp[s_ + 1]):
                    r_, c_ = g0 + m * ns + s_, p * nA + int(ci[q])
                    K[r_, c_] += cv[q]
                    K[c_, r_] += cv[q]
    for g in range(inst.n_g):
        K[g0 + g, g0 + g] = inst.corner_diag[g]
    return K


def pin_assembly_raw(inst):
    """arrowhead.block / border / corner / assemble equal, bit for bit, the
    matrix written out entry by entry from the raw CSC/CSR arrays (a doubled
    or dropped diagonal, a transposed or misplaced C block, a wrong corner
    all change an entry)."""
    Kraw = _dense_from_raw(inst)
    assert np.array_equal(ah.assemble(inst).toarray(), Kraw)
    nA = inst.n_A
    for n in range(inst.N):
        assert np.array_equal(ah.block(inst, n).toarray(), Kraw[n * nA:(n + 1) * nA, n * nA:(n + 1) * nA])


@pytest.mark.parametrize("case", [CASES[0], CASES[3], CASES[4]])
def test_assembly_matches_raw_arrays(case):
    pin_assembly_raw(kktgen.make_small(barrier_range=(1e-2, 1e2), **case))


def pin_backward_error_hand(inst=None):
    """omega = max_i |r_i| / (|K||x| + |b|)_i on a 2x2 system worked by hand:
    K = [[4, -1], [-1, -2]], x = (1, 2), b = (3, -6): K x = (2, -5),
    r = (1, -1), |K||x| + |b| = (6 + 3, 5 + 6) = (9, 11), omega = 1/9. With
    b = K x it is 0; a zero row (x = 0, b = 0) counts as 0; several
    right-hand sides take the largest."""
    import scipy.sparse as sp_
    K = sp_.csr_matrix(np.array([[4.0, -1.0], [-1.0, -2.0]]))
    assert ah.backward_error(None, np.array([[1.0, 2.0]]), np.array([[3.0, -6.0]]), K) == pytest.approx(1 / 9, rel=1e-15)
    assert ah.backward_error(None, np.array([[1.0, 2.0]]), np.array([[2.0, -5.0]]), K) == 0.0
    assert ah.backward_error(None, np.zeros((1, 2)), np.zeros((1, 2)), K) == 0.0
    # x = (1, 0), b = (4, 0): K x = (4, -1), r = (0, 1), rows (4 + 4, 1 + 0): omega = 1
    two = ah.backward_error(None, np.array([[1.0, 2.0], [1.0, 0.0]]), np.array([[3.0, -6.0], [4.0, 0.0]]), K)
    assert two == 1.0


def test_backward_error_hand_computed():
    pin_backward_error_hand()


def pin_residual_ld_exact(inst=None):
    """rel_residual_ld against the exact residual in rational arithmetic
    (fractions.Fraction, row by row) of an FP64 x near the solution of a
    wide-barrier system, where a plain FP64 evaluation is off by a large
    fraction of the residual itself."""
    from fractions import Fraction
    import math
    w = kktgen.make_workload(1, rep=1, barrier=(1e-8, 1e8), nrhs=1)
    out = sc.algorithm1(w)
    K = ah.assemble(w).tocsr()

    def exact_residual(x):
        r = []
        for i in range(K.shape[0]):
            acc = Fraction(float(w.b[0, i]))
            for q in range(K.indptr[i], K.indptr[i + 1]):
                acc -= Fraction(float(K.data[q])) * Fraction(float(x[0, K.indices[q]]))
            r.append(acc)
        return r

    # refine with exact residuals down to the rounding of x itself
    x = out["x"]
    for _ in range(3):
        r = np.array([[float(v) for v in exact_residual(x)]])
        x = x + sc.algorithm1(w, b=r, factors=out["factors"])["x"]
    r = exact_residual(x)
    exact = math.sqrt(sum(v * v for v in r) / sum(Fraction(float(v)) ** 2 for v in w.b[0]))
    got = ah.rel_residual_ld(w, x, w.b, K)
    # extended precision leaves ~ 1e-19 || |K||x| || / ||b|| (~ 1e-13 here):
    # resolved 1000 times below the 1e-10 target
    assert abs(got - exact) <= 2e-13, (got, exact)
    # a plain FP64 evaluation misses it by far more at this level
    fp64, _ = ah.rel_residual(w, x, w.b, K)
    assert abs(fp64 - exact) > 0.05 * exact, (fp64, exact)


def test_residual_ld_matches_exact_rational():
    pin_residual_ld_exact()


# --------------------------------------------------------------------------
# line-flow slacks: reduction and recovery (Eqs. SCOPFhessianReduced,
# SCOPFslackReduction) against the unreduced system (Eq. SCOPFslackAtEnd)
# --------------------------------------------------------------------------

SLACK_CASES = [dict(nb=8, nextra=3, ng=2, ns=2, N=3, nrhs=2, seed=31),
               dict(nb=12, nextra=6, ng=3, ns=0, N=2, nrhs=1, seed=32),
               dict(nb=10, nextra=5, ng=2, ns=1, N=4, nrhs=1, seed=33)]


def _slack_inst(case):
    return kktgen.make_small(barrier_range=(1e-2, 1e2), line_flow=True, ls_range=(1e-4, 1e2), keep_below=1e-3,
                             **case)


def pin_slack_reduction(inst):
    """Reduce (Eq. SCOPFhessianReduced), solve the reduced system by Algorithm
    1, recover the slacks (Eq. SCOPFslackReduction): the result is the LAPACK
    solution of the unreduced system (slacks last), entry for entry; the
    unreduced K has the inertia the IPM expects with the eliminated slacks
    counted as primal, i.e. the reduced inertia plus N n_elim positive."""
    red = ah.reduce_slacks(inst)
    out = sc.algorithm1(red)
    s_rec = ah.recover_slacks(red, out["x"])
    Kf = ah.assemble_unreduced(inst).toarray()
    full = np.linalg.solve(Kf, ah.rhs_unreduced(inst).T).T
    got = np.concatenate([out["x"], s_rec], axis=1)
    assert _rel(got, full) < 1e-10, _rel(got, full)
    ne = len(inst.meta["slack"]["lam_row"])
    expect_red = (inst.N * inst.n_primal, inst.N * (inst.n_A - inst.n_primal) + inst.n_g, 0)
    assert out["inertia"] == expect_red
    assert inertia_eig(Kf) == (expect_red[0] + inst.N * ne, expect_red[1], 0)


@pytest.mark.parametrize("case", SLACK_CASES)
def test_slack_reduction_equals_unreduced_solve(case):
    inst = _slack_inst(case)
    sl = inst.meta["slack"]
    assert sl["keep"].any() and (~sl["keep"]).any()      # both kinds of slack present
    pin_slack_reduction(inst)


# --------------------------------------------------------------------------
# planted mistakes: each must be caught by at least one pin
# --------------------------------------------------------------------------

def _mut_swap_c0_c1(monkeypatch):
    orig = ah.coupling
    monkeypatch.setattr(ah, "coupling", lambda inst: tuple(reversed(orig(inst))))


def _mut_border_transposed_periods(monkeypatch):
    orig = ah.border

    def wrong(inst, n):          # cumulative coupling on the wrong side
        return orig(inst, inst.N - 1 - n)
    monkeypatch.setattr(ah, "border", wrong)


def _mut_schur_sign(monkeypatch):
    orig = sc.place_local_schur
    monkeypatch.setattr(sc, "place_local_schur", lambda inst, n, Sb: -orig(inst, n, Sb))


def _mut_drop_s00(monkeypatch):
    orig = sc.place_local_schur

    def wrong(inst, n, Sbar):
        Sb = Sbar.copy()
        Sb[inst.ns:, inst.ns:] = 0.0
        return orig(inst, n, Sb)
    monkeypatch.setattr(sc, "place_local_schur", wrong)


def _mut_local_solve_sign(monkeypatch):
    orig = sc.algorithm1

    def wrong(inst, b=None, **kw):
        out = orig(inst, b=b, **kw)
        ug = out["ug"]
        b_ = inst.b if b is None else np.atleast_2d(b)
        for n in range(inst.N):        # A_n du_n = b_n + B_n^T du_g (wrong sign)
            rhs = b_[:, n * inst.n_A:(n + 1) * inst.n_A] + (ah.border(inst, n).T @ ug.T).T
            out["x"][:, n * inst.n_A:(n + 1) * inst.n_A] = out["factors"][n].solve(rhs.T).T
        return out
    monkeypatch.setattr(sc, "algorithm1", wrong)


def _mut_ldlt_update(monkeypatch):
    import oracle.ldlt as lm
    orig = lm.ldlt

    def wrong(A, signs=None, eps=1e-20, return_raw=False):
        A = np.array(A, dtype=float)
        if A.shape[0] > 3:
            A[3, 1] *= 1.0000001      # a dropped/garbled term
            A[1, 3] = A[3, 1]
        return orig(A, signs=signs, eps=eps, return_raw=return_raw)
    monkeypatch.setattr(sc, "ldlt", wrong)


def _mut_block_doubled_diagonal(monkeypatch):
    orig = ah.block_lower

    def wrong(inst, n):            # A_n = L + L^T without removing the diagonal once
        import scipy.sparse as sp_
        L = orig(inst, n)
        return (L + L.T).tocsr()
    monkeypatch.setattr(ah, "block", wrong)


def _mut_corner_sign(monkeypatch):
    import scipy.sparse as sp_
    monkeypatch.setattr(ah, "corner", lambda inst: sp_.diags(-inst.corner_diag).tocsr())


def _mut_inertia_sign(monkeypatch):
    monkeypatch.setattr(sc, "inertia_from_d", lambda d: (int(np.sum(np.asarray(d) < 0)),
                                                         int(np.sum(np.asarray(d) > 0)),
                                                         int(np.sum(np.asarray(d) == 0))))


def _mut_backward_error_no_b(monkeypatch):
    def wrong(inst, x, b, K=None):   # |b| left out of the denominator
        r = b - (K @ x.T).T
        den = (abs(K) @ np.abs(x).T).T
        with np.errstate(divide="ignore", invalid="ignore"):
            return float(np.max(np.where(den > 0, np.abs(r) / den, 0.0)))
    monkeypatch.setattr(ah, "backward_error", wrong)


def _mut_residual_ld_fp64(monkeypatch):
    def wrong(inst, x, b, K=None):   # summed in FP64 after all
        r = np.atleast_2d(b) - (K @ np.atleast_2d(x).T).T
        return float(np.max(np.linalg.norm(r, axis=-1) / np.linalg.norm(np.atleast_2d(b), axis=-1)))
    monkeypatch.setattr(ah, "rel_residual_ld", wrong)


def _mut_slack_recovery_sign(monkeypatch):
    orig = ah.recover_slacks

    def wrong(inst, x):               # L_s s = r - lambda_I (sign of the multiplier flipped)
        sl = inst.meta["slack"]
        N, nA, ne = inst.N, inst.n_A, len(sl["lam_row"])
        lam = np.stack([np.atleast_2d(x)[:, n * nA + sl["lam_row"]] for n in range(N)], axis=1)
        return ((sl["rs"].reshape(-1, N, ne) - lam) / sl["Ls"][None]).reshape(-1, N * ne)
    monkeypatch.setattr(ah, "recover_slacks", wrong)


def _mut_slack_reduce_rhs(monkeypatch):
    orig = ah.reduce_slacks

    def wrong(inst):                  # right-hand side not reduced
        out = orig(inst)
        out.b = inst.b.copy()
        return out
    monkeypatch.setattr(ah, "reduce_slacks", wrong)


def _pin_slack_first_case(inst=None):
    pin_slack_reduction(_slack_inst(SLACK_CASES[0]))


MUTANTS = [_mut_slack_recovery_sign, _mut_slack_reduce_rhs, _mut_swap_c0_c1, _mut_border_transposed_periods, _mut_schur_sign, _mut_drop_s00,
           _mut_local_solve_sign, _mut_ldlt_update, _mut_block_doubled_diagonal, _mut_corner_sign,
           _mut_inertia_sign, _mut_backward_error_no_b, _mut_residual_ld_fp64]


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda f: f.__name__)
def test_pins_catch_planted_mistakes(mutant, monkeypatch):
    inst = kktgen.make_small(nb=12, nextra=6, ng=3, ns=2, N=4, nrhs=1, seed=11, barrier_range=(1e-2, 1e2))
    mutant(monkeypatch)
    caught = 0
    for pin in (pin_decomposed_equals_monolithic, pin_plain_equals_structured, pin_local_schur_blocks,
                pin_inertia_additivity, pin_assembly_raw, pin_backward_error_hand, pin_residual_ld_exact,
                _pin_slack_first_case):
        try:
            pin(inst)
        except (AssertionError, np.linalg.LinAlgError):
            caught += 1
    assert caught >= 1
