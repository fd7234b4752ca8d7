"""Generator checks: pattern rules against the printed 9-bus KKT pattern
(Fig. KKTsystemOPF, first panel) and sizes against the workload definitions."""
import os

import numpy as np
import pytest

import kktgen

GOLD = os.path.join(os.path.dirname(__file__), "golden", "e1_case9_kkt_pattern.txt")


def _paper_pattern():
    pairs = np.loadtxt(GOLD, dtype=np.int64, comments="#")
    return set(map(tuple, pairs.tolist()))


def test_fixture_matches_printed_nz():
    s = _paper_pattern()
    assert len(s) == 576                      # "nz = 576"
    assert all((b, a) in s for a, b in s)     # symmetric


def _paper_to_ours(p):
    # x = rows 1..24 -> 0..23; lambda_E = rows 43..60 -> 24..41
    if 1 <= p <= 24:
        return p - 1
    if 43 <= p <= 60:
        return p - 43 + 24
    return None


def test_block_pattern_reproduces_printed_opf_kkt():
    """Recover the 9-bus topology and generator buses from the printed pattern,
    regenerate the x + lambda_E block with the generator's rules, compare
    entry by entry (360 entries: H 114, J_E and J_E^T 2 x 114, dual diag 18)."""
    s = _paper_pattern()
    sub = {(_paper_to_ours(a), _paper_to_ours(b)) for a, b in s}
    sub = {(a, b) for a, b in sub if a is not None and b is not None}
    assert len(sub) == 360
    lines = sorted({(a - 1, b - 1) for a, b in s if a < b <= 9})
    assert len(lines) == 9
    # generator k's P column is 19..21; P-balance row of bus j is 42 + j
    gen_bus = []
    for g in range(3):
        rows = [a for a, b in s if b == 19 + g and 43 <= a <= 51]
        assert len(rows) == 1
        gen_bus.append(rows[0] - 43)
    n_A, n_primal, colptr, rowind, kind = kktgen.block_pattern(9, np.array(lines), np.array(gen_bus),
                                                                np.array([], dtype=np.int64))
    assert (n_A, n_primal) == (42, 24)
    cols = np.repeat(np.arange(n_A), np.diff(colptr))
    ours = set()
    for i, j in zip(rowind.tolist(), cols.tolist()):
        ours.add((i, j))
        ours.add((j, i))
    assert ours == sub


def test_ring30_sizes():
    inst = kktgen.make_workload(1)
    assert inst.n_A == 136 and inst.n_primal == 76 and inst.n_A - inst.n_primal == 60
    assert inst.nnz == 794
    assert inst.n_g == 16 and inst.N == 8 and len(inst.lines) == 41
    assert inst.b.shape == (1, 8 * 136 + 16)


def test_mesh2000_sizes_and_degree_cap():
    inst = kktgen.make_workload(2, N=1, nrhs=1)
    assert inst.n_A == 9200 and inst.n_primal == 5200
    assert len(inst.lines) == 3000
    deg = np.bincount(inst.lines.ravel(), minlength=2000)
    assert deg.max() <= 6 and deg.min() >= 1
    assert inst.ns * 96 == 19200


def test_block_inertia_is_kkt_correct():
    """Values rule: each A_n has inertia (n_primal, n_dual, 0) (section 2.3)."""
    from oracle import arrowhead as ah
    inst = kktgen.make_workload(1)
    for n in range(inst.N):
        w = np.linalg.eigvalsh(ah.block(inst, n).toarray())
        assert (w > 0).sum() == inst.n_primal
        assert (w < 0).sum() == inst.n_A - inst.n_primal


def test_seeded_determinism():
    a = kktgen.make_workload(1)
    b = kktgen.make_workload(1)
    assert np.array_equal(a.vals, b.vals) and np.array_equal(a.b, b.b)
    c = kktgen.make_workload(1, rep=1)
    assert not np.array_equal(a.vals, c.vals)



def _paper_lines_in_order(s):
    """Lines in the order of the printed flow rows 61..69 (one per line, its
    (theta_f, theta_t) columns), from-bus first as printed."""
    out = []
    for r in range(61, 70):
        th = sorted(b for a, b in s if a == r and b <= 9)
        out.append((th[0] - 1, th[1] - 1))
    return out


def test_line_flow_slacks_reproduce_printed_opf_kkt():
    """With the line-flow rows and every slack kept in the block, the
    generator's pattern is the printed 78 x 78 one entry for entry (576
    nonzeros: x, slacks, lambda_E, lambda_I in the order of Eq.
    SCOPFhessianSymmetric); with every slack eliminated (Eq.
    SCOPFhessianReduced) it is the printed one without the slack rows and
    columns: 522 nonzeros, the count the figure prints for the reduced
    60 x 60 system. Moving the slacks last (Eq. SCOPFslackAtEnd) keeps 576."""
    s = _paper_pattern()
    lines = np.array(_paper_lines_in_order(s))
    gen_bus = []
    for g in range(3):
        gen_bus.append([a for a, b in s if b == 19 + g and 43 <= a <= 51][0] - 43)
    nb = 9

    def ours(keep):
        n_A, n_primal, colptr, rowind, kind = kktgen.block_pattern(nb, lines, np.array(gen_bus),
                                                                    np.array([], dtype=np.int64), True, keep)
        cols = np.repeat(np.arange(n_A), np.diff(colptr))
        e = set()
        for i, j in zip(rowind.tolist(), cols.tolist()):
            e.add((i + 1, j + 1))
            e.add((j + 1, i + 1))
        return n_A, n_primal, e

    n_A, n_primal, full = ours(np.ones(18, bool))
    assert (n_A, n_primal) == (78, 42)
    assert full == s and len(full) == 576
    n_A, n_primal, red = ours(np.zeros(18, bool))
    assert (n_A, n_primal) == (60, 24)
    renum = lambda p: p if p <= 24 else p - 18
    printed_red = {(renum(a), renum(b)) for a, b in s if not (25 <= a <= 42 or 25 <= b <= 42)}
    assert red == printed_red and len(red) == 522
    # slacks last: a symmetric permutation keeps the count
    perm = list(range(1, 25)) + list(range(43, 79)) + list(range(25, 43))
    pos = {p: q + 1 for q, p in enumerate(perm)}
    assert len({(pos[a], pos[b]) for a, b in s}) == 576
