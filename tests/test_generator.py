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
