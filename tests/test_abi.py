"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/kkt.h declares, and its planning query (the symbolic
analysis) produces a valid order whose factor pattern contains the exact fill."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import kktgen
import paper_1907_05420_amd as pk

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "kkt.h")


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(pk.LIB_PATH)
    names = set(re.findall(r"\b(kkt_[a-z_]+)\s*\(", open(HDR).read()))
    assert len(names) >= 14
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(pk._abi.SIGNATURES) == names


def test_strerror_and_defaults():
    assert pk.strerror(pk.KKT_ERR_ORDER) == "wrong call order"
    o = pk.kkt_default_options()
    assert o.precision == pk.KKT_FP64 and o.refine_tol == 1e-10 and o.refine_max == 20


def _plan(inst, want_perm=True):
    return pk.kkt_plan(inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, inst.rowind, inst.C0_rowptr,
                       inst.C0_colind, inst.C1_rowptr, inst.C1_colind, want_perm=want_perm)


def _exact_fill(inst, perm):
    """nnz of the Cholesky-pattern factor of P A P^T by dense boolean elimination."""
    n = inst.n_A
    cols = np.repeat(np.arange(n), np.diff(inst.colptr))
    B = np.zeros((n, n), bool)
    ip = np.empty(n, np.int64)
    ip[perm] = np.arange(n)
    B[ip[inst.rowind], ip[cols]] = True
    B |= B.T
    nnz = 0
    for k in range(n):
        rows = np.nonzero(B[k + 1:, k])[0] + k + 1
        nnz += 1 + len(rows)
        if len(rows):
            B[np.ix_(rows, rows)] = True
    return nnz


@pytest.mark.parametrize("case", [dict(nb=8, nextra=3, ng=2, ns=2, N=2, seed=0),
                                  dict(nb=60, nextra=30, ng=10, ns=5, N=3, seed=1),
                                  dict(nb=9, nextra=5, ng=3, ns=0, N=2, seed=3)])
def test_plan_order_and_fill(case):
    inst = kktgen.make_small(**case)
    st, perm = _plan(inst)
    assert sorted(perm.tolist()) == list(range(inst.n_A))
    # stored panels hold at least the exact fill of the ordered block
    # (the border rows add their own entries on top)
    assert st["nnz_L"] >= _exact_fill(inst, perm)
    assert st["max_front"] >= 2 * inst.ns
    assert st["device_bytes"] > 0


def test_plan_ring30_and_mesh2000():
    st1, _ = _plan(kktgen.make_workload(1), want_perm=False)
    assert st1["n_supernodes"] >= 2 and st1["max_front"] <= 136 + 4
    inst = kktgen.make_workload(2, N=1, nrhs=1)
    st2, perm = _plan(inst)
    assert sorted(perm.tolist()) == list(range(inst.n_A))
    assert st2["max_front"] < 2000 and st2["n_levels"] < 40


def test_plan_rejects_bad_structures():
    inst = kktgen.make_small(nb=8, nextra=3, ng=2, ns=2, N=2, seed=0)
    bad = inst.rowind.copy()
    bad[1] = bad[0]                      # duplicate row index in column 0
    with pytest.raises(pk.KKTError) as e:
        pk.kkt_plan(inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, bad, inst.C0_rowptr,
                    inst.C0_colind, inst.C1_rowptr, inst.C1_colind)
    assert e.value.code == pk.KKT_ERR_STRUCT
    c0 = inst.C0_colind.copy()
    c0[0] = inst.n_A + 5                 # coupling column out of range
    with pytest.raises(pk.KKTError) as e:
        pk.kkt_plan(inst.n_A, inst.n_primal, inst.N, inst.ns, inst.colptr, inst.rowind, inst.C0_rowptr,
                    c0, inst.C1_rowptr, inst.C1_colind)
    assert e.value.code == pk.KKT_ERR_STRUCT


def _dual_matching_ok(inst, perm):
    """Along the order, every eliminated dual is matched to its own eliminated
    primal neighbour (maximum bipartite matching by augmenting paths, in
    Python). Returns the number of duals that could not be matched."""
    n, npr = inst.n_A, inst.n_primal
    cols = np.repeat(np.arange(n), np.diff(inst.colptr))
    nbr = [[] for _ in range(n)]
    for i, j in zip(inst.rowind, cols):
        if i != j:
            nbr[i].append(int(j))
            nbr[int(j)].append(int(i))
    elim = np.zeros(n, bool)
    match_of_primal = {}

    def augment(d, seen):
        for u in nbr[d]:
            if u >= npr or not elim[u] or u in seen:
                continue
            seen.add(u)
            if u not in match_of_primal or augment(match_of_primal[u], seen):
                match_of_primal[u] = d
                return True
        return False

    unmatched = 0
    for v in perm:
        v = int(v)
        if v >= npr:
            elim[v] = True
            if not augment(v, set()):
                unmatched += 1
        else:
            elim[v] = True
    return unmatched


@pytest.mark.parametrize("case", [dict(nb=60, nextra=30, ng=10, ns=5, N=1, seed=1),
                                  dict(nb=160, nextra=90, ng=30, ns=12, N=1, seed=8),
                                  dict(nb=300, nextra=150, ng=60, ns=30, N=1, seed=5)])
def test_order_pairs_every_dual_with_an_eliminated_primal(case):
    """The default FP64 order: a dual waits for 4 of its primal neighbours and
    claims one eliminated primal neighbour no earlier dual claimed, so the
    eliminated duals never outnumber the eliminated primals they touch
    (their block of the partial Schur complement keeps full structural
    rank; without this a dual can be left with a pivot near -delta_c).
    Only the duals of the final clique (appended once every primal is
    gone) and duals forced for lack of any partner may stay unmatched: a
    handful at most."""
    inst = kktgen.make_small(**case)
    _, perm = _plan(inst)
    n_dual = inst.n_A - inst.n_primal
    assert _dual_matching_ok(inst, perm) <= max(2, n_dual // 200)
