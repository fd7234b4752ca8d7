"""GPU parity of the mixed-precision path (FP32 period factors and Schur
contributions, FP64 Schur factorisation, FP64 flexible-GMRES refinement)
against the FP64 oracle, through the C-ABI.

The paper has no mixed-precision result to pin against (parity unpinned);
the bar is the FP64 oracle: after refinement the relative residual meets the
same bar as the FP64 path, the solution matches the oracle's as closely as
the FP64 path's does, and the inertia of well-conditioned blocks is exact.
The local Schur blocks come out of FP32 factors and are compared at 1e-5 of
their largest entry (FP32 rounding amplified by the elimination).

Where the FP32 factor cannot be trusted (wrong inertia or perturbed pivots)
or refinement around it stops above the target, the library factors the
same values in FP64 and says so (fallback_used); the answer must then meet
the FP64 bar on the oracle's K all the same. Well-conditioned cases must not
fall back."""
import numpy as np
import pytest

import kktgen
from oracle import arrowhead as ah
from test_gpu_batch import oracle_best
from test_gpu_parity import SMALL, _rel, reference, residual_bar, run_gpu

pytestmark = pytest.mark.gpu

KKT_MIXED = 1


@pytest.mark.parametrize("case", SMALL)
def test_mixed_small(case):
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), **case)
    ref, xref, K = reference(inst)
    g = run_gpu(inst, precision=KKT_MIXED)
    rel = ah.rel_residual_ld(inst, g["x"], inst.b, K)
    assert rel <= 1e-10, rel
    assert g["info"]["rel_res"] <= 1e-10
    assert g["info"]["fallback_used"] == 0
    assert _rel(g["x"], xref) <= 1e-9, _rel(g["x"], xref)
    expect = (inst.N * inst.n_primal, inst.N * (inst.n_A - inst.n_primal) + inst.n_g, 0)
    inn = g["inertia"]
    assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == expect
    if inst.n_g:
        sb = ref["Sbar"]
        assert np.max(np.abs(g["Sbar"] - sb)) <= 1e-5 * np.max(np.abs(sb))


def test_mixed_wide_front():
    """FP32 factors with a 526-pivot front (growth-free order: the solves'
    256-pivot windows, inverted in FP32 after the factorisation): refinement
    reaches the FP64 bar on the oracle's K without falling back, x matches
    the oracle's, and the inertia is exact."""
    from test_gpu_parity import GROWTH_FREE
    inst = kktgen.make_small(nb=400, nextra=200, ng=50, ns=20, N=2, nrhs=3, seed=21, barrier_range=(1e-2, 1e2))
    ref, xref, K = reference(inst)
    g = run_gpu(inst, precision=KKT_MIXED, want_schur=False, dual_wait=GROWTH_FREE)
    rel = ah.rel_residual_ld(inst, g["x"], inst.b, K)
    assert rel <= 1e-10, rel
    assert g["info"]["fallback_used"] == 0 and g["rc_solve"] == 0
    assert _rel(g["x"], xref) <= 1e-9, _rel(g["x"], xref)
    expect = (inst.N * inst.n_primal, inst.N * (inst.n_A - inst.n_primal) + inst.n_g, 0)
    inn = g["inertia"]
    assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == expect


def test_mixed_ring30():
    inst = kktgen.make_workload(1)
    ref, xref, K = reference(inst)
    g = run_gpu(inst, precision=KKT_MIXED)
    rel = ah.rel_residual_ld(inst, g["x"], inst.b, K)
    assert rel <= residual_bar(ref), rel
    assert _rel(g["x"], xref) <= 1e-6
    assert g["rc_solve"] == 0


@pytest.mark.parametrize("barrier", [(1e-6, 1e6), (1e-8, 1e8)])
def test_mixed_wide_barrier_meets_fp64_bar(barrier):
    """258 buses over 24 periods (n_g 624) with late-IPM barrier ranges: the
    mixed path's answer (FP32 factor refined, or the FP64 fallback) meets
    the FP64 residual bar on the oracle's K, with the expected inertia."""
    inst = kktgen.uneven_batch(count=4, seed=31, nb_range=(250, 450), horizons=(12, 24), nrhs=1,
                               barrier=barrier)[3]
    g = run_gpu(inst, precision=KKT_MIXED, want_schur=False)
    best, K = oracle_best(inst)
    rel = ah.rel_residual_ld(inst, g["x"], inst.b, K)
    print(f"barrier {barrier}: fallback_used {g['info']['fallback_used']}, refine_iters "
          f"{g['info']['refine_iters']}, rel_res {rel:.2e}, oracle best {best:.2e}")
    assert rel <= max(1e-10, 2 * best), rel
    assert g["rc_solve"] == 0 or rel > 1e-10
    expect = (inst.N * inst.n_primal, inst.N * (inst.n_A - inst.n_primal) + inst.n_g, 0)
    inn = g["inertia"]
    assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == expect
