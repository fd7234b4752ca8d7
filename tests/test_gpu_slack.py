"""Slack elimination on the device (section 2.1) through the C-ABI:
kkt_slack_reduce (Eq. SCOPFhessianReduced), kkt_factor / kkt_solve of the
reduced system, kkt_slack_recover (Eq. SCOPFslackReduction), against the
oracle: the reduced values and right-hand sides equal the oracle's
reduction bit for bit (the same IEEE operations), the recovered slacks
equal the oracle's recovery from the same x bit for bit, and (x, s) matches
the LAPACK solution of the unreduced system (slacks last, Eq.
SCOPFslackAtEnd) element by element, with its residual in extended
precision <= 1e-10. Blocks keep the slacks whose L_s is near zero as
primal rows; the others are eliminated."""
import numpy as np
import pytest

import kktgen
from oracle import arrowhead as ah
from oracle import schur as sc
from test_gpu_parity import assert_x_close

pytestmark = pytest.mark.gpu

CASES = [dict(nb=8, nextra=3, ng=2, ns=2, N=3, nrhs=2, seed=31),
         dict(nb=12, nextra=6, ng=3, ns=0, N=2, nrhs=1, seed=32),
         dict(nb=40, nextra=25, ng=8, ns=6, N=7, nrhs=2, seed=34),
         dict(nb=90, nextra=50, ng=15, ns=10, N=5, nrhs=1, seed=35)]


def run_slack(inst):
    import torch
    import paper_1907_05420_amd as pk
    sl = inst.meta["slack"]
    s = pk.Solver(inst)
    pk.kkt_set_slacks(s.ctx, sl["lam_row"])
    d = pk.device_inputs(inst)
    Ls = torch.as_tensor(sl["Ls"]).cuda()
    rs = torch.as_tensor(sl["rs"]).cuda()
    A_red = torch.empty_like(d["vals"])
    b_red = torch.empty_like(d["b"])
    nrhs = d["b"].shape[0]
    pk.kkt_slack_reduce(s.ctx, d["vals"], Ls, d["b"], rs, A_red, b_red, nrhs)
    _, inn = s.factor(A_red, d["C0"], d["C1"], d["corner"])
    x, rc, info = s.solve(b_red)
    s_out = torch.empty_like(rs)
    pk.kkt_slack_recover(s.ctx, Ls, rs, x, s_out, nrhs)
    out = dict(A_red=A_red.cpu().numpy(), b_red=b_red.cpu().numpy(), x=x.cpu().numpy(), s=s_out.cpu().numpy(),
               inertia=inn, info=info, rc=rc)
    torch.cuda.synchronize()
    s.close()
    return out


@pytest.mark.parametrize("case", CASES)
def test_slack_elimination_against_unreduced_solve(case):
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), line_flow=True, ls_range=(1e-4, 1e2), keep_below=1e-3,
                             **case)
    sl = inst.meta["slack"]
    assert sl["keep"].any() and (~sl["keep"]).any()
    g = run_slack(inst)
    red = ah.reduce_slacks(inst)
    assert np.array_equal(g["A_red"], red.vals)
    assert np.array_equal(g["b_red"], red.b)
    assert np.array_equal(g["s"], ah.recover_slacks(red, g["x"]))
    Kf = ah.assemble_unreduced(inst)
    bf = ah.rhs_unreduced(inst)
    full = np.linalg.solve(Kf.toarray(), bf.T).T
    got = np.concatenate([g["x"], g["s"]], axis=1)
    assert_x_close(got, full, 1e-10, 1e-7)
    assert ah.rel_residual_ld(None, got, bf, Kf) <= 1e-10
    expect = (inst.N * inst.n_primal, inst.N * (inst.n_A - inst.n_primal) + inst.n_g, 0)
    inn = g["inertia"]
    assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == expect


def test_slack_elimination_wide_ranges():
    """250 buses, 8 periods, barrier and L_s over [1e-6, 1e6]: the unreduced
    residual of (x, s) meets the bar of the relative residual (1e-10, or twice
    the oracle's own best on the same route)."""
    rng = np.random.default_rng(36)
    lines = kktgen.tree_with_chords(250, 375, rng)
    inst = kktgen.make_instance(250, lines, 50, 25, 8, 1, 36, barrier_range=(1e-6, 1e6), rng=rng, line_flow=True,
                                ls_range=(1e-6, 1e6), keep_below=1e-4)
    g = run_slack(inst)
    Kf = ah.assemble_unreduced(inst)
    bf = ah.rhs_unreduced(inst)
    red = ah.reduce_slacks(inst)
    out = sc.algorithm1(red, dense_limit=0, assembly="prefix", schur_factor="cholesky")
    Kr = ah.assemble(red)
    solve = lambda r: sc.algorithm1(red, b=r, factors=out["factors"], schur=out["schur_fac"])["x"]
    best = np.inf
    x = out["x"]
    for _ in range(8):
        full = np.concatenate([x, ah.recover_slacks(red, x)], axis=1)
        best = min(best, ah.rel_residual_ld(None, full, bf, Kf))
        r, _ = ah.residual_ld(red, x, red.b, Kr)
        x = x + solve(r)
    got = np.concatenate([g["x"], g["s"]], axis=1)
    rel = ah.rel_residual_ld(None, got, bf, Kf)
    assert rel <= max(1e-10, 2 * best), (rel, best)
    assert g["inertia"]["inertia_ok"] == 1


def test_slack_error_paths():
    import torch
    import paper_1907_05420_amd as pk
    inst = kktgen.make_small(barrier_range=(1e-2, 1e2), line_flow=True, ls_range=(1e-4, 1e2), keep_below=1e-3,
                             **CASES[0])
    sl = inst.meta["slack"]
    s = pk.Solver(inst)
    with pytest.raises(pk.KKTError) as e:            # a primal row
        pk.kkt_set_slacks(s.ctx, np.array([0], np.int32))
    assert e.value.code == pk.KKT_ERR_ARG
    with pytest.raises(pk.KKTError) as e:            # two slacks on one row
        pk.kkt_set_slacks(s.ctx, np.array([sl["lam_row"][0]] * 2, np.int32))
    assert e.value.code == pk.KKT_ERR_ARG
    pk.kkt_set_slacks(s.ctx, sl["lam_row"])
    d = pk.device_inputs(inst)
    Ls = torch.as_tensor(sl["Ls"]).cuda()
    Ls[0, 0] = 0.0
    rs = torch.as_tensor(sl["rs"]).cuda()
    with pytest.raises(pk.KKTError) as e:
        pk.kkt_slack_reduce(s.ctx, d["vals"], Ls, d["b"], rs, d["vals"].clone(), d["b"].clone(), d["b"].shape[0])
    assert e.value.code == pk.KKT_ERR_NONFINITE
    torch.cuda.synchronize()
    s.close()
