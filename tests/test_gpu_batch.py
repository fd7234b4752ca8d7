"""Uneven batches through the C-ABI (kkt_batch_*): every instance of a batch
of different grids and horizons, run on several streams, gives bitwise the
result it gives alone (its kernels and their order do not depend on the other
instances), and that result meets the oracle's residual bar, also after the
values were changed in place (IPM iterations re-draw the barrier diagonals).
The HIP-graph form of the batch is switched off (see its skipped test).

At real sizes (the uneven mixture's barrier range [1e-6, 1e6], Schur
dimensions up to 888 so that the dense solves cross their 512-wide blocks,
fronts of 190 to 330 rows) every instance's solution is checked on the
oracle's assembled K in extended precision against the relative-residual
bar (1e-10, or twice the oracle's own best) and its inertia against the
expected triple."""
import numpy as np
import pytest

import kktgen
from oracle import arrowhead as ah
from oracle import schur as sc
from test_gpu_parity import reference, residual_bar

pytestmark = pytest.mark.gpu

STEPS = 3


def small_batch(count=6, seed=11):
    return kktgen.uneven_batch(count=count, seed=seed, nb_range=(20, 90), horizons=(2, 3, 5), nrhs=1,
                               barrier=(1e-2, 1e2))


def alone(inst, precision, vals=None):
    import torch
    import paper_1907_05420_amd as pk
    s = pk.Solver(inst, precision=precision)
    d = pk.device_inputs(inst)
    if vals is not None:
        d["vals"] = torch.as_tensor(vals).cuda()
    x = torch.empty_like(d["b"])
    pk.kkt_factor_async(s.ctx, d["vals"], d["C0"], d["C1"], d["corner"])
    pk.kkt_solve_async(s.ctx, d["b"], x, d["b"].shape[0], STEPS)
    rc, info = pk.kkt_solve_status(s.ctx)
    out = x.cpu().numpy()
    s.close()
    return out, info


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_alone_and_oracle(precision):
    """Eager multi-stream batch: bitwise equal to the instances alone, within
    the oracle's residual bar; a second run after new values in place."""
    import torch
    import paper_1907_05420_amd as pk
    insts = small_batch()
    ref_alone = [alone(inst, precision)[0] for inst in insts]
    b = pk.Batch(insts, nstreams=3, precision=precision)
    b.run(STEPS, use_graph=False)
    b.wait()
    eager = [x.cpu().numpy() for x in b.x]
    streams = {pk.kkt_batch_stream_of(b.h, i) for i in range(len(insts))}
    assert streams == {0, 1, 2}
    for xa, xe in zip(ref_alone, eager):
        assert np.array_equal(xa, xe)
    for inst, st, xe in zip(insts, b.status(), eager):
        ref, xref, K = reference(inst)
        rel = ah.rel_residual_ld(inst, xe, inst.b, K)
        assert rel <= residual_bar(ref), rel
        assert st["inertia"]["inertia_ok"] == 1
        assert st["info"]["rel_res"] <= 1e-10
    # new barrier values in place: the next run reads them
    rng = np.random.default_rng(5)
    new_vals = kktgen.redraw_barrier(insts[0], rng)
    b.inputs[0]["vals"].copy_(torch.as_tensor(new_vals))
    for x in b.x:
        x.fill_(0.0)
    torch.cuda.synchronize()
    b.run(STEPS, use_graph=False)
    b.wait()
    x_new, _ = alone(insts[0], precision, vals=new_vals)
    assert np.array_equal(b.x[0].cpu().numpy(), x_new)
    for x, xe in zip(b.x[1:], eager[1:]):
        assert np.array_equal(x.cpu().numpy(), xe)
    b.close()


@pytest.mark.skip(reason="graph capture of a batch ended in a host segmentation fault inside "
                         "kkt_batch_run; the graph path is switched off until its cause is found")
def test_batch_graph_replays_equal_eager():
    import torch
    import paper_1907_05420_amd as pk
    insts = small_batch()
    b = pk.Batch(insts, nstreams=3)
    b.run(STEPS, use_graph=False)
    b.wait()
    eager = [x.cpu().numpy() for x in b.x]
    for rep in range(3):
        for x in b.x:
            x.fill_(0.0)
        torch.cuda.synchronize()
        b.run(STEPS, use_graph=True)
        b.wait()
        for x, xe in zip(b.x, eager):
            assert np.array_equal(x.cpu().numpy(), xe), rep
    b.close()


def test_async_status_reports_nonfinite():
    import torch
    import paper_1907_05420_amd as pk
    inst = small_batch(count=1)[0]
    s = pk.Solver(inst)
    d = pk.device_inputs(inst)
    d["vals"][0, 0] = float("nan")
    pk.kkt_factor_async(s.ctx, d["vals"], d["C0"], d["C1"], d["corner"])
    with pytest.raises(pk.KKTError) as e:
        pk.kkt_factor_status(s.ctx)
    assert e.value.code == pk.KKT_ERR_NONFINITE
    torch.cuda.synchronize()
    s.close()


def oracle_best(inst):
    """Best relative residual the oracle's refined FP64 solution reaches
    (SuperLU blocks, Cholesky of -S, extended-precision residuals)."""
    out = sc.algorithm1(inst, dense_limit=0, assembly="prefix", schur_factor="cholesky")
    K = ah.assemble(inst)
    solve = lambda r: sc.algorithm1(inst, b=r, factors=out["factors"], schur=out["schur_fac"])["x"]
    _, hist = sc.refine(inst, out["x"], inst.b, solve, tol=1e-16, K=K, extended=True)
    return min(hist), K


def test_batch_real_sizes_against_oracle():
    """Four instances of 258 to 425 buses over 12 or 24 periods (n_g 444 to
    888, fronts up to 326 rows) on three streams with 5 refinement steps:
    each alone == in the batch bitwise, each within the oracle's residual bar
    on its assembled K, exact inertia."""
    import torch
    import paper_1907_05420_amd as pk
    steps = 5
    insts = kktgen.uneven_batch(count=4, seed=31, nb_range=(250, 450), horizons=(12, 24), nrhs=1,
                                barrier=(1e-6, 1e6))
    assert max(i.n_g for i in insts) > 512
    b = pk.Batch(insts, nstreams=3)
    b.run(steps, use_graph=False)
    b.wait()
    xs = [x.cpu().numpy() for x in b.x]
    st = b.status()
    b.close()
    for inst, xe, s in zip(insts, xs, st):
        best, K = oracle_best(inst)
        rel = ah.rel_residual_ld(inst, xe, inst.b, K)
        assert rel <= max(1e-10, 2 * best), (inst.nb, inst.N, rel, best)
        expect = (inst.N * inst.n_primal, inst.N * (inst.n_A - inst.n_primal) + inst.n_g, 0)
        inn = s["inertia"]
        assert (inn["n_pos"], inn["n_neg"], inn["n_zero"]) == expect and inn["inertia_ok"] == 1
        assert abs(s["info"]["rel_res"] - rel) <= 1e-2 * rel + 1e-16
        s_alone = pk.Solver(inst)
        d = pk.device_inputs(inst)
        x = torch.empty_like(d["b"])
        pk.kkt_factor_async(s_alone.ctx, d["vals"], d["C0"], d["C1"], d["corner"])
        pk.kkt_solve_async(s_alone.ctx, d["b"], x, 1, steps)
        pk.kkt_solve_status(s_alone.ctx)
        assert np.array_equal(x.cpu().numpy(), xe)
        s_alone.close()
