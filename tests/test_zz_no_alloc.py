"""kkt_solve_noalloc (the enqueue-only solve whose workspace is the library's
fixed device array, for callers that cannot allocate) against
kkt_solve_async, through the C-ABI: two calls in a row, the second on a
smaller system, so the second runs in an array that still holds the first
call's contents. The same kernels run on the same inputs, so the solutions
must agree bit for bit; the residual norms it leaves in the context agree
too, and the oracle's residual bar holds. A system whose workspace exceeds
the array is refused before anything is enqueued."""
import numpy as np
import pytest

import kktgen
from oracle import arrowhead as ah

pytestmark = pytest.mark.gpu

STEPS = 2


def _pair(inst):
    import torch
    import paper_1907_05420_amd as pk
    s = pk.Solver(inst)
    d = pk.device_inputs(inst)
    s.factor(d["vals"], d["C0"], d["C1"], d["corner"])
    nrhs = d["b"].shape[0]
    xa = torch.full_like(d["b"], 7.0)
    pk.kkt_solve_async(s.ctx, d["b"], xa, nrhs, STEPS)
    rc_a, info_a = pk.kkt_solve_status(s.ctx)
    xn = torch.full_like(d["b"], -3.0)
    pk.kkt_solve_noalloc(s.ctx, d["b"], xn, nrhs, STEPS)
    rc_n, info_n = pk.kkt_solve_status(s.ctx)
    torch.cuda.synchronize()
    out = (xa.cpu().numpy(), xn.cpu().numpy(), rc_a, rc_n, info_a, info_n)
    s.close()
    return out


def test_noalloc_equals_async_twice_second_smaller():
    big = kktgen.make_small(nb=70, nextra=40, ng=12, ns=9, N=9, nrhs=3, seed=6, barrier_range=(1e-2, 1e2))
    small = kktgen.make_small(nb=12, nextra=6, ng=3, ns=3, N=4, nrhs=1, seed=1, barrier_range=(1e-2, 1e2))
    for inst in (big, small):
        xa, xn, rc_a, rc_n, ia, inf_n = _pair(inst)
        assert np.array_equal(xa, xn)
        assert rc_a == rc_n == 0
        assert ia["rel_res"] == inf_n["rel_res"] and ia["omega"] == inf_n["omega"]
        assert ah.rel_residual_ld(inst, xn, inst.b) <= 1e-10


def test_noalloc_refuses_oversized_workspace():
    import torch
    import paper_1907_05420_amd as pk
    # 2000 buses, 24 periods, 4 right-hand sides: far above the 32 MiB array
    inst = kktgen.make_workload(2, N=24, nrhs=4)
    s = pk.Solver(inst)
    d = pk.device_inputs(inst)
    s.factor(d["vals"], d["C0"], d["C1"], d["corner"])
    x = torch.zeros_like(d["b"])
    with pytest.raises(pk.KKTError) as e:
        pk.kkt_solve_noalloc(s.ctx, d["b"], x, 4, 1)
    assert e.value.code == pk.KKT_ERR_TOOBIG
    torch.cuda.synchronize()
    assert float(x.abs().max()) == 0.0          # nothing was enqueued
    s.close()
