"""Serving loop (continuous batching) through the C-ABI: requests of
different grids and horizons arrive as a Poisson stream, are admitted by HBM
footprint into a few slots, and run their IPM-like iterations (re-drawn
barrier diagonals) side by side. Each request's final solution is bitwise the
one it gets when served alone, every iteration meets the residual bar, and
the admitted footprint never exceeds the budget. A mix with a real-size
request (Schur dimension 888, fronts up to 292 rows) is checked on the
oracle's assembled K in extended precision, with the values of the last
iteration, against the relative-residual bar, and for the inertia."""
import numpy as np
import pytest

import kktgen
from oracle import arrowhead as ah
from test_gpu_batch import oracle_best

pytestmark = pytest.mark.gpu


def make_requests(count=6, iterations=4, seed=21):
    from paper_1907_05420_amd import serve
    insts = kktgen.uneven_batch(count=count, seed=seed, nb_range=(20, 90), horizons=(2, 3, 5), nrhs=1,
                                barrier=(1e-2, 1e2))
    rng = np.random.default_rng(seed)
    arrivals = serve.poisson_arrivals(count, rate=200.0, rng=rng)
    reqs = []
    for i, (inst, t) in enumerate(zip(insts, arrivals)):
        vals = [kktgen.redraw_barrier(inst, np.random.default_rng(1000 * seed + 10 * i + k))
                for k in range(iterations)]
        reqs.append(serve.Request(i, inst, float(t), iterations, vals))
    return reqs


def test_serving_mix_equals_alone():
    from paper_1907_05420_amd import serve
    reqs = make_requests()
    budget = sorted(serve.footprint_bytes(r.inst) for r in reqs)[-1] * 3
    done, stats = serve.serve(reqs, slots=3, hbm_budget=budget, keep_x=True)
    assert stats["max_used"] <= budget
    assert stats["max_active"] >= 2            # requests overlapped on the device
    assert stats["iterations"] == sum(r.iterations for r in reqs)
    for r in done:
        assert r.finished is not None and r.admitted >= r.arrival - 1e-9
        assert max(r.rel_res) <= 1e-10, r.rel_res
        assert all(r.inertia_ok)
    for r in make_requests():
        alone, _ = serve.serve([r], slots=1, keep_x=True)
        mixed = [m for m in done if m.rid == r.rid][0]
        assert np.array_equal(alone[0].x, mixed.x)
        assert alone[0].rel_res == mixed.rel_res


def test_serving_to_tolerance_mix_equals_alone():
    """Requests refined to the residual tolerance (kkt_factor/kkt_solve in a
    host thread per admitted request) give, in the mix, bitwise what they give
    alone, and every iteration meets 1e-10."""
    from paper_1907_05420_amd import serve
    reqs = make_requests(seed=24)
    done, stats = serve.serve(reqs, slots=3, keep_x=True, refine="tolerance")
    assert stats["max_active"] >= 2
    assert stats["iterations"] == sum(r.iterations for r in reqs)
    for r in done:
        assert len(r.rel_res) == r.iterations and max(r.rel_res) <= 1e-10, r.rel_res
        assert all(r.inertia_ok)
    for r in make_requests(seed=24):
        alone, _ = serve.serve([r], slots=1, keep_x=True, refine="tolerance")
        mixed = [m for m in done if m.rid == r.rid][0]
        assert np.array_equal(alone[0].x, mixed.x)
        assert alone[0].rel_res == mixed.rel_res


def test_serving_admission_respects_budget():
    from paper_1907_05420_amd import serve
    reqs = make_requests(count=5, iterations=2, seed=22)
    foot = [serve.footprint_bytes(r.inst) for r in reqs]
    budget = max(foot) + min(foot)             # at most two requests fit at once
    done, stats = serve.serve(reqs, slots=4, hbm_budget=budget)
    assert stats["max_used"] <= budget
    assert all(r.finished is not None for r in done)


def test_serving_rejects_oversized_request():
    from paper_1907_05420_amd import serve
    reqs = make_requests(count=1, iterations=1, seed=23)
    with pytest.raises(ValueError):
        serve.serve(reqs, slots=1, hbm_budget=1024)


def test_serving_real_size_against_oracle():
    """Two small requests and one of 372 buses over 24 periods (n_g 888),
    3 iterations each with re-drawn barriers, refined to the tolerance: the
    last solution of every request meets the residual bar on the oracle's K
    (assembled with that iteration's values), the inertia is exact in every
    iteration, and the big request's solution equals its solution alone."""
    import copy
    from paper_1907_05420_amd import serve
    small = kktgen.uneven_batch(count=2, seed=41, nb_range=(40, 90), horizons=(3, 5), nrhs=1, barrier=(1e-6, 1e6))
    big = kktgen.uneven_batch(count=4, seed=31, nb_range=(250, 450), horizons=(12, 24), nrhs=1,
                              barrier=(1e-6, 1e6))[2]
    assert big.n_g == 888

    def requests():
        out = []
        for i, inst in enumerate([small[0], big, small[1]]):
            vals = [kktgen.redraw_barrier(inst, np.random.default_rng(500 + 10 * i + k)) for k in range(3)]
            out.append(serve.Request(i, inst, 0.001 * i, 3, vals))
        return out

    reqs = requests()
    done, stats = serve.serve(reqs, slots=3, keep_x=True, refine="tolerance")
    assert stats["max_active"] >= 2
    for r in done:
        assert all(r.inertia_ok)
        last = copy.copy(r.inst)
        last.vals = r.values[-1]
        best, K = oracle_best(last)
        rel = ah.rel_residual_ld(last, r.x, last.b, K)
        assert rel <= max(1e-10, 2 * best), (r.rid, rel, best)
    alone, _ = serve.serve([requests()[1]], slots=1, keep_x=True, refine="tolerance")
    assert np.array_equal(alone[0].x, [m for m in done if m.rid == 1][0].x)
