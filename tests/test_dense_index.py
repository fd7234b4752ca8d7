"""Host check of the address ranges of the triangular solves with the dense
Schur factor (no GPU needed): the header with the kernels' launch geometry
and global addresses is compiled with the host compiler, and for every
launch of a forward and a backward pass over Schur dimensions that end
inside, at and past the 1024-wide inverted diagonal blocks, every address a
thread loads lies inside the n_g x n_g factor; every unmasked load lies in
the part of the factor the product uses (the block's rows below it, the
strict lower triangle of the inverted diagonal block, one column segment of
a dot product); and every entry of those parts is loaded by exactly one
unmasked load. An out-of-range row pointer on a ragged last block faulted
the GPU once; this pins the clamping that prevents it."""
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1907_05420_amd", "csrc")

PROG = r"""
#include "dense_index.hpp"
#include <cstdio>
#include <cstdint>
#include <vector>
using namespace kkt;
static long bad = 0;
#define CHECK(c, ...) do { if (!(c)) { if (bad < 20) printf(__VA_ARGS__); ++bad; } } while (0)

// counts of unmasked loads per factor entry (ng <= 4200), or bounds only
struct Cov {
    int64_t ng; std::vector<unsigned char> n; bool on;
    Cov(int64_t g, bool o) : ng(g), on(o) { if (on) n.assign((size_t)(g * g), 0); }
    void hit(int64_t a) { if (on) n[(size_t)a]++; }
};

static void pass(int64_t ng, bool cover) {
    Cov cv(ng, cover);
    const int64_t NS = ng * ng;
    // forward: the first block's in-block product, then one launch per step:
    // the rows below block [j0, j1) (their first row workgroups, the
    // producers, cover the next block exactly), then the next block's
    // in-block product (the product's geometry with row0 = col0)
    auto tri = [&](int64_t j0, int nbw) {
        for (int64_t b = 0; b < gemv_grid(nbw); ++b)
            for (int tid = 0; tid < 512; ++tid) {
                if (!gemv_tri_used(b, tid)) continue;  // groups right of the diagonal load nothing
                const int64_t i = b * GV_R + tid % GV_R;
                const int qa = 64 * (tid / GV_R);
                const int ncq = (int)ds_max(1, ds_min(64, nbw - qa));
                for (int u = 0; u < 64; ++u) {
                    const int64_t a = gemv_s_addr(ng, j0, nbw, j0, nbw, b, tid, u);
                    CHECK(a >= 0 && a < NS, "tri ng %lld j0 %lld b %lld tid %d u %d addr %lld\n", (long long)ng,
                          (long long)j0, (long long)b, tid, u, (long long)a);
                    const int64_t q = qa + u;
                    if (qa < nbw && u < ncq && q < i && i < nbw) {  // unmasked
                        CHECK(a == (j0 + i) + (j0 + q) * ng, "tri addr ng %lld\n", (long long)ng);
                        cv.hit(a);
                    }
                }
            }
    };
    tri(0, (int)ds_min(DENSE_BLOCK, ng));
    for (int64_t j0 = 0; j0 + DENSE_BLOCK < ng; j0 += DENSE_BLOCK) {
        const int nbw = DENSE_BLOCK;
        const int64_t row0 = j0 + nbw, nrow = ng - row0;
        const int nbw1 = (int)ds_min(DENSE_BLOCK, nrow);
        const int64_t G = gemv_grid(nrow), P = gemv_grid(nbw1);
        CHECK(fwd_step_grid(ng, row0) == G + P, "fwd grid ng %lld\n", (long long)ng);
        // the producers' rows are the next block's rows, and no other workgroup writes them
        CHECK(ds_min(P * GV_R, nrow) >= nbw1 && (P - 1) * GV_R < nbw1, "producers ng %lld j0 %lld\n", (long long)ng,
              (long long)j0);
        for (int64_t b = 0; b < G; ++b)
            for (int tid = 0; tid < 512; ++tid) {
                const int64_t i = b * GV_R + tid % GV_R;
                const int qa = 64 * (tid / GV_R);
                const int ncq = (int)ds_max(1, ds_min(64, nbw - qa));
                for (int u = 0; u < 64; ++u) {
                    const int64_t a = gemv_s_addr(ng, row0, nrow, j0, nbw, b, tid, u);
                    CHECK(a >= 0 && a < NS, "gemv ng %lld j0 %lld b %lld tid %d u %d\n", (long long)ng,
                          (long long)j0, (long long)b, tid, u);
                    if (qa < nbw && u < ncq && i < nrow) {
                        CHECK(a == (row0 + i) + (j0 + qa + u) * ng, "gemv addr ng %lld\n", (long long)ng);
                        cv.hit(a);
                    }
                }
            }
        tri(row0, nbw1);
    }
    if (cover) {  // every strictly lower entry once (diagonal D is read by the division)
        for (int64_t q = 0; q < ng; ++q)
            for (int64_t r = 0; r < ng; ++r) {
                const int want = r > q ? 1 : 0;
                CHECK(cv.n[(size_t)(r + q * ng)] == want, "fwd coverage ng %lld (%lld, %lld): %d\n", (long long)ng,
                      (long long)r, (long long)q, cv.n[(size_t)(r + q * ng)]);
            }
        cv.n.assign((size_t)(ng * ng), 0);
    }
    // backward: the last block's in-block product with X^T, then one launch
    // per step: the columns [0, j0) above block [j0, ..) in reverse order of
    // workgroups (the first tdot_grid(DENSE_BLOCK), the producers, cover the
    // block before it exactly), then that block's in-block product
    auto tdot = [&](int64_t row0, int nq, int64_t col0, int ncols, bool blk, bool rev) {
        const int64_t G = tdot_grid(ncols);
        for (int64_t bb = 0; bb < G; ++bb) {
            const int64_t b = rev ? G - 1 - bb : bb;
            for (int wv = 0; wv < 4; ++wv)
                for (int c = 0; c < TD_CPW; ++c)
                    for (int lane = 0; lane < 64; ++lane)
                        for (int k = 0; k < DENSE_BLOCK / 64; ++k) {
                            const int64_t a = tdot_s_addr(ng, row0, nq, col0, ncols, b, wv, c, lane, k);
                            CHECK(a >= 0 && a < NS, "tdot ng %lld row0 %lld\n", (long long)ng, (long long)row0);
                            const int64_t i = (b * 4 + wv) * TD_CPW + c, q = lane + 64 * k;
                            if (rev && bb < tdot_grid(DENSE_BLOCK))  // producers: the last DENSE_BLOCK columns
                                CHECK(i >= ncols - DENSE_BLOCK, "bwd producers ng %lld\n", (long long)ng);
                            if (i < ncols && q < nq && (!blk || q > i)) {
                                CHECK(a == (row0 + q) + (col0 + i) * ng, "tdot addr ng %lld\n", (long long)ng);
                                cv.hit(a);
                            }
                        }
        }
    };
    const int64_t jl = ((ng - 1) / DENSE_BLOCK) * DENSE_BLOCK;
    tdot(jl, (int)(ng - jl), jl, (int)(ng - jl), true, false);
    for (int64_t j0 = jl; j0 >= DENSE_BLOCK; j0 -= DENSE_BLOCK) {
        const int nbw = (int)ds_min(DENSE_BLOCK, ng - j0);
        CHECK(bwd_step_grid(j0) == tdot_grid(j0) + tdot_grid(DENSE_BLOCK), "bwd grid ng %lld\n", (long long)ng);
        tdot(j0, nbw, 0, (int)j0, false, true);
        tdot(j0 - DENSE_BLOCK, DENSE_BLOCK, j0 - DENSE_BLOCK, DENSE_BLOCK, true, false);
    }
    if (cover)
        for (int64_t q = 0; q < ng; ++q)
            for (int64_t r = 0; r < ng; ++r) {
                const int want = r > q ? 1 : 0;
                CHECK(cv.n[(size_t)(r + q * ng)] == want, "bwd coverage ng %lld (%lld, %lld): %d\n", (long long)ng,
                      (long long)r, (long long)q, cv.n[(size_t)(r + q * ng)]);
            }
}

int main() {
    const int64_t cover_sizes[] = {1, 2, 15, 16, 17, 63, 64, 65, 81, 312, 480, 512, 516, 800, 1023, 1024, 1025,
                                   1040, 1536, 2047, 2048, 2049, 2100, 3071, 4200};
    for (int64_t ng : cover_sizes) pass(ng, true);
    const int64_t big[] = {12000, 19200, 19201};  // the workloads' sizes: bounds and places only
    for (int64_t ng : big) pass(ng, false);
    printf("bad %ld\n", bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_dense_solve_addresses_stay_in_the_factor(tmp_path):
    src = tmp_path / "dense_index.cpp"
    src.write_text(PROG)
    exe = tmp_path / "dense_index"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "bad 0" in r.stdout
