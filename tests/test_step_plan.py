"""Host check of the step plan of the blocked factorisation (no GPU needed):
the header with the plan and the update geometry is compiled with the host
compiler, every step of the plans of several front groups is applied to a
record of which pivot columns have updated which entry, and every entry
(r, q), r >= q, of every front must have received each pivot k < min(q, c)
exactly once and no other. Front groups: period-like sets of fronts of
different sizes (outer panels of 512 columns in sub-panels of 256, some
with 1024 or more rows below a sub-panel so that those rows take one
launch), the same fronts in 256-wide panels, and single dense fronts with
the lookahead split of the dense Schur factor. A double update of the
update block's first columns by fronts that end inside the second sub-panel
of an outer panel was caught this way."""
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1907_05420_amd", "csrc")

PROG = r"""
#include "step_plan.hpp"
#include <cstdio>
#include <cstdint>
#include <vector>
using namespace kkt;
struct FD { int m, c; };
static long bad = 0;
#define CHECK(c, ...) do { if (!(c)) { if (bad < 20) printf(__VA_ARGS__); ++bad; } } while (0)

// pivot-column bitsets of the lower triangle of a front
struct Cov {
    int m, c, w;
    std::vector<uint64_t> b;
    Cov(int m_, int c_) : m(m_), c(c_), w((c_ + 63) / 64), b((size_t)m_ * (m_ + 1) / 2 * ((c_ + 63) / 64), 0) {}
    size_t at(int r, int q) const { return ((size_t)q * (2 * (size_t)m - q + 1) / 2 + (r - q)) * w; }
    // pivots [k0, k1) applied to entry (r, q)
    void mark(int r, int q, int k0, int k1, const char *what) {
        const int need = q < c ? q : c;
        CHECK(k0 >= 0 && k1 <= need, "%s: entry (%d,%d) of (%d,%d) gets pivots [%d,%d), needs < %d\n", what, r, q, m,
              c, k0, k1, need);
        uint64_t *e = &b[at(r, q)];
        for (int k = k0; k < k1 && k < c; ++k) {
            const uint64_t bit = 1ull << (k & 63);
            CHECK(!(e[k >> 6] & bit), "%s: entry (%d,%d) of (%d,%d) gets pivot %d twice\n", what, r, q, m, c, k);
            e[k >> 6] |= bit;
        }
    }
    void done(const char *name) {
        for (int q = 0; q < m; ++q)
            for (int r = q; r < m; ++r) {
                const uint64_t *e = &b[at(r, q)];
                const int need = q < c ? q : c;
                for (int k = 0; k < c; ++k) {
                    const bool set = (e[k >> 6] >> (k & 63)) & 1;
                    CHECK(set == (k < need), "%s: entry (%d,%d) of (%d,%d) pivot %d %s\n", name, r, q, m, c, k,
                          set ? "extra" : "missing");
                }
            }
    }
};

static void run(const char *name, const std::vector<FD> &fd, bool lookahead, int outer, int inner,
                int big_rows_chain = 0) {
    std::vector<int32_t> fl, buf;
    for (int i = 0; i < (int)fd.size(); ++i) fl.push_back(i);
    std::vector<StepHost> steps;
    plan_steps(fd, fl, buf, steps, lookahead, 512, outer, inner, big_rows_chain);
    std::vector<Cov> cov;
    for (const FD &f : fd) cov.emplace_back(f.m, f.c);
    for (const StepHost &s : steps) {
        if (s.kind == SYNC_TO_SIDE || s.kind == SYNC_TO_MAIN) continue;
        int tot = 0;
        for (int i = 0; i < s.nf; ++i) {
            const int f = buf[s.fl_off + i];
            const int m = fd[f].m, c = fd[f].c, t0 = s.t0, pe = s.pe;
            const int nt = step_tasks(s.kind, t0, pe, c, m, s.win);
            CHECK(c > t0 && nt > 0, "%s: front %d listed in a step with no work\n", name, f);
            CHECK(buf[s.pre_off + i] == tot, "%s: task prefix\n", name);
            tot += nt;
            Cov &cv = cov[f];
            const int nb = std::min(PIVOT_NB, c - t0);
            if (s.kind == 0) {
                for (int q = t0; q < t0 + nb; ++q)
                    for (int r = q; r < t0 + nb; ++r) cv.mark(r, q, t0, q, "pivot block");
            } else if (s.kind == 1) {
                const int mr = s.win == 3 ? std::min(pe, c) : m;
                for (int q = t0; q < t0 + nb; ++q)
                    for (int r = t0 + nb; r < mr; ++r) cv.mark(r, q, t0, q, "rows below a block");
            } else if (s.kind == 7) {
                const int cend = std::min(pe, c);
                for (int q = t0; q < cend; ++q)
                    for (int r = cend; r < m; ++r) cv.mark(r, q, t0, q, "rows below a sub-panel");
            } else {
                const UpdGeom g = upd_geom(s.kind == 2 ? 2 : 3, t0, pe, c, m, s.win);
                const int mr = (s.kind == 2 && s.win == 3) ? g.qhi : m;
                for (int q = g.lo; q < g.qhi; ++q)
                    for (int r = q; r < mr; ++r) cv.mark(r, q, t0, t0 + g.K, s.kind == 2 ? "panel update" : "trailing update");
            }
        }
        CHECK(tot == s.ntasks, "%s: task count %d vs %d\n", name, tot, s.ntasks);
    }
    for (Cov &cv : cov) cv.done(name);
}

int main() {
    const std::vector<FD> periods = {{700, 600}, {640, 300}, {520, 512}, {600, 257}, {300, 250}, {700, 700},
                                     {130, 65},  {200, 64},  {1300, 260}, {1350, 513}};
    run("periods 512/256", periods, false, 512, 256);
    run("periods 256/256", periods, false, 256, 256);
    run("periods 512/256 with lookahead", periods, true, 512, 256);
    for (int n : {1100, 1024, 1300, 800, 2600}) {
        run("dense with lookahead", std::vector<FD>{{n, n}}, true, 512, 256);
        run("dense with lookahead, 64x64 chain updates below 1500 rows", std::vector<FD>{{n, n}}, true, 512, 256, 1500);
        // three sub-panels asked for: the plan keeps two per outer panel
        run("dense with lookahead, 768-wide outer panels asked for", std::vector<FD>{{n, n}}, true, 768, 256);
    }
    printf("bad %ld\n", bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_step_plan_applies_every_pivot_once(tmp_path):
    src = tmp_path / "step_plan.cpp"
    src.write_text(PROG)
    exe = tmp_path / "step_plan"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:]
    assert "bad 0" in r.stdout
