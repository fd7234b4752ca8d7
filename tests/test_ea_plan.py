"""Host check of the extend-add task lists (no GPU needed): the header that
plans them is compiled with the host compiler together with the symbolic
analysis, the lists of every level are built for real structures, and then

  * every entry (i, j), j <= i, of every child's update block is added by
    exactly one segment, inside the tile that holds its target (rel[i],
    rel[j]) in the parent front;
  * every entry (r, q), c <= q <= r, of every large front's update block
    lies in exactly one listed tile (the tile clears it before the adds);
  * no tile is listed twice.

Structures: the 2000-bus network in the elimination orders with dual wait 4
(the library default) and 2, and a 160-bus network (several large fronts)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import kktgen

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_1907_05420_amd", "csrc")

PROG = r"""
#include "symbolic.hpp"
#include "ea_plan.hpp"
#include <cstdio>
#include <fstream>
#include <map>
#include <tuple>
#include <vector>
using namespace kkt;

static long bad = 0;
#define CHECK(c, ...) do { if (!(c)) { if (bad < 20) printf(__VA_ARGS__); ++bad; } } while (0)

template <class T> static std::vector<T> rd(const std::string &f) {
    std::ifstream s(f, std::ios::binary | std::ios::ate);
    const size_t n = s.tellg();
    s.seekg(0);
    std::vector<T> v(n / sizeof(T));
    s.read((char *)v.data(), n);
    return v;
}

int main(int argc, char **argv) {
    const std::string dir = argv[1];
    long nA, np_, Ns;
    std::ifstream dims(dir + "/dims.txt");
    dims >> nA >> np_ >> Ns;
    const auto cp = rd<int64_t>(dir + "/colptr.bin");
    const auto ri = rd<int32_t>(dir + "/rowind.bin");
    const auto c0p = rd<int64_t>(dir + "/C0p.bin"), c1p = rd<int64_t>(dir + "/C1p.bin");
    const auto c0i = rd<int32_t>(dir + "/C0i.bin"), c1i = rd<int32_t>(dir + "/C1i.bin");
    SymbolicInput in;
    in.nA = nA; in.n_primal = np_; in.Ns = Ns;
    in.colptr = cp.data(); in.rowind = ri.data();
    in.C0p = c0p.data(); in.C0i = c0i.data(); in.C1p = c1p.data(); in.C1i = c1i.data();
    in.dual_wait = atoi(argv[2]);
    Symbolic S;
    const std::string err = analyze(in, S);
    if (!err.empty()) { printf("analysis: %s\n", err.c_str()); return 1; }
    long ntiles = 0, nadds = 0;
    for (int l = 0; l < S.nlevels; ++l) {
        std::vector<int32_t> large, buf;
        for (int q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q)
            if (S.nrow[S.level_list[q]] > 64) large.push_back(S.level_list[q]);
        const int nt = plan_extend_add(S, large, buf);
        ntiles += nt;
        // adds of every child entry, per child (lower triangles, i * uc + j)
        std::map<int, std::vector<unsigned char>> added;
        std::map<std::tuple<int, int, int>, int> seen;
        std::map<int, std::vector<unsigned char>> cleared;  // per front, (r - c) * u + (q - c)
        for (int32_t t : large) {
            const int u = S.nrow[t] - S.ncol[t];
            cleared[t].assign((size_t)u * u, 0);
            for (int32_t k = S.child_ptr[t]; k < S.child_ptr[t + 1]; ++k) {
                const int ch = S.child_list[k], uc = S.nrow[ch] - S.ncol[ch];
                added[ch].assign((size_t)uc * uc, 0);
            }
        }
        for (int x = 0; x < nt; ++x) {
            const int32_t *tk = buf.data() + 8 * x;
            const int t = tk[0], r0 = tk[1], c0 = tk[2], seg = tk[3], nseg = tk[4];
            const int m = S.nrow[t], c = S.ncol[t];
            const int r1 = std::min(r0 + 64, m), c1 = std::min(c0 + EA_CW, r1);
            CHECK(r0 % 64 == 0 && c0 % EA_CW == 0 && c0 < r1, "level %d: tile (%d, %d) of front %d misplaced\n", l,
                  r0, c0, t);
            CHECK(seen[std::make_tuple(t, r0, c0)]++ == 0, "level %d: tile (%d, %d) of front %d twice\n", l, r0,
                  c0, t);
            for (int r = std::max(r0, c); r < r1; ++r)
                for (int q = std::max(c0, c); q < c1 && q <= r; ++q) cleared[t][(size_t)(r - c) * (m - c) + (q - c)]++;
            for (int k = 0; k < nseg; ++k) {
                const int32_t *sg = buf.data() + seg + EA_SEG * k;  // tiles start at buf[0]
                const int ch = sg[0], ilo = sg[1], ihi = sg[2], jlo = sg[3], jhi = sg[4];
                const int uc = S.nrow[ch] - S.ncol[ch];
                const int32_t *rl = S.rel.data() + S.relptr[ch];
                CHECK(S.parent[ch] == t, "level %d: segment of child %d in front %d\n", l, ch, t);
                CHECK(0 <= ilo && ilo < ihi && ihi <= uc && 0 <= jlo && jlo < jhi && jhi <= ihi,
                      "level %d: segment ranges of child %d\n", l, ch);
                for (int i = ilo; i < ihi; ++i) {
                    CHECK(rl[i] >= r0 && rl[i] < r1, "level %d: child %d row %d outside its tile\n", l, ch, i);
                    for (int j = jlo; j < jhi && j <= i; ++j) {
                        CHECK(rl[j] >= c0 && rl[j] < c1, "level %d: child %d column %d outside its tile\n", l, ch, j);
                        added[ch][(size_t)i * uc + j]++;
                        ++nadds;
                    }
                }
            }
        }
        for (auto &kv : added) {
            const int ch = kv.first, uc = S.nrow[ch] - S.ncol[ch];
            for (int i = 0; i < uc; ++i)
                for (int j = 0; j <= i; ++j)
                    CHECK(kv.second[(size_t)i * uc + j] == 1, "level %d: child %d entry (%d,%d) added %d times\n", l,
                          ch, i, j, kv.second[(size_t)i * uc + j]);
        }
        for (auto &kv : cleared) {
            const int t = kv.first, u = S.nrow[t] - S.ncol[t];
            for (int r = 0; r < u; ++r)
                for (int q = 0; q <= r; ++q)
                    CHECK(kv.second[(size_t)r * u + q] == 1, "level %d: front %d update entry (%d,%d) in %d tiles\n",
                          l, t, r, q, kv.second[(size_t)r * u + q]);
        }
    }
    printf("tiles %ld adds %ld bad %ld\n", ntiles, nadds, bad);
    return bad != 0;
}
"""


def _dump(inst, d):
    os.makedirs(d, exist_ok=True)
    np.asarray(inst.colptr, dtype=np.int64).tofile(os.path.join(d, "colptr.bin"))
    np.asarray(inst.rowind, dtype=np.int32).tofile(os.path.join(d, "rowind.bin"))
    for name, a, dt in (("C0p", inst.C0_rowptr, np.int64), ("C0i", inst.C0_colind, np.int32),
                        ("C1p", inst.C1_rowptr, np.int64), ("C1i", inst.C1_colind, np.int32)):
        np.asarray(a, dtype=dt).tofile(os.path.join(d, name + ".bin"))
    with open(os.path.join(d, "dims.txt"), "w") as f:
        f.write(f"{inst.n_A} {inst.n_primal} {inst.ns}\n")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_extend_add_tiles_cover_every_entry_once(tmp_path):
    src = tmp_path / "ea_plan.cpp"
    src.write_text(PROG)
    exe = tmp_path / "ea_plan"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), os.path.join(CSRC, "symbolic.cpp"), "-o",
                    str(exe)], check=True)
    cases = [(kktgen.make_workload(2, N=2), 4), (kktgen.make_workload(2, N=2), 2),
             (kktgen.make_small(nb=160, nextra=90, ng=30, ns=12, N=2, nrhs=1, seed=8), 4)]
    for k, (inst, dw) in enumerate(cases):
        d = str(tmp_path / f"s{k}")
        _dump(inst, d)
        r = subprocess.run([str(exe), d, str(dw)], capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, (k, r.stdout[-3000:])
        assert "bad 0" in r.stdout
