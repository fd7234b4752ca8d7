"""Host check of the dense trailing update's XCD-aware tile order (no GPU
needed): the header is compiled with the host compiler, and for every
trapezoid of Tr row tiles and Tc <= Tr column tiles the workgroup ids
0..T-1 must map one-to-one onto the tiles (ti, tj) with tj < Tc and
tj <= ti < Tr. A tile visited twice or missed would leave part of the
trailing matrix updated twice or not at all."""
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1907_05420_amd", "csrc")

PROG = r"""
#define __host__
#define __device__
#include "tile_order.hpp"
#include <cstdio>
#include <vector>
int main() {
    long bad = 0, cases = 0;
    for (int Tr = 1; Tr <= 240; ++Tr)
        for (int Tc = 1; Tc <= Tr; ++Tc) {
            const int T = Tc * Tr - Tc * (Tc - 1) / 2;
            std::vector<int> seen((size_t)Tr * Tc, 0);
            for (int b = 0; b < T; ++b) {
                int ti = -1, tj = -1;
                kkt::trap_decode_xcd(b, Tr, Tc, ti, tj);
                if (ti < 0 || ti >= Tr || tj < 0 || tj >= Tc || tj > ti) { ++bad; continue; }
                seen[(size_t)ti * Tc + tj]++;
            }
            for (int ti = 0; ti < Tr; ++ti)
                for (int tj = 0; tj < Tc && tj <= ti; ++tj) bad += seen[(size_t)ti * Tc + tj] != 1;
            ++cases;
        }
    // the first 64 tiles of every XCD in a 150 x 150 trapezoid (the first
    // panel of a 19200-wide S) touch at most 22 distinct row and column
    // panels (8 columns and 8 to 12 rows; the column-by-column order gives 65)
    for (int x = 0; x < 8; ++x) {
        const int Tr = 150, Tc = 150;
        std::vector<int> rows(Tr, 0), cols(Tc, 0);
        int nr = 0, nc = 0;
        for (int k = 0; k < 64; ++k) {
            int ti, tj;
            kkt::trap_decode_xcd(8 * k + x, Tr, Tc, ti, tj);
            nr += !rows[ti]++;
            nc += !cols[tj]++;
        }
        if (nr + nc > 22) { printf("xcd %d panels %d %d\n", x, nr, nc); ++bad; }
    }
    printf("cases %ld bad %ld\n", cases, bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_xcd_tile_order_is_a_bijection_onto_the_trapezoid(tmp_path):
    src = tmp_path / "order.cpp"
    src.write_text(PROG)
    exe = tmp_path / "order"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout
