// Tile order of the dense trailing update (host and device; the host side
// serves the tests of the order).
#pragma once

namespace kkt {

// Tile order of a single-front trailing update (one launch row): workgroup b
// runs on XCD b % 8 (the dispatcher deals workgroups round-robin over the 8
// XCDs), and XCD x takes a contiguous share of an order that walks the
// trapezoid in groups of 8 tile columns, row by row inside a group. The tiles
// resident on one XCD at a time then span about 8 row and 8 column panels,
// which its L2 serves to all of them, instead of one column and every row.
__host__ __device__ inline void trap_decode_xcd(int b, int Tr, int Tc, int &ti, int &tj) {
    const int T = Tc * Tr - Tc * (Tc - 1) / 2;
    const int q = T >> 3, r = T & 7, x = b & 7, k = b >> 3;
    int L = x * q + (x < r ? x : r) + k;
    for (int c0 = 0; c0 < Tc; c0 += 8) {
        const int wg = Tc - c0 < 8 ? Tc - c0 : 8;
        const int tri = wg * (wg + 1) / 2;
        const int size = tri + wg * (Tr - c0 - wg);
        if (L < size) {
            if (L < tri) {
                int s = 0;
                while ((s + 1) * (s + 2) / 2 <= L) ++s;
                ti = c0 + s;
                tj = c0 + L - s * (s + 1) / 2;
            } else {
                const int u = L - tri;
                ti = c0 + wg + u / wg;
                tj = c0 + u % wg;
            }
            return;
        }
        L -= size;
    }
    ti = Tr;  // only for b outside the trapezoid's tile count
    tj = 0;
}

}  // namespace kkt
