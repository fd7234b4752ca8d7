// Task lists of the extend-add (host side; the layout is shared with the
// kernel). The children's update blocks are added into tiles of 64 rows by
// EA_CW columns of the lower triangle of each large front; a tile lists the
// children whose update rows and columns reach it, with those ranges (the
// relative indices of a child increase, so each range is contiguous).
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

namespace kkt {

// Extend-add into the tile of rows [r0, r0 + 64) and columns [c0, c0 +
// EA_CW) of front f: nseg segments of EA_SEG int32 at seg int32 past the
// first task of the list, each (child, i_lo, i_hi, j_lo, j_hi): the child's
// update rows [i_lo, i_hi) land in the tile's rows and its update columns
// [j_lo, j_hi) in the tile's columns; children in increasing order.
struct EaTask {
    int32_t f, r0, c0, seg, nseg, pad0, pad1, pad2;
};
constexpr int EA_CW = 256;  // columns of an extend-add tile
constexpr int EA_SEG = 5;   // int32 per segment

// Tiles (EaTask as 8 int32 each, segment offsets counted from the first
// task) followed by their segments, for the fronts `large` of a supernodal
// structure SY (fields nrow, ncol, child_ptr, child_list, relptr, rel). A
// tile without segments is kept where it holds entries of the front's
// update block (rows and columns at or past the pivots): the kernel clears
// those first. Returns the number of tiles.
template <class SY>
int plan_extend_add(const SY &S, const std::vector<int32_t> &large, std::vector<int32_t> &out) {
    std::vector<int32_t> tiles, segs, rows_of;  // rows_of: (child, i_lo, i_hi) of a row tile
    for (int32_t t : large)
        for (int r0 = 0; r0 < S.nrow[t]; r0 += 64) {
            const int r1 = std::min(r0 + 64, (int)S.nrow[t]);
            rows_of.clear();
            for (int32_t k = S.child_ptr[t]; k < S.child_ptr[t + 1]; ++k) {
                const int32_t ch = S.child_list[k];
                const int32_t *rl = S.rel.data() + S.relptr[ch];
                const int uc = S.nrow[ch] - S.ncol[ch];
                const int lo = (int)(std::lower_bound(rl, rl + uc, r0) - rl);
                const int hi = (int)(std::lower_bound(rl + lo, rl + uc, r1) - rl);
                if (lo < hi) rows_of.insert(rows_of.end(), {ch, lo, hi});
            }
            for (int c0 = 0; c0 < r1; c0 += EA_CW) {
                const int c1 = std::min(c0 + EA_CW, r1);
                const int32_t s0 = (int32_t)segs.size();
                for (size_t q = 0; q < rows_of.size(); q += 3) {
                    const int32_t ch = rows_of[q], lo = rows_of[q + 1], hi = rows_of[q + 2];
                    const int32_t *rl = S.rel.data() + S.relptr[ch];
                    // columns j < hi only: the kernel takes j <= i
                    const int jl = (int)(std::lower_bound(rl, rl + hi, c0) - rl);
                    const int jh = (int)(std::lower_bound(rl + jl, rl + hi, c1) - rl);
                    if (jl < jh) segs.insert(segs.end(), {ch, lo, hi, jl, jh});
                }
                const int nseg = ((int32_t)segs.size() - s0) / EA_SEG;
                const bool clears = r1 > S.ncol[t] && c1 > S.ncol[t];
                if (nseg > 0 || clears) tiles.insert(tiles.end(), {t, r0, c0, s0, nseg, 0, 0, 0});
            }
        }
    for (size_t q = 0; q < tiles.size(); q += 8) tiles[q + 3] += (int32_t)tiles.size();
    out.insert(out.end(), tiles.begin(), tiles.end());
    out.insert(out.end(), segs.begin(), segs.end());
    return (int)(tiles.size() / 8);
}

}  // namespace kkt
