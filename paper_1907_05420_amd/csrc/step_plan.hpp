// Step plan of the blocked factorisation of a group of fronts (host) and the
// update geometry its kernels share (host and device; the host side serves
// the tests of the plan). A front of m rows holds its c pivot columns as a
// column-major panel and its update block beyond them; a step is one launch
// over all listed fronts that still have pivots at its first column.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#endif

namespace kkt {

constexpr int PIVOT_NB = 64;   // pivot block width
constexpr int BIG_TILE = 128;  // tile edge of the large trailing-update kernel

// Geometry of an update after the pivot columns [t0, t0+K): target rows and
// columns start at lo; columns end at qhi. kind 2: inside the sub-panel
// ending at pe; kind 3: the trailing matrix after the panel [t0, pe).
struct UpdGeom {
    int lo, qhi, K;
};
// win (trailing updates only): 0 the whole trailing matrix; 1 the columns of
// the next panel of the same width (up to the front's last pivot); 2
// everything right of the next panel.
__host__ __device__ inline UpdGeom upd_geom(int kind, int t0, int pe, int c, int m, int win = 0) {
    const int cend = pe < c ? pe : c;
    UpdGeom g;
    if (kind == 2) {
        g.K = (c - t0) < PIVOT_NB ? (c - t0) : PIVOT_NB;
        g.lo = t0 + g.K;
        g.qhi = cend;
        (void)win;  // win 3 (rows below the panel left out) is applied by the caller's row limit
    } else {
        g.K = cend - t0;
        g.lo = cend;
        g.qhi = m;
        // the next panel has the width of this one (pe - t0); its columns
        // end at the front's last pivot, and the rest (win 2) starts there
        // at the latest: the update block's columns take the whole outer
        // panel's update with the rest
        const int nxt = pe + (pe - t0) < m ? pe + (pe - t0) : m;
        if (win == 1) g.qhi = nxt < c ? nxt : c;
        else if (win == 2) g.lo = nxt < c ? nxt : c;
    }
    return g;
}

// workgroups of a step on one front
inline int step_tasks_big(int t0, int pe, int c, int m, int win) {
    const UpdGeom g = upd_geom(3, t0, pe, c, m, win);
    if (g.K <= 0 || g.qhi <= g.lo) return 0;
    const int Tr = (m - g.lo + BIG_TILE - 1) / BIG_TILE, Tc = (g.qhi - g.lo + BIG_TILE - 1) / BIG_TILE;
    return Tc * Tr - Tc * (Tc - 1) / 2;
}
inline int step_tasks(int kind, int t0, int pe, int c, int m, int win = 0) {
    if (kind == 4) return step_tasks_big(t0, pe, c, m, win);
    if (kind == 0) return c > t0 ? 1 : 0;
    if (kind == 1) {
        const int nb = std::min(PIVOT_NB, c - t0);
        const int rows = (win == 3 ? std::min(pe, c) : m) - t0 - nb;
        return rows > 0 ? (rows + 63) / 64 : 0;
    }
    if (kind == 7) {
        const int rows = m - std::min(pe, c);
        return c > t0 && rows > 0 ? (rows + 63) / 64 : 0;
    }
    const UpdGeom g = upd_geom(kind, t0, pe, c, m, win);
    if (g.K <= 0 || g.qhi <= g.lo) return 0;
    const int mr = (kind == 2 && win == 3) ? g.qhi : m;
    const int Tr = (mr - g.lo + 63) / 64, Tc = (g.qhi - g.lo + 63) / 64;
    return Tc * Tr - Tc * (Tc - 1) / 2;
}

// kind 0-7: launches (see StepDev); SYNC_TO_SIDE: the side stream waits for
// the main stream's work so far; SYNC_TO_MAIN: the main stream waits for the
// side stream's work so far.
constexpr int SYNC_TO_SIDE = 100, SYNC_TO_MAIN = 101;
constexpr int PANEL_ROWS = 1024;  // rows below a sub-panel from which its rows below take one launch
struct StepHost {
    int kind, win, t0, pe, nf, ntasks;
    int side;                 // 0: main stream, 1: side stream
    int64_t fl_off, pre_off;  // offsets (int32 elements) into the task buffer
};

// launch sequence of the blocked factorisation of a set of fronts
// With lookahead (dense Schur), each trailing update is split: the next
// panel's columns on the main stream, the rest on the side stream, so that the
// latency-bound factorisation of the next panel overlaps the large update.
// big_rows_chain (0: big_rows) is the threshold for the updates on the
// panel chain (the next sub-panel's and, with lookahead, the next panel's
// columns): there the launch's parallelism decides, and 64x64 tiles give
// four times the workgroups of 128x128 ones.
template <class FD>
void plan_steps(const std::vector<FD> &fd, const std::vector<int32_t> &fl, std::vector<int32_t> &buf,
                std::vector<StepHost> &steps, bool lookahead, int big_rows, int outer_w, int inner_w,
                int big_rows_chain = 0) {
    if (big_rows_chain <= 0) big_rows_chain = big_rows;
    // sub-panels of at most four pivot blocks (k_panel_trsm), at most two per
    // outer panel: a finished sub-panel updates only the next sub-panel's
    // columns (the next panel of its width, upd_geom win 1)
    if (inner_w > 4 * PIVOT_NB) inner_w = 4 * PIVOT_NB;
    if (outer_w > 2 * inner_w) outer_w = 2 * inner_w;
    int cmax = 0;
    for (int32_t f : fl) cmax = std::max(cmax, fd[f].c);
    auto sync = [&](int kind) {
        StepHost s{};
        s.kind = kind;
        steps.push_back(s);
    };
    auto add = [&](int kind, int t0, int pe, int win = 0, int side = 0) {
        std::vector<int32_t> act;
        std::vector<int> cnt;
        for (int32_t f : fl) {
            if (fd[f].c <= t0) continue;
            int k = step_tasks(kind, t0, pe, fd[f].c, fd[f].m, win);
            if (k <= 0) continue;
            act.push_back(f);
            cnt.push_back(k);
        }
        if (act.empty()) return;
        StepHost s{};
        s.kind = kind;
        s.win = win;
        s.side = side;
        s.t0 = t0;
        s.pe = pe;
        s.nf = (int)act.size();
        s.fl_off = (int64_t)buf.size();
        buf.insert(buf.end(), act.begin(), act.end());
        s.pre_off = (int64_t)buf.size();
        int acc = 0;
        for (int k : cnt) { buf.push_back(acc); acc += k; }
        buf.push_back(acc);
        s.ntasks = acc;
        steps.push_back(s);
    };
    // large trailing matrices (rows below column `col`) take the 128x128 tile kernel
    auto big_from = [&](int t0, int col, int rows = -1) {
        if (rows < 0) rows = big_rows;
        for (int32_t f : fl)
            if (fd[f].c > t0 && fd[f].m - std::min(col, fd[f].c) >= rows) return 1;
        return 0;
    };
    for (int k = 0; k < cmax; k += outer_w) {
        const int pe = k + outer_w;
        // the panel's columns were brought up to date by the main stream's
        // update from the previous panel, after the side stream had finished
        // the updates of the panels before it; the side stream's update from
        // the previous panel (columns beyond this panel) runs meanwhile.
        // Inside the panel, sub-panels of inner_w columns: 64-column steps
        // update only their own sub-panel, and each finished sub-panel updates
        // the next sub-panel's columns in one rank-inner_w product.
        for (int s0 = k; s0 < std::min(pe, cmax); s0 += inner_w) {
            const int se = std::min(s0 + inner_w, pe);
            // where the fronts have many rows below the sub-panel (the dense
            // Schur factor, the largest period fronts) the 64-column steps
            // stay inside the sub-panel's diagonal block, and the rows below
            // it take all of the sub-panel's columns in one launch. Fronts
            // with few rows below (most period fronts, the structured Schur's
            // 2 N_s x N_s fronts) keep the per-block steps: there the
            // one-launch form's per-tile chain of products is the slower one.
            int below = 0;
            for (int32_t f : fl)
                if (fd[f].c > s0) below = std::max(below, fd[f].m - std::min(se, fd[f].c));
            const bool one_launch = lookahead || below >= PANEL_ROWS;
            for (int j0 = s0; j0 < std::min(se, cmax); j0 += 64) {
                add(0, j0, se);
                add(1, j0, se, one_launch ? 3 : 0);
                add(2, j0, se, one_launch ? 3 : 0);
            }
            if (one_launch) add(7, s0, se);
            if (se < std::min(pe, cmax)) add(big_from(s0, se, big_rows_chain) ? 4 : 3, s0, se, 1, 0);
        }
        const int big = big_from(k, pe);
        if (!lookahead) {
            add(big ? 4 : 3, k, pe);
            continue;
        }
        // the next panel's columns: the side stream's update from the
        // previous panel must be done before this panel's update of them
        if (k > 0) sync(SYNC_TO_MAIN);
        add(big_from(k, pe, big_rows_chain) ? 4 : 3, k, pe, 1, 0);  // next panel's columns, main stream
        // the side stream updates the columns beyond the next panel once the
        // main stream's update of the next panel's columns is done: started
        // together, the large update takes the compute units first and the
        // next panel (the critical path) waits behind it
        sync(SYNC_TO_SIDE);
        add(big ? 4 : 3, k, pe, 2, 1);  // the rest, side stream
    }
    if (lookahead) sync(SYNC_TO_MAIN);
}

}  // namespace kkt
