// C-ABI context: symbolic analysis upload, the numeric factorisation of all
// period blocks and of the Schur complement, and the refined solve
// (Algorithm 1 of section 4.2 on one device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/kkt.h"
#include "device.hpp"
#include "step_plan.hpp"
#include "footprint.hpp"
#include "kernels.hpp"
#include "symbolic.hpp"

namespace kkt {
SymbolicInput make_input(const kkt_structure *s, const kkt_options &o);
void fill_stats(const Symbolic &S, kkt_symbolic_stats *st);
}

using namespace kkt;

#define HIPCHK(x)                                                                                 \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) {                                                                   \
            if (ctx && ctx->opt.verbose) std::fprintf(stderr, "kkt: %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
            return e_ == hipErrorOutOfMemory ? KKT_ERR_NOMEM : KKT_ERR_HIP;                       \
        }                                                                                         \
    } while (0)

namespace {

struct LevelPlan {
    int64_t small_off = 0, all_off = 0, ea_off = 0, large_off = 0;  // int32 offsets into the task buffer
    int64_t rrow_off = 0, rcol_off = 0;                             // RowTask lists of the solve
    int nsmall = 0, nall = 0, nea = 0, nlarge = 0, nrrow = 0, nrcol = 0;
    int nsmall_cls[3] = {0, 0, 0};  // small fronts of <= 16, <= 32, <= 64 rows (listed in that order)
    int maxm = 0, maxm_large = 0, maxc_large = 0;
    int step_begin = 0, step_end = 0;
    int win_begin = 0, win_end = 0;  // pivot windows of the wide fronts (solve)
    int maxc_wide = 0;
};

// a pivot window of the solve's wide fronts as offsets into the task buffer
struct WindowPlan {
    int p0 = 0, nfront = 0, nrows = 0, ncols = 0;
    int64_t f_off = 0, r_off = 0, c_off = 0;
};

}  // namespace

struct kkt_ctx {
    hipStream_t stream = nullptr;
    bool dry = false;  // planning only: allocations and uploads are counted, not made
    kkt_options opt{};
    int device = 0;
    bool analyzed = false, factored = false;
    Symbolic sy;
    int64_t N = 0, ng = 0, ntot = 0;
    // periods whose factors and update matrices are held at a time: N, or
    // fewer with recompute_periods (factors recomputed in every solve pass,
    // the memory-saving variant of section 4.3); the chunk of periods whose
    // factor the storage holds now (-1: none); the local Schur blocks of
    // every period, copied out of the update storage chunk by chunk
    int64_t P = 0;
    int64_t resident = -1;
    void *d_sbar = nullptr;
    double eps = 1e-14;
    std::vector<std::pair<void *, size_t>> allocs;  // static allocations
    size_t bytes_static = 0, bytes_ws = 0;

    // symbolic device data
    int64_t *d_amap = nullptr, *d_c0map = nullptr, *d_c1map = nullptr, *d_rowptr = nullptr, *d_relptr = nullptr;
    int8_t *d_adiag = nullptr, *d_pivsign = nullptr;
    int32_t *d_adpiv = nullptr, *d_rows = nullptr, *d_cptr = nullptr, *d_clist = nullptr, *d_rel = nullptr;
    int32_t *d_vea = nullptr;  // children's update rows of every front in groups (TreeArgs::vea)
    int32_t *d_perm = nullptr, *d_tasks = nullptr;
    FrontDesc *d_sd = nullptr;
    std::vector<LevelPlan> levels;
    std::vector<WindowPlan> win_plan;
    std::vector<TriWindow> win;            // win_plan with device pointers
    std::vector<StepHost> steps, ssteps;   // sparse levels, Schur
    int32_t *d_stasks = nullptr;           // Schur step tasks
    FrontDesc *d_sdS = nullptr;
    // residual: K's pattern as sliced ELLPACK (64-row slices) with the values
    // of every period in that order (shifts included), rebuilt per factorisation
    int64_t nnz_sell = 0;
    int64_t *d_sl_off = nullptr;
    int32_t *d_sl_ci = nullptr, *d_sl_vi = nullptr;
    double *d_Asell = nullptr;
    int64_t *d_c1tp = nullptr, *d_c0tp = nullptr, *d_c1tk = nullptr,
            *d_c0tk = nullptr, *d_c0p = nullptr, *d_c1p = nullptr;
    int32_t *d_c1ts = nullptr, *d_c0ts = nullptr, *d_c0i = nullptr, *d_c1i = nullptr;
    // numeric
    void *d_L = nullptr, *d_U = nullptr;
    double *d_tau = nullptr, *d_amax = nullptr;
    int64_t *d_cnt = nullptr;
    int *d_flag = nullptr;
    double *d_A = nullptr, *d_C0 = nullptr, *d_C1 = nullptr, *d_corner = nullptr;
    bool has_corner = false;
    double dw = 0.0, dc = 0.0;
    double *d_S = nullptr, *d_prefix = nullptr, *d_tauS = nullptr, *d_amaxS = nullptr;
    double *d_invtmp = nullptr;  // staging of the block-inverse combinations
    int *d_dsync = nullptr;      // dense Schur solves: [0] failure flag, then the step counters
    // structured Schur (section 4.3): the N fronts [A_j; B_j] (2 Ns x Ns, ld
    // 2 Ns; Ns x Ns for the last), G_j = W_j Linv_j and its transpose, the
    // running U_j and the update block of the current front, and the solve's
    // recurrences; two planned fronts (full, last) and their launch sequences
    bool structured = false;
    double *d_sfront = nullptr, *d_sG = nullptr, *d_sGT = nullptr, *d_sU = nullptr, *d_sUb = nullptr;
    double *d_sM = nullptr, *d_sMT = nullptr, *d_sce = nullptr;  // column pairs of the structured solves
    double *d_ssa = nullptr, *d_saa = nullptr;
    FrontDesc *d_sfd = nullptr;
    int32_t *d_sftasks = nullptr;
    std::vector<StepHost> sf_steps[2];
    int64_t *d_cntS = nullptr;
    // solve workspace
    int64_t ws_nrhs = 0;
    std::vector<void *> ws;
    double *d_xp = nullptr, *d_uv = nullptr, *d_bh = nullptr, *d_y = nullptr, *d_xg = nullptr, *d_res = nullptr,
           *d_dx = nullptr, *d_norms = nullptr, *d_work = nullptr;
    // flexible GMRES: bases V (KRYLOV_M + 1 blocks) and Z (KRYLOV_M blocks) of
    // [nrhs][ntot]; coefficients h1, h2 ([nrhs][ldh] each), norms [nrhs], y
    // [nrhs][ldh] on the device with a pinned host mirror; reduction partials
    double *d_V = nullptr, *d_Z = nullptr, *d_h = nullptr, *d_kpart = nullptr, *h_pin = nullptr;
    // side stream and events of the lookahead
    hipStream_t side = nullptr;
    hipEvent_t ev_main = nullptr, ev_side = nullptr, ev_asm = nullptr;
    // timing
    bool timing = false;
    hipEvent_t ev[8] = {};
    double times[5] = {0, 0, 0, 0, 0};
    // per-launch events of the Schur trailing-update kernel (timing only)
    std::vector<hipEvent_t> kev;
    int64_t kcount = 0;
    kkt_kernel_stat kstat{};
    // trailing matrices with at least this many rows use the 128x128 tiles
    int big_rows = 512;
    // last kkt_solve_async / kkt_solve_noalloc: its right-hand sides, steps
    // and where it left the norms of the final residual (the workspace's
    // norms, or d_snorms, a context-owned buffer for 64 right-hand sides)
    int64_t async_nrhs = 0;
    int async_steps = 0;
    double *d_snorms = nullptr;
    const double *status_norms = nullptr;
    // FP64 fallback of the mixed path: a copy of the pattern, an FP64
    // context created on first use (its own FP64 order and factors), whether
    // the current values are factored there and the last solve used it
    std::vector<int64_t> pat_colptr, pat_C0p, pat_C1p;
    std::vector<int32_t> pat_rowind, pat_C0i, pat_C1i;
    int64_t pat_n_primal = 0, pat_Ns = 0;
    kkt_ctx *fb = nullptr;
    bool fb_factored = false;
    kkt_inertia fb_inertia{};
    // eliminated slacks (kkt_set_slacks): their flow rows and the positions
    // of those rows' diagonal entries in A_vals
    int64_t n_slack = 0;
    int32_t *d_slack_row = nullptr;
    int64_t *d_slack_dpos = nullptr;
    std::vector<void *> slack_allocs;
};

namespace {

int dalloc(kkt_ctx *ctx, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return KKT_OK;
    bytes = align_up(bytes);
    if (ctx->dry) {
        ctx->bytes_static += bytes;
        return KKT_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) { *p = nullptr; return e == hipErrorOutOfMemory ? KKT_ERR_NOMEM : KKT_ERR_HIP; }
    ctx->allocs.emplace_back(*p, bytes);
    ctx->bytes_static += bytes;
    return KKT_OK;
}

template <typename V>
int upload(kkt_ctx *ctx, V **dst, const std::vector<V> &src) {
    int rc = dalloc(ctx, (void **)dst, sizeof(V) * std::max<size_t>(src.size(), 1));
    if (rc) return rc;
    if (!src.empty() && !ctx->dry)
        HIPCHK(hipMemcpy(*dst, src.data(), sizeof(V) * src.size(), hipMemcpyHostToDevice));
    return KKT_OK;
}

void free_static(kkt_ctx *ctx) {
    for (auto &a : ctx->allocs) (void)hipFree(a.first);
    ctx->allocs.clear();
    ctx->bytes_static = 0;
}

void free_ws(kkt_ctx *ctx) {
    for (void *p : ctx->ws) (void)hipFree(p);
    ctx->ws.clear();
    if (ctx->h_pin) (void)hipHostFree(ctx->h_pin);
    ctx->h_pin = nullptr;
    ctx->d_V = ctx->d_Z = ctx->d_h = ctx->d_kpart = nullptr;
    ctx->bytes_ws = 0;
    ctx->ws_nrhs = 0;
}

StepDev step_dev(const StepHost &s, const int32_t *base) {
    StepDev d;
    d.kind = s.kind;
    d.win = s.win;
    d.t0 = s.t0;
    d.pe = s.pe;
    d.nf = s.nf;
    d.fl = base + s.fl_off;
    d.pre = base + s.pre_off;
    d.ntasks = s.ntasks;
    return d;
}

bool recomputes(const kkt_ctx *ctx) { return ctx->opt.recompute_periods > 0; }

// where the local Schur blocks S_bar_n live: the border node's update matrix
// in each period's update storage, or the copies of the recomputing mode
struct SbarSrc {
    const void *p;
    int64_t stride, off;
};
SbarSrc sbar_src(const kkt_ctx *ctx) {
    const Symbolic &S = ctx->sy;
    if (recomputes(ctx)) return SbarSrc{ctx->d_sbar, S.nbord * S.nbord, 0};
    return SbarSrc{ctx->d_U, S.Usize, S.Uoff[S.border_sn]};
}

TreeArgs tree_args(const kkt_ctx *ctx) {
    TreeArgs t;
    t.cptr = ctx->d_cptr;
    t.clist = ctx->d_clist;
    t.relptr = ctx->d_relptr;
    t.rel = ctx->d_rel;
    t.vea = ctx->d_vea;
    t.rows = ctx->d_rows;
    t.rowptr = ctx->d_rowptr;
    return t;
}

int build_device_symbolic(kkt_ctx *ctx, const kkt_structure *s) {
    const Symbolic &S = ctx->sy;
    int rc;
    std::vector<int32_t> adpiv(S.nnzA, -1);
    for (int64_t j = 0; j < S.nA; ++j)
        for (int64_t k = s->A_colptr[j]; k < s->A_colptr[j + 1]; ++k)
            if (s->A_rowind[k] == j) adpiv[k] = S.iperm[j];
    if ((rc = upload(ctx, &ctx->d_amap, S.amap))) return rc;
    if ((rc = upload(ctx, &ctx->d_adiag, S.adiag))) return rc;
    if ((rc = upload(ctx, &ctx->d_adpiv, adpiv))) return rc;
    if ((rc = upload(ctx, &ctx->d_c0map, S.c0map))) return rc;
    if ((rc = upload(ctx, &ctx->d_c1map, S.c1map))) return rc;
    if ((rc = upload(ctx, &ctx->d_rows, S.rows))) return rc;
    if ((rc = upload(ctx, &ctx->d_rowptr, S.rowptr))) return rc;
    if ((rc = upload(ctx, &ctx->d_cptr, S.child_ptr))) return rc;
    if ((rc = upload(ctx, &ctx->d_clist, S.child_list))) return rc;
    if ((rc = upload(ctx, &ctx->d_relptr, S.relptr))) return rc;
    if ((rc = upload(ctx, &ctx->d_rel, S.rel))) return rc;
    {
        // the children's update rows of every front, in groups of children
        // whose rows are disjoint: a child goes into the group after the last
        // one holding an earlier child that shares a row with it, so every
        // row receives its children's entries in the children's order
        std::vector<int32_t> vea(S.nsup), last_group(S.max_front + 1);
        for (int32_t t = 0; t < S.nsup; ++t) {
            vea[t] = (int32_t)vea.size();
            std::vector<std::vector<int32_t>> groups;  // (src, dst) pairs per group
            std::fill(last_group.begin(), last_group.begin() + S.nrow[t], 0);
            for (int32_t k = S.child_ptr[t]; k < S.child_ptr[t + 1]; ++k) {
                const int32_t ch = S.child_list[k];
                const int32_t *rl = S.rel.data() + S.relptr[ch];
                const int uc = S.nrow[ch] - S.ncol[ch];
                int32_t g = 0;
                for (int i = 0; i < uc; ++i) g = std::max(g, last_group[rl[i]]);
                if (g == (int32_t)groups.size()) groups.emplace_back();
                for (int i = 0; i < uc; ++i) {
                    groups[g].push_back((int32_t)(S.relptr[ch] + i));
                    groups[g].push_back(rl[i]);
                    last_group[rl[i]] = g + 1;
                }
            }
            vea.push_back((int32_t)groups.size());
            int32_t e = 0;
            for (const auto &gr : groups) vea.push_back(e += (int32_t)(gr.size() / 2));
            for (const auto &gr : groups) vea.insert(vea.end(), gr.begin(), gr.end());
        }
        if ((rc = upload(ctx, &ctx->d_vea, vea))) return rc;
    }
    if ((rc = upload(ctx, &ctx->d_perm, S.perm))) return rc;
    if ((rc = upload(ctx, &ctx->d_pivsign, S.pivsign))) return rc;
    std::vector<FrontDesc> fd(S.nsup);
    for (int32_t t = 0; t < S.nsup; ++t) {
        fd[t].Loff = S.Loff[t];
        fd[t].Uoff = S.Uoff[t];
        fd[t].m = S.nrow[t];
        fd[t].c = S.ncol[t];
        fd[t].piv0 = S.first[t];
        fd[t].sn = t;
    }
    if ((rc = upload(ctx, &ctx->d_sd, fd))) return rc;
    // per-level task lists
    std::vector<int32_t> buf;
    ctx->levels.assign(S.nlevels, LevelPlan());
    ctx->steps.clear();
    ctx->win_plan.clear();
    for (int32_t l = 0; l < S.nlevels; ++l) {
        LevelPlan &lp = ctx->levels[l];
        std::vector<int32_t> small, large, all;
        for (int32_t q = S.level_ptr[l]; q < S.level_ptr[l + 1]; ++q) {
            int32_t t = S.level_list[q];
            all.push_back(t);
            lp.maxm = std::max(lp.maxm, S.nrow[t]);
            if (S.nrow[t] <= 64) small.push_back(t);
            else {
                large.push_back(t);
                if (!wide_front(S.nrow[t], S.ncol[t])) {  // the solve vectors held in LDS
                    lp.maxm_large = std::max(lp.maxm_large, S.nrow[t]);
                    lp.maxc_large = std::max(lp.maxc_large, S.ncol[t]);
                }
            }
        }
        lp.small_off = (int64_t)buf.size();
        lp.nsmall = (int)small.size();
        for (int cls = 0; cls < 3; ++cls) {
            const int lo = cls == 0 ? 0 : (16 << (cls - 1)), hi = 16 << cls;
            for (int32_t t : small)
                if (S.nrow[t] > lo && S.nrow[t] <= hi) {
                    buf.push_back(t);
                    ++lp.nsmall_cls[cls];
                }
        }
        lp.all_off = (int64_t)buf.size();
        lp.nall = (int)all.size();
        buf.insert(buf.end(), all.begin(), all.end());
        // the solve's pivot part: wide fronts window by window, the others whole
        std::vector<int32_t> plain, wide;
        for (int32_t t : large) (wide_front(S.nrow[t], S.ncol[t]) ? wide : plain).push_back(t);
        lp.large_off = (int64_t)buf.size();
        lp.nlarge = (int)plain.size();
        buf.insert(buf.end(), plain.begin(), plain.end());
        // extend-add tiles and their children's segments (ea_plan.hpp)
        while (buf.size() % 8) buf.push_back(0);  // EaTask alignment
        lp.ea_off = (int64_t)buf.size();
        lp.nea = plan_extend_add(S, large, buf);
        if (buf.size() % 2) buf.push_back(0);  // RowTask alignment (pairs of int32)
        // solve: 64 update rows / 64 pivot columns of each large front (the
        // update rows of wide fronts go with their windows' products)
        lp.rrow_off = (int64_t)buf.size();
        for (int32_t t : plain)
            if (S.ncol[t] > 0)
                for (int r0 = S.ncol[t]; r0 < S.nrow[t]; r0 += 64) { buf.push_back(t); buf.push_back(r0); ++lp.nrrow; }
        lp.rcol_off = (int64_t)buf.size();
        for (int32_t t : large)
            if (S.nrow[t] > S.ncol[t])
                for (int q0 = 0; q0 < S.ncol[t]; q0 += 64) { buf.push_back(t); buf.push_back(q0); ++lp.nrcol; }
        lp.win_begin = (int)ctx->win_plan.size();
        for (int32_t t : wide) lp.maxc_wide = std::max(lp.maxc_wide, S.ncol[t]);
        for (int p0 = 0; p0 < lp.maxc_wide; p0 += TRI_W) {
            WindowPlan w;
            w.p0 = p0;
            w.f_off = (int64_t)buf.size();
            for (int32_t t : wide)
                if (S.ncol[t] > p0) { buf.push_back(t); ++w.nfront; }
            if (buf.size() % 2) buf.push_back(0);  // RowTask alignment
            w.r_off = (int64_t)buf.size();
            for (int32_t t : wide)
                if (S.ncol[t] > p0)
                    for (int r0 = std::min(p0 + TRI_W, S.ncol[t]); r0 < S.nrow[t]; r0 += 64) {
                        buf.push_back(t);
                        buf.push_back(r0);
                        ++w.nrows;
                    }
            w.c_off = (int64_t)buf.size();
            for (int32_t t : wide)
                if (S.ncol[t] > p0)
                    for (int q0 = 0; q0 < p0; q0 += 64) { buf.push_back(t); buf.push_back(q0); ++w.ncols; }
            ctx->win_plan.push_back(w);
        }
        lp.win_end = (int)ctx->win_plan.size();
        // levels with a front of many pivots take the lookahead plan: its
        // trailing updates beyond the next panel go on the side stream while
        // the main stream factors the next panel
        bool lookahead = false;
        for (int32_t t : large) lookahead = lookahead || S.ncol[t] >= LOOKAHEAD_PIVOTS;
        lp.step_begin = (int)ctx->steps.size();
        plan_steps(fd, large, buf, ctx->steps, lookahead, ctx->big_rows, OUTER_W, INNER_W);
        lp.step_end = (int)ctx->steps.size();
    }
    if ((rc = upload(ctx, &ctx->d_tasks, buf))) return rc;
    ctx->win.clear();
    for (const WindowPlan &w : ctx->win_plan) {
        TriWindow tw;
        tw.p0 = w.p0;
        tw.fronts = ctx->d_tasks + w.f_off;
        tw.rows = (const RowTask *)(ctx->d_tasks + w.r_off);
        tw.cols = (const RowTask *)(ctx->d_tasks + w.c_off);
        tw.nfront = w.nfront;
        tw.nrows = w.nrows;
        tw.ncols = w.ncols;
        ctx->win.push_back(tw);
    }
    // Schur front and its steps
    if (ctx->ng > 0 && ctx->structured) {
        const int32_t ns = (int32_t)S.Ns;
        std::vector<FrontDesc> sf(2);
        for (int k = 0; k < 2; ++k) {
            sf[k].Loff = 0;
            sf[k].Uoff = 0;
            sf[k].m = k == 0 ? 2 * ns : ns;
            sf[k].c = ns;
            sf[k].piv0 = 0;
            sf[k].sn = 0;
        }
        if ((rc = upload(ctx, &ctx->d_sfd, sf))) return rc;
        std::vector<int32_t> sbuf;
        for (int k = 0; k < 2; ++k) {
            ctx->sf_steps[k].clear();
            plan_steps(sf, std::vector<int32_t>{k}, sbuf, ctx->sf_steps[k], false, ctx->big_rows, INNER_W, INNER_W);
        }
        if ((rc = upload(ctx, &ctx->d_sftasks, sbuf))) return rc;
    } else if (ctx->ng > 0) {
        std::vector<FrontDesc> sdS(1);
        sdS[0].Loff = 0;
        sdS[0].Uoff = 0;
        sdS[0].m = (int32_t)ctx->ng;
        sdS[0].c = (int32_t)ctx->ng;
        sdS[0].piv0 = 0;
        sdS[0].sn = 0;
        if ((rc = upload(ctx, &ctx->d_sdS, sdS))) return rc;
        std::vector<int32_t> sbuf;
        ctx->ssteps.clear();
        plan_steps(sdS, std::vector<int32_t>{0}, sbuf, ctx->ssteps, true, ctx->big_rows, SCHUR_OUTER_W, INNER_W,
                   std::max(ctx->big_rows, SCHUR_CHAIN_BIG_ROWS));
        if ((rc = upload(ctx, &ctx->d_stasks, sbuf))) return rc;
    }
    // residual: full symmetric CSR of the pattern (caller order) and C^T by column
    {
        const int64_t nA = S.nA;
        std::vector<int64_t> rp(nA + 1, 0);
        for (int64_t j = 0; j < nA; ++j)
            for (int64_t k = s->A_colptr[j]; k < s->A_colptr[j + 1]; ++k) {
                int32_t i = s->A_rowind[k];
                rp[i + 1]++;
                if (i != j) rp[j + 1]++;
            }
        for (int64_t i = 0; i < nA; ++i) rp[i + 1] += rp[i];
        std::vector<int32_t> ci(rp[nA]);
        std::vector<int64_t> vi(rp[nA]);
        std::vector<int64_t> q(rp.begin(), rp.end() - 1);
        for (int64_t j = 0; j < nA; ++j)
            for (int64_t k = s->A_colptr[j]; k < s->A_colptr[j + 1]; ++k) {
                int32_t i = s->A_rowind[k];
                ci[q[i]] = (int32_t)j;
                vi[q[i]++] = k;
                if (i != j) { ci[q[j]] = i; vi[q[j]++] = k; }
            }
        // sliced ELLPACK of that CSR: 64-row slices, entry u of row 64 s + l at
        // sl_off[s] + 64 u + l, padded with the row itself and no value
        const int64_t nsl = (nA + 63) / 64;
        std::vector<int64_t> sl_off(nsl + 1, 0);
        for (int64_t sl = 0; sl < nsl; ++sl) {
            int64_t w = 0;
            for (int64_t i = 64 * sl; i < std::min(nA, 64 * sl + 64); ++i) w = std::max(w, rp[i + 1] - rp[i]);
            sl_off[sl + 1] = sl_off[sl] + 64 * w;
        }
        std::vector<int32_t> sl_ci(sl_off[nsl]), sl_vi(sl_off[nsl], -1);
        for (int64_t sl = 0; sl < nsl; ++sl) {
            const int64_t w = (sl_off[sl + 1] - sl_off[sl]) / 64;
            for (int64_t l = 0; l < 64; ++l) {
                const int64_t i = std::min(nA - 1, 64 * sl + l);
                for (int64_t u = 0; u < w; ++u) {
                    const int64_t p = sl_off[sl] + 64 * u + l;
                    const bool has = 64 * sl + l < nA && rp[i] + u < rp[i + 1];
                    sl_ci[p] = has ? ci[rp[i] + u] : (int32_t)i;
                    sl_vi[p] = has ? (int32_t)vi[rp[i] + u] : -1;
                }
            }
        }
        ctx->nnz_sell = sl_off[nsl];
        if ((rc = upload(ctx, &ctx->d_sl_off, sl_off))) return rc;
        if ((rc = upload(ctx, &ctx->d_sl_ci, sl_ci))) return rc;
        if ((rc = upload(ctx, &ctx->d_sl_vi, sl_vi))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_Asell, 8 * ctx->nnz_sell * ctx->N))) return rc;
        const int64_t Ns = S.Ns;
        auto transpose = [&](const int64_t *p, const int32_t *c, std::vector<int64_t> &tp, std::vector<int32_t> &ts,
                             std::vector<int64_t> &tk) {
            tp.assign(nA + 1, 0);
            for (int64_t sidx = 0; sidx < Ns; ++sidx)
                for (int64_t k = p[sidx]; k < p[sidx + 1]; ++k) tp[c[k] + 1]++;
            for (int64_t i = 0; i < nA; ++i) tp[i + 1] += tp[i];
            ts.assign(tp[nA], 0);
            tk.assign(tp[nA], 0);
            std::vector<int64_t> qq(tp.begin(), tp.end() - 1);
            for (int64_t sidx = 0; sidx < Ns; ++sidx)
                for (int64_t k = p[sidx]; k < p[sidx + 1]; ++k) { ts[qq[c[k]]] = (int32_t)sidx; tk[qq[c[k]]++] = k; }
        };
        std::vector<int64_t> c1tp, c0tp, c1tk, c0tk, c0p, c1p;
        std::vector<int32_t> c1ts, c0ts, c0i, c1i;
        if (Ns > 0) {
            transpose(s->C1_rowptr, s->C1_colind, c1tp, c1ts, c1tk);
            transpose(s->C0_rowptr, s->C0_colind, c0tp, c0ts, c0tk);
            c0p.assign(s->C0_rowptr, s->C0_rowptr + Ns + 1);
            c1p.assign(s->C1_rowptr, s->C1_rowptr + Ns + 1);
            c0i.assign(s->C0_colind, s->C0_colind + c0p[Ns]);
            c1i.assign(s->C1_colind, s->C1_colind + c1p[Ns]);
        } else {
            c1tp.assign(nA + 1, 0);
            c0tp.assign(nA + 1, 0);
            c0p.assign(1, 0);
            c1p.assign(1, 0);
        }
        if ((rc = upload(ctx, &ctx->d_c1tp, c1tp))) return rc;
        if ((rc = upload(ctx, &ctx->d_c0tp, c0tp))) return rc;
        if ((rc = upload(ctx, &ctx->d_c1ts, c1ts))) return rc;
        if ((rc = upload(ctx, &ctx->d_c0ts, c0ts))) return rc;
        if ((rc = upload(ctx, &ctx->d_c1tk, c1tk))) return rc;
        if ((rc = upload(ctx, &ctx->d_c0tk, c0tk))) return rc;
        if ((rc = upload(ctx, &ctx->d_c0p, c0p))) return rc;
        if ((rc = upload(ctx, &ctx->d_c1p, c1p))) return rc;
        if ((rc = upload(ctx, &ctx->d_c0i, c0i))) return rc;
        if ((rc = upload(ctx, &ctx->d_c1i, c1i))) return rc;
    }
    // numeric storage
    const size_t w = ctx->opt.precision == KKT_MIXED ? 4 : 8;
    ctx->P = ctx->opt.recompute_periods > 0 ? std::min<int64_t>(ctx->opt.recompute_periods, ctx->N) : ctx->N;
    ctx->resident = -1;
    if ((rc = dalloc(ctx, &ctx->d_L, w * S.Lsize * ctx->P))) return rc;
    if ((rc = dalloc(ctx, &ctx->d_U, w * std::max<int64_t>(S.Usize, 1) * ctx->P))) return rc;
    if ((rc = dalloc(ctx, (void **)&ctx->d_tau, 8 * S.nA * ctx->P))) return rc;
    if ((rc = dalloc(ctx, (void **)&ctx->d_amax, 8 * (ctx->P + 1)))) return rc;
    // pivot counters of every period, then P more that refactorisations
    // inside the solves count into (and nobody reads)
    if ((rc = dalloc(ctx, (void **)&ctx->d_cnt, 8 * 4 * (ctx->N + 1 + ctx->P)))) return rc;
    if (recomputes(ctx) && ctx->ng > 0 &&
        (rc = dalloc(ctx, &ctx->d_sbar, w * S.nbord * S.nbord * ctx->N)))
        return rc;
    if ((rc = dalloc(ctx, (void **)&ctx->d_flag, 256))) return rc;
    if ((rc = dalloc(ctx, (void **)&ctx->d_snorms, 8 * (4 * 64 + 8)))) return rc;
    if ((rc = dalloc(ctx, (void **)&ctx->d_A, 8 * S.nnzA * ctx->N))) return rc;
    if ((rc = dalloc(ctx, (void **)&ctx->d_C0, 8 * std::max<int64_t>(S.nnzC0, 1)))) return rc;
    if ((rc = dalloc(ctx, (void **)&ctx->d_C1, 8 * std::max<int64_t>(S.nnzC1, 1)))) return rc;
    if (ctx->ng > 0 && ctx->structured) {
        const int64_t ns = S.Ns;
        if ((rc = dalloc(ctx, (void **)&ctx->d_corner, 8 * ctx->ng))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_sfront, 8 * ctx->N * 2 * ns * ns))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_sG, 8 * ctx->N * ns * ns))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_sGT, 8 * ctx->N * ns * ns))) return rc;
        // U and the fronts' update blocks, two of each (column parity)
        if ((rc = dalloc(ctx, (void **)&ctx->d_sU, 8 * 2 * ns * ns))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_sUb, 8 * 2 * ns * ns))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_ssa, 8 * 4 * ctx->ng))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_saa, 8 * 4 * ctx->ng))) return rc;
        if (struct_pairs(ctx->N)) {
            if ((rc = dalloc(ctx, (void **)&ctx->d_sM, 8 * (ctx->N / 2) * ns * ns))) return rc;
            if ((rc = dalloc(ctx, (void **)&ctx->d_sMT, 8 * (ctx->N / 2) * ns * ns))) return rc;
            if ((rc = dalloc(ctx, (void **)&ctx->d_sce, 8 * 4 * (ctx->N / 2) * ns))) return rc;
        }
        if ((rc = dalloc(ctx, (void **)&ctx->d_prefix, 8 * (ctx->N + 1) * S.Ns * S.Ns))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_tauS, 8 * ctx->ng))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_amaxS, 256))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_cntS, 256))) return rc;
        if (ns > INV_W && (rc = dalloc(ctx, (void **)&ctx->d_invtmp, 8 * INV_W * INV_W))) return rc;
    } else if (ctx->ng > 0) {
        if ((rc = dalloc(ctx, (void **)&ctx->d_corner, 8 * ctx->ng))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_S, 8 * ctx->ng * ctx->ng))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_prefix, 8 * (ctx->N + 1) * S.Ns * S.Ns))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_tauS, 8 * ctx->ng))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_amaxS, 256))) return rc;
        if ((rc = dalloc(ctx, (void **)&ctx->d_cntS, 256))) return rc;
        int64_t tmp = 0;
        for (int64_t W = INV_W; 2 * W <= DENSE_INV_W; W *= 2)
            tmp = std::max(tmp, W * W * ((ctx->ng + 2 * W - 1) / (2 * W)));
        if ((rc = dalloc(ctx, (void **)&ctx->d_invtmp, 8 * tmp))) return rc;
        const int64_t nblk = (ctx->ng + DENSE_INV_W - 1) / DENSE_INV_W;
        if ((rc = dalloc(ctx, (void **)&ctx->d_dsync, 4 * (1 + 2 * nblk)))) return rc;
    }
    return KKT_OK;
}

int ensure_ws(kkt_ctx *ctx, int64_t nrhs) {
    if (ctx->ws_nrhs >= nrhs) return KKT_OK;
    free_ws(ctx);
    const Symbolic &S = ctx->sy;
    auto get = [&](double **p, int64_t count) -> int {
        size_t bytes = align_up(8 * std::max<int64_t>(count, 1));
        if (ctx->dry) {
            *p = nullptr;
            ctx->bytes_ws += bytes;
            return KKT_OK;
        }
        hipError_t e = hipMalloc((void **)p, bytes);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? KKT_ERR_NOMEM : KKT_ERR_HIP;
        ctx->ws.push_back(*p);
        ctx->bytes_ws += bytes;
        return KKT_OK;
    };
    int rc;
    if ((rc = get(&ctx->d_xp, (S.nA + S.nbord) * ctx->N * nrhs))) return rc;
    if ((rc = get(&ctx->d_uv, S.Usize_vec() * ctx->N * nrhs))) return rc;
    if ((rc = get(&ctx->d_bh, ctx->ng * nrhs))) return rc;
    if ((rc = get(&ctx->d_y, ctx->ng * nrhs))) return rc;
    if ((rc = get(&ctx->d_xg, ctx->ng * nrhs))) return rc;
    if ((rc = get(&ctx->d_res, ctx->ntot * nrhs))) return rc;
    if ((rc = get(&ctx->d_dx, ctx->ntot * nrhs))) return rc;
    if ((rc = get(&ctx->d_norms, 4 * nrhs + 8))) return rc;
    if ((rc = get(&ctx->d_work, residual_work(ctx->N, S.nA, S.Ns, nrhs)))) return rc;
    if (uses_krylov(ctx->opt)) {
        const int64_t ldh = KRYLOV_M + 1;
        if ((rc = get(&ctx->d_V, (KRYLOV_M + 1) * ctx->ntot * nrhs))) return rc;
        if ((rc = get(&ctx->d_Z, KRYLOV_M * ctx->ntot * nrhs))) return rc;
        if ((rc = get(&ctx->d_h, 3 * ldh * nrhs + nrhs))) return rc;
        if ((rc = get(&ctx->d_kpart, (int64_t)KRYLOV_PART * ldh * nrhs))) return rc;
        if (!ctx->dry &&
            hipHostMalloc((void **)&ctx->h_pin, 8 * (3 * ldh * nrhs + nrhs), hipHostMallocDefault) != hipSuccess) {
            ctx->h_pin = nullptr;
            return KKT_ERR_NOMEM;
        }
    }
    ctx->ws_nrhs = nrhs;
    return KKT_OK;
}

template <typename T>
FactorArgs<T> factor_args(kkt_ctx *ctx) {
    FactorArgs<T> fa;
    fa.L = (T *)ctx->d_L;
    fa.U = (T *)ctx->d_U;
    fa.Lstride = ctx->sy.Lsize;
    fa.Ustride = ctx->sy.Usize;
    fa.tau = ctx->d_tau;
    fa.tstride = ctx->sy.nA;
    fa.amax = ctx->d_amax;
    fa.sign = ctx->d_pivsign;
    fa.cnt = ctx->d_cnt;
    fa.eps = ctx->eps;
    return fa;
}

FactorArgs<double> schur_args(kkt_ctx *ctx) {
    FactorArgs<double> fa;
    fa.L = ctx->d_S;
    fa.U = nullptr;
    fa.Lstride = 0;
    fa.Ustride = 0;
    fa.tau = ctx->d_tauS;
    fa.tstride = 0;
    fa.amax = ctx->d_amaxS;
    fa.sign = nullptr;
    fa.cnt = ctx->d_cntS;
    fa.eps = ctx->eps;
    return fa;
}

void mark(kkt_ctx *ctx, int i) {
    if (ctx->timing) (void)hipEventRecord(ctx->ev[i], ctx->stream);
}

// numeric factorisation of periods [p0, p0 + np) into the factor storage
// (which holds np <= P periods), pivot counters at cnt ([np][4])
template <typename T>
int factor_range(kkt_ctx *ctx, int64_t p0, int64_t np, int64_t *cnt) {
    const Symbolic &S = ctx->sy;
    hipStream_t st = ctx->stream;
    FactorArgs<T> fa = factor_args<T>(ctx);
    fa.cnt = cnt;
    launch_zero<T>((T *)ctx->d_L, S.Lsize * np, st);
    launch_zero<double>(ctx->d_tau, S.nA * np, st);
    launch_zero<double>(ctx->d_amax, np + 1, st);
    ScatterArgs sa;
    sa.A = ctx->d_A + p0 * S.nnzA;
    sa.nnz = S.nnzA;
    sa.amap = ctx->d_amap;
    sa.adiag = ctx->d_adiag;
    sa.adpiv = ctx->d_adpiv;
    sa.dw = ctx->dw;
    sa.dc = ctx->dc;
    sa.C0 = ctx->d_C0;
    sa.C1 = ctx->d_C1;
    sa.n0 = S.nnzC0;
    sa.n1 = S.nnzC1;
    sa.c0map = ctx->d_c0map;
    sa.c1map = ctx->d_c1map;
    launch_scatter<T>(sa, fa, np, st);
    TreeArgs tr = tree_args(ctx);
    for (const LevelPlan &lp : ctx->levels) {
        launch_small_fronts<T>(fa, ctx->d_sd, ctx->d_tasks + lp.small_off, lp.nsmall_cls, np, tr, st);
        launch_extend_add<T>(fa, ctx->d_sd, (const EaTask *)(ctx->d_tasks + lp.ea_off), lp.nea, np, tr, st);
        for (int q = lp.step_begin; q < lp.step_end; ++q) {
            const StepHost &s = ctx->steps[q];
            if (s.kind == SYNC_TO_SIDE) {
                HIPCHK(hipEventRecord(ctx->ev_main, st));
                HIPCHK(hipStreamWaitEvent(ctx->side, ctx->ev_main, 0));
            } else if (s.kind == SYNC_TO_MAIN) {
                HIPCHK(hipEventRecord(ctx->ev_side, ctx->side));
                HIPCHK(hipStreamWaitEvent(st, ctx->ev_side, 0));
            } else {
                launch_step<T>(fa, ctx->d_sd, step_dev(s, ctx->d_tasks), np, s.side ? ctx->side : st);
            }
        }
        if (lp.win_end > lp.win_begin) {
            // the solves' windows of the wide fronts: their diagonal blocks inverted
            const WindowPlan &w0 = ctx->win_plan[lp.win_begin];
            launch_window_inverses<T>(fa, ctx->d_sd, ctx->d_tasks + w0.f_off, w0.nfront, lp.maxc_wide, np, st);
        }
    }
    return KKT_OK;
}

// the factorisation of every period; with recompute_periods chunk by chunk,
// each chunk's local Schur blocks copied out of the update storage
template <typename T>
int factor_blocks(kkt_ctx *ctx) {
    const Symbolic &S = ctx->sy;
    launch_zero<int64_t>(ctx->d_cnt, 4 * (ctx->N + 1 + ctx->P), ctx->stream);
    for (int64_t p0 = 0; p0 < ctx->N; p0 += ctx->P) {
        const int64_t np = std::min(ctx->P, ctx->N - p0);
        int rc = factor_range<T>(ctx, p0, np, ctx->d_cnt + 4 * p0);
        if (rc) return rc;
        if (recomputes(ctx) && ctx->ng > 0) {
            const size_t ub = S.nbord * S.nbord * sizeof(T);
            HIPCHK(hipMemcpy2DAsync((T *)ctx->d_sbar + p0 * S.nbord * S.nbord, ub,
                                    (const T *)ctx->d_U + S.Uoff[S.border_sn], S.Usize * sizeof(T), ub, np,
                                    hipMemcpyDeviceToDevice, ctx->stream));
        }
        ctx->resident = p0 / ctx->P;
    }
    return KKT_OK;
}

// structured Schur elimination (section 4.3): one front per block column,
// factored on the main stream; the pivot-block inverse and G_j = W_j Linv_j
// (used only by the solves) on the side stream
int factor_schur_structured(kkt_ctx *ctx) {
    hipStream_t st = ctx->stream;
    const Symbolic &S = ctx->sy;
    const int64_t ns = S.Ns, N = ctx->N;
    const double *corner = ctx->has_corner ? ctx->d_corner : nullptr;
    const SbarSrc sb = sbar_src(ctx);
    launch_struct_tau(sb.p, sb.stride, sb.off, N, ns, ctx->opt.precision, ctx->d_prefix, corner, ctx->d_tauS, ctx->eps,
                      ctx->d_amaxS, st);
    mark(ctx, 2);
    // U_j and front j's update block (which holds -B_j A_j^-1 B_j^T) live in
    // buffer j % 2; front j's assembly reads U_{j-1} and block j-1 from the
    // other one (both zero for j = 0) and forms U_j on the way
    launch_zero<double>(ctx->d_sU, 2 * ns * ns, st);
    launch_zero<double>(ctx->d_sUb, 2 * ns * ns, st);
    FactorArgs<double> fa = schur_args(ctx);
    for (int64_t j = 0; j < N; ++j) {
        const int last = j + 1 == N ? 1 : 0;
        const int64_t cur = (j & 1) * ns * ns, prev = ((j + 1) & 1) * ns * ns;
        double *Fj = ctx->d_sfront + j * 2 * ns * ns;
        launch_struct_front(sb.p, sb.stride, sb.off, ns, j, last, ctx->opt.precision, ctx->d_prefix, corner,
                            ctx->d_sU + prev, ctx->d_sUb + prev, ctx->d_sU + cur, Fj, ctx->d_sUb + cur, st);
        fa.L = Fj;
        fa.U = ctx->d_sUb + cur;
        fa.tau = ctx->d_tauS + j * ns;
        for (const StepHost &s : ctx->sf_steps[last]) launch_step<double>(fa, ctx->d_sfd, step_dev(s, ctx->d_sftasks), 1, st);
        // the front is final: its inverse and G_j on the side stream
        HIPCHK(hipEventRecord(ctx->ev_main, st));
        HIPCHK(hipStreamWaitEvent(ctx->side, ctx->ev_main, 0));
        const int32_t *fl = ctx->d_sftasks + ctx->sf_steps[last].front().fl_off;  // this front's index list {last}
        launch_inv256(fa, ctx->d_sfd, fl, 0, ctx->side);
        if (ns > INV_W) {
            launch_inv256(fa, ctx->d_sfd, fl, INV_W, ctx->side);
            launch_inv_combine(fa, ctx->d_sfd, fl, 0, (int)ns, ctx->d_invtmp, ctx->side);
        }
        if (!last)
            launch_struct_g(Fj, (int)(2 * ns), (int)ns, ctx->d_sG + j * ns * ns, ctx->d_sGT + j * ns * ns, ctx->side);
    }
    HIPCHK(hipEventRecord(ctx->ev_side, ctx->side));
    HIPCHK(hipStreamWaitEvent(st, ctx->ev_side, 0));
    // pair matrices of the solves' two-column chain steps
    if (struct_pairs(N)) launch_struct_pair(ctx->d_sG, (int)ns, (int)N, ctx->d_sM, ctx->d_sMT, st);
    return KKT_OK;
}

int factor_schur(kkt_ctx *ctx) {
    if (ctx->ng == 0) return KKT_OK;
    hipStream_t st = ctx->stream;
    const Symbolic &S = ctx->sy;
    const SbarSrc sb = sbar_src(ctx);
    launch_zero<double>(ctx->d_amaxS, 1, st);
    launch_zero<int64_t>(ctx->d_cntS, 4, st);
    if (ctx->structured) {
        launch_schur_prefix(sb.p, sb.stride, sb.off, ctx->N, S.Ns, ctx->opt.precision, ctx->d_prefix, st);
        return factor_schur_structured(ctx);
    }
    launch_schur_prefix(sb.p, sb.stride, sb.off, ctx->N, S.Ns, ctx->opt.precision, ctx->d_prefix, st);
    // the pivot thresholds from S's diagonal, the first panel's columns on
    // the main stream, the other columns on the side stream while the first
    // panel is factored; the main stream waits for them before its first
    // update beyond the first panel
    const double *corner = ctx->has_corner ? ctx->d_corner : nullptr;
    const int64_t w0 = std::min<int64_t>(SCHUR_OUTER_W, ctx->ng);
    launch_schur_diag(sb.p, sb.stride, sb.off, ctx->N, S.Ns, ctx->opt.precision, ctx->d_prefix, corner, ctx->d_tauS,
                      ctx->eps, ctx->d_amaxS, st);
    launch_schur_assemble(sb.p, sb.stride, sb.off, ctx->N, S.Ns, ctx->opt.precision, ctx->d_prefix, corner, ctx->d_S,
                          nullptr, 0.0, nullptr, 0, st, 0, w0);
    HIPCHK(hipEventRecord(ctx->ev_main, st));
    HIPCHK(hipStreamWaitEvent(ctx->side, ctx->ev_main, 0));
    launch_schur_assemble(sb.p, sb.stride, sb.off, ctx->N, S.Ns, ctx->opt.precision, ctx->d_prefix, corner, ctx->d_S,
                          nullptr, 0.0, nullptr, 0, ctx->side, w0, -1);
    HIPCHK(hipEventRecord(ctx->ev_asm, ctx->side));
    bool assembled = false;
    mark(ctx, 2);
    ctx->kcount = 0;
    ctx->kstat = kkt_kernel_stat{};
    FactorArgs<double> fa = schur_args(ctx);
    for (const StepHost &s : ctx->ssteps) {
        if (s.kind == SYNC_TO_SIDE) {
            HIPCHK(hipEventRecord(ctx->ev_main, st));
            HIPCHK(hipStreamWaitEvent(ctx->side, ctx->ev_main, 0));
        } else if (s.kind == SYNC_TO_MAIN) {
            HIPCHK(hipEventRecord(ctx->ev_side, ctx->side));
            HIPCHK(hipStreamWaitEvent(st, ctx->ev_side, 0));
        } else {
            hipStream_t ss = s.side ? ctx->side : st;
            if (!assembled && !s.side && (s.kind == 3 || s.kind == 4) && s.pe >= w0) {
                HIPCHK(hipStreamWaitEvent(st, ctx->ev_asm, 0));
                assembled = true;
            }
            const bool timed = ctx->timing && s.kind == 4;
            if (timed) {
                if ((size_t)(2 * ctx->kcount + 2) > ctx->kev.size()) {
                    hipEvent_t e0, e1;
                    HIPCHK(hipEventCreate(&e0));
                    HIPCHK(hipEventCreate(&e1));
                    ctx->kev.push_back(e0);
                    ctx->kev.push_back(e1);
                }
                HIPCHK(hipEventRecord(ctx->kev[2 * ctx->kcount], ss));
            }
            launch_step<double>(fa, ctx->d_sdS, step_dev(s, ctx->d_stasks), 1, ss);
            if (timed) {
                HIPCHK(hipEventRecord(ctx->kev[2 * ctx->kcount + 1], ss));
                double f = 0.0, b = 0.0;
                update_work(s.t0, s.pe, (int)ctx->ng, (int)ctx->ng, s.win, &f, &b);
                ctx->kstat.flops += f;
                ctx->kstat.bytes += b;
                ++ctx->kcount;
            }
        }
    }
    // the inverses of the diagonal blocks, which only the dense solves use,
    // for all blocks at once
    launch_inverses_all(fa, ctx->d_sdS, ctx->d_stasks + ctx->ssteps.front().fl_off, (int)ctx->ng, ctx->d_invtmp, st);
    return KKT_OK;
}

// one pass of Algorithm 1's solve for the right-hand sides in `b` (device,
// [nrhs][ntot]) into `x`. With recompute_periods the factor storage holds one
// chunk of periods at a time: every chunk is factored again before its
// forward sweep and before its backward sweep (the memory-saving variant of
// section 4.3, which recomputes the period factors in the solve steps),
// starting each sweep with the chunk that is still resident.
template <typename T>
int solve_once(kkt_ctx *ctx, const double *b, double *x, int64_t nrhs) {
    const Symbolic &S = ctx->sy;
    hipStream_t st = ctx->stream;
    SolveArgs sa;
    sa.N = ctx->N;
    sa.nrhs = nrhs;
    sa.nv = S.nA + S.nbord;
    sa.usz = S.Usize_vec();
    sa.xp = ctx->d_xp;
    sa.uv = ctx->d_uv;
    TreeArgs tr = tree_args(ctx);
    const T *L = (const T *)ctx->d_L;
    launch_gather_rhs<T>(b, ctx->ntot, S.nA, ctx->d_perm, sa, st);
    auto tasks_of = [&](const LevelPlan &lp) {
        LevelTasks lt;
        lt.small = ctx->d_tasks + lp.small_off;
        lt.large = ctx->d_tasks + lp.large_off;
        lt.rect_rows = (const RowTask *)(ctx->d_tasks + lp.rrow_off);
        lt.rect_cols = (const RowTask *)(ctx->d_tasks + lp.rcol_off);
        lt.nsmall = lp.nsmall;
        lt.nlarge = lp.nlarge;
        lt.nrect_rows = lp.nrrow;
        lt.nrect_cols = lp.nrcol;
        lt.win = ctx->win.data() + lp.win_begin;
        lt.nwin = lp.win_end - lp.win_begin;
        lt.maxm = lp.maxm_large;
        lt.maxc = lp.maxc_large;
        return lt;
    };
    // the chunks of periods, the resident one first; each made resident
    const int64_t nch = (ctx->N + ctx->P - 1) / ctx->P;
    auto chunk_order = [&]() {
        std::vector<int64_t> ord;
        if (ctx->resident >= 0) ord.push_back(ctx->resident);
        for (int64_t c = 0; c < nch; ++c)
            if (c != ctx->resident) ord.push_back(c);
        return ord;
    };
    auto make_resident = [&](int64_t c) -> int {
        if (ctx->resident == c) return KKT_OK;
        const int64_t p0 = c * ctx->P;
        int rc = factor_range<T>(ctx, p0, std::min(ctx->P, ctx->N - p0), ctx->d_cnt + 4 * (ctx->N + 1));
        ctx->resident = c;
        return rc;
    };
    auto chunk_args = [&](int64_t c) {
        SolveArgs sc = sa;
        const int64_t p0 = c * ctx->P;
        sc.N = std::min(ctx->P, ctx->N - p0);
        sc.xp = sa.xp + p0 * nrhs * sa.nv;
        sc.uv = sa.uv + p0 * nrhs * sa.usz;
        return sc;
    };
    for (int64_t c : chunk_order()) {
        int rc = make_resident(c);
        if (rc) return rc;
        const SolveArgs sc = chunk_args(c);
        for (const LevelPlan &lp : ctx->levels) launch_fwd_level<T>(L, S.Lsize, ctx->d_sd, tasks_of(lp), tr, sc, st);
    }
    if (ctx->ng > 0) {
        launch_schur_rhs(b, ctx->ntot, S.nA, sa, S.Ns, S.relptr[S.border_sn], ctx->d_bh, st);
        if (ctx->structured) {
            launch_struct_solve(ctx->d_sfront, ctx->d_sG, ctx->d_sGT, ctx->d_sM, ctx->d_sMT, ctx->N, S.Ns, ctx->d_bh,
                                ctx->d_xg, ctx->d_ssa, ctx->d_saa, ctx->d_sce, nrhs, st);
        } else {
            launch_dense_fwd(ctx->d_S, ctx->ng, ctx->d_bh, ctx->d_y, nrhs, ctx->d_dsync, st);
            launch_dense_bwd(ctx->d_S, ctx->ng, ctx->d_y, ctx->d_xg, nrhs, ctx->d_dsync, st);
        }
        launch_border_values(ctx->d_xg, sa, S.nA, S.Ns, st);
    }
    for (int64_t c : chunk_order()) {
        int rc = make_resident(c);
        if (rc) return rc;
        const SolveArgs sc = chunk_args(c);
        for (int l = (int)ctx->levels.size() - 1; l >= 0; --l) {
            const LevelPlan &lp = ctx->levels[l];
            launch_bwd_level<T>(L, S.Lsize, ctx->d_sd, tasks_of(lp), tr, sc, st);
        }
    }
    launch_scatter_x(x, ctx->ntot, S.nA, ctx->d_perm, sa, ctx->d_xg, ctx->ng, st);
    return KKT_OK;
}

ResidualArgs residual_args(kkt_ctx *ctx, int64_t nrhs) {
    const Symbolic &S = ctx->sy;
    ResidualArgs ra;
    ra.N = ctx->N;
    ra.nA = S.nA;
    ra.Ns = S.Ns;
    ra.ntot = ctx->ntot;
    ra.nrhs = nrhs;
    ra.A = ctx->d_A;
    ra.nnz = S.nnzA;
    ra.sl_off = ctx->d_sl_off;
    ra.sl_ci = ctx->d_sl_ci;
    ra.Asell = ctx->d_Asell;
    ra.nnz_sell = ctx->nnz_sell;
    ra.c1tp = ctx->d_c1tp;
    ra.c0tp = ctx->d_c0tp;
    ra.c1ts = ctx->d_c1ts;
    ra.c0ts = ctx->d_c0ts;
    ra.c1tk = ctx->d_c1tk;
    ra.c0tk = ctx->d_c0tk;
    ra.c0p = ctx->d_c0p;
    ra.c1p = ctx->d_c1p;
    ra.c0i = ctx->d_c0i;
    ra.c1i = ctx->d_c1i;
    ra.C0v = ctx->d_C0;
    ra.C1v = ctx->d_C1;
    ra.corner = ctx->has_corner ? ctx->d_corner : nullptr;
    ra.dw = ctx->dw;
    ra.dc = ctx->dc;
    ra.n_primal = S.n_primal;
    return ra;
}

double elapsed(kkt_ctx *ctx, int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[a], ctx->ev[b]) != hipSuccess) return 0.0;
    return (double)ms;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" int kkt_create(kkt_ctx **out, void *stream, const kkt_options *opt) {
    if (!out) return KKT_ERR_ARG;
    *out = nullptr;
    kkt_ctx *ctx = new (std::nothrow) kkt_ctx();
    if (!ctx) return KKT_ERR_NOMEM;
    kkt_default_options(&ctx->opt);
    if (opt) ctx->opt = *opt;
    if (ctx->opt.precision != KKT_FP64 && ctx->opt.precision != KKT_MIXED) { delete ctx; return KKT_ERR_ARG; }
    if (ctx->opt.refine_tol <= 0) ctx->opt.refine_tol = 1e-10;
    if (ctx->opt.big_tile_rows < 0 || ctx->opt.recompute_periods < 0 || ctx->opt.dual_wait < 0) {
        delete ctx;
        return KKT_ERR_ARG;
    }
    if (ctx->opt.schur_mode != KKT_SCHUR_DENSE && ctx->opt.schur_mode != KKT_SCHUR_STRUCTURED) {
        delete ctx;
        return KKT_ERR_ARG;
    }
    ctx->structured = ctx->opt.schur_mode == KKT_SCHUR_STRUCTURED;
    ctx->big_rows = ctx->opt.big_tile_rows > 0 ? ctx->opt.big_tile_rows : 512;
    if (ctx->opt.refine_max < 0) ctx->opt.refine_max = 0;
    ctx->eps = ctx->opt.pivot_eps > 0 ? ctx->opt.pivot_eps : (ctx->opt.precision == KKT_MIXED ? 1e-10 : 1e-20);
    ctx->stream = (hipStream_t)stream;
    if (hipGetDevice(&ctx->device) != hipSuccess) { delete ctx; return KKT_ERR_HIP; }
    if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_main, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_side, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_asm, hipEventDisableTiming) != hipSuccess) {
        kkt_destroy(ctx);
        return KKT_ERR_HIP;
    }
    for (auto &e : ctx->ev)
        if (hipEventCreate(&e) != hipSuccess) { delete ctx; return KKT_ERR_HIP; }
    *out = ctx;
    return KKT_OK;
}

// symbolic analysis with the structure checks and the kernels' size limits
int analyze_checked(const kkt_structure *s, const kkt_options &o, Symbolic &S) {
    if (!s || s->N < 1 || s->Ns < 0 || s->nA < 1) return KKT_ERR_ARG;
    if (!s->A_colptr || !s->A_rowind) return KKT_ERR_ARG;
    if (s->Ns > 0 && (!s->C0_rowptr || !s->C0_colind || !s->C1_rowptr || !s->C1_colind)) return KKT_ERR_ARG;
    std::string err;
    try {
        err = analyze(make_input(s, o), S);
    } catch (...) {
        return KKT_ERR_NOMEM;
    }
    if (!err.empty()) {
        if (o.verbose) std::fprintf(stderr, "kkt_analyze: %s\n", err.c_str());
        return KKT_ERR_STRUCT;
    }
    // fronts whose solve vectors must fit in LDS (all but the wide ones, whose
    // solves go window by window through HBM; those need their factor panel
    // below 2^31 bytes for 32-bit buffer offsets); 32-bit launch and index
    // limits of the dense S; the structured Schur's block inverses cover
    // Ns <= 2 INV_W
    const bool structured = o.schur_mode == KKT_SCHUR_STRUCTURED;
    bool fronts_ok = true;
    for (int32_t t = 0; t < S.nsup && fronts_ok; ++t) {
        const int m = S.nrow[t], c = S.ncol[t];
        fronts_ok = wide_front(m, c) ? (int64_t)m * c * 8 < ((int64_t)1 << 31)
                                     : (m <= MAX_FRONT_ROWS && c <= MAX_FRONT_PIVOTS);
    }
    if (!fronts_ok || (!structured && s->N * s->Ns > 46000) || (structured && s->Ns > 2 * INV_W)) {
        if (o.verbose)
            std::fprintf(stderr, "kkt_analyze: front of %lld rows / %lld pivots or Schur size %lld over the limits\n",
                         (long long)S.max_front, (long long)S.max_pivots, (long long)(s->N * s->Ns));
        return KKT_ERR_ARG;
    }
    return KKT_OK;
}

extern "C" int kkt_analyze(kkt_ctx *ctx, const kkt_structure *s) {
    if (!ctx) return KKT_ERR_ARG;
    Symbolic S;
    const int arc = analyze_checked(s, ctx->opt, S);
    if (arc) return arc;
    (void)hipStreamSynchronize(ctx->stream);
    free_ws(ctx);
    free_static(ctx);
    ctx->analyzed = ctx->factored = false;
    ctx->sy = std::move(S);
    ctx->N = s->N;
    ctx->ng = s->N * s->Ns;
    ctx->ntot = s->N * s->nA + ctx->ng;
    int rc = build_device_symbolic(ctx, s);
    if (rc) { free_static(ctx); return rc; }
    if (ctx->fb) { kkt_destroy(ctx->fb); ctx->fb = nullptr; }
    ctx->fb_factored = false;
    for (void *q : ctx->slack_allocs) (void)hipFree(q);
    ctx->slack_allocs.clear();
    ctx->n_slack = 0;
    ctx->d_slack_row = nullptr;
    ctx->d_slack_dpos = nullptr;
    ctx->pat_colptr.assign(s->A_colptr, s->A_colptr + s->nA + 1);
    if (ctx->opt.precision == KKT_MIXED) {
        // the pattern, for an FP64 fallback analysis
        const int64_t nnz = s->A_colptr[s->nA];
        ctx->pat_rowind.assign(s->A_rowind, s->A_rowind + nnz);
        ctx->pat_n_primal = s->n_primal;
        ctx->pat_Ns = s->Ns;
        if (s->Ns > 0) {
            ctx->pat_C0p.assign(s->C0_rowptr, s->C0_rowptr + s->Ns + 1);
            ctx->pat_C1p.assign(s->C1_rowptr, s->C1_rowptr + s->Ns + 1);
            ctx->pat_C0i.assign(s->C0_colind, s->C0_colind + ctx->pat_C0p[s->Ns]);
            ctx->pat_C1i.assign(s->C1_colind, s->C1_colind + ctx->pat_C1p[s->Ns]);
        }
    }
    ctx->analyzed = true;
    return KKT_OK;
}

namespace kkt {
int plan_device_bytes(const kkt_structure *s, const kkt_options &o, int64_t nrhs, size_t *bytes) {
    if (!bytes || nrhs < 1) return KKT_ERR_ARG;
    kkt_ctx ctx;
    ctx.dry = true;
    ctx.opt = o;
    ctx.structured = o.schur_mode == KKT_SCHUR_STRUCTURED;
    ctx.big_rows = o.big_tile_rows > 0 ? o.big_tile_rows : 512;
    Symbolic S;
    int rc = analyze_checked(s, o, S);
    if (rc) return rc;
    ctx.sy = std::move(S);
    ctx.N = s->N;
    ctx.ng = s->N * s->Ns;
    ctx.ntot = s->N * s->nA + ctx.ng;
    if ((rc = build_device_symbolic(&ctx, s))) return rc;
    if ((rc = ensure_ws(&ctx, nrhs))) return rc;
    *bytes = ctx.bytes_static + ctx.bytes_ws;
    return KKT_OK;
}
}  // namespace kkt

extern "C" int kkt_footprint(const kkt_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return KKT_ERR_ARG;
    *bytes = ctx->bytes_static + ctx->bytes_ws;
    if (ctx->fb) *bytes += ctx->fb->bytes_static + ctx->fb->bytes_ws;
    return KKT_OK;
}

extern "C" int kkt_stats(const kkt_ctx *ctx, kkt_symbolic_stats *st) {
    if (!ctx || !st) return KKT_ERR_ARG;
    if (!ctx->analyzed) return KKT_ERR_ORDER;
    fill_stats(ctx->sy, st);
    st->device_bytes = (int64_t)(ctx->bytes_static + ctx->bytes_ws);
    return KKT_OK;
}

namespace {

// enqueue the whole factorisation; with `check` the non-finite test is read
// back (one synchronisation) before any state changes, else its result stays
// on the device for kkt_factor_status
int factor_enqueue(kkt_ctx *ctx, const double *A_vals, const double *C0_vals, const double *C1_vals,
                   const double *corner_diag, double delta_w, double delta_c, bool check) {
    if (!ctx) return KKT_ERR_ARG;
    if (!ctx->analyzed) return KKT_ERR_ORDER;
    const Symbolic &S = ctx->sy;
    if (!A_vals || (S.Ns > 0 && (!C0_vals || !C1_vals))) return KKT_ERR_ARG;
    if (!std::isfinite(delta_w) || !std::isfinite(delta_c) || delta_w < 0 || delta_c < 0) return KKT_ERR_ARG;
    hipStream_t st = ctx->stream;
    launch_zero<int>(ctx->d_flag, 1, st);
    launch_check_finite(A_vals, S.nnzA * ctx->N, ctx->d_flag, st);
    if (S.Ns > 0) {
        launch_check_finite(C0_vals, S.nnzC0, ctx->d_flag, st);
        launch_check_finite(C1_vals, S.nnzC1, ctx->d_flag, st);
    }
    if (corner_diag && ctx->ng) launch_check_finite(corner_diag, ctx->ng, ctx->d_flag, st);
    if (check) {
        int flag = 0;
        HIPCHK(hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (flag) return KKT_ERR_NONFINITE;
    }
    HIPCHK(hipMemcpyAsync(ctx->d_A, A_vals, 8 * S.nnzA * ctx->N, hipMemcpyDeviceToDevice, st));
    if (S.Ns > 0) {
        HIPCHK(hipMemcpyAsync(ctx->d_C0, C0_vals, 8 * S.nnzC0, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(ctx->d_C1, C1_vals, 8 * S.nnzC1, hipMemcpyDeviceToDevice, st));
    }
    ctx->has_corner = corner_diag != nullptr && ctx->ng > 0;
    if (ctx->has_corner) HIPCHK(hipMemcpyAsync(ctx->d_corner, corner_diag, 8 * ctx->ng, hipMemcpyDeviceToDevice, st));
    ctx->dw = delta_w;
    ctx->dc = delta_c;
    launch_sell_values(ctx->d_A, S.nnzA, ctx->N, S.nA, S.n_primal, ctx->d_sl_off, ctx->d_sl_ci, ctx->d_sl_vi,
                       ctx->nnz_sell, delta_w, delta_c, ctx->d_Asell, st);
    mark(ctx, 0);
    int rc = ctx->opt.precision == KKT_MIXED ? factor_blocks<float>(ctx) : factor_blocks<double>(ctx);
    if (rc) return rc;
    mark(ctx, 1);
    rc = factor_schur(ctx);
    if (rc) return rc;
    mark(ctx, 3);
    HIPCHK(hipGetLastError());
    ctx->factored = true;
    return KKT_OK;
}

// read the pivot counters of the last factorisation (synchronises)
int factor_readback(kkt_ctx *ctx, kkt_inertia *out) {
    hipStream_t st = ctx->stream;
    const Symbolic &S = ctx->sy;
    std::vector<int64_t> cnt(4 * (ctx->N + 1), 0), cs(4, 0);
    HIPCHK(hipMemcpyAsync(cnt.data(), ctx->d_cnt, 8 * 4 * ctx->N, hipMemcpyDeviceToHost, st));
    if (ctx->ng) HIPCHK(hipMemcpyAsync(cs.data(), ctx->d_cntS, 8 * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    kkt_inertia in{};
    for (int64_t n = 0; n < ctx->N; ++n) {
        in.n_pos += cnt[4 * n + 0];
        in.n_neg += cnt[4 * n + 1];
        in.n_zero += cnt[4 * n + 2];
        in.n_perturbed += cnt[4 * n + 3];
    }
    in.n_pos += cs[0];
    in.n_neg += cs[1];
    in.n_zero += cs[2];
    in.n_perturbed += cs[3];
    const int64_t epos = ctx->N * S.n_primal, eneg = ctx->N * (S.nA - S.n_primal) + ctx->ng;
    in.inertia_ok = (in.n_pos == epos && in.n_neg == eneg && in.n_zero == 0) ? 1 : 0;
    if (out) *out = in;
    if (!in.inertia_ok) return KKT_WARN_INERTIA;
    if (in.n_perturbed) return KKT_WARN_PERTURBED;
    return KKT_OK;
}

}  // namespace

namespace {

// FP64 factorisation of the context's current values in its fallback
// context (created, with its own FP64 analysis, on first use)
int fallback_factor(kkt_ctx *ctx) {
    if (!ctx->fb) {
        kkt_options o = ctx->opt;
        o.precision = KKT_FP64;
        o.pivot_eps = 0.0;
        o.dual_wait = 0;
        kkt_ctx *fb = nullptr;
        int rc = kkt_create(&fb, ctx->stream, &o);
        if (rc) return rc;
        kkt_structure st{};
        st.nA = ctx->sy.nA;
        st.n_primal = ctx->pat_n_primal;
        st.N = ctx->N;
        st.Ns = ctx->pat_Ns;
        st.A_colptr = ctx->pat_colptr.data();
        st.A_rowind = ctx->pat_rowind.data();
        if (st.Ns > 0) {
            st.C0_rowptr = ctx->pat_C0p.data();
            st.C0_colind = ctx->pat_C0i.data();
            st.C1_rowptr = ctx->pat_C1p.data();
            st.C1_colind = ctx->pat_C1i.data();
        }
        rc = kkt_analyze(fb, &st);
        if (rc) { kkt_destroy(fb); return rc; }
        ctx->fb = fb;
    }
    ctx->fb->stream = ctx->stream;
    int rc = kkt_factor(ctx->fb, ctx->d_A, ctx->d_C0, ctx->d_C1, ctx->has_corner ? ctx->d_corner : nullptr, ctx->dw,
                        ctx->dc, &ctx->fb_inertia);
    if (rc < 0) return rc;
    ctx->fb_factored = true;
    return rc;
}

}  // namespace

extern "C" int kkt_factor(kkt_ctx *ctx, const double *A_vals, const double *C0_vals, const double *C1_vals,
                          const double *corner_diag, double delta_w, double delta_c, kkt_inertia *out) {
    int rc = factor_enqueue(ctx, A_vals, C0_vals, C1_vals, corner_diag, delta_w, delta_c, true);
    if (rc) return rc;
    ctx->fb_factored = false;
    if (ctx->opt.precision == KKT_MIXED) {
        // An FP32 factor whose inertia differs from the expected one, or that
        // needed perturbed pivots, cannot be trusted for the inertia test of
        // the interior point method: the values are factored in FP64 as well
        // and that factor's inertia is reported (and used by kkt_solve).
        kkt_inertia in32{};
        const int rc32 = factor_readback(ctx, &in32);
        if (rc32 != KKT_OK) {
            rc = fallback_factor(ctx);
            if (rc < 0) return rc;
            if (out) *out = ctx->fb_inertia;
            return rc;
        }
    }
    hipStream_t st = ctx->stream;
    if (ctx->timing) {
        HIPCHK(hipStreamSynchronize(st));
        ctx->times[0] = elapsed(ctx, 0, 1);
        ctx->times[1] = ctx->ng ? elapsed(ctx, 1, 2) : 0.0;
        ctx->times[2] = ctx->ng ? elapsed(ctx, 2, 3) : 0.0;
        double kms = 0.0;
        for (int64_t j = 0; j < ctx->kcount; ++j) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ctx->kev[2 * j], ctx->kev[2 * j + 1]) == hipSuccess) kms += ms;
        }
        ctx->kstat.launches = ctx->kcount;
        ctx->kstat.total_ms = kms;
        ctx->times[4] = kms;
    }
    if (!out) return KKT_OK;
    return factor_readback(ctx, out);
}

extern "C" int kkt_factor_async(kkt_ctx *ctx, const double *A_vals, const double *C0_vals, const double *C1_vals,
                                const double *corner_diag, double delta_w, double delta_c) {
    if (ctx && ctx->timing) return KKT_ERR_ARG;  // timing synchronises
    return factor_enqueue(ctx, A_vals, C0_vals, C1_vals, corner_diag, delta_w, delta_c, false);
}

extern "C" int kkt_factor_status(kkt_ctx *ctx, kkt_inertia *out) {
    if (!ctx) return KKT_ERR_ARG;
    if (!ctx->factored) return KKT_ERR_ORDER;
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (flag) return KKT_ERR_NONFINITE;
    return factor_readback(ctx, out);
}

extern "C" int kkt_set_stream(kkt_ctx *ctx, void *stream) {
    if (!ctx) return KKT_ERR_ARG;
    ctx->stream = (hipStream_t)stream;
    return KKT_OK;
}

namespace {

constexpr double EPS64 = 2.220446049250313e-16;

struct RefineState {
    int it = 0, status = KKT_OK;
    double rel = 0.0, omega = 0.0;
    double floor = 0.0;  // max_k eps || |K||x_k| + |b_k| ||_2 / ||b_k||_2
};

// true residual r = b - K x (compensated sums) with its norms
int true_residual(kkt_ctx *ctx, const ResidualArgs &ra, const double *b, const double *x, double *r, int64_t nrhs,
                  std::vector<double> &nh, RefineState &rs) {
    hipStream_t st = ctx->stream;
    launch_residual(ra, b, x, r, ctx->d_work, ctx->d_norms, st);
    HIPCHK(hipMemcpyAsync(nh.data(), ctx->d_norms, 8 * 4 * nrhs, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rs.rel = 0.0;
    rs.omega = 0.0;
    rs.floor = 0.0;
    for (int64_t k = 0; k < nrhs; ++k) {
        const double bn = nh[4 * k + 1] > 0 ? nh[4 * k + 1] : 1.0;
        rs.rel = std::max(rs.rel, nh[4 * k + 0] / bn);
        rs.omega = std::max(rs.omega, nh[4 * k + 2]);
        rs.floor = std::max(rs.floor, EPS64 * nh[4 * k + 3] / bn);
    }
    if (ctx->opt.verbose)
        std::fprintf(stderr, "kkt_solve: step %d rel_res %.3e omega %.3e floor %.3e\n", rs.it, rs.rel, rs.omega,
                     rs.floor);
    return KKT_OK;
}

// common stopping tests on a true residual; true = stop. The residual is
// evaluated with compensated sums, so it resolves the residual of x itself
// down to the rounding of x to FP64; refinement runs until the target, the
// step limit, or stagnation (the callers' tests).
bool refine_done(kkt_ctx *ctx, RefineState &rs) {
    if (!std::isfinite(rs.rel)) { rs.status = KKT_WARN_REFINE; return true; }
    if (rs.rel <= ctx->opt.refine_tol) return true;
    if (rs.it >= ctx->opt.refine_max) { rs.status = KKT_WARN_REFINE; return true; }
    return false;
}

// classic refinement: x += M^-1 (b - K x)
template <typename T>
int refine_classic(kkt_ctx *ctx, const double *b, double *x, int64_t nrhs, RefineState &rs) {
    ResidualArgs ra = residual_args(ctx, nrhs);
    std::vector<double> nh(4 * nrhs), hist;
    int rc;
    while (true) {
        if ((rc = true_residual(ctx, ra, b, x, ctx->d_res, nrhs, nh, rs))) return rc;
        if (refine_done(ctx, rs)) break;
        hist.push_back(rs.rel);
        // stagnation: near the rounding floor one step without a 2x gain ends
        // refinement; above it, two consecutive such steps
        size_t h = hist.size();
        if (h >= 2 && hist[h - 1] < 1e-6 && hist[h - 1] > 0.5 * hist[h - 2]) { rs.status = KKT_WARN_REFINE; break; }
        if (h >= 3 && hist[h - 1] > 0.5 * hist[h - 2] && hist[h - 2] > 0.5 * hist[h - 3]) {
            rs.status = KKT_WARN_REFINE;
            break;
        }
        if ((rc = solve_once<T>(ctx, ctx->d_res, ctx->d_dx, nrhs))) return rc;
        launch_axpy(x, ctx->d_dx, ctx->ntot * nrhs, ctx->stream);
        ++rs.it;
    }
    return KKT_OK;
}

// Flexible GMRES on K x = b with the factorisation M as right
// preconditioner (z_j = M^-1 v_j, x = x0 + Z y), classical Gram-Schmidt with
// one reorthogonalisation, Givens rotations for the small least-squares
// problem on the host, restarted from the true FP64 residual every
// KRYLOV_M steps or once the estimated residual falls below half the target.
// The right-hand sides run side by side, each with its own Hessenberg matrix.
template <typename T>
int refine_fgmres(kkt_ctx *ctx, const double *b, double *x, int64_t nrhs, RefineState &rs) {
    hipStream_t st = ctx->stream;
    ResidualArgs ra = residual_args(ctx, nrhs);
    const int64_t n = ctx->ntot, blk = n * nrhs;
    constexpr int M = KRYLOV_M, ldh = KRYLOV_M + 1;
    double *V = ctx->d_V, *Z = ctx->d_Z;
    double *h1 = ctx->d_h, *h2 = h1 + ldh * nrhs, *nrm = h2 + ldh * nrhs, *yd = nrm + nrhs;
    const double *hh1 = ctx->h_pin, *hh2 = hh1 + ldh * nrhs, *hnrm = hh2 + ldh * nrhs;
    double *hy = ctx->h_pin + (yd - h1);
    std::vector<double> nh(4 * nrhs), bnorm(nrhs), H((size_t)nrhs * M * ldh), g((size_t)nrhs * ldh),
        cs((size_t)nrhs * M), sn((size_t)nrhs * M);
    double prev_cycle = INFINITY;
    int rc;
    while (true) {
        if ((rc = true_residual(ctx, ra, b, x, V, nrhs, nh, rs))) return rc;
        if (refine_done(ctx, rs)) break;
        // a restart that did not halve the residual ends refinement
        if (rs.rel > 0.5 * prev_cycle) { rs.status = KKT_WARN_REFINE; break; }
        prev_cycle = rs.rel;
        launch_norm(V, nrhs, n, ctx->d_kpart, nrm, 1, st);
        std::fill(g.begin(), g.end(), 0.0);
        for (int64_t k = 0; k < nrhs; ++k) {
            bnorm[k] = nh[4 * k + 1] > 0 ? nh[4 * k + 1] : 1.0;
            g[k * ldh] = nh[4 * k + 0];
        }
        int j = 0;
        while (j < M && rs.it < ctx->opt.refine_max) {
            double *Vj = V + j * blk, *Zj = Z + j * blk, *W = V + (j + 1) * blk;
            if ((rc = solve_once<T>(ctx, Vj, Zj, nrhs))) return rc;
            launch_matvec(ra, Zj, W, ctx->d_work, st);
            launch_dots(W, V, j + 1, nrhs, n, ctx->d_kpart, h1, ldh, st);
            launch_combine(W, V, j + 1, nrhs, n, h1, ldh, -1.0, st);
            launch_dots(W, V, j + 1, nrhs, n, ctx->d_kpart, h2, ldh, st);
            launch_combine(W, V, j + 1, nrhs, n, h2, ldh, -1.0, st);
            launch_norm(W, nrhs, n, ctx->d_kpart, nrm, 1, st);
            HIPCHK(hipMemcpyAsync(ctx->h_pin, h1, 8 * (2 * ldh * nrhs + nrhs), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            ++rs.it;
            double est = 0.0;
            for (int64_t k = 0; k < nrhs; ++k) {
                double *col = &H[((size_t)k * M + j) * ldh];
                double *c = &cs[(size_t)k * M], *s = &sn[(size_t)k * M], *gk = &g[(size_t)k * ldh];
                for (int i = 0; i <= j; ++i) col[i] = hh1[k * ldh + i] + hh2[k * ldh + i];
                col[j + 1] = hnrm[k];
                for (int i = 0; i < j; ++i) {
                    const double t = c[i] * col[i] + s[i] * col[i + 1];
                    col[i + 1] = -s[i] * col[i] + c[i] * col[i + 1];
                    col[i] = t;
                }
                const double r = std::hypot(col[j], col[j + 1]);
                c[j] = r > 0 ? col[j] / r : 1.0;
                s[j] = r > 0 ? col[j + 1] / r : 0.0;
                col[j] = r;
                col[j + 1] = 0.0;
                gk[j + 1] = -s[j] * gk[j];
                gk[j] = c[j] * gk[j];
                est = std::max(est, std::fabs(gk[j + 1]) / bnorm[k]);
            }
            ++j;
            if (ctx->opt.verbose) std::fprintf(stderr, "kkt_solve:   fgmres %d estimate %.3e\n", rs.it, est);
            if (!std::isfinite(est)) break;
            if (est <= 0.5 * ctx->opt.refine_tol) break;
        }
        // y = R^-1 g (upper triangular R in the rotated H), x += Z y
        for (int64_t k = 0; k < nrhs; ++k) {
            const double *gk = &g[(size_t)k * ldh];
            double *y = hy + k * ldh;
            for (int i = j - 1; i >= 0; --i) {
                double a = gk[i];
                for (int l = i + 1; l < j; ++l) a -= H[((size_t)k * M + l) * ldh + i] * y[l];
                const double d = H[((size_t)k * M + i) * ldh + i];
                y[i] = d != 0.0 && std::isfinite(a) ? a / d : 0.0;
            }
        }
        HIPCHK(hipMemcpyAsync(yd, hy, 8 * ldh * nrhs, hipMemcpyHostToDevice, st));
        launch_combine(x, Z, j, nrhs, n, yd, ldh, 1.0, st);
    }
    return KKT_OK;
}

}  // namespace

namespace {
// a dense Schur solve step whose in-block product waited past its bound
// (the wait between the workgroups of one launch); synchronises
bool dense_wait_failed(kkt_ctx *ctx) {
    if (!ctx->d_dsync) return false;
    int f = 0;
    if (hipMemcpyAsync(&f, ctx->d_dsync, sizeof(int), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return true;
    return f != 0;
}
}  // namespace

extern "C" int kkt_solve(kkt_ctx *ctx, const double *b, double *x, int64_t nrhs, kkt_solve_info *info) {
    if (!ctx) return KKT_ERR_ARG;
    if (!ctx->analyzed || !ctx->factored) return KKT_ERR_ORDER;
    if (!b || !x || b == x || nrhs < 1 || nrhs > 64) return KKT_ERR_ARG;
    if (ctx->fb_factored) {
        // the mixed path's values are factored in FP64 (see kkt_factor)
        ctx->fb->stream = ctx->stream;
        int rc = kkt_solve(ctx->fb, b, x, nrhs, info);
        if (info && rc >= 0) info->fallback_used = 1;
        return rc;
    }
    int rc = ensure_ws(ctx, nrhs);
    if (rc) return rc;
    hipStream_t st = ctx->stream;
    const bool mixed = ctx->opt.precision == KKT_MIXED;
    // non-finite right-hand sides are rejected before anything is written
    {
        int flag = 0;
        launch_zero<int>(ctx->d_flag + 1, 1, st);
        launch_check_finite(b, ctx->ntot * nrhs, ctx->d_flag + 1, st);
        HIPCHK(hipMemcpyAsync(&flag, ctx->d_flag + 1, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (flag) return KKT_ERR_NONFINITE;
    }
    mark(ctx, 4);
    if (ctx->d_dsync) launch_zero<int>(ctx->d_dsync, 1, st);
    rc = mixed ? solve_once<float>(ctx, b, x, nrhs) : solve_once<double>(ctx, b, x, nrhs);
    if (rc) return rc;
    RefineState rs;
    if (uses_krylov(ctx->opt))
        rc = mixed ? refine_fgmres<float>(ctx, b, x, nrhs, rs) : refine_fgmres<double>(ctx, b, x, nrhs, rs);
    else
        rc = mixed ? refine_classic<float>(ctx, b, x, nrhs, rs) : refine_classic<double>(ctx, b, x, nrhs, rs);
    if (rc) return rc;
    mark(ctx, 5);
    HIPCHK(hipGetLastError());
    if (ctx->timing) {
        HIPCHK(hipStreamSynchronize(st));
        ctx->times[3] = elapsed(ctx, 4, 5);
    }
    if (dense_wait_failed(ctx)) return KKT_ERR_HIP;
    if (mixed && rs.status == KKT_WARN_REFINE) {
        // refinement around the FP32 factor stopped above the target:
        // factor the same values in FP64 and solve again with that factor
        rc = fallback_factor(ctx);
        if (rc < 0) return rc;
        kkt_solve_info fi{};
        rc = kkt_solve(ctx->fb, b, x, nrhs, &fi);
        if (rc < 0) return rc;
        if (info) {
            *info = fi;
            info->refine_iters += rs.it;
            info->fallback_used = 1;
        }
        return rc;
    }
    if (info) {
        info->refine_iters = rs.it;
        info->rel_res = rs.rel;
        info->omega = rs.omega;
        info->fallback_used = 0;
        info->rel_floor = rs.floor;
    }
    return rs.status;
}

namespace {

// solve + `steps` classic refinement steps, entirely on the stream, with the
// workspace the context's pointers name at the time of the call; the norms
// of the final residual go to `norms` (4 nrhs + 8 doubles)
int solve_fixed_steps(kkt_ctx *ctx, const double *b, double *x, int64_t nrhs, int steps, double *norms) {
    hipStream_t st = ctx->stream;
    const bool mixed = ctx->opt.precision == KKT_MIXED;
    // a non-finite right-hand side is recorded for kkt_solve_status
    launch_zero<int>(ctx->d_flag + 1, 1, st);
    launch_check_finite(b, ctx->ntot * nrhs, ctx->d_flag + 1, st);
    if (ctx->d_dsync) launch_zero<int>(ctx->d_dsync, 1, st);
    int rc = mixed ? solve_once<float>(ctx, b, x, nrhs) : solve_once<double>(ctx, b, x, nrhs);
    if (rc) return rc;
    ResidualArgs ra = residual_args(ctx, nrhs);
    for (int k = 0; k < steps; ++k) {
        launch_residual(ra, b, x, ctx->d_res, ctx->d_work, norms, st);
        rc = mixed ? solve_once<float>(ctx, ctx->d_res, ctx->d_dx, nrhs) : solve_once<double>(ctx, ctx->d_res, ctx->d_dx, nrhs);
        if (rc) return rc;
        launch_axpy(x, ctx->d_dx, ctx->ntot * nrhs, st);
    }
    launch_residual(ra, b, x, ctx->d_res, ctx->d_work, norms, st);
    ctx->async_nrhs = nrhs;
    ctx->async_steps = steps;
    ctx->status_norms = norms;
    HIPCHK(hipGetLastError());
    return KKT_OK;
}

}  // namespace

// solve + `steps` classic refinement steps, entirely on the stream; the norms
// of the final residual stay on the device for kkt_solve_status
extern "C" int kkt_solve_async(kkt_ctx *ctx, const double *b, double *x, int64_t nrhs, int steps) {
    if (!ctx) return KKT_ERR_ARG;
    if (!ctx->analyzed || !ctx->factored) return KKT_ERR_ORDER;
    if (!b || !x || b == x || nrhs < 1 || nrhs > 64 || steps < 0 || ctx->timing) return KKT_ERR_ARG;
    if (ctx->ws_nrhs < nrhs) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIPCHK(hipStreamIsCapturing(ctx->stream, &cs));
        if (cs != hipStreamCaptureStatusNone) return KKT_ERR_ARG;  // workspace must exist before capture
        int rc = ensure_ws(ctx, nrhs);
        if (rc) return rc;
    }
    return solve_fixed_steps(ctx, b, x, nrhs, steps, ctx->d_norms);
}

// ---------------------------------------------------------------------------
// kkt_solve_noalloc: kkt_solve_async with its workspace in a fixed device
// array instead of memory the context allocates. Each device holds its own
// copy of the array (from the library's load until the process ends); host
// code reaches it only through the address hipGetSymbolAddress returns for
// the current device, never through the array's name.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t SCRATCH_DOUBLES = (int64_t)4 << 20;  // 32 MiB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_dev[MAX_DEVICES] = {};

// the array's device address on the current device, looked up once per device
int scratch_base(kkt_ctx *ctx, double **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return KKT_ERR_ARG;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        scratch_dev[dev] = (double *)p;
    }
    *out = scratch_dev[dev];
    return KKT_OK;
}

struct WsPtrs {
    double *xp, *uv, *bh, *y, *xg, *res, *dx, *norms, *work;
};
WsPtrs save_ws(const kkt_ctx *ctx) {
    return WsPtrs{ctx->d_xp, ctx->d_uv, ctx->d_bh, ctx->d_y, ctx->d_xg, ctx->d_res, ctx->d_dx, ctx->d_norms, ctx->d_work};
}
void restore_ws(kkt_ctx *ctx, const WsPtrs &w) {
    ctx->d_xp = w.xp;
    ctx->d_uv = w.uv;
    ctx->d_bh = w.bh;
    ctx->d_y = w.y;
    ctx->d_xg = w.xg;
    ctx->d_res = w.res;
    ctx->d_dx = w.dx;
    ctx->d_norms = w.norms;
    ctx->d_work = w.work;
}

}  // namespace

extern "C" int kkt_solve_noalloc(kkt_ctx *ctx, const double *b, double *x, int64_t nrhs, int steps) {
    if (!ctx) return KKT_ERR_ARG;
    if (!ctx->analyzed || !ctx->factored) return KKT_ERR_ORDER;
    if (!b || !x || b == x || nrhs < 1 || nrhs > 64 || steps < 0 || ctx->timing) return KKT_ERR_ARG;
    const Symbolic &S = ctx->sy;
    // the workspace of kkt_solve_async, carved from the array in 256-byte
    // aligned pieces: xp, uv, bh, y, xg, res, dx, work
    const int64_t count[8] = {(S.nA + S.nbord) * ctx->N * nrhs, S.Usize_vec() * ctx->N * nrhs, ctx->ng * nrhs,
                              ctx->ng * nrhs, ctx->ng * nrhs, ctx->ntot * nrhs, ctx->ntot * nrhs,
                              residual_work(ctx->N, S.nA, S.Ns, nrhs)};
    int64_t off[8], used = 0;
    for (int q = 0; q < 8; ++q) {
        off[q] = used;
        used += (int64_t)(align_up(8 * std::max<int64_t>(count[q], 1)) / 8);
    }
    if (used > SCRATCH_DOUBLES) {
        if (ctx->opt.verbose)
            std::fprintf(stderr, "kkt_solve_noalloc: needs %lld bytes of workspace, the fixed array holds %lld\n",
                         (long long)(8 * used), (long long)(8 * SCRATCH_DOUBLES));
        return KKT_ERR_TOOBIG;
    }
    double *base = nullptr;
    int rc = scratch_base(ctx, &base);
    if (rc) return rc;
    const WsPtrs saved = save_ws(ctx);
    WsPtrs w{base + off[0], base + off[1], base + off[2], base + off[3], base + off[4],
             base + off[5], base + off[6], ctx->d_snorms, base + off[7]};
    restore_ws(ctx, w);
    rc = solve_fixed_steps(ctx, b, x, nrhs, steps, ctx->d_snorms);
    restore_ws(ctx, saved);
    return rc;
}

extern "C" int kkt_solve_status(kkt_ctx *ctx, kkt_solve_info *info) {
    if (!ctx) return KKT_ERR_ARG;
    if (ctx->async_nrhs < 1) return KKT_ERR_ORDER;
    const int64_t nrhs = ctx->async_nrhs;
    std::vector<double> nh(4 * nrhs);
    int flag = 0;
    HIPCHK(hipMemcpyAsync(nh.data(), ctx->status_norms, 8 * 4 * nrhs, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(&flag, ctx->d_flag + 1, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (flag) return KKT_ERR_NONFINITE;
    if (dense_wait_failed(ctx)) return KKT_ERR_HIP;
    double rel = 0.0, omega = 0.0, fl = 0.0;
    for (int64_t k = 0; k < nrhs; ++k) {
        const double bn = nh[4 * k + 1] > 0 ? nh[4 * k + 1] : 1.0;
        rel = std::max(rel, nh[4 * k + 0] / bn);
        omega = std::max(omega, nh[4 * k + 2]);
        fl = std::max(fl, EPS64 * nh[4 * k + 3] / bn);
    }
    if (info) {
        info->refine_iters = ctx->async_steps;
        info->rel_res = rel;
        info->omega = omega;
        info->fallback_used = 0;
        info->rel_floor = fl;
    }
    if (!std::isfinite(rel) || rel > ctx->opt.refine_tol) return KKT_WARN_REFINE;
    return KKT_OK;
}

extern "C" int kkt_schur(kkt_ctx *ctx, double *S_out) {
    if (!ctx || !S_out) return KKT_ERR_ARG;
    if (!ctx->factored) return KKT_ERR_ORDER;
    if (ctx->ng == 0) return KKT_OK;
    const Symbolic &S = ctx->sy;
    const SbarSrc sb = sbar_src(ctx);
    launch_schur_prefix(sb.p, sb.stride, sb.off, ctx->N, S.Ns, ctx->opt.precision, ctx->d_prefix, ctx->stream);
    launch_schur_assemble(sb.p, sb.stride, sb.off, ctx->N, S.Ns, ctx->opt.precision, ctx->d_prefix,
                          ctx->has_corner ? ctx->d_corner : nullptr, S_out, nullptr, 0.0, nullptr, 1, ctx->stream);
    HIPCHK(hipGetLastError());
    return KKT_OK;
}

extern "C" int kkt_schur_blocks(kkt_ctx *ctx, double *out) {
    if (!ctx || !out) return KKT_ERR_ARG;
    if (!ctx->factored) return KKT_ERR_ORDER;
    if (ctx->ng == 0) return KKT_OK;
    const Symbolic &S = ctx->sy;
    const SbarSrc sb = sbar_src(ctx);
    launch_copy_sbar(sb.p, sb.stride, sb.off, ctx->N, S.nbord, ctx->opt.precision, out, ctx->stream);
    HIPCHK(hipGetLastError());
    return KKT_OK;
}

// ---------------------------------------------------------------------------
// slack elimination (section 2.1, Eqs. SCOPFslackAtEnd, SCOPFhessianReduced,
// SCOPFslackReduction)
// ---------------------------------------------------------------------------

extern "C" int kkt_set_slacks(kkt_ctx *ctx, int64_t n_slack, const int32_t *lam_row) {
    if (!ctx) return KKT_ERR_ARG;
    if (!ctx->analyzed) return KKT_ERR_ORDER;
    if (n_slack < 0 || (n_slack > 0 && !lam_row)) return KKT_ERR_ARG;
    const Symbolic &S = ctx->sy;
    std::vector<char> seen(S.nA, 0);
    std::vector<int64_t> dpos(n_slack);
    for (int64_t j = 0; j < n_slack; ++j) {
        const int32_t r = lam_row[j];
        // a multiplier row (negative pivot), at most one slack each
        if (r < S.n_primal || r >= S.nA || seen[r]) return KKT_ERR_ARG;
        seen[r] = 1;
        dpos[j] = ctx->pat_colptr[r];  // the diagonal leads its column
    }
    (void)hipStreamSynchronize(ctx->stream);
    for (void *q : ctx->slack_allocs) (void)hipFree(q);
    ctx->slack_allocs.clear();
    ctx->n_slack = 0;
    if (n_slack == 0) return KKT_OK;
    void *pr = nullptr, *pd = nullptr;
    if (hipMalloc(&pr, 4 * n_slack) != hipSuccess) return KKT_ERR_NOMEM;
    ctx->slack_allocs.push_back(pr);
    if (hipMalloc(&pd, 8 * n_slack) != hipSuccess) return KKT_ERR_NOMEM;
    ctx->slack_allocs.push_back(pd);
    HIPCHK(hipMemcpy(pr, lam_row, 4 * n_slack, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(pd, dpos.data(), 8 * n_slack, hipMemcpyHostToDevice));
    ctx->d_slack_row = (int32_t *)pr;
    ctx->d_slack_dpos = (int64_t *)pd;
    ctx->n_slack = n_slack;
    return KKT_OK;
}

extern "C" int kkt_slack_reduce(kkt_ctx *ctx, const double *A_vals, const double *Ls, const double *b,
                                const double *rs, double *A_out, double *b_out, int64_t nrhs) {
    if (!ctx) return KKT_ERR_ARG;
    if (!ctx->analyzed) return KKT_ERR_ORDER;
    if (!A_vals || !A_out || nrhs < 0 || (nrhs > 0 && (!b || !b_out)) ||
        (ctx->n_slack > 0 && (!Ls || (nrhs > 0 && !rs))))
        return KKT_ERR_ARG;
    const Symbolic &S = ctx->sy;
    hipStream_t st = ctx->stream;
    if (A_out != A_vals)
        HIPCHK(hipMemcpyAsync(A_out, A_vals, 8 * S.nnzA * ctx->N, hipMemcpyDeviceToDevice, st));
    if (nrhs > 0 && b_out != b)
        HIPCHK(hipMemcpyAsync(b_out, b, 8 * ctx->ntot * nrhs, hipMemcpyDeviceToDevice, st));
    launch_zero<int>(ctx->d_flag + 2, 1, st);
    launch_slack_reduce(Ls, rs, ctx->n_slack, ctx->N, nrhs, ctx->d_slack_row, ctx->d_slack_dpos, S.nnzA, S.nA,
                        ctx->ntot, A_out, b_out, ctx->d_flag + 2, st);
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, ctx->d_flag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return flag ? KKT_ERR_NONFINITE : KKT_OK;
}

extern "C" int kkt_slack_recover(kkt_ctx *ctx, const double *Ls, const double *rs, const double *x, double *s_out,
                                 int64_t nrhs) {
    if (!ctx) return KKT_ERR_ARG;
    if (!ctx->analyzed) return KKT_ERR_ORDER;
    if (nrhs < 1 || !x || (ctx->n_slack > 0 && (!Ls || !rs || !s_out))) return KKT_ERR_ARG;
    const Symbolic &S = ctx->sy;
    launch_slack_recover(Ls, rs, ctx->n_slack, ctx->N, nrhs, ctx->d_slack_row, S.nA, ctx->ntot, x, s_out,
                         ctx->stream);
    HIPCHK(hipGetLastError());
    return KKT_OK;
}

extern "C" int kkt_enable_timing(kkt_ctx *ctx, int on) {
    if (!ctx) return KKT_ERR_ARG;
    ctx->timing = on != 0;
    return KKT_OK;
}

extern "C" int kkt_phase_times(kkt_ctx *ctx, double *t) {
    if (!ctx || !t) return KKT_ERR_ARG;
    for (int i = 0; i < 5; ++i) t[i] = ctx->times[i];
    return KKT_OK;
}

extern "C" int kkt_dominant_kernel(kkt_ctx *ctx, kkt_kernel_stat *out) {
    if (!ctx || !out) return KKT_ERR_ARG;
    *out = ctx->kstat;
    return KKT_OK;
}

extern "C" void kkt_destroy(kkt_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->fb) kkt_destroy(ctx->fb);
    for (void *q : ctx->slack_allocs) (void)hipFree(q);
    free_ws(ctx);
    free_static(ctx);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : ctx->kev) (void)hipEventDestroy(e);
    if (ctx->ev_main) (void)hipEventDestroy(ctx->ev_main);
    if (ctx->ev_side) (void)hipEventDestroy(ctx->ev_side);
    if (ctx->ev_asm) (void)hipEventDestroy(ctx->ev_asm);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    delete ctx;
}
