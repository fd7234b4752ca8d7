// Host-side launchers of the device kernels (declarations).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "device.hpp"

namespace kkt {

struct ScatterArgs {
    const double *A;
    int64_t nnz;
    const int64_t *amap;
    const int8_t *adiag;
    const int32_t *adpiv;
    double dw, dc;
    const double *C0, *C1;
    int64_t n0, n1;
    const int64_t *c0map, *c1map;
};

// LDS of one workgroup (gfx950). The triangular solves of a large front keep
// the front's vector in LDS: the forward pass its m rows beside a 64x65
// staging tile, the backward pass its c pivot rows beside a 128x64 tile and
// the partial sums, at one right-hand side per pass at the limit.
constexpr int64_t LDS_BYTES = 160 * 1024;
constexpr int64_t MAX_FRONT_ROWS = (LDS_BYTES - 8 * 64 * 65) / 8;
constexpr int64_t MAX_FRONT_PIVOTS = (LDS_BYTES - 8 * (129 * 64 + 8 * 64)) / 8;

struct TreeArgs {
    const int32_t *cptr, *clist;
    const int64_t *relptr;
    const int32_t *rel;
    const int32_t *rows;
    const int64_t *rowptr;
    // children's update rows by front: vea[vea[s]] = ng groups, then the
    // groups' cumulative entry counts, then (update-vector offset, front row)
    // pairs; within a group no two entries share a front row
    const int32_t *vea;
};

// One launch of the blocked right-looking factorisation over a group of large
// fronts. Pivot columns go in 64-wide blocks inside outer panels (OUTER_W
// columns for the period fronts, SCHUR_OUTER_W for the dense Schur factor)
// of sub-panels of INNER_W columns: per block the pivot block (kind 0), the
// rows below it (kind 1) and the rest of the sub-panel (kind 2); after a
// sub-panel the next sub-panel's columns, after each outer panel one
// trailing update of rank <= the panel width (kind 3 on 64x64 tiles, kind 4
// on 128x128 tiles for large trailing matrices). The dense Schur factor's
// diagonal-block inverses, which only the dense solves use, follow its last
// panel (launch_inverses_all).
constexpr int OUTER_W = 512;
constexpr int INNER_W = 256;  // at most four pivot blocks (k_panel_trsm)
constexpr int SCHUR_OUTER_W = 512;
// period levels with a front of at least this many pivots use the lookahead plan
constexpr int LOOKAHEAD_PIVOTS = 2048;
// the dense Schur factor's panel-chain updates take 128x128 tiles only with
// at least this many rows below the panel (enough tiles for every CU)
constexpr int SCHUR_CHAIN_BIG_ROWS = 12288;
constexpr int MAX_OUTER_W = 512;
static_assert(OUTER_W <= 2 * INNER_W && SCHUR_OUTER_W <= 2 * INNER_W && SCHUR_OUTER_W <= MAX_OUTER_W,
              "at most two sub-panels per outer panel");
constexpr int INV_W = 256;
// width of the inverted diagonal blocks of the dense Schur factor that its
// solves use (built from INV_W ones by doubling)
constexpr int DENSE_INV_W = 4 * INV_W;
struct StepDev {
    int kind;
    int win;                // trailing updates: 0 all, 1 next panel's columns, 2 the rest
    int t0, pe;             // first column of the block (kinds 0-2) or panel (3); panel end
    int nf;                 // fronts in this launch
    const int32_t *fl;      // their FrontDesc indices
    const int32_t *pre;     // prefix sums of the per-front task counts (kinds 1-4)
    int ntasks;
};
// algorithmic flops and HBM bytes of one trailing-update launch on a front
void update_work(int t0, int pe, int c, int m, int win, double *flops, double *bytes);

template <typename T> void launch_zero(T *p, int64_t n, hipStream_t st);
void launch_check_finite(const double *v, int64_t n, int *flag, hipStream_t st);
template <typename T> void launch_scatter(const ScatterArgs &a, FactorArgs<T> fa, int64_t N, hipStream_t st);
template <typename T>
void launch_small_fronts(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *tasks, const int *ncls, int64_t N,
                         const TreeArgs &tr, hipStream_t st);
template <typename T>
void launch_extend_add(FactorArgs<T> fa, const FrontDesc *sd, const EaTask *tasks, int ntasks, int64_t N,
                       const TreeArgs &tr, hipStream_t st);
template <typename T>
void launch_step(FactorArgs<T> fa, const FrontDesc *sd, const StepDev &s, int64_t N, hipStream_t st);

// ---- solve -------------------------------------------------------------------
struct SolveArgs {
    int64_t N, nrhs, nv;     // nv = nA + nbord (length of a period's permuted vector)
    int64_t usz;             // sum of update rows (per period, per rhs)
    double *xp;              // [N][nrhs][nv]
    double *uv;              // [N][nrhs][usz]
};

template <typename T>
void launch_gather_rhs(const double *b, int64_t ntot, int64_t nA, const int32_t *perm, SolveArgs sa,
                       hipStream_t st);
// Fronts with more than TRI_W pivots (and rows below them) go through the
// pivot part of the solves in windows of TRI_W pivots: the window's diagonal
// block is inverted after the factorisation, one workgroup per front applies
// the inverse, and the products of the window with the rest of the pivot
// part are spread over many workgroups.
constexpr int TRI_W = 256;
static_assert(TRI_W == INV_W, "the solves' windows are the factor's inverted diagonal blocks");
// a front whose pivot part the solves take window by window (its vectors
// then never need to fit in LDS)
inline bool wide_front(int m, int c) { return c > TRI_W && m > c; }
struct TriWindow {
    int p0;                      // first pivot of the window
    const int32_t *fronts;       // wide fronts with more than p0 pivots
    const RowTask *rows;         // (front, first row) of 64 rows after the window (pivot and update rows)
    const RowTask *cols;         // (front, first column) of 64 pivot columns before the window
    int nfront, nrows, ncols;
};
// device task lists of one level for the solve kernels
struct LevelTasks {
    const int32_t *small;        // fronts of at most 64 rows
    const int32_t *large;        // the others, except the wide ones
    const RowTask *rect_rows;    // (front, first row) of 64 update rows of the large fronts that are not wide
    const RowTask *rect_cols;    // (front, first column) of 64 pivot columns of large and wide fronts
    const TriWindow *win;        // pivot windows of the wide fronts (host array)
    int nsmall, nlarge, nrect_rows, nrect_cols, nwin;
    int maxm, maxc;              // largest rows / pivots of the large fronts that are not wide
};

template <typename T>
void launch_fwd_level(const T *L, int64_t Lstride, const FrontDesc *sd, const LevelTasks &lt, const TreeArgs &tr,
                      SolveArgs sa, hipStream_t st);
template <typename T>
void launch_bwd_level(const T *L, int64_t Lstride, const FrontDesc *sd, const LevelTasks &lt, const TreeArgs &tr,
                      SolveArgs sa, hipStream_t st);
void launch_scatter_x(double *x, int64_t ntot, int64_t nA, const int32_t *perm, SolveArgs sa, const double *xg,
                      int64_t ng, hipStream_t st);
// border glue: rhs of the Schur system and the border values for the backward pass
void launch_schur_rhs(const double *b, int64_t ntot, int64_t nA, SolveArgs sa, int64_t Ns, int64_t uoff_border,
                      double *bh, hipStream_t st);
void launch_border_values(const double *xg, SolveArgs sa, int64_t nA, int64_t Ns, hipStream_t st);

// dense Schur: assembly, factor steps reuse launch_step, triangular solves
void launch_schur_prefix(const void *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns, int precision,
                         double *prefix, hipStream_t st);
// columns [q0, q1) of S (q1 < 0: to the last); the diagonal's entries set
// tau_s and amax_s when those are given
void launch_schur_assemble(const void *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns, int precision,
                           const double *prefix, const double *corner, double *S, double *tau_s, double eps,
                           double *amax_s, int mirror, hipStream_t st, int64_t q0 = 0, int64_t q1 = -1);
// the diagonal of S only: tau_s and amax_s (S itself is not written)
void launch_schur_diag(const void *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns, int precision,
                       const double *prefix, const double *corner, double *tau_s, double eps, double *amax_s,
                       hipStream_t st);
void launch_copy_sbar(const void *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t nb, int precision,
                      double *out, hipStream_t st);
// inverse of the INV_W diagonal block at j0 of the (single) front fl[0]
void launch_inv256(FactorArgs<double> fa, const FrontDesc *sd, const int32_t *fl, int j0, hipStream_t st);
// the TRI_W-wide diagonal-block inverses of the pivot part of every listed
// front of N periods (in place below the diagonal, after the front's
// factorisation, and transposed above it): the solves' windows of wide fronts
template <typename T>
void launch_window_inverses(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fronts, int nfront, int maxc,
                            int64_t N, hipStream_t st);
// the DENSE_INV_W diagonal-block inverses of the dense factor of one front
// with c pivots, after its factorisation (through INV_W and 2 INV_W ones;
// tmp: W^2 doubles per 2W block at each doubling, W < DENSE_INV_W)
void launch_inverses_all(FactorArgs<double> fa, const FrontDesc *sd, const int32_t *fl, int c, double *tmp,
                         hipStream_t st);
// structured Schur (section 4.3): thresholds from S's diagonal, front j
// [S_d[j] - U; S_o[j] - U], U accumulation, G_j = W_j Linv_j, and the solve
void launch_struct_tau(const void *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns, int precision,
                       const double *prefix, const double *corner, double *tau_s, double eps, double *amax_s,
                       hipStream_t st);
void launch_struct_front(const void *U, int64_t Ustride, int64_t uoff, int64_t Ns, int64_t j, int last, int precision,
                         const double *prefix, const double *corner, const double *Uprev, const double *Ubprev,
                         double *Uout, double *F, double *Ubz, hipStream_t st);
void launch_struct_g(const double *F, int m, int ns, double *G, double *GT, hipStream_t st);
// M_p = (I - G_{2p+1})(I - G_{2p}) and its transpose for the N/2 column pairs
void launch_struct_pair(const double *G, int ns, int N, double *M, double *MT, hipStream_t st);
// structured solves; with N even (N >= 4) two block columns per chain step
// (M, MT from launch_struct_pair; ce: [4][N/2][Ns] workspace)
bool struct_pairs(int64_t N);
void launch_struct_solve(const double *F, const double *G, const double *GT, const double *M, const double *MT,
                         int64_t N, int64_t Ns, const double *bh, double *xg, double *sa, double *aa, double *ce,
                         int64_t nrhs, hipStream_t st);
// inverse of the 2*INV_W diagonal block at j0 from its two INV_W inverses
// (tmp: INV_W x INV_W doubles)
void launch_inv_combine(FactorArgs<double> fa, const FrontDesc *sd, const int32_t *fl, int j0, int c, double *tmp,
                        hipStream_t st);
// sync: [0] failure flag (set if an in-block product's wait passed its
// bound), then 2 (ceil(ng / DENSE_INV_W) - 1) step counters, zeroed by the
// forward launcher
void launch_dense_fwd(const double *S, int64_t ng, double *v, double *y, int64_t nrhs, int *sync, hipStream_t st);
void launch_dense_bwd(const double *S, int64_t ng, double *z, double *x, int64_t nrhs, int *sync, hipStream_t st);

// ---- residual ------------------------------------------------------------------
struct ResidualArgs {
    int64_t N, nA, Ns, ntot, nrhs;
    const double *A;           // [N][nnz]
    int64_t nnz;
    // K's blocks as sliced ELLPACK (old order): 64-row slices, entry u of row
    // 64 s + l at sl_off[s] + 64 u + l; Asell [N][nnz_sell] the values with
    // the shifts on the diagonal, zero in the padding (column = the row)
    const int64_t *sl_off;
    const int32_t *sl_ci;
    const double *Asell;
    int64_t nnz_sell;
    const int64_t *c1tp, *c0tp;   // C_1^T, C_0^T by A column: (s, k)
    const int32_t *c1ts, *c0ts;
    const int64_t *c1tk, *c0tk;
    const int64_t *c0p, *c1p;  // C_0 / C_1 CSR
    const int32_t *c0i, *c1i;
    const double *C0v, *C1v;
    const double *corner;      // [ng] or null
    double dw, dc;
    int64_t n_primal;
};
// r = b - K x, plus per-rhs partial sums for ||r||_2, ||b||_2 and max omega;
// `work` holds residual_work(...) doubles
int64_t residual_work(int64_t N, int64_t nA, int64_t Ns, int64_t nrhs);
void launch_residual(const ResidualArgs &ra, const double *b, const double *x, double *r, double *work,
                     double *norms, hipStream_t st);
void launch_axpy(double *x, const double *dx, int64_t n, hipStream_t st);
// Asell[n][p] = A[n][sl_vi[p]] (+ delta_w / -delta_c on the diagonal), 0 in the padding
void launch_sell_values(const double *A, int64_t nnzA, int64_t N, int64_t nA, int64_t n_primal,
                        const int64_t *sl_off, const int32_t *sl_ci, const int32_t *sl_vi, int64_t nnz_sell,
                        double dw, double dc, double *Asell, hipStream_t st);
void launch_matvec(const ResidualArgs &ra, const double *x, double *y, double *work, hipStream_t st);

// ---- slack elimination (Eqs. SCOPFhessianReduced, SCOPFslackReduction) ----------
// A_out[n][dpos[j]] -= 1/Ls[n][j]; b_out rows n nA + lam_row[j] += rs / Ls;
// flag |= 1 where an L_s is not positive and finite
void launch_slack_reduce(const double *Ls, const double *rs, int64_t ns, int64_t N, int64_t nrhs,
                         const int32_t *lam_row, const int64_t *dpos, int64_t nnzA, int64_t nA, int64_t ntot,
                         double *A_out, double *b_out, int *flag, hipStream_t st);
// s_out = (rs + x[rows n nA + lam_row[j]]) / Ls
void launch_slack_recover(const double *Ls, const double *rs, int64_t ns, int64_t N, int64_t nrhs,
                          const int32_t *lam_row, int64_t nA, int64_t ntot, const double *x, double *s_out,
                          hipStream_t st);

// ---- Krylov helpers (vectors are [nrhs][n] blocks; coefficient arrays on device)
// h[k * ldh + i] = <W_k, V_i,k> for i < nv (deterministic two-stage sums;
// part holds nrhs * nv * 512 doubles)
void launch_dots(const double *W, const double *V, int nv, int64_t nrhs, int64_t n, double *part, double *h,
                 int ldh, hipStream_t st);
// W_k -= sum_i h[k * ldh + i] V_i,k   (sign = -1) or  += (sign = +1)
void launch_combine(double *W, const double *V, int nv, int64_t nrhs, int64_t n, const double *h, int ldh,
                    double sign, hipStream_t st);
// nrm[k] = ||W_k||_2 ; then W_k /= nrm[k] when normalize
void launch_norm(double *W, int64_t nrhs, int64_t n, double *part, double *nrm, int normalize, hipStream_t st);

}  // namespace kkt
