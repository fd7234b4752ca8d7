/*
 * libkkt -- MI355X (gfx950) solver for the block-bordered (arrowhead) KKT
 * system of a multiperiod AC optimal-power-flow problem with storage.
 *
 * The system (Eq. hessianPerm, section 4.1) in the ordering
 * u = (u_1, ..., u_N, u_g) of Eq. orderingMPOPF:
 *
 *     [ A_1                B_1^T ] [du_1]   [b_1]
 *     [      ...            ...  ] [ .. ] = [ ..]
 *     [            A_N     B_N^T ] [du_N]   [b_N]
 *     [ B_1  ...   B_N     C     ] [du_g]   [b_C]
 *
 * Every A_n (nA x nA, symmetric indefinite) shares one sparsity pattern. The
 * border follows Eq. B12N: B_n is (N*Ns) x nA with block row m equal to 0 for
 * m < n, C_1 for m = n and C_0 for m > n (C_0, C_1: Ns x nA, the same for every
 * period). C is the corner (zero, or a diagonal; section 4.1 gives a zero block
 * for MPOPF, the dual regularisation -delta_c I of section 2.3 makes it
 * negative definite).
 *
 * The solve is the Schur-complement decomposition of Algorithm 1 (section
 * 4.2, Eqs. SCform, SCsolve, SCsolve1): factor every A_n, form
 * S = C - sum_n B_n A_n^-1 B_n^T, factor S, solve for du_g, back-substitute
 * du_n = A_n^-1 (b_n - B_n^T du_g). The per-period contribution is built from
 * the 2*Ns distinct right-hand sides of Eq. LocalSchurBs3 and placed by the
 * structure of Eq. LocalSchurBs, then refined in FP64 (section 2.1).
 *
 * Conventions
 *  - All sizes are int64_t; index arrays are int32_t.
 *  - Device pointers are HIP device allocations owned by the caller and must
 *    stay valid until the work enqueued on the context's stream completes.
 *  - Host pointers are read during the call only (copied where kept).
 *  - Return codes: 0 OK; negative = error, outputs untouched, the context
 *    keeps its previous state; positive = warning, outputs valid.
 *  - One context per stream; calls on one context are not thread safe.
 *    Separate contexts are independent and may share a device.
 */
#ifndef KKT_H
#define KKT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define KKT_OK 0
#define KKT_ERR_ARG (-1)          /* bad argument (null pointer, bad size)   */
#define KKT_ERR_NOMEM (-2)        /* device allocation failed                */
#define KKT_ERR_ORDER (-3)        /* factor before analyze, solve before factor */
#define KKT_ERR_STRUCT (-4)       /* empty column, entry above the diagonal, */
                                  /* unsorted/duplicate row index, bad C col  */
#define KKT_ERR_HIP (-5)          /* HIP runtime error                        */
#define KKT_ERR_NONFINITE (-6)    /* NaN/Inf in the values or the RHS         */
#define KKT_ERR_TOOBIG (-7)       /* the system needs more workspace than the  */
                                  /* fixed array of kkt_solve_noalloc holds    */
#define KKT_WARN_PERTURBED 1      /* static pivots were perturbed             */
#define KKT_WARN_INERTIA 2        /* inertia differs from (N*n_primal,        */
                                  /*   N*(nA-n_primal)+N*Ns, 0)              */
#define KKT_WARN_REFINE 3         /* refinement stopped above refine_tol      */

/* ---- options ------------------------------------------------------------ */
#define KKT_FP64 0   /* every factor and solve in FP64                         */
#define KKT_MIXED 1  /* block factors and Schur contributions in FP32, FP64    */
                     /* refinement residual, FP64 dense Schur factorisation;   */
                     /* the elimination order then postpones every dual until  */
                     /* all its primal neighbours are eliminated (no growth     */
                     /* from early duals, more fill than the FP64 order).       */
                     /* FP64 fallback (kkt_factor, kkt_solve): when the FP32    */
                     /* factor's inertia differs from the expected one or it   */
                     /* perturbed pivots, or when refinement around it stops   */
                     /* above refine_tol, the same values are factored in FP64 */
                     /* (an internal FP64 analysis and factor, allocated on    */
                     /* first use and counted by kkt_footprint) and solved     */
                     /* with that factor; kkt_solve_info.fallback_used says so.*/
                     /* The enqueue-only calls have no fallback.                */

typedef struct kkt_options {
    int precision;      /* KKT_FP64 or KKT_MIXED                              */
    double pivot_eps;   /* static-pivot threshold factor (see kkt_factor);    */
                        /* 0 selects the default (1e-20 FP64, 1e-10 mixed)      */
    double refine_tol;  /* target max_k ||b_k - K x_k||_2 / ||b_k||_2, 1e-10   */
    int refine_max;     /* refinement steps at most (default 20)              */
    int verbose;        /* 0 quiet                                            */
    int refine_method;  /* KKT_REFINE_FGMRES (default) or KKT_REFINE_CLASSIC   */
    int big_tile_rows;  /* trailing updates of at least this many rows use     */
                        /* 128x128 tiles, smaller ones 64x64; 0 = default 512   */
                        /* (a tile-shape knob for autotuning)                   */
    int schur_mode;     /* KKT_SCHUR_DENSE (default) or KKT_SCHUR_STRUCTURED    */
    int recompute_periods; /* 0 (default): the factors and update matrices of */
                        /* every period stay in device memory. P > 0: only P  */
                        /* periods' are held at a time and the period factors */
                        /* are recomputed, chunk by chunk, before the forward */
                        /* and the backward sweep of every solve pass (the    */
                        /* memory-saving variant of section 4.3): about       */
                        /* N / P times less factor memory, two more block     */
                        /* factorisations per solve pass                       */
    int dual_wait;      /* elimination order: a dual becomes eligible once     */
                        /* min(dual_wait, its primal neighbours) of its primal */
                        /* neighbours are eliminated and it can claim one of   */
                        /* them that no earlier dual claimed; 0 = default      */
                        /* (FP64: 4, mixed: all of them). Larger values trade  */
                        /* fill for smaller pivot growth                       */
} kkt_options;

/* Factorisation of the Schur complement S (Algorithm 1 step 12):
 * KKT_SCHUR_DENSE: assemble the dense n_g x n_g S and factor it (LDL^T on
 *   FP64 MFMA, n_g^3/3 flops, n_g^2 doubles of device memory).
 * KKT_SCHUR_STRUCTURED: section 4.3 (Eq. GlobalSchur): every block below the
 *   diagonal of a block column of S is the same N_s x N_s matrix, so block
 *   elimination keeps that structure and only needs, for j = 1..N, the
 *   N_s x N_s pivot block S_jj - U_j, the common block below it S_j+1,j - U_j,
 *   and U_j+1 = U_j + (S_j+1,j - U_j)(S_jj - U_j)^-1 (S_j+1,j - U_j)^T:
 *   O(N N_s^3) flops and O(N N_s^2) memory. Same solution and inertia up to
 *   rounding; requires N_s <= 512 (kkt_analyze returns KKT_ERR_ARG beyond). */
#define KKT_SCHUR_DENSE 0
#define KKT_SCHUR_STRUCTURED 1

#define KKT_REFINE_FGMRES 0  /* flexible GMRES on K, right-preconditioned by the */
                             /* factorisation; CGS2 orthogonalisation            */
#define KKT_REFINE_CLASSIC 1 /* x += solve(b - K x)                              */

/* Fill *opt with the defaults above. */
void kkt_default_options(kkt_options *opt);

/* ---- structure (host pointers, copied by kkt_analyze) -------------------- */
typedef struct kkt_structure {
    int64_t nA;              /* rows of every A_n                              */
    int64_t n_primal;        /* leading rows of A_n with positive pivots       */
                             /* (primal: Hessian + barrier); the rest are duals */
    int64_t N;               /* number of periods (>= 1)                       */
    int64_t Ns;              /* rows of C_0 / C_1 (storage units, >= 0)         */
    const int64_t *A_colptr; /* [nA+1] lower-triangular CSC of A_n's pattern,   */
    const int32_t *A_rowind; /* [nnz]  rows sorted ascending, diagonal present  */
    const int64_t *C0_rowptr;/* [Ns+1] CSR of C_0 (may be NULL when Ns = 0)     */
    const int32_t *C0_colind;
    const int64_t *C1_rowptr;/* [Ns+1] CSR of C_1                              */
    const int32_t *C1_colind;
} kkt_structure;

typedef struct kkt_inertia {
    int64_t n_pos, n_neg, n_zero;  /* sign count of the computed pivots of all */
                                   /* A_n and of S (Haynsworth: = inertia of K) */
    int64_t n_perturbed;           /* pivots replaced by the static rule        */
    int inertia_ok;                /* 1 when equal to the expected inertia      */
} kkt_inertia;

typedef struct kkt_solve_info {
    int refine_iters;    /* refinement corrections applied                      */
    double rel_res;      /* max over right-hand sides of ||b-Kx||_2/||b||_2,     */
                         /* FP64, on the unscaled K                             */
    double omega;        /* componentwise backward error max_i |r_i|/(|K||x|+|b|)_i */
    int fallback_used;   /* 1 when the mixed path solved with FP64 factors of   */
                         /* the same values (see KKT_MIXED); refine_iters then  */
                         /* counts the steps of both attempts                  */
    double rel_floor;    /* max over right-hand sides of                        */
                         /* eps || |K||x| + |b| ||_2 / ||b||_2: a bound on the  */
                         /* relative residual that rounding x to FP64 alone can */
                         /* cause (and the error a residual summed in plain     */
                         /* FP64 would carry); informational                    */
} kkt_solve_info;

typedef struct kkt_symbolic_stats {
    int64_t n_supernodes;     /* supernodes of one period block (+1 border node) */
    int64_t n_levels;         /* height of the supernodal elimination tree       */
    int64_t nnz_L;            /* stored entries of one period's factor panels    */
    int64_t u_entries;        /* stored entries of one period's update matrices  */
    int64_t max_front;        /* largest front (rows)                            */
    int64_t max_pivots;       /* most pivots in one supernode                    */
    double flops_factor;      /* FP ops of one period's block factorisation      */
    int64_t device_bytes;     /* device memory a context of this structure holds */
} kkt_symbolic_stats;

typedef struct kkt_ctx kkt_ctx;

/* ---- lifecycle ------------------------------------------------------------
 * kkt_create: bind a context to `stream` (a hipStream_t; NULL = the default
 * stream) on the current device. `opt` may be NULL (defaults).            */
int kkt_create(kkt_ctx **ctx, void *stream, const kkt_options *opt);

/* kkt_analyze: symbolic analysis shared by all N periods (section 4.1's
 * arrowhead structure; Algorithm 1 step 1 on one device): a fill-reducing
 * approximate-minimum-degree order of A_n with the 2*Ns border rows
 * [C_1; C_0] appended last, the supernodal elimination tree, front row sets
 * and extend-add maps; then allocates device factors and workspace. Host
 * time only plus one host->device copy of the maps. May be called again
 * (re-analysis frees the previous state). Returns KKT_ERR_ARG when a front
 * with at most 256 pivots, or without rows below its pivots, has more than
 * 16 320 rows or 11 712 pivots (the triangular solves keep such a front's
 * vector in the 160 KiB of LDS of one workgroup), when a front with more
 * pivots and rows below them has a factor panel of 2^31 bytes or more
 * (rows x pivots x 8; its solves stream the vector through HBM with 32-bit
 * offsets), or when N*Ns > 46 000. */
int kkt_analyze(kkt_ctx *ctx, const kkt_structure *s);

/* Exact device bytes the context holds after kkt_analyze (for admission). */
int kkt_footprint(const kkt_ctx *ctx, size_t *bytes);

/* Host-only planning query: the same symbolic analysis without a context or
 * a device; fills *st (device_bytes for `opt`'s precision, nrhs_max RHS) and,
 * when perm != NULL, the fill-reducing order perm[new] = old (nA entries). */
int kkt_plan(const kkt_structure *s, const kkt_options *opt, int64_t nrhs_max,
             kkt_symbolic_stats *st, int32_t *perm);

/* kkt_factor: numeric factorisation for new values (Algorithm 1 steps 2-7,
 * section 4.2):
 *   A_vals     device [N][nnz_A] FP64, values of each A_n in the pattern
 *              order of kkt_analyze (lower triangle).
 *   C0_vals    device [nnz_C0], C1_vals device [nnz_C1] (NULL when Ns = 0).
 *   corner_diag device [N*Ns] diagonal of C, or NULL for C = 0.
 *   delta_w, delta_c: inertia-correction shifts (section 2.3) added as
 *              +delta_w to the first n_primal diagonal entries of every A_n
 *              and -delta_c to the remaining ones, without re-uploading.
 *   out        optional (host); when non-NULL the call synchronises the
 *              stream and reports the inertia counts.
 * Pivoting is static: a pivot d_k with |d_k| <= tau_k, tau_k = pivot_eps *
 * |a_kk| (the diagonal entry of the matrix being factored; pivot_eps * max|A|
 * when a_kk = 0), keeps its sign and takes magnitude tau_k. Inertia counts
 * the computed pivots before perturbation. With KKT_MIXED the call always
 * synchronises to read the FP32 factor's pivot counts, and reports the FP64
 * factor's inertia when it fell back (see KKT_MIXED).
 * Returns 0, KKT_WARN_PERTURBED or KKT_WARN_INERTIA (warnings only when out
 * is non-NULL, or on a fallback), or an error. */
int kkt_factor(kkt_ctx *ctx, const double *A_vals, const double *C0_vals,
               const double *C1_vals, const double *corner_diag,
               double delta_w, double delta_c, kkt_inertia *out);

/* kkt_solve: x = K^-1 b for nrhs right-hand sides (Eqs. SCsolve, SCsolve1)
 * with FP64 iterative refinement on the unscaled K until rel_res <=
 * refine_tol or refine_max steps (section 2.1): by default flexible GMRES
 * preconditioned with the factorisation, restarted with the true residual;
 * refinement also stops when a restart does not halve the residual (classic
 * refinement: when steps stop halving it). True residuals b - K x are summed
 * with compensated (twice-working-precision) arithmetic, so rel_res resolves
 * the residual of the FP64 solution itself. refine_max = 0 returns the
 * unrefined solution of the factorisation.
 *   b, x  device [nrhs][N*nA + N*Ns] FP64, column-major in u order; b != x.
 *   info  optional (host). The refinement loop reads one scalar per step
 *         from the device (a stream synchronisation per step).
 * Returns 0, KKT_WARN_REFINE, or an error; KKT_ERR_NONFINITE (x untouched)
 * when b holds a NaN or an infinity. */
int kkt_solve(kkt_ctx *ctx, const double *b, double *x, int64_t nrhs,
              kkt_solve_info *info);

/* ---- enqueue-only variants (no host synchronisation), for batches, graphs
 * and serving loops that keep many systems in flight ---------------------- */

/* kkt_set_stream: later calls of ctx enqueue on `stream` (a hipStream_t);
 * the caller orders any earlier work of the context on its old stream. */
int kkt_set_stream(kkt_ctx *ctx, void *stream);

/* kkt_factor_async: kkt_factor without any host synchronisation, so it can be
 * captured into a HIP graph. Non-finite input is not rejected up front: it is
 * recorded on the device and reported by kkt_factor_status, which also reads
 * the inertia (synchronises; returns as kkt_factor would, including
 * KKT_ERR_NONFINITE). Fails with KKT_ERR_ARG while timing is enabled. */
int kkt_factor_async(kkt_ctx *ctx, const double *A_vals, const double *C0_vals,
                     const double *C1_vals, const double *corner_diag,
                     double delta_w, double delta_c);
int kkt_factor_status(kkt_ctx *ctx, kkt_inertia *out);

/* kkt_solve_async: x = K^-1 b (Eqs. SCsolve, SCsolve1) followed by exactly
 * `steps` FP64 refinement steps x += solve(b - K x) (section 2.1), all on the
 * stream; the norms of the final residual stay on the device for
 * kkt_solve_status (synchronises; returns KKT_WARN_REFINE when rel_res is
 * above refine_tol, KKT_ERR_NONFINITE when b held a NaN or an infinity). The solve workspace for nrhs right-hand sides must exist
 * before a graph capture (any earlier kkt_solve or kkt_solve_async with at
 * least nrhs right-hand sides creates it); otherwise KKT_ERR_ARG. */
int kkt_solve_async(kkt_ctx *ctx, const double *b, double *x, int64_t nrhs, int steps);
int kkt_solve_status(kkt_ctx *ctx, kkt_solve_info *info);

/* kkt_solve_noalloc: kkt_solve_async (the same kernels and arithmetic, so
 * the same x bit for bit) for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc. The call allocates nothing: its solve workspace is a fixed
 * 32 MiB device array inside the library (one per device, held from the
 * library's first use on that device until the process ends), and the norms
 * of the final residual stay in the context (read them with
 * kkt_solve_status). The caller passes b and x as for kkt_solve_async; the
 * context must be analysed and factored (kkt_analyze / kkt_factor allocate as
 * usual). Every call on a device shares that device's array and leaves its
 * contents behind (each call writes all of the workspace it reads), so calls
 * that overlap on one device, from any context or stream, race: the caller
 * orders them (e.g. one stream, or an event between them).
 * Returns KKT_ERR_TOOBIG, with nothing enqueued, when the workspace for
 * nrhs right-hand sides exceeds the array: about
 * 8 * nrhs * (3 N nA + N u + 9 N Ns) bytes plus 9 KB per right-hand side,
 * with u the update-vector length of one period (a few times nA); e.g. 30
 * buses, 8 periods and 4 right-hand sides need well under 1 MiB. Other
 * errors as kkt_solve_async. */
int kkt_solve_noalloc(kkt_ctx *ctx, const double *b, double *x, int64_t nrhs, int steps);

/* ---- uneven batches (many independent systems, one submission) ----------- */

typedef struct kkt_batch kkt_batch;

/* kkt_batch_create: a batch with nstreams HIP streams (1..64) of default
 * priority. kkt_batch_add registers an analysed context with device
 * pointers to its values (as kkt_factor), right-hand sides and solution (as
 * kkt_solve); the pointers stay in use for the life of the batch and are read
 * or written on every run. Instances are placed on the streams by estimated
 * work, largest first onto the least loaded stream. */
int kkt_batch_create(kkt_batch **b, int nstreams);
int kkt_batch_add(kkt_batch *b, kkt_ctx *ctx, const double *A_vals, const double *C0_vals,
                  const double *C1_vals, const double *corner_diag, const double *rhs,
                  double *x, int64_t nrhs);

/* kkt_batch_run: enqueue kkt_factor_async + kkt_solve_async(refine_steps) of
 * every instance on its stream. Results are ready after kkt_batch_wait;
 * per-instance status through kkt_factor_status and kkt_solve_status of the
 * instance's context. use_graph (capture the sequence once into a HIP graph
 * and replay it) is currently switched off and returns KKT_ERR_ARG. */
int kkt_batch_run(kkt_batch *b, int refine_steps, int use_graph);
int kkt_batch_wait(kkt_batch *b);
/* stream index (0..nstreams-1) instance i runs on, -1 before the first run */
int kkt_batch_stream_of(const kkt_batch *b, int64_t i);
void kkt_batch_destroy(kkt_batch *b);

/* ---- slack elimination (section 2.1) --------------------------------------
 * A period block with line-flow (inequality) rows has a slack s_j per row,
 * linked to its multiplier row i by -1 with the diagonal L_s,j = S^-1 Y > 0
 * (Eq. SCOPFhessianSymmetric, slacks last in Eq. SCOPFslackAtEnd):
 *     [ A_n   E  ] [u_n]   [b_n]      E: -1 at (lam_row[j], j)
 *     [ E^T  L_s ] [s_n] = [r_n]
 * Eliminating the slacks whose L_s is well away from zero leaves
 * A_n - E L_s^-1 E^T (1/L_s,j subtracted from the diagonal of row lam_row[j])
 * and b_n - E L_s^-1 r_n (r_j / L_s,j added to that row): Eq.
 * SCOPFhessianReduced; afterwards L_s,j s_j = r_j + u_n[lam_row[j]] (Eq.
 * SCOPFslackReduction). Slacks near zero are left in A_n by the caller as
 * primal rows of the pattern. The reduced K is what kkt_factor / kkt_solve
 * see: its inertia lacks the N * n_slack positive eigenvalues of the
 * eliminated slacks.
 *
 * kkt_set_slacks: after kkt_analyze, the row of A_n (a multiplier row,
 * >= n_primal, at most one slack each; host array, copied) of each of the
 * n_slack eliminated slacks of every period. KKT_ERR_ARG otherwise. Holds
 * 12 bytes per slack of device memory beyond kkt_footprint.
 * kkt_slack_reduce: A_out = A_vals reduced, b_out = b reduced (device
 * pointers; A_out may be A_vals and b_out may be b, in place):
 *   A_vals, A_out  [N][nnz_A] as kkt_factor; Ls [N][n_slack];
 *   b, b_out       [nrhs][N*nA + N*Ns] as kkt_solve (nrhs may be 0: values only);
 *   rs             [nrhs][N*n_slack], period-major (r_n of period n at n*n_slack).
 * Synchronises; KKT_ERR_NONFINITE when an L_s is not positive and finite.
 * kkt_slack_recover: s_out [nrhs][N*n_slack] from the solution x of the
 * reduced system (device pointers, enqueued on the stream). */
int kkt_set_slacks(kkt_ctx *ctx, int64_t n_slack, const int32_t *lam_row);
int kkt_slack_reduce(kkt_ctx *ctx, const double *A_vals, const double *Ls, const double *b,
                     const double *rs, double *A_out, double *b_out, int64_t nrhs);
int kkt_slack_recover(kkt_ctx *ctx, const double *Ls, const double *rs, const double *x,
                      double *s_out, int64_t nrhs);

/* kkt_schur: write the assembled Schur complement S of the last kkt_factor
 * (dense n_g x n_g, column-major, both triangles; n_g = N*Ns) into the
 * caller's device buffer S_out. Diagnostic; enqueued on the stream. */
int kkt_schur(kkt_ctx *ctx, double *S_out);

/* kkt_schur_blocks: write the per-period local Schur blocks
 * S_bar_n = [[S_11,n, S_10,n^T], [S_10,n, S_00,n]], S_ij,n = -C_i A_n^-1 C_j^T
 * (Eq. LocalSchurBs3), as device [N][2Ns][2Ns] column-major. Diagnostic. */
int kkt_schur_blocks(kkt_ctx *ctx, double *Sbar_out);

/* kkt_stats: symbolic statistics of the analysed structure (host). */
int kkt_stats(const kkt_ctx *ctx, kkt_symbolic_stats *st);

/* kkt_phase_times: milliseconds of the phases of the last factor/solve,
 * measured with HIP events on the context's stream (syncs the stream):
 * [0] block factor, [1] Schur assembly, [2] Schur factor, [3] last solve
 * (all refinement steps), [4] summed launch durations of the Schur
 * trailing-update kernel (see kkt_dominant_kernel) in the last factor; t must
 * hold 5 doubles. Timing is off unless enabled with kkt_enable_timing(ctx, 1). */
int kkt_enable_timing(kkt_ctx *ctx, int on);
int kkt_phase_times(kkt_ctx *ctx, double *t);

/* Work and time of the dominant kernel of kkt_factor: the trailing update
 * F -= L D L^T of the dense Schur LDL^T (Algorithm 1 step 12) on 128x128
 * tiles, over its launches in the last kkt_factor with timing enabled.
 * Durations come from HIP events recorded around every launch on the stream it
 * is launched on. flops counts 2 K per updated lower-triangle entry; bytes
 * counts one read and one write of every updated entry plus one read of the
 * panel operands (the kernel's algorithmic HBM traffic). */
typedef struct {
    int64_t launches;
    double total_ms;
    double flops;
    double bytes;
} kkt_kernel_stat;
int kkt_dominant_kernel(kkt_ctx *ctx, kkt_kernel_stat *out);

void kkt_destroy(kkt_ctx *ctx);
const char *kkt_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* KKT_H */
