// Block solves through the multifrontal factors (Algorithm 1 steps 8 and 16,
// Eqs. SCsolve and SCsolve1), the border glue of the MPOPF coupling, and the
// triangular solves with the dense Schur factor (step 13).
//
// Forward pass (leaves to root) on the augmented factor [L 0; X I] of
// [A Bh^T; Bh 0]: the border rows end with -Bh A^-1 b_n = -(C_1 y_n, C_0 y_n),
// y_n = A_n^-1 b_n, which give r of Eq. SCsolve by a running sum over periods.
// Backward pass (root to leaves) with the border rows set to
// (du_g[n], sum_{m>n} du_g[m]) yields du_n = A_n^-1 (b_n - B_n^T du_g), i.e.
// Eq. SCsolve1 with B_n^T du_g = C_1^T du_g[n] + C_0^T sum_{m>n} du_g[m] (Eq. B12N).
// Vectors are FP64; factors are read in their stored precision.
#include "dense_index.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace kkt {

template <typename T>
__global__ void k_gather_rhs(const double *b, int64_t ntot, int64_t nA, const int32_t *perm, SolveArgs sa) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y, k = blockIdx.z;
    if (q >= sa.nv) return;
    double v = q < nA ? b[(int64_t)k * ntot + (int64_t)n * nA + perm[q]] : 0.0;
    sa.xp[((int64_t)n * sa.nrhs + k) * sa.nv + q] = v;
}

// Up to RB right-hand sides go through a front together (the factor is read
// once per pass); v[i * RBT + r] holds row i of right-hand side r, with zeros
// for the right-hand sides beyond the last.
constexpr int RB = 4;

constexpr int SNT = 512;  // threads of a front's triangular solve

// Inner loops load their factor entries in batches of LB from clamped,
// always-valid addresses and mask the surplus entries to zero afterwards, so
// that the loads of a batch are in flight together.
constexpr int LB = 16;
constexpr int SLB = 8;   // batch of the one-wavefront kernels of small fronts

// Stage a ROWS x 64 tile of a front (column-major, leading dimension m) into
// LDS as Lt[a + q * (ROWS + 1)]: rows r0 + a (a < nrow), columns c0 + q
// (q < ncol), and only q < a when `strict`; everything else is zero.
// nrow, ncol >= 1.
template <typename T, int NT, int ROWS = 64>
__device__ inline void stage_tile(double *Lt, const T *P, int m, int r0, int c0, int nrow, int ncol, bool strict,
                                  int tid) {
    constexpr int PER = ROWS * 64 / NT;
    T val[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * NT, a = idx % ROWS, q = idx / ROWS;
        val[u] = P[(r0 + min(a, nrow - 1)) + (int64_t)(c0 + min(q, ncol - 1)) * m];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int idx = tid + u * NT, a = idx % ROWS, q = idx / ROWS;
        const bool ok = a < nrow && q < ncol && (!strict || q < a);
        Lt[a + q * (ROWS + 1)] = ok ? (double)val[u] : 0.0;
    }
}

// acc[r] += sum_{q < nq} P[q * m] * w[q * RBT + r] for one row (P points at
// the row's entry in the first column); w is in LDS.
template <typename T, int RBT, int NB = LB>
__device__ inline void row_dot(const T *P, int64_t m, int nq, const double *w, double *acc) {
    for (int q0 = 0; q0 < nq; q0 += NB) {
        T l[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) l[u] = P[(int64_t)min(q0 + u, nq - 1) * m];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int q = min(q0 + u, nq - 1);
            const double x = q0 + u < nq ? (double)l[u] : 0.0;
#pragma unroll
            for (int r = 0; r < RBT; ++r) acc[r] += x * w[q * RBT + r];
        }
    }
}

// dst[i * RBT + r] = src[r * nv + idx[i]] for i < n, r < nr; zero for the
// other rows i < nrows and right-hand sides. Index loads, then value loads,
// four rows per thread at a time.
template <int RBT, int NT>
__device__ inline void gather_rows(double *dst, int nrows, int n, const int32_t *idx, const double *src, int64_t nv,
                                   int nr, int tid) {
    for (int i0 = 0; i0 < nrows; i0 += 4 * NT) {
        int32_t ri[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ri[u] = n > 0 ? idx[min(i0 + tid + u * NT, n - 1)] : 0;
        double val[4][RBT];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < RBT; ++r) val[u][r] = n > 0 ? src[(int64_t)min(r, nr - 1) * nv + ri[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + tid + u * NT;
            if (i < nrows)
#pragma unroll
                for (int r = 0; r < RBT; ++r) dst[i * RBT + r] = (i < n && r < nr) ? val[u][r] : 0.0;
        }
    }
}

// v[rel[i] * RBT + r] += U[r * usz + i] for the uc update rows of a child
// (rel is injective, so the rows of one child never collide)
template <int RBT, int NT>
__device__ inline void add_child(double *v, int uc, const int32_t *rel, const double *U, int64_t usz, int nr,
                                 int tid) {
    for (int i0 = 0; i0 < uc; i0 += 4 * NT) {
        int32_t ri[4];
        double uv[4][RBT];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = min(i0 + tid + u * NT, uc - 1);
            ri[u] = rel[i];
#pragma unroll
            for (int r = 0; r < RBT; ++r) uv[u][r] = U[(int64_t)min(r, nr - 1) * usz + i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + tid + u * NT < uc)
#pragma unroll
                for (int r = 0; r < RBT; ++r)
                    if (r < nr) v[ri[u] * RBT + r] += uv[u][r];
    }
}

// Forward pass of a front larger than 64 rows, pivot part: extend-add of the
// children's update vectors, then y = L11^-1 v over 64-column blocks with the
// stored inverses of the pivot blocks. Rows below the pivots leave with the
// children's contributions only; k_fwd_rect subtracts L21 y from them.
// With npiv = 0 only the extend-add is done, in place in HBM (a wide front,
// whose pivot part k_win solves window by window): the front's update
// vector cleared, then the children's groups added to it and to the pivot
// rows' x, with no vector in LDS (any front size).
template <typename T, int RBT>
__global__ __launch_bounds__(SNT) void k_fwd_tri(const T *L, int64_t Lstride, const FrontDesc *sd,
                                                 const int32_t *tasks, TreeArgs tr, SolveArgs sa, int npiv) {
    extern __shared__ double smem[];
    double *Lt = smem;             // 64 x 65 staging tile
    double *v = smem + 64 * 65;    // m x RBT
    int tx, n;
    period_task(tx, n);
    const int s = tasks[tx];
    const int tid = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    const T *P = L + (int64_t)n * Lstride + d.Loff;
    const int32_t *R = tr.rows + tr.rowptr[s];
    const int64_t ro = tr.relptr[s];
    const int p1 = min(c, npiv);
    if (npiv == 0) {
        const int32_t *rec = tr.vea + tr.vea[s];
        const int ng = rec[0];
        const int32_t *pr = rec + 1 + ng;
        for (int k0r = 0; k0r < sa.nrhs; k0r += RBT) {
            const int nr = min(RBT, (int)sa.nrhs - k0r);
            double *x0 = sa.xp + ((int64_t)n * sa.nrhs + k0r) * sa.nv;
            double *U0 = sa.uv + ((int64_t)n * sa.nrhs + k0r) * sa.usz;
            for (int idx = tid; idx < (m - c) * nr; idx += SNT) {
                const int i = idx / nr, r = idx % nr;
                U0[(int64_t)r * sa.usz + ro + i] = 0.0;
            }
            __syncthreads();
            for (int g = 0, e0 = 0; g < ng; ++g) {
                const int e1 = rec[1 + g];
                for (int idx = tid; idx < (e1 - e0) * nr; idx += SNT) {
                    const int e = e0 + idx / nr, r = idx % nr;
                    const int row = pr[2 * e + 1];
                    const double u = U0[(int64_t)r * sa.usz + pr[2 * e]];
                    if (row < c) x0[(int64_t)r * sa.nv + R[row]] += u;
                    else U0[(int64_t)r * sa.usz + ro + (row - c)] += u;
                }
                __syncthreads();
                e0 = e1;
            }
        }
        return;
    }
    for (int k0r = 0; k0r < sa.nrhs; k0r += RBT) {
        const int nr = min(RBT, (int)sa.nrhs - k0r);
        double *x0 = sa.xp + ((int64_t)n * sa.nrhs + k0r) * sa.nv;
        double *U0 = sa.uv + ((int64_t)n * sa.nrhs + k0r) * sa.usz;
        for (int idx = tid; idx < m * RBT; idx += SNT) {
            const int i = idx / RBT, r = idx % RBT;
            v[idx] = (r < nr && i < c) ? x0[(int64_t)r * sa.nv + R[i]] : 0.0;
        }
        __syncthreads();
        {
            // children's update vectors, one group of row-disjoint children at a time
            const int32_t *rec = tr.vea + tr.vea[s];
            const int ng = rec[0];
            const int32_t *pr = rec + 1 + ng;
            for (int g = 0, e0 = 0; g < ng; ++g) {
                const int e1 = rec[1 + g];
                for (int idx = tid; idx < (e1 - e0) * nr; idx += SNT) {
                    const int e = e0 + idx / nr, r = idx % nr;
                    v[pr[2 * e + 1] * RBT + r] += U0[(int64_t)r * sa.usz + pr[2 * e]];
                }
                __syncthreads();
                e0 = e1;
            }
        }
        for (int k0 = 0; k0 < p1; k0 += 64) {
            const int nb = min(64, p1 - k0);
            stage_tile<T, SNT>(Lt, P, m, k0, k0, nb, nb, true, tid);
            __syncthreads();
            const int i = tid & 63, r = tid >> 6;
            double yv = 0.0;
            if (i < nb && r < nr) {
                yv = v[(k0 + i) * RBT + r];
                for (int q = 0; q < i; ++q) yv += Lt[i + q * 65] * v[(k0 + q) * RBT + r];
            }
            __syncthreads();
            if (i < nb && r < nr) v[(k0 + i) * RBT + r] = yv;
            __syncthreads();
            for (int i2 = k0 + nb + tid; i2 < p1; i2 += SNT) {
                double acc[RBT];
#pragma unroll
                for (int rr = 0; rr < RBT; ++rr) acc[rr] = 0.0;
                row_dot<T, RBT>(P + i2 + (int64_t)k0 * m, m, nb, v + k0 * RBT, acc);
#pragma unroll
                for (int rr = 0; rr < RBT; ++rr) v[i2 * RBT + rr] -= acc[rr];
            }
            __syncthreads();
        }
        for (int idx = tid; idx < m * nr; idx += SNT) {
            const int i = idx / nr, r = idx % nr;
            if (i < c) x0[(int64_t)r * sa.nv + R[i]] = v[i * RBT + r];
            else U0[(int64_t)r * sa.usz + ro + (i - c)] = v[i * RBT + r];
        }
        __syncthreads();
    }
}

// Forward pass, rows below the pivots: u -= L21 y for 64 update rows of a
// front per workgroup (four column groups, reduced at the end). With qw > 0
// the rows lie below the window [q0w, q0w + qw) of a wide front and take
// that window's product only: v -= L[rows, window] y_window, on pivot rows
// and update rows alike.
template <typename T, int RBT>
__global__ __launch_bounds__(256) void k_fwd_rect(const T *L, int64_t Lstride, const FrontDesc *sd,
                                                  const RowTask *tasks, TreeArgs tr, SolveArgs sa, int q0w, int qw) {
    __shared__ double yb[256 * RBT];
    __shared__ double red[4 * 64 * RBT];
    int tx, n;
    period_task(tx, n);
    const RowTask tk = tasks[tx];
    const int s = tk.f, i0 = tk.r0;
    const int tid = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    const T *P = L + (int64_t)n * Lstride + d.Loff;
    const int32_t *R = tr.rows + tr.rowptr[s];
    const int64_t ro = tr.relptr[s];
    const int a = tid & 63, g = tid >> 6;
    const int i = i0 + a;
    const T *rowp = P + min(i, m - 1);
    const int qb = qw > 0 ? q0w : 0, qe = qw > 0 ? min(c, q0w + qw) : c;
    for (int k0r = 0; k0r < sa.nrhs; k0r += RBT) {
        const int nr = min(RBT, (int)sa.nrhs - k0r);
        double *x0 = sa.xp + ((int64_t)n * sa.nrhs + k0r) * sa.nv;
        double *U0 = sa.uv + ((int64_t)n * sa.nrhs + k0r) * sa.usz;
        double acc[RBT];
#pragma unroll
        for (int rr = 0; rr < RBT; ++rr) acc[rr] = 0.0;
        for (int q0 = qb; q0 < qe; q0 += 256) {
            const int nq = min(256, qe - q0);
            gather_rows<RBT, 256>(yb, 256, nq, R + q0, x0, sa.nv, nr, tid);
            __syncthreads();
            const int qa = 64 * g;
            if (qa < nq) row_dot<T, RBT>(rowp + (int64_t)(q0 + qa) * m, m, min(64, nq - qa), yb + qa * RBT, acc);
            __syncthreads();
        }
#pragma unroll
        for (int rr = 0; rr < RBT; ++rr) red[(g * 64 + a) * RBT + rr] = acc[rr];
        __syncthreads();
        if (g == 0 && i < m) {
            for (int rr = 0; rr < nr; ++rr) {
                const double t = red[(0 * 64 + a) * RBT + rr] + red[(1 * 64 + a) * RBT + rr] +
                                 red[(2 * 64 + a) * RBT + rr] + red[(3 * 64 + a) * RBT + rr];
                if (i < c) x0[(int64_t)rr * sa.nv + R[i]] -= t;
                else U0[(int64_t)rr * sa.usz + ro + (i - c)] -= t;
            }
        }
        __syncthreads();
    }
}

// Backward pass, rows below the pivots: for 64 pivot columns per workgroup,
// z = D^-1 v - L21^T x_below with x_below the ancestors' final values (L
// tiles staged through LDS so that global reads run down the columns). z
// replaces v in place; k_bwd_tri finishes with L11^T. With qw > 0 the rows
// are a solved pivot window [q0w, q0w + qw) of a wide front and the columns
// lie before it: z -= L[window, columns]^T x_window, without the division.
template <typename T, int RBT>
__global__ __launch_bounds__(256) void k_bwd_rect(const T *L, int64_t Lstride, const FrontDesc *sd,
                                                  const RowTask *tasks, TreeArgs tr, SolveArgs sa, int q0w, int qw) {
    __shared__ double Lt[64 * 65];  // the staged tile; the partial sums at the end
    __shared__ double xb[64 * RBT];
    double *red = Lt;
    int tx, n;
    period_task(tx, n);
    const RowTask tk = tasks[tx];
    const int s = tk.f, q0 = tk.r0;
    const int tid = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    if (qw == 0 && m == c) return;
    const T *P = L + (int64_t)n * Lstride + d.Loff;
    const BufRes rs = make_bufres(P, (int64_t)m * c * sizeof(T));
    const int32_t *R = tr.rows + tr.rowptr[s];
    const int q = tid & 63, g = tid >> 6;
    const int ncol = min(64, (qw > 0 ? q0w : c) - q0);
    const int ib0 = qw > 0 ? q0w : c, ib1 = qw > 0 ? min(c, q0w + qw) : m;
    for (int k0r = 0; k0r < sa.nrhs; k0r += RBT) {
        const int nr = min(RBT, (int)sa.nrhs - k0r);
        double *x0 = sa.xp + ((int64_t)n * sa.nrhs + k0r) * sa.nv;
        double acc[RBT];
#pragma unroll
        for (int rr = 0; rr < RBT; ++rr) acc[rr] = 0.0;
        // the next tile's factor entries (16 per thread: row q, columns g + 4 u
        // of the 64 x 64 tile, by buffer loads at 32-bit offsets from the
        // front, whose at most 16 320 x 11 712 entries stay below 2^31 bytes)
        // and, for the first 64 threads, its row's x values: loaded while the
        // current tile is used
        T lv[16];
        double xv[RBT];
        auto fetch = [&](int ib) {
            const int nrow = min(64, ib1 - ib);
            const int base = (int)sizeof(T) * (ib + min(q, nrow - 1) + q0 * m);
#pragma unroll
            for (int u = 0; u < 16; ++u)
                lv[u] = buf_load(rs, base + (int)sizeof(T) * min(g + 4 * u, ncol - 1) * m, T(0));
            if (tid < 64) {
                const int32_t ri = R[ib + min(tid, nrow - 1)];
#pragma unroll
                for (int rr = 0; rr < RBT; ++rr)
                    xv[rr] = (tid < nrow && rr < nr) ? x0[(int64_t)rr * sa.nv + ri] : 0.0;
            }
        };
        if (ib0 < ib1) fetch(ib0);
        for (int ib = ib0; ib < ib1; ib += 64) {
            const int nrow = min(64, ib1 - ib);
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int qq = g + 4 * u;
                Lt[q + qq * 65] = (q < nrow && qq < ncol) ? (double)lv[u] : 0.0;
            }
            if (tid < 64)
#pragma unroll
                for (int rr = 0; rr < RBT; ++rr) xb[tid * RBT + rr] = xv[rr];
            __syncthreads();
            if (ib + 64 < ib1) fetch(ib + 64);
#pragma unroll 4
            for (int a = 16 * g; a < 16 * g + 16; ++a) {
                const double l = Lt[a + q * 65];
#pragma unroll
                for (int rr = 0; rr < RBT; ++rr) acc[rr] += l * xb[a * RBT + rr];
            }
            __syncthreads();
        }
#pragma unroll
        for (int rr = 0; rr < RBT; ++rr) red[(g * 64 + q) * RBT + rr] = acc[rr];
        __syncthreads();
        if (g == 0 && q < ncol) {
            const double dq = qw > 0 ? 1.0 : (double)P[(q0 + q) + (int64_t)(q0 + q) * m];
            for (int rr = 0; rr < nr; ++rr) {
                const double t = red[(0 * 64 + q) * RBT + rr] + red[(1 * 64 + q) * RBT + rr] +
                                 red[(2 * 64 + q) * RBT + rr] + red[(3 * 64 + q) * RBT + rr];
                double *xp = x0 + (int64_t)rr * sa.nv + R[q0 + q];
                *xp = (qw > 0 ? *xp : *xp / dq) - t;
            }
        }
        __syncthreads();
    }
}

// Backward pass of a front larger than 64 rows, pivot part: left-looking over
// 64-column blocks from the last, z_b -= L[below b, b]^T x (rows < c only),
// then x_b = X_b^T z_b with X_b the stored inverse of the pivot block. The
// division by D and the rows below the pivots were applied by k_bwd_rect,
// except for fronts without such rows.
template <typename T, int RBT>
__global__ __launch_bounds__(SNT) void k_bwd_tri(const T *L, int64_t Lstride, const FrontDesc *sd,
                                                 const int32_t *tasks, TreeArgs tr, SolveArgs sa) {
    extern __shared__ double smem[];
    double *Lt = smem;                 // 128 x 64 staging tile (ld 129)
    double *red = smem + 129 * 64;     // 8 groups x 64 columns x RBT partial sums
    double *v = red + 8 * 64 * RBT;    // c x RBT
    int tx, n;
    period_task(tx, n);
    const int s = tasks[tx];
    const int tid = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    if (c == 0) return;
    const T *P = L + (int64_t)n * Lstride + d.Loff;
    const int32_t *R = tr.rows + tr.rowptr[s];
    const int q = tid & 63, g = tid >> 6;
    const bool divide = m == c;
    for (int k0r = 0; k0r < sa.nrhs; k0r += RBT) {
        const int nr = min(RBT, (int)sa.nrhs - k0r);
        double *x0 = sa.xp + ((int64_t)n * sa.nrhs + k0r) * sa.nv;
        gather_rows<RBT, SNT>(v, c, c, R, x0, sa.nv, nr, tid);
        if (divide) {
            __syncthreads();
            for (int i = tid; i < c; i += SNT) {
                const double dd = (double)P[i + (int64_t)i * m];
#pragma unroll
                for (int r = 0; r < RBT; ++r) v[i * RBT + r] /= dd;
            }
        }
        __syncthreads();
        for (int kb = ((c - 1) / 64) * 64; kb >= 0; kb -= 64) {
            const int nb = min(64, c - kb);
            double acc[RBT];
#pragma unroll
            for (int rr = 0; rr < RBT; ++rr) acc[rr] = 0.0;
            for (int ib = kb + nb; ib < c; ib += 128) {
                const int nrow = min(128, c - ib);
                stage_tile<T, SNT, 128>(Lt, P, m, ib, kb, nrow, nb, false, tid);
                __syncthreads();
                const int a1 = min(16 * g + 16, nrow);
                for (int a = 16 * g; a < a1; ++a) {
                    const double l = Lt[a + q * 129];
#pragma unroll
                    for (int rr = 0; rr < RBT; ++rr) acc[rr] += l * v[(ib + a) * RBT + rr];
                }
                __syncthreads();
            }
#pragma unroll
            for (int rr = 0; rr < RBT; ++rr) red[(g * 64 + q) * RBT + rr] = acc[rr];
            stage_tile<T, SNT>(Lt, P, m, kb, kb, nb, nb, true, tid);
            __syncthreads();
            if (g < nr && q < nb) {
                double t = 0.0;
#pragma unroll
                for (int gg = 0; gg < 8; ++gg) t += red[(gg * 64 + q) * RBT + g];
                v[(kb + q) * RBT + g] -= t;
            }
            __syncthreads();
            double xv = 0.0;
            if (g < nr && q < nb) {
                xv = v[(kb + q) * RBT + g];
                for (int i = q + 1; i < nb; ++i) xv += Lt[i + q * 65] * v[(kb + i) * RBT + g];
            }
            __syncthreads();
            if (g < nr && q < nb) v[(kb + q) * RBT + g] = xv;
            __syncthreads();
        }
        for (int idx = tid; idx < c * nr; idx += SNT) {
            const int i = idx / nr, r = idx % nr;
            x0[(int64_t)r * sa.nv + R[i]] = v[i * RBT + r];
        }
        __syncthreads();
    }
}

// Pivot window [p0, p0 + TRI_W) of a wide front, whose diagonal block holds
// the inverse X of its unit lower triangle below the diagonal and X^T above
// it (built after the factorisation): y = X v (forward, UPPER false) or
// x = X^T z (backward, UPPER true) in place for the window's rows, as
// products along the rows of the stored triangle: 1024 threads as 256 rows
// by four 64-column quarters, the loads of a quarter in flight in batches.
template <typename T, int RBT, bool UPPER>
__global__ __launch_bounds__(1024) void k_win(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *fronts,
                                              TreeArgs tr, SolveArgs sa, int p0) {
    __shared__ double v[TRI_W * RBT];
    __shared__ double part[4 * TRI_W * RBT];
    int tx, n;
    period_task(tx, n);
    const int s = fronts[tx];
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    const int nw = min(TRI_W, c - p0);
    const T *P = L + (int64_t)n * Lstride + d.Loff + p0 + (int64_t)p0 * m;  // the window's diagonal block
    const int32_t *R = tr.rows + tr.rowptr[s] + p0;
    const int tid = threadIdx.x, i = tid & (TRI_W - 1), g = tid >> 8;
    // columns [qa, qb) of row i: below the diagonal (q < i) or above it (q > i)
    const int qa = UPPER ? max(64 * g, i + 1) : 64 * g;
    const int qb = UPPER ? min(64 * g + 64, nw) : min(64 * g + 64, min(i, nw));
    for (int k0r = 0; k0r < sa.nrhs; k0r += RBT) {
        const int nr = min(RBT, (int)sa.nrhs - k0r);
        double *x0 = sa.xp + ((int64_t)n * sa.nrhs + k0r) * sa.nv;
        if (g == 0)
#pragma unroll
            for (int r = 0; r < RBT; ++r) v[i * RBT + r] = (i < nw && r < nr) ? x0[(int64_t)r * sa.nv + R[i]] : 0.0;
        __syncthreads();
        double acc[RBT];
#pragma unroll
        for (int r = 0; r < RBT; ++r) acc[r] = 0.0;
        if (i < nw && qb > qa) row_dot<T, RBT>(P + i + (int64_t)qa * m, m, qb - qa, v + qa * RBT, acc);
#pragma unroll
        for (int r = 0; r < RBT; ++r) part[(g * TRI_W + i) * RBT + r] = acc[r];
        __syncthreads();
        if (g == 0 && i < nw)
            for (int r = 0; r < nr; ++r)
                x0[(int64_t)r * sa.nv + R[i]] = v[i * RBT + r] + ((part[i * RBT + r] + part[(TRI_W + i) * RBT + r]) +
                                                                  (part[(2 * TRI_W + i) * RBT + r] +
                                                                   part[(3 * TRI_W + i) * RBT + r]));
        __syncthreads();
    }
}

// Fronts of at most 64 rows: one wavefront per front, lane i owns row i
// (forward) or pivot column i (backward).
template <typename T>
__global__ __launch_bounds__(64) void k_fwd_small(const T *L, int64_t Lstride, const FrontDesc *sd,
                                                  const int32_t *tasks, TreeArgs tr, SolveArgs sa) {
    __shared__ double vs[64 * RB];
    int tx, n;
    period_task(tx, n);
    const int s = tasks[tx];
    const int i = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    const T *P = L + (int64_t)n * Lstride + d.Loff;
    const T *rowp = P + min(i, m - 1);
    const int32_t *R = tr.rows + tr.rowptr[s];
    const int64_t ro = tr.relptr[s];
    for (int k0r = 0; k0r < sa.nrhs; k0r += RB) {
        const int nr = min(RB, (int)sa.nrhs - k0r);
        double *x0 = sa.xp + ((int64_t)n * sa.nrhs + k0r) * sa.nv;
        double *U0 = sa.uv + ((int64_t)n * sa.nrhs + k0r) * sa.usz;
        const int32_t Ri = i < c ? R[i] : 0;
#pragma unroll
        for (int r = 0; r < RB; ++r) vs[i * RB + r] = (i < c && r < nr) ? x0[(int64_t)r * sa.nv + Ri] : 0.0;
        __syncthreads();
        for (int qc = tr.cptr[s]; qc < tr.cptr[s + 1]; ++qc) {
            const int ch = tr.clist[qc];
            const int uc = sd[ch].m - sd[ch].c;
            if (i < uc) {
                const int row = tr.rel[tr.relptr[ch] + i];
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    if (r < nr) vs[row * RB + r] += U0[(int64_t)r * sa.usz + tr.relptr[ch] + i];
            }
            __syncthreads();
        }
        // y = X v on the pivot rows (X[i][q] for q < i)
        double y[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) y[r] = vs[i * RB + r];
        for (int q0 = 0; q0 < c; q0 += SLB) {
            T l[SLB];
#pragma unroll
            for (int u = 0; u < SLB; ++u) l[u] = rowp[(int64_t)min(q0 + u, c - 1) * m];
#pragma unroll
            for (int u = 0; u < SLB; ++u) {
                const int q = min(q0 + u, c - 1);
                const double x = (q0 + u < i && i < c) ? (double)l[u] : 0.0;
#pragma unroll
                for (int r = 0; r < RB; ++r) y[r] += x * vs[q * RB + r];
            }
        }
        __syncthreads();
        if (i < c) {
#pragma unroll
            for (int r = 0; r < RB; ++r) vs[i * RB + r] = y[r];
        }
        __syncthreads();
        // update rows: u -= L21 y
        if (i >= c) {
            double acc[RB] = {0.0, 0.0, 0.0, 0.0};
            row_dot<T, RB, SLB>(rowp, m, c, vs, acc);
#pragma unroll
            for (int r = 0; r < RB; ++r) y[r] -= acc[r];
        }
        if (i < m) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                if (r >= nr) continue;
                if (i < c) x0[(int64_t)r * sa.nv + Ri] = y[r];
                else U0[(int64_t)r * sa.usz + ro + (i - c)] = y[r];
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(64) void k_bwd_small(const T *L, int64_t Lstride, const FrontDesc *sd,
                                                  const int32_t *tasks, TreeArgs tr, SolveArgs sa) {
    __shared__ double vs[64 * RB];
    int tx, n;
    period_task(tx, n);
    const int s = tasks[tx];
    const int i = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    if (c == 0) return;
    const T *P = L + (int64_t)n * Lstride + d.Loff;
    const T *col = P + (int64_t)min(i, c - 1) * m;   // pivot column of lane i
    const int32_t *R = tr.rows + tr.rowptr[s];
    for (int k0r = 0; k0r < sa.nrhs; k0r += RB) {
        const int nr = min(RB, (int)sa.nrhs - k0r);
        double *x0 = sa.xp + ((int64_t)n * sa.nrhs + k0r) * sa.nv;
        const int32_t Ri = i < m ? R[i] : 0;
        const double dd = i < c ? (double)P[i + (int64_t)i * m] : 1.0;
#pragma unroll
        for (int r = 0; r < RB; ++r) vs[i * RB + r] = (i < m && r < nr) ? x0[(int64_t)r * sa.nv + Ri] / dd : 0.0;
        __syncthreads();
        // z = D^-1 v - L21^T x_below
        double z[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) z[r] = vs[i * RB + r];
        for (int j0 = c; j0 < m; j0 += SLB) {
            T l[SLB];
#pragma unroll
            for (int u = 0; u < SLB; ++u) l[u] = col[min(j0 + u, m - 1)];
#pragma unroll
            for (int u = 0; u < SLB; ++u) {
                const int j = min(j0 + u, m - 1);
                const double x = j0 + u < m ? (double)l[u] : 0.0;
#pragma unroll
                for (int r = 0; r < RB; ++r) z[r] -= x * vs[j * RB + r];
            }
        }
        __syncthreads();
        if (i < c) {
#pragma unroll
            for (int r = 0; r < RB; ++r) vs[i * RB + r] = z[r];
        }
        __syncthreads();
        // x = X^T z on the pivot block (X[j][i] for j > i)
        for (int j0 = 0; j0 < c; j0 += SLB) {
            T l[SLB];
#pragma unroll
            for (int u = 0; u < SLB; ++u) l[u] = col[min(j0 + u, c - 1)];
#pragma unroll
            for (int u = 0; u < SLB; ++u) {
                const int j = min(j0 + u, c - 1);
                const double x = (j0 + u > i && j0 + u < c) ? (double)l[u] : 0.0;
#pragma unroll
                for (int r = 0; r < RB; ++r) z[r] += x * vs[j * RB + r];
            }
        }
        if (i < c) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
                if (r < nr) x0[(int64_t)r * sa.nv + Ri] = z[r];
        }
        __syncthreads();
    }
}

__global__ void k_scatter_x(double *x, int64_t ntot, int64_t nA, const int32_t *perm, SolveArgs sa,
                            const double *xg, int64_t ng) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y, k = blockIdx.z;
    if (q < nA) x[(int64_t)k * ntot + (int64_t)n * nA + perm[q]] = sa.xp[((int64_t)n * sa.nrhs + k) * sa.nv + q];
    if (n == 0 && q < ng) x[(int64_t)k * ntot + sa.N * nA + q] = xg[(int64_t)k * ng + q];
}

// bh = b_C - r, r block m = C_1 y_m + sum_{n<m} C_0 y_n; the border node's
// update vector of period n holds -(C_1 y_n, C_0 y_n).
// (the running sums walk the periods in order; the loads of PB periods are
// issued together)
constexpr int PB = 16;
__global__ void k_schur_rhs(const double *b, int64_t ntot, int64_t nA, SolveArgs sa, int64_t Ns,
                            int64_t uoff_border, double *bh) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= Ns) return;
    const int64_t ng = sa.N * Ns;
    double acc = 0.0;
    for (int64_t m0 = 0; m0 < sa.N; m0 += PB) {
        double u0[PB], u1[PB], bc[PB];
#pragma unroll
        for (int t = 0; t < PB; ++t) {
            const int64_t m = min(m0 + t, sa.N - 1);
            const double *ub = sa.uv + ((int64_t)m * sa.nrhs + k) * sa.usz + uoff_border;
            u0[t] = ub[i];
            u1[t] = ub[Ns + i];
            bc[t] = b[(int64_t)k * ntot + sa.N * nA + m * Ns + i];
        }
#pragma unroll
        for (int t = 0; t < PB; ++t)
            if (m0 + t < sa.N) {
                bh[(int64_t)k * ng + (m0 + t) * Ns + i] = bc[t] + u0[t] + acc;
                acc += u1[t];
            }
    }
}

// border rows of every period for the backward pass: (du_g[n], sum_{m>n} du_g[m])
__global__ void k_border_values(const double *xg, SolveArgs sa, int64_t nA, int64_t Ns) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= Ns) return;
    const int64_t ng = sa.N * Ns;
    double acc = 0.0;
    for (int64_t n1 = sa.N - 1; n1 >= 0; n1 -= PB) {
        double g[PB];
#pragma unroll
        for (int t = 0; t < PB; ++t) g[t] = xg[(int64_t)k * ng + max(n1 - t, (int64_t)0) * Ns + i];
#pragma unroll
        for (int t = 0; t < PB; ++t)
            if (n1 - t >= 0) {
                double *x = sa.xp + ((n1 - t) * sa.nrhs + k) * sa.nv;
                x[nA + i] = g[t];
                x[nA + Ns + i] = acc;
                acc += g[t];
            }
    }
}

// ---- dense Schur factor solves ----------------------------------------------
// The factor of S (column-major, ld ng) keeps D on its diagonal, the inverse
// X_J of every unit lower DBW x DBW diagonal block J strictly below that
// block's diagonal, and L elsewhere strictly below the diagonal (the upper
// triangle is not read). Steps go over DBW-wide blocks: forward y_J = X_J v_J
// then v_below -= L[below, J] y_J (rows of a column block); backward x_J =
// X_J^T z_J then z_above -= L[J, above]^T x_J (dot products down columns).
constexpr int DBW = DENSE_INV_W;  // the factor holds the inverses of its DBW-wide diagonal blocks
static_assert(DBW == DENSE_BLOCK && RB == DS_RB, "dense solve geometry");

// Signals between the workgroups of one launch. A producer workgroup, once
// its outputs are stored, adds one to a counter with an agent-scope release
// (its stores become visible to every XCD before the add); a consumer
// workgroup waits with agent-scope acquires until the counter reaches the
// number of producers. Producers never wait and come first in the
// launch's workgroup order, so they are all dispatched before any consumer
// and every wait ends; the wait is still bounded (about a second), after
// which the consumer sets the launch's failure flag and leaves its outputs
// unwritten.
constexpr int WAIT_LIMIT = 1 << 22;
__device__ __forceinline__ void signal_done(int *cnt) {
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool wait_done(int *cnt, int need, int *flag) {
    __shared__ int ok;
    if (threadIdx.x == 0) {
        // relaxed polling (no cache invalidation per poll, which would
        // evict the producers' operands), one acquire once the count is in
        int it = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need && it < WAIT_LIMIT) {
            __builtin_amdgcn_s_sleep(4);
            ++it;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = it < WAIT_LIMIT;
        if (!ok) __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return ok != 0;
}

// Row product of workgroup `blk` (GV_R rows, GV_G groups of 64 columns,
// reduced at the end; geometry and addresses in dense_index.hpp; all global
// loads of a workgroup are issued before the first use):
//   TRI false: out[row0 + i] -= sum_{q < ncol} S[row0 + i, col0 + q] w[q],
//   TRI true (row0 = col0, nrow = ncol, w = in + col0, the in-block product
//   with the stored inverse): out[row0 + i] = in[row0 + i] + sum_{q < i}
//   S[row0 + i, row0 + q] in[row0 + q], loading only the groups left of the
//   diagonal.
__device__ __forceinline__ void gemv_body(bool TRI, const double *S, int64_t ng, int64_t row0, int64_t nrow,
                                          int64_t col0, int ncol, const double *w, const double *in, double *out,
                                          int nrhs, int64_t blk, double *wb, double *red) {
    const int tid = threadIdx.x;
    const int a = tid % GV_R, g = tid / GV_R;
    const int64_t i = blk * GV_R + a;
    const int qa = 64 * g;
    const int ncq = max(1, min(64, ncol - qa));
    const bool used = TRI ? gemv_tri_used(blk, tid) : true;
    // terms u < nu of this thread's group are used (for TRI: left of the diagonal)
    const int nu = TRI ? (int)max((int64_t)0, min((int64_t)ncq, i - qa)) : ncq;
    // groups past the last column (a ragged last block) read, and then
    // ignore, that column: every address stays inside the factor
    double l[64];
    if (used) {
#pragma unroll
        for (int u = 0; u < 64; ++u) l[u] = S[gemv_s_addr(ng, row0, nrow, col0, ncol, blk, tid, u)];
    } else {
#pragma unroll
        for (int u = 0; u < 64; ++u) l[u] = 0.0;
    }
    for (int k0r = 0; k0r < nrhs; k0r += RB) {
        const int nr = min(RB, nrhs - k0r);
        for (int idx = tid; idx < DBW * RB; idx += 512) {
            const int q = idx / RB, r = idx % RB;
            wb[idx] = (q < ncol && r < nr) ? w[(int64_t)(k0r + r) * ng + q] : 0.0;
        }
        __syncthreads();
        double acc[RB] = {0.0, 0.0, 0.0, 0.0};
        if (qa < ncol && used) {
#pragma unroll
            for (int u = 0; u < 64; ++u) {
                const double x = u < nu ? l[u] : 0.0;
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) acc[rr] += x * wb[(qa + min(u, ncq - 1)) * RB + rr];
            }
        }
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) red[(g * GV_R + a) * RB + rr] = acc[rr];
        __syncthreads();
        if (g == 0 && i < nrow)
            for (int rr = 0; rr < nr; ++rr) {
                double t = 0.0;
#pragma unroll
                for (int gg = 0; gg < GV_G; ++gg) t += red[(gg * GV_R + a) * RB + rr];
                const int64_t o = (int64_t)(k0r + rr) * ng + row0 + i;
                out[o] = TRI ? in[o] + t : out[o] - t;
            }
        __syncthreads();
    }
}

// In-block product of the first block (the other blocks' in-block products
// run inside the forward step launches)
__global__ __launch_bounds__(512) void k_dense_tri(const double *S, int64_t ng, int64_t j0, int nbw, const double *in,
                                                   double *out, int nrhs) {
    __shared__ double wb[DBW * RB];
    __shared__ double red[GV_G * GV_R * RB];
    gemv_body(true, S, ng, j0, nbw, j0, nbw, in + j0, in, out, nrhs, blockIdx.x, wb, red);
}

// Forward step after block [j0, j0 + nbw), whose y_J is final: v_below -=
// L[below, J] y_J, then the next block's in-block product y = X v on it by
// the last workgroups, once the workgroups of its rows have stored them.
__global__ __launch_bounds__(512) void k_dense_fwd_step(const double *S, int64_t ng, int64_t j0, int nbw, double *v,
                                                        double *y, int nrhs, int *cnt, int *flag) {
    __shared__ double wb[DBW * RB];
    __shared__ double red[GV_G * GV_R * RB];
    const int64_t j1 = j0 + nbw, below = ng - j1;
    const int nbw1 = (int)min((int64_t)DBW, below);
    const int64_t G = gemv_grid(below), P = gemv_grid(nbw1);
    const int64_t b = blockIdx.x;
    const bool tri = b >= G;
    if (tri && !wait_done(cnt, (int)P, flag)) return;
    gemv_body(tri, S, ng, j1, tri ? nbw1 : below, tri ? j1 : j0, tri ? nbw1 : nbw, tri ? v + j1 : y + j0, v,
              tri ? y : v, nrhs, tri ? b - G : b, wb, red);
    if (b < P) signal_done(cnt);
}

// Products with the transpose of the stored lower triangle, for the
// backward solves: output i is the dot product of the contiguous column
// segment S[row0 .. row0 + nq, col0 + i] with a vector, so every read runs
// down a column. Four waves per workgroup, TD_CPW outputs per wave, the nq <=
// DBW terms of a dot product split over the 64 lanes (16 each) and summed
// across the wave at the end.
//   BLK false: out[col0 + i] -= sum_{q < nq} S[row0 + q, col0 + i] w[q]
//   BLK true (row0 = col0 = j0, the in-block product with X_J^T):
//              out[j0 + i] = in[j0 + i] + sum_{i < q < nq} S[j0 + q, j0 + i] in[j0 + q]
template <bool BLK>
__device__ __forceinline__ void tdot_body(const double *S, int64_t ng, int64_t row0, int nq, int64_t col0, int ncols,
                                 const double *w, const double *in, double *out, int nrhs, int64_t blk, double *wb) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i0 = ((int)blk * 4 + wv) * TD_CPW;
    // the column segments of this wave's outputs (clamped, always-valid
    // addresses; terms past nq, and for BLK those with q <= i, are masked)
    double v[TD_CPW][DBW / 64];
#pragma unroll
    for (int c = 0; c < TD_CPW; ++c)
#pragma unroll
        for (int k = 0; k < DBW / 64; ++k) v[c][k] = S[tdot_s_addr(ng, row0, nq, col0, ncols, blk, wv, c, lane, k)];
    for (int k0r = 0; k0r < nrhs; k0r += RB) {
        const int nr = min(RB, nrhs - k0r);
        const double *src = BLK ? in + row0 : w;
        for (int idx = tid; idx < DBW * RB; idx += 256) {
            const int q = idx / RB, r = idx % RB;
            wb[idx] = (q < nq && r < nr) ? src[(int64_t)(k0r + r) * ng + q] : 0.0;
        }
        __syncthreads();
        double acc[TD_CPW][RB];
#pragma unroll
        for (int c = 0; c < TD_CPW; ++c) {
#pragma unroll
            for (int r = 0; r < RB; ++r) acc[c][r] = 0.0;
#pragma unroll
            for (int k = 0; k < DBW / 64; ++k) {
                const int q = lane + 64 * k;
                const bool ok = q < nq && (!BLK || q > i0 + c);
                const double x = ok ? v[c][k] : 0.0;
#pragma unroll
                for (int r = 0; r < RB; ++r) acc[c][r] += x * wb[min(q, DBW - 1) * RB + r];
            }
        }
        // sums across the wave, in a fixed order
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
            for (int c = 0; c < TD_CPW; ++c)
#pragma unroll
                for (int r = 0; r < RB; ++r) acc[c][r] += __shfl_xor(acc[c][r], off);
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < TD_CPW; ++c)
                if (i0 + c < ncols)
                    for (int r = 0; r < nr; ++r) {
                        const int64_t o = (int64_t)(k0r + r) * ng + col0 + i0 + c;
                        out[o] = BLK ? in[o] + acc[c][r] : out[o] - acc[c][r];
                    }
        __syncthreads();
    }
}

template <bool BLK>
__global__ __launch_bounds__(256) void k_dense_tdot(const double *S, int64_t ng, int64_t row0, int nq, int64_t col0,
                                                    int ncols, const double *w, const double *in, double *out,
                                                    int nrhs) {
    __shared__ double wb[DBW * RB];
    tdot_body<BLK>(S, ng, row0, nq, col0, ncols, w, in, out, nrhs, blockIdx.x, wb);
}

// Backward step with block [j0, j0 + nbw), whose x_J is final: z_above -=
// L[J, above]^T x_J over the columns [0, j0) (last columns first), then the
// in-block product x = X^T z of block [j0 - DBW, j0) by the last
// workgroups, once the workgroups of its columns have stored them.
__global__ __launch_bounds__(256) void k_dense_bwd_step(const double *S, int64_t ng, int64_t j0, int nbw, double *z,
                                                        double *x, int nrhs, int *cnt, int *flag) {
    __shared__ double wb[DBW * RB];
    const int64_t G = tdot_grid(j0), P = tdot_grid(DBW);
    const int64_t b = blockIdx.x;
    if (b < G) {
        tdot_body<false>(S, ng, j0, nbw, 0, (int)j0, x + j0, nullptr, z, nrhs, G - 1 - b, wb);
        if (b < P) signal_done(cnt);
    } else {
        if (!wait_done(cnt, (int)P, flag)) return;
        const int64_t jp = j0 - DBW;
        tdot_body<true>(S, ng, jp, DBW, jp, DBW, nullptr, z, x, nrhs, b - G, wb);
    }
}

__global__ void k_div_diag(const double *S, int64_t ng, const double *y, double *z, int nrhs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng) return;
    const double dd = S[i + i * ng];
    for (int k = 0; k < nrhs; ++k) z[(int64_t)k * ng + i] = y[(int64_t)k * ng + i] / dd;
}

// ---- launchers ---------------------------------------------------------------
template <typename T>
void launch_gather_rhs(const double *b, int64_t ntot, int64_t nA, const int32_t *perm, SolveArgs sa,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_gather_rhs<T>, dim3((unsigned)((sa.nv + 255) / 256), (unsigned)sa.N, (unsigned)sa.nrhs),
                       dim3(256), 0, st, b, ntot, nA, perm, sa);
}

// right-hand sides per pass of a kernel whose LDS holds `rows` x RBT doubles
// beside `fixed` bytes
static int rhs_block(int64_t nrhs, int rows, size_t fixed) {
    int rb = (int)std::min<int64_t>(nrhs, RB);
    if (rb == 3) rb = 4;
    while (rb > 1 && (size_t)rows * rb * 8 + fixed > (size_t)LDS_BYTES) rb /= 2;
    return rb;
}

template <typename T, int RBT>
static void fwd_tri(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *fronts, int nfront, int maxm,
                    int npiv, const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    const size_t lds = sizeof(double) * ((size_t)maxm * RBT + 64 * 65);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)k_fwd_tri<T, RBT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_fwd_tri<T, RBT>), dim3(nfront, (unsigned)sa.N), dim3(SNT), lds, st, L, Lstride, sd, fronts,
                       tr, sa, npiv);
}

template <typename T, int RBT>
static void bwd_tri(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *fronts, int nfront, int maxc,
                    const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    const size_t lds = sizeof(double) * ((size_t)maxc * RBT + 129 * 64 + 8 * 64 * RBT);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)k_bwd_tri<T, RBT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_bwd_tri<T, RBT>), dim3(nfront, (unsigned)sa.N), dim3(SNT), lds, st, L, Lstride, sd, fronts,
                       tr, sa);
}

template <typename T>
static void fwd_tri_rb(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *fronts, int nfront, int maxm,
                       int npiv, const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    if (nfront <= 0) return;
    const int rb = rhs_block(sa.nrhs, maxm, sizeof(double) * 64 * 65);
    if (rb == 4) fwd_tri<T, 4>(L, Lstride, sd, fronts, nfront, maxm, npiv, tr, sa, st);
    else if (rb == 2) fwd_tri<T, 2>(L, Lstride, sd, fronts, nfront, maxm, npiv, tr, sa, st);
    else fwd_tri<T, 1>(L, Lstride, sd, fronts, nfront, maxm, npiv, tr, sa, st);
}

template <typename T>
static void bwd_tri_rb(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *fronts, int nfront, int maxc,
                       const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    if (nfront <= 0) return;
    const int rb = rhs_block(sa.nrhs, maxc, sizeof(double) * (129 * 64 + 8 * 64 * RB));
    if (rb == 4) bwd_tri<T, 4>(L, Lstride, sd, fronts, nfront, maxc, tr, sa, st);
    else if (rb == 2) bwd_tri<T, 2>(L, Lstride, sd, fronts, nfront, maxc, tr, sa, st);
    else bwd_tri<T, 1>(L, Lstride, sd, fronts, nfront, maxc, tr, sa, st);
}

// the window kernels: up to four right-hand sides per pass (LDS 40 KiB)
template <typename T>
static void win_solve(bool fwd, const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *fronts, int nfront,
                      int p0, const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    if (nfront <= 0) return;
    const dim3 g(nfront, (unsigned)sa.N);
    if (sa.nrhs >= 3) {
        if (fwd) hipLaunchKernelGGL((k_win<T, 4, false>), g, dim3(1024), 0, st, L, Lstride, sd, fronts, tr, sa, p0);
        else hipLaunchKernelGGL((k_win<T, 4, true>), g, dim3(1024), 0, st, L, Lstride, sd, fronts, tr, sa, p0);
    } else if (sa.nrhs == 2) {
        if (fwd) hipLaunchKernelGGL((k_win<T, 2, false>), g, dim3(1024), 0, st, L, Lstride, sd, fronts, tr, sa, p0);
        else hipLaunchKernelGGL((k_win<T, 2, true>), g, dim3(1024), 0, st, L, Lstride, sd, fronts, tr, sa, p0);
    } else {
        if (fwd) hipLaunchKernelGGL((k_win<T, 1, false>), g, dim3(1024), 0, st, L, Lstride, sd, fronts, tr, sa, p0);
        else hipLaunchKernelGGL((k_win<T, 1, true>), g, dim3(1024), 0, st, L, Lstride, sd, fronts, tr, sa, p0);
    }
}

template <typename T>
static void fwd_rect(const T *L, int64_t Lstride, const FrontDesc *sd, const RowTask *rows, int nrows, int q0w, int qw,
                     const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    if (nrows <= 0) return;
    const dim3 g(nrows, (unsigned)sa.N);
    if (sa.nrhs >= 3)
        hipLaunchKernelGGL((k_fwd_rect<T, 4>), g, dim3(256), 0, st, L, Lstride, sd, rows, tr, sa, q0w, qw);
    else if (sa.nrhs >= 2)
        hipLaunchKernelGGL((k_fwd_rect<T, 2>), g, dim3(256), 0, st, L, Lstride, sd, rows, tr, sa, q0w, qw);
    else
        hipLaunchKernelGGL((k_fwd_rect<T, 1>), g, dim3(256), 0, st, L, Lstride, sd, rows, tr, sa, q0w, qw);
}

template <typename T>
static void bwd_rect(const T *L, int64_t Lstride, const FrontDesc *sd, const RowTask *cols, int ncols, int q0w, int qw,
                     const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    if (ncols <= 0) return;
    const dim3 g(ncols, (unsigned)sa.N);
    if (sa.nrhs >= 3)
        hipLaunchKernelGGL((k_bwd_rect<T, 4>), g, dim3(256), 0, st, L, Lstride, sd, cols, tr, sa, q0w, qw);
    else if (sa.nrhs >= 2)
        hipLaunchKernelGGL((k_bwd_rect<T, 2>), g, dim3(256), 0, st, L, Lstride, sd, cols, tr, sa, q0w, qw);
    else
        hipLaunchKernelGGL((k_bwd_rect<T, 1>), g, dim3(256), 0, st, L, Lstride, sd, cols, tr, sa, q0w, qw);
}

constexpr int WHOLE = 1 << 30;  // no limit on the pivots solved

// Forward level: small fronts, the pivot part of the other fronts and their
// update rows (a wide front's extend-add, then window by window: the
// window's inverse, then its products with every row below it over 64-row
// workgroups).
template <typename T>
void launch_fwd_level(const T *L, int64_t Lstride, const FrontDesc *sd, const LevelTasks &lt, const TreeArgs &tr,
                      SolveArgs sa, hipStream_t st) {
    if (lt.nsmall > 0)
        hipLaunchKernelGGL(k_fwd_small<T>, dim3(lt.nsmall, (unsigned)sa.N), dim3(64), 0, st, L, Lstride, sd, lt.small,
                           tr, sa);
    fwd_tri_rb<T>(L, Lstride, sd, lt.large, lt.nlarge, lt.maxm, WHOLE, tr, sa, st);
    if (lt.nwin > 0) fwd_tri_rb<T>(L, Lstride, sd, lt.win[0].fronts, lt.win[0].nfront, 0, 0, tr, sa, st);
    for (int w = 0; w < lt.nwin; ++w) {
        const TriWindow &tw = lt.win[w];
        win_solve<T>(true, L, Lstride, sd, tw.fronts, tw.nfront, tw.p0, tr, sa, st);
        fwd_rect<T>(L, Lstride, sd, tw.rows, tw.nrows, tw.p0, TRI_W, tr, sa, st);
    }
    fwd_rect<T>(L, Lstride, sd, lt.rect_rows, lt.nrect_rows, 0, 0, tr, sa, st);
}

// Backward level: small fronts, the update rows of the other fronts, then
// their pivot part (a wide front window by window from the last: the
// window's inverse, then its products with the pivot columns before it over
// 64-column workgroups).
template <typename T>
void launch_bwd_level(const T *L, int64_t Lstride, const FrontDesc *sd, const LevelTasks &lt, const TreeArgs &tr,
                      SolveArgs sa, hipStream_t st) {
    if (lt.nsmall > 0)
        hipLaunchKernelGGL(k_bwd_small<T>, dim3(lt.nsmall, (unsigned)sa.N), dim3(64), 0, st, L, Lstride, sd, lt.small,
                           tr, sa);
    bwd_rect<T>(L, Lstride, sd, lt.rect_cols, lt.nrect_cols, 0, 0, tr, sa, st);
    bwd_tri_rb<T>(L, Lstride, sd, lt.large, lt.nlarge, lt.maxc, tr, sa, st);
    for (int w = lt.nwin - 1; w >= 0; --w) {
        const TriWindow &tw = lt.win[w];
        win_solve<T>(false, L, Lstride, sd, tw.fronts, tw.nfront, tw.p0, tr, sa, st);
        bwd_rect<T>(L, Lstride, sd, tw.cols, tw.ncols, tw.p0, TRI_W, tr, sa, st);
    }
}

void launch_scatter_x(double *x, int64_t ntot, int64_t nA, const int32_t *perm, SolveArgs sa, const double *xg,
                      int64_t ng, hipStream_t st) {
    int64_t mx = std::max<int64_t>(nA, ng);
    hipLaunchKernelGGL(k_scatter_x, dim3((unsigned)((mx + 255) / 256), (unsigned)sa.N, (unsigned)sa.nrhs),
                       dim3(256), 0, st, x, ntot, nA, perm, sa, xg, ng);
}

void launch_schur_rhs(const double *b, int64_t ntot, int64_t nA, SolveArgs sa, int64_t Ns, int64_t uoff_border,
                      double *bh, hipStream_t st) {
    hipLaunchKernelGGL(k_schur_rhs, dim3((unsigned)((Ns + 127) / 128), (unsigned)sa.nrhs), dim3(128), 0, st, b,
                       ntot, nA, sa, Ns, uoff_border, bh);
}

void launch_border_values(const double *xg, SolveArgs sa, int64_t nA, int64_t Ns, hipStream_t st) {
    hipLaunchKernelGGL(k_border_values, dim3((unsigned)((Ns + 127) / 128), (unsigned)sa.nrhs), dim3(128), 0, st,
                       xg, sa, nA, Ns);
}

void launch_dense_fwd(const double *S, int64_t ng, double *v, double *y, int64_t nrhs, int *sync, hipStream_t st) {
    const int64_t nblk = (ng + DBW - 1) / DBW;
    if (nblk > 1) launch_zero<int>(sync + 1, 2 * (nblk - 1), st);
    const int nbw0 = (int)std::min<int64_t>(DBW, ng);
    hipLaunchKernelGGL(k_dense_tri, dim3((unsigned)gemv_grid(nbw0)), dim3(512), 0, st, S, ng, (int64_t)0, nbw0,
                       (const double *)v, y, (int)nrhs);
    for (int64_t k = 0; k + 1 < nblk; ++k) {
        const int64_t j0 = k * DBW;
        hipLaunchKernelGGL(k_dense_fwd_step, dim3((unsigned)fwd_step_grid(ng, j0 + DBW)), dim3(512), 0, st, S, ng, j0,
                           (int)DBW, v, y, (int)nrhs, sync + 1 + k, sync);
    }
}

void launch_dense_bwd(const double *S, int64_t ng, double *z, double *x, int64_t nrhs, int *sync, hipStream_t st) {
    const int64_t nblk = (ng + DBW - 1) / DBW;
    int *cnt = sync + 1 + (nblk > 1 ? nblk - 1 : 0);
    hipLaunchKernelGGL(k_div_diag, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, S, ng, z, z, (int)nrhs);
    const int64_t jl = (nblk - 1) * DBW;
    const int nbwl = (int)(ng - jl);
    // x_J = X_J^T z_J for the last block, then one step per block: z_above
    // -= L[J, above]^T x_J and the in-block product of the block before it,
    // both read down the columns of the stored lower triangle
    hipLaunchKernelGGL(k_dense_tdot<true>, dim3((unsigned)tdot_grid(nbwl)), dim3(256), 0, st, S, ng, jl, nbwl, jl,
                       nbwl, (const double *)nullptr, (const double *)z, x, (int)nrhs);
    for (int64_t k = nblk - 1; k >= 1; --k) {
        const int64_t j0 = k * DBW;
        const int nbw = (int)std::min<int64_t>(DBW, ng - j0);
        hipLaunchKernelGGL(k_dense_bwd_step, dim3((unsigned)bwd_step_grid(j0)), dim3(256), 0, st, S, ng, j0, nbw, z, x,
                           (int)nrhs, cnt + (k - 1), sync);
    }
}

template void launch_gather_rhs<double>(const double *, int64_t, int64_t, const int32_t *, SolveArgs, hipStream_t);
template void launch_gather_rhs<float>(const double *, int64_t, int64_t, const int32_t *, SolveArgs, hipStream_t);
#define KKT_SOLVE_INST(T)                                                                                   \
    template void launch_fwd_level<T>(const T *, int64_t, const FrontDesc *, const LevelTasks &,            \
                                      const TreeArgs &, SolveArgs, hipStream_t);                            \
    template void launch_bwd_level<T>(const T *, int64_t, const FrontDesc *, const LevelTasks &,            \
                                      const TreeArgs &, SolveArgs, hipStream_t);
KKT_SOLVE_INST(double)
KKT_SOLVE_INST(float)

}  // namespace kkt
