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
// once per pass); v[i * RB + r] holds row i of right-hand side r.
constexpr int RB = 4;

constexpr int SNT = 512;  // threads of a front solve

template <typename T>
__global__ __launch_bounds__(SNT) void k_fwd(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *tasks,
                                             TreeArgs tr, SolveArgs sa, int rb) {
    extern __shared__ double smem[];
    double *Lt = smem;             // 64 x 65 staging tile
    double *v = smem + 64 * 65;
    const int s = tasks[blockIdx.x];
    const int n = blockIdx.y, tid = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    const T *P = L + (int64_t)n * Lstride + d.Loff;
    const int32_t *R = tr.rows + tr.rowptr[s];
    for (int k0r = 0; k0r < sa.nrhs; k0r += rb) {
        const int nr = min(rb, (int)sa.nrhs - k0r);
        double *x0 = sa.xp + ((int64_t)n * sa.nrhs + k0r) * sa.nv;
        double *U0 = sa.uv + ((int64_t)n * sa.nrhs + k0r) * sa.usz;
        for (int idx = tid; idx < m * rb; idx += SNT) {
            const int i = idx / rb, r = idx % rb;
            v[idx] = (r < nr && i < c) ? x0[(int64_t)r * sa.nv + R[i]] : 0.0;
        }
        __syncthreads();
        for (int q = tr.cptr[s]; q < tr.cptr[s + 1]; ++q) {
            const int ch = tr.clist[q];
            const int uc = sd[ch].m - sd[ch].c;
            const int32_t *rl = tr.rel + tr.relptr[ch];
            for (int idx = tid; idx < uc * nr; idx += SNT) {
                const int i = idx / nr, r = idx % nr;
                v[rl[i] * rb + r] += U0[(int64_t)r * sa.usz + tr.relptr[ch] + i];
            }
            __syncthreads();
        }
        for (int k0 = 0; k0 < c; k0 += 64) {
            const int nb = min(64, c - k0);
            const int i = tid & 63, r = tid >> 6;
            for (int idx = tid; idx < 64 * 64; idx += SNT) {
                const int a = idx & 63, q = idx >> 6;
                Lt[a + q * 65] = (q < a && a < nb) ? (double)P[(k0 + a) + (int64_t)(k0 + q) * m] : 0.0;
            }
            __syncthreads();
            double yv = 0.0;
            if (i < nb && r < nr) {
                yv = v[(k0 + i) * rb + r];
                for (int q = 0; q < i; ++q) yv += Lt[i + q * 65] * v[(k0 + q) * rb + r];
            }
            __syncthreads();
            if (i < nb && r < nr) v[(k0 + i) * rb + r] = yv;
            __syncthreads();
            for (int i2 = k0 + nb + tid; i2 < m; i2 += SNT) {
                double acc[RB] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
                for (int q = 0; q < nb; ++q) {
                    const double l = (double)P[i2 + (int64_t)(k0 + q) * m];
#pragma unroll
                    for (int rr = 0; rr < RB; ++rr)
                        if (rr < nr) acc[rr] += l * v[(k0 + q) * rb + rr];
                }
#pragma unroll
                for (int rr = 0; rr < RB; ++rr)
                    if (rr < nr) v[i2 * rb + rr] -= acc[rr];
            }
            __syncthreads();
        }
        for (int idx = tid; idx < m * nr; idx += SNT) {
            const int i = idx / nr, r = idx % nr;
            if (i < c) x0[(int64_t)r * sa.nv + R[i]] = v[i * rb + r];
            else U0[(int64_t)r * sa.usz + tr.relptr[s] + (i - c)] = v[i * rb + r];
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(SNT) void k_bwd(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *tasks,
                                             TreeArgs tr, SolveArgs sa, int rb) {
    extern __shared__ double smem[];
    double *Lt = smem;             // 64 x 65 staging tile
    double *v = smem + 64 * 65;
    const int s = tasks[blockIdx.x];
    const int n = blockIdx.y, tid = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    if (c == 0) return;
    const T *P = L + (int64_t)n * Lstride + d.Loff;
    const int32_t *R = tr.rows + tr.rowptr[s];
    for (int k0r = 0; k0r < sa.nrhs; k0r += rb) {
        const int nr = min(rb, (int)sa.nrhs - k0r);
        double *x0 = sa.xp + ((int64_t)n * sa.nrhs + k0r) * sa.nv;
        for (int idx = tid; idx < m * rb; idx += SNT) {
            const int i = idx / rb, r = idx % rb;
            double val = 0.0;
            if (r < nr) {
                val = x0[(int64_t)r * sa.nv + R[i]];
                if (i < c) val /= (double)P[i + (int64_t)i * m];
            }
            v[idx] = val;
        }
        __syncthreads();
        // contributions of the update rows (ancestors' final values)
        for (int q = tid; q < c; q += SNT) {
            double acc[RB] = {0.0, 0.0, 0.0, 0.0};
            const T *col = P + (int64_t)q * m;
#pragma unroll 8
            for (int i = c; i < m; ++i) {
                const double l = (double)col[i];
#pragma unroll
                for (int rr = 0; rr < RB; ++rr)
                    if (rr < nr) acc[rr] += l * v[i * rb + rr];
            }
#pragma unroll
            for (int rr = 0; rr < RB; ++rr)
                if (rr < nr) v[q * rb + rr] -= acc[rr];
        }
        __syncthreads();
        for (int kb = ((c - 1) / 64) * 64; kb >= 0; kb -= 64) {
            const int nb = min(64, c - kb);
            const int q = tid & 63, r = tid >> 6;
            for (int idx = tid; idx < 64 * 64; idx += SNT) {
                const int a = idx & 63, qq = idx >> 6;
                Lt[a + qq * 65] = (qq < a && a < nb) ? (double)P[(kb + a) + (int64_t)(kb + qq) * m] : 0.0;
            }
            __syncthreads();
            double xv = 0.0;
            if (q < nb && r < nr) {
                xv = v[(kb + q) * rb + r];
                for (int i = q + 1; i < nb; ++i) xv += Lt[i + q * 65] * v[(kb + i) * rb + r];
            }
            __syncthreads();
            if (q < nb && r < nr) v[(kb + q) * rb + r] = xv;
            __syncthreads();
            for (int q2 = tid; q2 < kb; q2 += SNT) {
                double acc[RB] = {0.0, 0.0, 0.0, 0.0};
                const T *col = P + (int64_t)q2 * m + kb;
#pragma unroll 8
                for (int i = 0; i < nb; ++i) {
                    const double l = (double)col[i];
#pragma unroll
                    for (int rr = 0; rr < RB; ++rr)
                        if (rr < nr) acc[rr] += l * v[(kb + i) * rb + rr];
                }
#pragma unroll
                for (int rr = 0; rr < RB; ++rr)
                    if (rr < nr) v[q2 * rb + rr] -= acc[rr];
            }
            __syncthreads();
        }
        for (int idx = tid; idx < c * nr; idx += SNT) {
            const int i = idx / nr, r = idx % nr;
            x0[(int64_t)r * sa.nv + R[i]] = v[i * rb + r];
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
__global__ void k_schur_rhs(const double *b, int64_t ntot, int64_t nA, SolveArgs sa, int64_t Ns,
                            int64_t uoff_border, double *bh) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= Ns) return;
    const int64_t ng = sa.N * Ns;
    double acc = 0.0;
    for (int64_t m = 0; m < sa.N; ++m) {
        const double *ub = sa.uv + ((int64_t)m * sa.nrhs + k) * sa.usz + uoff_border;
        const double bc = b[(int64_t)k * ntot + sa.N * nA + m * Ns + i];
        bh[(int64_t)k * ng + m * Ns + i] = bc + ub[i] + acc;
        acc += ub[Ns + i];
    }
}

// border rows of every period for the backward pass: (du_g[n], sum_{m>n} du_g[m])
__global__ void k_border_values(const double *xg, SolveArgs sa, int64_t nA, int64_t Ns) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= Ns) return;
    const int64_t ng = sa.N * Ns;
    double acc = 0.0;
    for (int64_t n = sa.N - 1; n >= 0; --n) {
        double *x = sa.xp + ((int64_t)n * sa.nrhs + k) * sa.nv;
        x[nA + i] = xg[(int64_t)k * ng + n * Ns + i];
        x[nA + Ns + i] = acc;
        acc += xg[(int64_t)k * ng + n * Ns + i];
    }
}

// ---- dense Schur factor solves ----------------------------------------------
// The factor of S keeps D on its diagonal, L^-1 of every 64x64 diagonal block
// below the diagonal of that block, and L elsewhere below the diagonal. Steps
// go over 256-row blocks; every workgroup of a step redoes the small in-block
// solve and then updates its own 256 rows (forward) or columns (backward).
constexpr int DBW = 256;

// The factor of S keeps L^-1 of every 256x256 diagonal block below that
// block's diagonal. y[j0:j0+nbw) = X v[j0:j0+nbw) with X unit lower: 16 rows
// per workgroup, 16 partial sums per row.
__global__ __launch_bounds__(256) void k_dense_yblk(const double *S, int64_t ng, const double *v, double *y, int nrhs,
                                                    int64_t j0) {
    __shared__ double vb[DBW * RB];
    __shared__ double red[16 * 16 * RB];
    const int tid = threadIdx.x;
    const int nbw = (int)min((int64_t)DBW, ng - j0);
    const int rl = tid & 15, g = tid >> 4;          // row in tile, column group
    const int i = blockIdx.x * 16 + rl;             // row in block
    for (int k0r = 0; k0r < nrhs; k0r += RB) {
        const int nr = min(RB, nrhs - k0r);
        for (int idx = tid; idx < nbw * RB; idx += 256) {
            const int q = idx / RB, r = idx % RB;
            vb[idx] = r < nr ? v[(int64_t)(k0r + r) * ng + j0 + q] : 0.0;
        }
        __syncthreads();
        double acc[RB] = {0.0, 0.0, 0.0, 0.0};
        if (i < nbw) {
            const double *row = S + (j0 + i);
            for (int q = g; q < i; q += 16) {
                const double l = row[(j0 + q) * ng];
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) acc[rr] += l * vb[q * RB + rr];
            }
        }
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) red[(g * 16 + rl) * RB + rr] = acc[rr];
        __syncthreads();
        if (g == 0 && i < nbw)
            for (int rr = 0; rr < nr; ++rr) {
                double t = vb[i * RB + rr];
                for (int gg = 0; gg < 16; ++gg) t += red[(gg * 16 + rl) * RB + rr];
                y[(int64_t)(k0r + rr) * ng + j0 + i] = t;
            }
        __syncthreads();
    }
}

// rows below the block: v[i] -= L[i, j0:j0+nbw] y[j0:j0+nbw], 64 rows per
// workgroup, four partial sums per row
__global__ __launch_bounds__(256) void k_dense_rows_fwd(const double *S, int64_t ng, double *v, const double *y,
                                                        int nrhs, int64_t j0) {
    __shared__ double yb[DBW * RB];
    __shared__ double red[4 * 64 * RB];
    const int tid = threadIdx.x;
    const int nbw = (int)min((int64_t)DBW, ng - j0);
    const int row = tid & 63, g = tid >> 6;
    const int64_t i = j0 + nbw + (int64_t)blockIdx.x * 64 + row;
    for (int k0r = 0; k0r < nrhs; k0r += RB) {
        const int nr = min(RB, nrhs - k0r);
        for (int idx = tid; idx < nbw * RB; idx += 256) {
            const int q = idx / RB, r = idx % RB;
            yb[idx] = r < nr ? y[(int64_t)(k0r + r) * ng + j0 + q] : 0.0;
        }
        __syncthreads();
        double acc[RB] = {0.0, 0.0, 0.0, 0.0};
        if (i < ng) {
            const int qlo = 64 * g, qhi = min(nbw, qlo + 64);
#pragma unroll 8
            for (int q = qlo; q < qhi; ++q) {
                const double l = S[i + (j0 + q) * ng];
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) acc[rr] += l * yb[q * RB + rr];
            }
        }
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) red[(g * 64 + row) * RB + rr] = acc[rr];
        __syncthreads();
        if (g == 0 && i < ng)
            for (int rr = 0; rr < nr; ++rr) {
                const double t = red[(0 * 64 + row) * RB + rr] + red[(1 * 64 + row) * RB + rr] +
                                 red[(2 * 64 + row) * RB + rr] + red[(3 * 64 + row) * RB + rr];
                v[(int64_t)(k0r + rr) * ng + i] -= t;
            }
        __syncthreads();
    }
}

__global__ void k_div_diag(const double *S, int64_t ng, const double *y, double *z, int nrhs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng) return;
    const double dd = S[i + i * ng];
    for (int k = 0; k < nrhs; ++k) z[(int64_t)k * ng + i] = y[(int64_t)k * ng + i] / dd;
}

// x[j0:j0+nbw) = X^T z[j0:j0+nbw): 16 columns per workgroup, 16 partial sums
__global__ __launch_bounds__(256) void k_dense_xblk(const double *S, int64_t ng, const double *z, double *x, int nrhs,
                                                    int64_t j0) {
    __shared__ double zb[DBW * RB];
    __shared__ double red[16 * 16 * RB];
    const int tid = threadIdx.x;
    const int nbw = (int)min((int64_t)DBW, ng - j0);
    const int cl = tid & 15, g = tid >> 4;
    const int q = blockIdx.x * 16 + cl;
    for (int k0r = 0; k0r < nrhs; k0r += RB) {
        const int nr = min(RB, nrhs - k0r);
        for (int idx = tid; idx < nbw * RB; idx += 256) {
            const int i = idx / RB, r = idx % RB;
            zb[idx] = r < nr ? z[(int64_t)(k0r + r) * ng + j0 + i] : 0.0;
        }
        __syncthreads();
        double acc[RB] = {0.0, 0.0, 0.0, 0.0};
        if (q < nbw) {
            const double *col = S + j0 + (j0 + q) * ng;
            for (int i = q + 1 + g; i < nbw; i += 16) {
                const double l = col[i];
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) acc[rr] += l * zb[i * RB + rr];
            }
        }
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) red[(g * 16 + cl) * RB + rr] = acc[rr];
        __syncthreads();
        if (g == 0 && q < nbw)
            for (int rr = 0; rr < nr; ++rr) {
                double t = zb[q * RB + rr];
                for (int gg = 0; gg < 16; ++gg) t += red[(gg * 16 + cl) * RB + rr];
                x[(int64_t)(k0r + rr) * ng + j0 + q] = t;
            }
        __syncthreads();
    }
}

// columns before the block: z[q] -= L[j0:j0+nbw, q]^T x[j0:j0+nbw], 64
// columns per workgroup, four partial sums per column
__global__ __launch_bounds__(256) void k_dense_cols_bwd(const double *S, int64_t ng, double *z, const double *x,
                                                        int nrhs, int64_t j0) {
    __shared__ double xb[DBW * RB];
    __shared__ double red[4 * 64 * RB];
    const int tid = threadIdx.x;
    const int nbw = (int)min((int64_t)DBW, ng - j0);
    const int cl = tid & 63, g = tid >> 6;
    const int64_t q = (int64_t)blockIdx.x * 64 + cl;
    for (int k0r = 0; k0r < nrhs; k0r += RB) {
        const int nr = min(RB, nrhs - k0r);
        for (int idx = tid; idx < nbw * RB; idx += 256) {
            const int i = idx / RB, r = idx % RB;
            xb[idx] = r < nr ? x[(int64_t)(k0r + r) * ng + j0 + i] : 0.0;
        }
        __syncthreads();
        double acc[RB] = {0.0, 0.0, 0.0, 0.0};
        if (q < j0) {
            const int ilo = 64 * g, ihi = min(nbw, ilo + 64);
            const double *col = S + j0 + q * ng;
#pragma unroll 8
            for (int i = ilo; i < ihi; ++i) {
                const double l = col[i];
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) acc[rr] += l * xb[i * RB + rr];
            }
        }
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) red[(g * 64 + cl) * RB + rr] = acc[rr];
        __syncthreads();
        if (g == 0 && q < j0)
            for (int rr = 0; rr < nr; ++rr) {
                const double t = red[(0 * 64 + cl) * RB + rr] + red[(1 * 64 + cl) * RB + rr] +
                                 red[(2 * 64 + cl) * RB + rr] + red[(3 * 64 + cl) * RB + rr];
                z[(int64_t)(k0r + rr) * ng + q] -= t;
            }
        __syncthreads();
    }
}

// ---- launchers ---------------------------------------------------------------
template <typename T>
void launch_gather_rhs(const double *b, int64_t ntot, int64_t nA, const int32_t *perm, SolveArgs sa,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_gather_rhs<T>, dim3((unsigned)((sa.nv + 255) / 256), (unsigned)sa.N, (unsigned)sa.nrhs),
                       dim3(256), 0, st, b, ntot, nA, perm, sa);
}

static int rhs_block(int64_t nrhs, int maxm) {
    int rb = (int)std::min<int64_t>(nrhs, RB);
    while (rb > 1 && (int64_t)maxm * rb * 8 > 96 * 1024) --rb;
    return rb;
}
static size_t front_lds(int maxm, int rb) { return sizeof(double) * ((size_t)maxm * rb + 64 * 65); }

template <typename T>
void launch_fwd_level(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *tasks, int ntasks, int maxm,
                      const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    if (ntasks <= 0) return;
    const int rb = rhs_block(sa.nrhs, maxm);
    const size_t lds = front_lds(maxm, rb);
    if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void *)k_fwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_fwd<T>, dim3(ntasks, (unsigned)sa.N), dim3(SNT), lds, st, L, Lstride, sd, tasks, tr, sa, rb);
}

template <typename T>
void launch_bwd_level(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *tasks, int ntasks, int maxm,
                      const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    if (ntasks <= 0) return;
    const int rb = rhs_block(sa.nrhs, maxm);
    const size_t lds = front_lds(maxm, rb);
    if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void *)k_bwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_bwd<T>, dim3(ntasks, (unsigned)sa.N), dim3(SNT), lds, st, L, Lstride, sd, tasks, tr, sa, rb);
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

void launch_dense_fwd(const double *S, int64_t ng, double *v, double *y, int64_t nrhs, hipStream_t st) {
    for (int64_t j0 = 0; j0 < ng; j0 += DBW) {
        const int64_t nbw = std::min<int64_t>(DBW, ng - j0);
        hipLaunchKernelGGL(k_dense_yblk, dim3((unsigned)((nbw + 15) / 16)), dim3(256), 0, st, S, ng, v, y, (int)nrhs,
                           j0);
        const int64_t below = ng - j0 - DBW;
        if (below > 0)
            hipLaunchKernelGGL(k_dense_rows_fwd, dim3((unsigned)((below + 63) / 64)), dim3(256), 0, st, S, ng, v, y,
                               (int)nrhs, j0);
    }
}

void launch_dense_bwd(const double *S, int64_t ng, double *z, double *x, int64_t nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_div_diag, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, S, ng, z, z, (int)nrhs);
    for (int64_t j0 = ((ng - 1) / DBW) * DBW; j0 >= 0; j0 -= DBW) {
        const int64_t nbw = std::min<int64_t>(DBW, ng - j0);
        hipLaunchKernelGGL(k_dense_xblk, dim3((unsigned)((nbw + 15) / 16)), dim3(256), 0, st, S, ng, z, x, (int)nrhs,
                           j0);
        if (j0 > 0)
            hipLaunchKernelGGL(k_dense_cols_bwd, dim3((unsigned)((j0 + 63) / 64)), dim3(256), 0, st, S, ng, z, x,
                               (int)nrhs, j0);
    }
}

template void launch_gather_rhs<double>(const double *, int64_t, int64_t, const int32_t *, SolveArgs, hipStream_t);
template void launch_gather_rhs<float>(const double *, int64_t, int64_t, const int32_t *, SolveArgs, hipStream_t);
#define KKT_SOLVE_INST(T)                                                                                   \
    template void launch_fwd_level<T>(const T *, int64_t, const FrontDesc *, const int32_t *, int, int,     \
                                      const TreeArgs &, SolveArgs, hipStream_t);                            \
    template void launch_bwd_level<T>(const T *, int64_t, const FrontDesc *, const int32_t *, int, int,     \
                                      const TreeArgs &, SolveArgs, hipStream_t);
KKT_SOLVE_INST(double)
KKT_SOLVE_INST(float)

}  // namespace kkt
