// Batched multifrontal LDL^T of all period blocks (Algorithm 1 step 2,
// section 4.2) and the dense LDL^T of the Schur complement (step 12).
//
// Every kernel is batched over the N periods through blockIdx.y; all periods
// share the symbolic structure, so one launch covers the same fronts of every
// period.  Fronts with at most 64 rows are assembled and factored entirely in
// LDS by one wavefront; larger fronts are assembled by row tiles and factored
// right-looking in 64-column steps (pivot block in LDS, row-parallel
// triangular solve, trailing update on MFMA), grouped over all large fronts of
// one tree level.
#include "device.hpp"
#include "kernels.hpp"

namespace kkt {

constexpr int SMALL_M = 64;
constexpr int NB = 64;      // pivot block width
constexpr int LDT = 65;     // LDS leading dimension of a 64x64 tile

// --------------------------------------------------------------------------
// static pivoting rule (oracle's reading): |d| <= tau -> sign(d) * tau,
// inertia from the computed pivot before perturbation.
// --------------------------------------------------------------------------
__device__ inline double pivot_rule(double raw, double tau_k, double amax, double eps, int sgn, int64_t *cnt) {
    double t = tau_k > 0.0 ? tau_k : eps * amax;
    if (raw > 0.0) atomicAdd((unsigned long long *)(cnt + 0), 1ull);
    else if (raw < 0.0) atomicAdd((unsigned long long *)(cnt + 1), 1ull);
    else atomicAdd((unsigned long long *)(cnt + 2), 1ull);
    if (!(fabs(raw) > t)) {  // also catches NaN
        double s = raw > 0.0 ? 1.0 : (raw < 0.0 ? -1.0 : (double)sgn);
        double mag = t > 0.0 ? t : 1e-300;
        atomicAdd((unsigned long long *)(cnt + 3), 1ull);
        return s * mag;
    }
    return raw;
}

template <typename T>
__device__ inline T do_pivot(const FactorArgs<T> &fa, int n, int gpiv, T raw) {
    int sgn = fa.sign ? (int)fa.sign[gpiv] : -1;
    double v = pivot_rule((double)raw, fa.tau[(int64_t)n * fa.tstride + gpiv], fa.amax[n], fa.eps, sgn,
                          fa.cnt + 4 * n);
    return (T)v;
}

// --------------------------------------------------------------------------
// utility kernels
// --------------------------------------------------------------------------
template <typename T>
__global__ void k_zero(T *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

__global__ void k_check_finite(const double *v, int64_t n, int *flag) {
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(v[i]);
    if (bad) atomicOr(flag, 1);
}

// A values of every period into the panels (+delta_w on primal, -delta_c on
// dual diagonals), per-pivot thresholds and the per-period max |a_ij|.
template <typename T>
__global__ __launch_bounds__(256) void k_scatter_A(const double *A, int64_t nnz, const int64_t *amap,
                                                   const int8_t *adiag, const int32_t *adpiv, T *L,
                                                   int64_t Lstride, double *tau, int64_t tstride, double *amax,
                                                   double dw, double dc, double eps) {
    __shared__ double red[256];
    const int n = blockIdx.y;
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double a = 0.0;
    if (k < nnz) {
        double v = A[(int64_t)n * nnz + k];
        int8_t dg = adiag[k];
        if (dg == 1) v += dw;
        else if (dg == -1) v -= dc;
        L[(int64_t)n * Lstride + amap[k]] = (T)v;
        if (dg) tau[(int64_t)n * tstride + adpiv[k]] = eps * fabs(v);
        a = fabs(v);
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomic_max_nonneg(amax + n, red[0]);
}

template <typename T>
__global__ void k_scatter_C(const double *C0, int64_t n0, const int64_t *c0map, const double *C1, int64_t n1,
                            const int64_t *c1map, T *L, int64_t Lstride) {
    const int n = blockIdx.y;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n0) L[(int64_t)n * Lstride + c0map[k]] = (T)C0[k];
    else if (k < n0 + n1) L[(int64_t)n * Lstride + c1map[k - n0]] = (T)C1[k - n0];
}

// --------------------------------------------------------------------------
// small fronts (m <= 64): extend-add + full partial factorisation in LDS
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_small_front(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *tasks,
                                                    const int32_t *cptr, const int32_t *clist,
                                                    const int64_t *relptr, const int32_t *rel) {
    __shared__ T F[SMALL_M * LDT];
    __shared__ T piv;
    const int s = tasks[blockIdx.x];
    const int n = blockIdx.y;
    const int tid = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c, u = m - c;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    for (int idx = tid; idx < m * m; idx += 64) {
        int r = idx % m, q = idx / m;
        if (r >= q) F[r + q * LDT] = q < c ? P[r + (int64_t)q * m] : T(0);
    }
    __syncthreads();
    for (int k = cptr[s]; k < cptr[s + 1]; ++k) {
        const int ch = clist[k];
        const FrontDesc dc = sd[ch];
        const int uc = dc.m - dc.c;
        const T *Uc = fa.U + (int64_t)n * fa.Ustride + dc.Uoff;
        const int32_t *rl = rel + relptr[ch];
        for (int idx = tid; idx < uc * uc; idx += 64) {
            int i = idx % uc, j = idx / uc;
            if (i >= j) F[rl[i] + rl[j] * LDT] += Uc[i + (int64_t)j * uc];
        }
        __syncthreads();
    }
    for (int j = 0; j < c; ++j) {
        if (tid == 0) {
            T v = do_pivot(fa, n, d.piv0 + j, F[j + j * LDT]);
            F[j + j * LDT] = v;
            piv = v;
        }
        __syncthreads();
        const T dj = piv;
        for (int i = j + 1 + tid; i < m; i += 64) F[i + j * LDT] /= dj;
        __syncthreads();
        const int nt = m - j - 1;
        for (int idx = tid; idx < nt * nt; idx += 64) {
            int ii = idx % nt, qq = idx / nt;
            if (ii >= qq) {
                int i = j + 1 + ii, q = j + 1 + qq;
                F[i + q * LDT] -= F[i + j * LDT] * dj * F[q + j * LDT];
            }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < m * c; idx += 64) {
        int r = idx % m, q = idx / m;
        if (r >= q) P[r + (int64_t)q * m] = F[r + q * LDT];
    }
    T *Us = fa.U + (int64_t)n * fa.Ustride + d.Uoff;
    for (int idx = tid; idx < u * u; idx += 64) {
        int i = idx % u, j = idx / u;
        if (i >= j) Us[i + (int64_t)j * u] = F[(c + i) + (c + j) * LDT];
    }
}

// --------------------------------------------------------------------------
// large fronts
// --------------------------------------------------------------------------
template <typename T>
__device__ inline T *front_addr(T *P, T *Ub, int m, int c, int r, int q) {
    return q < c ? P + r + (int64_t)q * m : Ub + (r - c) + (int64_t)(q - c) * (m - c);
}

// Extend-add of the children's update blocks into 64-row tiles of a large
// front.  The child rows landing in a tile form one contiguous range (the
// relative indices increase), so every tile owns its target rows; children
// are added one after another in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_extend_add(FactorArgs<T> fa, const FrontDesc *sd, const RowTask *tasks,
                                                    const int32_t *cptr, const int32_t *clist,
                                                    const int64_t *relptr, const int32_t *rel) {
    const RowTask tk = tasks[blockIdx.x];
    const int n = blockIdx.y;
    const FrontDesc d = sd[tk.f];
    const int r0 = tk.r0, r1 = min(r0 + 64, d.m);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    T *Ub = fa.U + (int64_t)n * fa.Ustride + d.Uoff;
    for (int k = cptr[d.sn]; k < cptr[d.sn + 1]; ++k) {
        const int ch = clist[k];
        const FrontDesc dc = sd[ch];
        const int uc = dc.m - dc.c;
        const T *Uc = fa.U + (int64_t)n * fa.Ustride + dc.Uoff;
        const int32_t *rl = rel + relptr[ch];
        int lo = 0, hi = uc;  // first child row with rl >= r0
        while (lo < hi) { int mid = (lo + hi) >> 1; if (rl[mid] < r0) lo = mid + 1; else hi = mid; }
        const int i_lo = lo;
        hi = uc;
        while (lo < hi) { int mid = (lo + hi) >> 1; if (rl[mid] < r1) lo = mid + 1; else hi = mid; }
        const int i_hi = lo;
        const int i = i_lo + lane;
        if (i < i_hi) {
            const int R = rl[i];
            for (int j = wv; j <= i; j += 4) {
                const int Q = rl[j];
                *front_addr(P, Ub, d.m, d.c, R, Q) += Uc[i + (int64_t)j * uc];
            }
        }
        __syncthreads();
    }
}

// LDL^T of the 64x64 (or smaller) pivot block at column k0 of every listed front.
template <typename T>
__global__ __launch_bounds__(256) void k_diag(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fl, int k0) {
    __shared__ T F[NB * LDT];
    __shared__ T piv;
    const FrontDesc d = sd[fl[blockIdx.x]];
    const int n = blockIdx.y, tid = threadIdx.x;
    const int nb = min(NB, d.c - k0);
    const int m = d.m;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    for (int idx = tid; idx < nb * nb; idx += 256) {
        int r = idx % nb, q = idx / nb;
        if (r >= q) F[r + q * LDT] = P[(k0 + r) + (int64_t)(k0 + q) * m];
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (tid == 0) {
            T v = do_pivot(fa, n, d.piv0 + k0 + j, F[j + j * LDT]);
            F[j + j * LDT] = v;
            piv = v;
        }
        __syncthreads();
        const T dj = piv;
        for (int i = j + 1 + tid; i < nb; i += 256) F[i + j * LDT] /= dj;
        __syncthreads();
        const int nt = nb - j - 1;
        for (int idx = tid; idx < nt * nt; idx += 256) {
            int ii = idx % nt, qq = idx / nt;
            if (ii >= qq) {
                int i = j + 1 + ii, q = j + 1 + qq;
                F[i + q * LDT] -= F[i + j * LDT] * dj * F[q + j * LDT];
            }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < nb * nb; idx += 256) {
        int r = idx % nb, q = idx / nb;
        if (r >= q) P[(k0 + r) + (int64_t)(k0 + q) * m] = F[r + q * LDT];
    }
}

// Locate the front of a flattened task index through per-step prefix sums.
__device__ inline int find_front(const int32_t *pre, int nf, int b) {
    int lo = 0, hi = nf - 1;
    while (lo < hi) { int mid = (lo + hi + 1) >> 1; if (pre[mid] <= b) lo = mid; else hi = mid - 1; }
    return lo;
}

// Rows below the pivot block: X = F21 L11^-T, then L21 = X D^-1 (one row per thread).
template <typename T>
__global__ __launch_bounds__(256) void k_trsm(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fl,
                                              const int32_t *pre, int nf, int k0) {
    __shared__ T Ls[NB * LDT];
    __shared__ T Ds[NB];
    const int fi = find_front(pre, nf, blockIdx.x);
    const FrontDesc d = sd[fl[fi]];
    const int n = blockIdx.y, tid = threadIdx.x;
    const int nb = min(NB, d.c - k0), m = d.m;
    const int r = k0 + nb + (blockIdx.x - pre[fi]) * 256 + tid;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    for (int idx = tid; idx < NB * NB; idx += 256) {
        int i = idx % NB, q = idx / NB;
        T v = T(0);
        if (i < nb && q < nb && i > q) v = P[(k0 + i) + (int64_t)(k0 + q) * m];
        Ls[i + q * LDT] = v;
    }
    if (tid < NB) Ds[tid] = tid < nb ? P[(k0 + tid) + (int64_t)(k0 + tid) * m] : T(1);
    __syncthreads();
    if (r >= m) return;
    T x[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) x[j] = j < nb ? P[r + (int64_t)(k0 + j) * m] : T(0);
#pragma unroll
    for (int j = 1; j < NB; ++j) {
        T acc = x[j];
#pragma unroll
        for (int q = 0; q < j; ++q) acc -= x[q] * Ls[j + q * LDT];
        x[j] = acc;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (j < nb) P[r + (int64_t)(k0 + j) * m] = x[j] / Ds[j];
}

// Trailing update of every listed front after the pivot block at k0:
// F(r, q) -= sum_k L(r, k) d_k L(q, k) for r >= q >= k0 + nb, one 64x64 tile
// per workgroup, FP64/FP32 MFMA 16x16x4, four waves of 32x32.
template <typename T>
__global__ __launch_bounds__(256) void k_update(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fl,
                                                const int32_t *pre, int nf, int k0) {
    typedef typename Acc<T>::type acc_t;
    constexpr int LDS = 68;
    __shared__ T sA[NB * LDS];
    __shared__ T sB[NB * LDS];
    const int fi = find_front(pre, nf, blockIdx.x);
    const FrontDesc d = sd[fl[fi]];
    const int n = blockIdx.y, tid = threadIdx.x;
    const int nb = min(NB, d.c - k0), m = d.m, c = d.c;
    const int r0 = k0 + nb;
    // triangular decode of the tile index
    const int t = blockIdx.x - pre[fi];
    int ti = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    const int tj = t - ti * (ti + 1) / 2;
    const int R0 = r0 + 64 * ti, Q0 = r0 + 64 * tj;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    T *Ub = fa.U + (int64_t)n * fa.Ustride + d.Uoff;
    {
        const int row = tid & 63, kk = tid >> 6;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k = kk + 4 * j;
            T a = T(0), b = T(0);
            if (k < nb) {
                const T dk = P[(k0 + k) + (int64_t)(k0 + k) * m];
                if (R0 + row < m) a = P[(R0 + row) + (int64_t)(k0 + k) * m] * dk;
                if (Q0 + row < m) b = P[(Q0 + row) + (int64_t)(k0 + k) * m];
            }
            sA[k * LDS + row] = a;
            sB[k * LDS + row] = b;
        }
    }
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    acc_t acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int k = 0; k < NB; k += 4) {
        T a0 = sA[(k + lk) * LDS + wr + li];
        T a1 = sA[(k + lk) * LDS + wr + 16 + li];
        T b0 = sB[(k + lk) * LDS + wc + li];
        T b1 = sB[(k + lk) * LDS + wc + 16 + li];
        acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
        acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
        acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
        acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int r = R0 + wr + bi * 16 + mfma_row(T(0), lk, rr);
                const int q = Q0 + wc + bj * 16 + li;
                if (r < m && q <= r) *front_addr(P, Ub, m, c, r, q) -= acc[bi][bj][rr];
            }
}

// --------------------------------------------------------------------------
// host launchers
// --------------------------------------------------------------------------
template <typename T>
void launch_zero(T *p, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
}

void launch_check_finite(const double *v, int64_t n, int *flag, hipStream_t st) {
    if (n <= 0 || !v) return;
    int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)blocks), dim3(256), 0, st, v, n, flag);
}

template <typename T>
void launch_scatter(const ScatterArgs &a, FactorArgs<T> fa, int64_t N, hipStream_t st) {
    if (a.nnz > 0)
        hipLaunchKernelGGL(k_scatter_A<T>, dim3((unsigned)((a.nnz + 255) / 256), (unsigned)N), dim3(256), 0, st,
                           a.A, a.nnz, a.amap, a.adiag, a.adpiv, fa.L, fa.Lstride, (double *)fa.tau, fa.tstride,
                           (double *)fa.amax, a.dw, a.dc, fa.eps);
    int64_t nc = a.n0 + a.n1;
    if (nc > 0 && a.C0 && a.C1)
        hipLaunchKernelGGL(k_scatter_C<T>, dim3((unsigned)((nc + 255) / 256), (unsigned)N), dim3(256), 0, st,
                           a.C0, a.n0, a.c0map, a.C1, a.n1, a.c1map, fa.L, fa.Lstride);
}

template <typename T>
void launch_small_fronts(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *tasks, int ntasks, int64_t N,
                         const TreeArgs &tr, hipStream_t st) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_small_front<T>, dim3(ntasks, (unsigned)N), dim3(64), 0, st, fa, sd, tasks, tr.cptr,
                       tr.clist, tr.relptr, tr.rel);
}

template <typename T>
void launch_extend_add(FactorArgs<T> fa, const FrontDesc *sd, const RowTask *tasks, int ntasks, int64_t N,
                       const TreeArgs &tr, hipStream_t st) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_extend_add<T>, dim3(ntasks, (unsigned)N), dim3(256), 0, st, fa, sd, tasks, tr.cptr,
                       tr.clist, tr.relptr, tr.rel);
}

template <typename T>
void launch_step(FactorArgs<T> fa, const FrontDesc *sd, const StepDev &s, int64_t N, hipStream_t st) {
    if (s.nf <= 0) return;
    hipLaunchKernelGGL(k_diag<T>, dim3(s.nf, (unsigned)N), dim3(256), 0, st, fa, sd, s.fl, s.k0);
    if (s.ntrsm > 0)
        hipLaunchKernelGGL(k_trsm<T>, dim3(s.ntrsm, (unsigned)N), dim3(256), 0, st, fa, sd, s.fl, s.pre_trsm,
                           s.nf, s.k0);
    if (s.ntile > 0)
        hipLaunchKernelGGL(k_update<T>, dim3(s.ntile, (unsigned)N), dim3(256), 0, st, fa, sd, s.fl, s.pre_tile,
                           s.nf, s.k0);
}

#define KKT_INST(T)                                                                                        \
    template void launch_zero<T>(T *, int64_t, hipStream_t);                                              \
    template void launch_scatter<T>(const ScatterArgs &, FactorArgs<T>, int64_t, hipStream_t);            \
    template void launch_small_fronts<T>(FactorArgs<T>, const FrontDesc *, const int32_t *, int, int64_t, \
                                         const TreeArgs &, hipStream_t);                                  \
    template void launch_extend_add<T>(FactorArgs<T>, const FrontDesc *, const RowTask *, int, int64_t,   \
                                       const TreeArgs &, hipStream_t);                                    \
    template void launch_step<T>(FactorArgs<T>, const FrontDesc *, const StepDev &, int64_t, hipStream_t);
KKT_INST(double)
KKT_INST(float)
template void launch_zero<int64_t>(int64_t *, int64_t, hipStream_t);
template void launch_zero<int>(int *, int64_t, hipStream_t);

}  // namespace kkt
