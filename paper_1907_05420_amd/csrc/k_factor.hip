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
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"
#include "step_plan.hpp"
#include "tile_order.hpp"

namespace kkt {

constexpr int SMALL_M = 64;
constexpr int NB = PIVOT_NB;  // pivot block width
constexpr int LDT = 65;     // LDS leading dimension of a 64x64 tile

// --------------------------------------------------------------------------
// static pivoting rule (oracle's reading): |d| <= tau -> sign(d) * tau,
// inertia from the computed pivot before perturbation.
// --------------------------------------------------------------------------
__device__ inline double pivot_rule(double raw, double t, int sgn, int &cls, int &pert) {
    cls = raw > 0.0 ? 0 : (raw < 0.0 ? 1 : 2);
    pert = 0;
    if (!(fabs(raw) > t)) {  // also catches NaN
        double s = raw > 0.0 ? 1.0 : (raw < 0.0 ? -1.0 : (double)sgn);
        double mag = t > 0.0 ? t : 1e-300;
        pert = 1;
        return s * mag;
    }
    return raw;
}

// per-thread tallies of pivot signs, flushed with one atomic per counter
struct PivTally {
    int c[4] = {0, 0, 0, 0};
    // no dynamic index: the counters stay in registers
    __device__ void add(int cls, int pert) {
        c[0] += cls == 0;
        c[1] += cls == 1;
        c[2] += cls == 2;
        c[3] += pert;
    }
};

// expected sign of pivot gpiv (dual pivots and the Schur complement: -1)
template <typename T>
__device__ inline int pivot_sign(const FactorArgs<T> &fa, int gpiv) {
    return fa.sign ? (int)fa.sign[gpiv] : -1;
}

// raw pivot -> stored pivot; tau_k the pivot's own threshold, tfb the
// threshold used where tau_k is zero (eps * max|A| of the block)
template <typename T>
__device__ inline T do_pivot(T raw, double tau_k, int sgn, double tfb, PivTally &tl) {
    const double t = tau_k > 0.0 ? tau_k : tfb;
    int cls, pert;
    const double v = pivot_rule((double)raw, t, sgn, cls, pert);
    tl.add(cls, pert);
    return (T)v;
}

// block-wide sum of the tallies, one atomic per counter
__device__ inline void flush_tally(PivTally &tl, int64_t *cnt) {
    __shared__ int tot[4];
    if (threadIdx.x < 4) tot[threadIdx.x] = 0;
    __syncthreads();
    for (int k = 0; k < 4; ++k)
        if (tl.c[k]) atomicAdd(&tot[k], tl.c[k]);
    __syncthreads();
    if (threadIdx.x < 4 && tot[threadIdx.x]) atomicAdd((unsigned long long *)(cnt + threadIdx.x), (unsigned long long)tot[threadIdx.x]);
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
// small fronts (m <= MAXM <= 64): extend-add + full partial factorisation in
// LDS, one wavefront per front, lane r owning row r. The LDS tile is sized by
// the front's size class (16, 32 or 64 rows) so that many fronts of the lower
// tree levels share a compute unit.
// --------------------------------------------------------------------------
template <typename T, int MAXM>
__global__ __launch_bounds__(64) void k_small_front(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *tasks,
                                                    const int32_t *cptr, const int32_t *clist,
                                                    const int64_t *relptr, const int32_t *rel) {
    constexpr int LD = MAXM + 1;
    __shared__ T F[MAXM * LD];
    __shared__ T piv;
    __shared__ double taus[MAXM];
    __shared__ int sgns[MAXM];
    const int s = tasks[blockIdx.x];
    const int n = blockIdx.y;
    const int tid = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c, u = m - c;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    // row tid of the pivot columns (loads in batches of 8 from clamped
    // addresses), zero in the update columns
    const int rc = min(tid, m - 1);
    for (int q0 = 0; q0 < m; q0 += 8) {
        T v[8];
#pragma unroll
        for (int u2 = 0; u2 < 8; ++u2) v[u2] = c > 0 ? P[rc + (int64_t)min(q0 + u2, c - 1) * m] : T(0);
#pragma unroll
        for (int u2 = 0; u2 < 8; ++u2) {
            const int q = q0 + u2;
            if (tid < m && q <= tid) F[tid + q * LD] = q < c ? v[u2] : T(0);
        }
    }
    __syncthreads();
    for (int k = cptr[s]; k < cptr[s + 1]; ++k) {
        const int ch = clist[k];
        const FrontDesc dc = sd[ch];
        const int uc = dc.m - dc.c;   // at most m: the child's update rows are rows of this front
        const T *Uc = fa.U + (int64_t)n * fa.Ustride + dc.Uoff;
        const int ri = tid < uc ? rel[relptr[ch] + tid] : 0;
        const T *Ui = Uc + min(tid, uc - 1);
        for (int j0 = 0; j0 < uc; j0 += 8) {
            T v[8];
#pragma unroll
            for (int u2 = 0; u2 < 8; ++u2) v[u2] = Ui[(int64_t)min(j0 + u2, uc - 1) * uc];
#pragma unroll
            for (int u2 = 0; u2 < 8; ++u2) {
                const int j = j0 + u2;
                const int rj = __shfl(ri, min(j, 63), 64);
                if (tid < uc && j <= tid) F[ri + rj * LD] += v[u2];
            }
        }
        __syncthreads();
    }
    PivTally tl;
    if (tid < c) {
        taus[tid] = fa.tau[(int64_t)n * fa.tstride + d.piv0 + tid];
        sgns[tid] = pivot_sign(fa, d.piv0 + tid);
    }
    const double tfb = fa.eps * fa.amax[n];
    __syncthreads();
    for (int j = 0; j < c; ++j) {
        if (tid == 0) {
            T v = do_pivot(F[j + j * LD], taus[j], sgns[j], tfb, tl);
            F[j + j * LD] = v;
            piv = v;
        }
        __syncthreads();
        const T dj = piv;
        // multiplier of row tid, then its rank-1 update of columns j < q <= tid
        T li = T(0);
        if (tid > j && tid < m) {
            li = F[tid + j * LD] / dj;
            F[tid + j * LD] = li;
        }
        __syncthreads();
        const T ld = li * dj;
        if (tid > j && tid < m)
            for (int q = j + 1; q <= tid; ++q) F[tid + q * LD] -= ld * F[q + j * LD];
        __syncthreads();
    }
    flush_tally(tl, fa.cnt + 4 * n);
    // inverse of the unit lower pivot block in place, column by column from
    // the right: X[i][q] = -(L[i][q] + sum_{q<t<i} X[i][t] L[t][q])
    for (int q = c - 2; q >= 0; --q) {
        T x = T(0);
        const int i = tid;
        if (i > q && i < c) {
            x = F[i + q * LD];
            for (int t = q + 1; t < i; ++t) x += F[i + t * LD] * F[t + q * LD];
            x = -x;
        }
        __syncthreads();
        if (i > q && i < c) F[i + q * LD] = x;
        __syncthreads();
    }
    // stores down the columns, lane = row
    if (tid < m)
        for (int q = 0; q < c && q <= tid; ++q) P[tid + (int64_t)q * m] = F[tid + q * LD];
    T *Us = fa.U + (int64_t)n * fa.Ustride + d.Uoff;
    if (tid < u)
        for (int j = 0; j <= tid; ++j) Us[tid + (int64_t)j * u] = F[(c + tid) + (c + j) * LD];
}

// --------------------------------------------------------------------------
// large fronts
// --------------------------------------------------------------------------

template <typename T>
__device__ inline T *front_addr(T *P, T *Ub, int m, int c, int r, int q);

// Epilogue of the update kernels: F(r, qb + j) -= sC[j * ldc] for the NJ
// columns j = j0 + js * jj of row r, restricted to q <= r, q < qhi, r < m.
// All target loads are issued (from clamped, valid addresses) before the
// first store.
template <typename T, int NJ>
__device__ inline void rmw_sub_row(T *P, T *Ub, int m, int c, int r, int qb, int j0, int js, int qhi, const T *sC,
                                   int ldc, int rlim = -1) {
    const int rl = rlim < 0 ? m : rlim;  // rows below rl are not updated
    const int rc = min(r, rl - 1);
    const int lim = min(rc, qhi - 1);
    T o[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) o[jj] = *front_addr(P, Ub, m, c, rc, min(qb + j0 + js * jj, lim));
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int j = j0 + js * jj, q = qb + j;
        if (r < rl && q <= r && q < qhi) *front_addr(P, Ub, m, c, r, q) = o[jj] - sC[j * ldc];
    }
}

template <typename T>
__device__ inline T *front_addr(T *P, T *Ub, int m, int c, int r, int q) {
    return q < c ? P + r + (int64_t)q * m : Ub + (r - c) + (int64_t)(q - c) * (m - c);
}

// The kernels of the panel chain (pivot blocks, their rows and the updates
// inside a sub-panel) raise their waves' issue priority: on the dense Schur
// factor they share compute units with the other stream's trailing update,
// whose MFMA waves would otherwise take most issue slots from them.
__device__ inline void chain_priority() { __builtin_amdgcn_s_setprio(2); }

// Extend-add of the children's update blocks into tiles of 64 rows by EA_CW
// columns of a large front. The child rows and columns landing in a tile
// each form one contiguous range (the relative indices increase), so every
// tile owns its target entries; the task lists those ranges for the children
// that reach the tile, and they are added one after another in increasing
// order. The tile first clears its entries of the front's update block
// (rows and columns at or past the pivots, lower triangle): nothing else
// writes them before, so the update blocks need no clearing pass (their
// strict upper triangles are never read).
template <typename T>
__global__ __launch_bounds__(256) void k_extend_add(FactorArgs<T> fa, const FrontDesc *sd, const EaTask *tasks,
                                                    const int32_t *segs, const int64_t *relptr, const int32_t *rel) {
    __shared__ int32_t rls[EA_CW];
    const EaTask tk = tasks[blockIdx.x];
    const int n = blockIdx.y;
    const FrontDesc d = sd[tk.f];
    const int m = d.m, c = d.c;
    const int r1 = min(tk.r0 + 64, m), c1 = min(tk.c0 + EA_CW, r1);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    T *Ub = fa.U + (int64_t)n * fa.Ustride + d.Uoff;
    {
        const int r = max(tk.r0, c) + lane, q0 = max(tk.c0, c);
        if (r < r1)
            for (int q = q0 + wv; q < c1 && q <= r; q += 4) Ub[(r - c) + (int64_t)(q - c) * (m - c)] = T(0);
    }
    for (int k = 0; k < tk.nseg; ++k) {
        const int32_t *sg = segs + tk.seg + EA_SEG * k;
        const int ch = sg[0], i_lo = sg[1], i_hi = sg[2], j_lo = sg[3], jn = sg[4] - sg[3];
        const FrontDesc dc = sd[ch];
        const int uc = dc.m - dc.c;
        const T *Uc = fa.U + (int64_t)n * fa.Ustride + dc.Uoff;
        const int32_t *rl = rel + relptr[ch];
        __syncthreads();
        for (int t = threadIdx.x; t < jn; t += 256) rls[t] = rl[j_lo + t];
        __syncthreads();
        const int i = i_lo + lane;
        if (i < i_hi) {
            const int R = rl[i];
            const T *Ui = Uc + i;
            const int jend = min(jn, i - j_lo + 1);  // columns j <= i
            for (int jj = wv; jj < jend; jj += 32) {
                T v[8];
                T *ad[8];
#pragma unroll
                for (int u2 = 0; u2 < 8; ++u2) {
                    const int jc = min(jj + 4 * u2, jend - 1);
                    v[u2] = Ui[(int64_t)(j_lo + jc) * uc];
                    ad[u2] = front_addr(P, Ub, m, c, R, rls[jc]);
                }
                T o[8];
#pragma unroll
                for (int u2 = 0; u2 < 8; ++u2) o[u2] = *ad[u2];
#pragma unroll
                for (int u2 = 0; u2 < 8; ++u2)
                    if (jj + 4 * u2 < jend) *ad[u2] = o[u2] + v[u2];
            }
        }
    }
}

// Pivot block at column t0 of every listed front (one wavefront per front and
// period, row i of the block in lane i's registers): LDL^T with the static
// pivot rule, then the inverse of the unit lower triangle, row by row. The
// block keeps D on its diagonal and L^-1 below it; the solves and the
// row-block kernel use the inverse instead of a serial substitution.
// Four waves: lane i holds row i, wave w holds columns [16w, 16w+16) of both
// the block F and X = L^-1, built alongside the elimination (the row
// operations of step j applied to the identity).
// value of v in lane `lane` (wave-uniform) of the calling wavefront
__device__ inline double lane_value(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}
__device__ inline float lane_value(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ inline int lane_value(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// the pivot block at column t0 of front d in period n, by the whole
// 256-thread workgroup; Ls [2][16][NB] and Ds [2][16] in LDS
template <typename T>
__device__ inline void diag_core(const FactorArgs<T> &fa, const FrontDesc &d, int n, int t0, T (*Ls)[16][NB],
                                 T (*Ds)[16]) {
    const int i = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nb = min(NB, d.c - t0), m = d.m;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    T R[16], X[16];
    PivTally tl;
    const double my_tau = (i < nb) ? fa.tau[(int64_t)n * fa.tstride + d.piv0 + t0 + i] : 0.0;
    const int my_sgn = (i < nb) ? pivot_sign(fa, d.piv0 + t0 + i) : -1;
    const double tfb = fa.eps * fa.amax[n];
    {
        const T *Pi = P + (t0 + min(i, nb - 1)) + (int64_t)(t0 + 16 * w) * m;
        T v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = Pi[(int64_t)min(16 * w + k, nb - 1) * m - (int64_t)(16 * w) * m];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int q = 16 * w + k;
            R[k] = (i < nb && q <= i) ? v[k] : T(0);
            X[k] = (q == i) ? T(1) : T(0);
        }
    }
    // Block jb of 16 columns belongs to wave jb (lane = row). That wave
    // eliminates its 16 columns alone, with cross-lane reads and no barrier:
    // step j takes the pivot from lane j, forms the multipliers of column j
    // for all rows and updates its own later columns. It publishes the
    // block's multipliers and pivots once; then the waves right of it apply
    // the block's 16 rank-1 updates to their columns, and the waves up to it
    // the block's row operations on X = L^-1, both in step order (the same
    // operations in the same order as one step at a time).
#pragma unroll 1
    for (int jb = 0; jb < 4; ++jb) {
        if (16 * jb >= nb) break;
        const int bf = jb & 1;
        if (w == jb) {
#pragma unroll
            for (int kj = 0; kj < 16; ++kj) {
                const int j = 16 * jb + kj;
                if (j < nb) {
                    const double tj = lane_value(my_tau, j);
                    const int sj = lane_value(my_sgn, j);
                    int cls, pert;
                    const T dj = (T)pivot_rule((double)lane_value(R[kj], j), tj > 0.0 ? tj : tfb, sj, cls, pert);
                    if (i == j) {
                        tl.add(cls, pert);
                        R[kj] = dj;
                    }
                    const T l = (i > j && i < nb) ? R[kj] / dj : T(0);
                    if (i > j) R[kj] = l;
                    Ls[bf][kj][i] = l;
                    if (i == 0) Ds[bf][kj] = dj;
                    const T ld = l * dj;
                    // the block's later multipliers, read back as LDS
                    // broadcasts: LDS operations of one wave complete in
                    // order, and the wavefront-scope fence keeps the compiler
                    // from moving these reads above the store of other lanes
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
                    for (int k = kj + 1; k < 16; ++k) R[k] -= ld * Ls[bf][kj][16 * jb + k];
                }
            }
        }
        __syncthreads();
        if (w > jb) {
#pragma unroll
            for (int kj = 0; kj < 16; ++kj) {
                if (16 * jb + kj < nb) {
                    const T ld = Ls[bf][kj][i] * Ds[bf][kj];
                    T cq[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) cq[k] = Ls[bf][kj][16 * w + k];
#pragma unroll
                    for (int k = 0; k < 16; ++k) R[k] -= ld * cq[k];
                }
            }
        } else if (w < jb) {
#pragma unroll
            for (int kj = 0; kj < 16; ++kj) {
                const int j = 16 * jb + kj;
                if (j < nb) {
                    const T li = Ls[bf][kj][i];
#pragma unroll
                    for (int k = 0; k < 16; ++k) X[k] -= li * lane_value(X[k], j);
                }
            }
        } else {
#pragma unroll
            for (int kj = 0; kj < 16; ++kj) {
                const int j = 16 * jb + kj;
                if (j < nb) {
                    const T li = Ls[bf][kj][i];
#pragma unroll
                    for (int k = 0; k <= kj; ++k) X[k] -= li * lane_value(X[k], j);
                }
            }
        }
    }
    if (i < nb) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int q = 16 * w + k;
            if (q < i) P[(t0 + i) + (int64_t)(t0 + q) * m] = X[k];
            else if (q == i) P[(t0 + i) + (int64_t)(t0 + q) * m] = R[k];
        }
    }
    flush_tally(tl, fa.cnt + 4 * n);
}

template <typename T>
__global__ __launch_bounds__(256) void k_diag(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fl, int t0) {
    // multipliers and pivots of a 16-column block, double-buffered by block
    __shared__ T Ls[2][16][NB];
    __shared__ T Ds[2][16];
    chain_priority();
    diag_core<T>(fa, sd[fl[blockIdx.x]], blockIdx.y, t0, Ls, Ds);
}

// Locate the front of a flattened task index through per-step prefix sums.
__device__ inline int find_front(const int32_t *pre, int nf, int b) {
    int lo = 0, hi = nf - 1;
    while (lo < hi) { int mid = (lo + hi + 1) >> 1; if (pre[mid] <= b) lo = mid; else hi = mid - 1; }
    return lo;
}

// 64x64 MFMA tile product acc(r, q) = sum_k sA[k][r] sB[k][q] (k-major LDS
// tiles of ld LDS_LD); each of the four waves owns a 32x32 quadrant.
constexpr int LDS_LD = 68;
template <typename T>
__device__ inline void tile_mma(const T *sA, const T *sB, typename Acc<T>::type (&acc)[2][2], int lane, int w) {
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int k = 0; k < NB; k += 4) {
        const T a0 = sA[(k + lk) * LDS_LD + wr + li];
        const T a1 = sA[(k + lk) * LDS_LD + wr + 16 + li];
        const T b0 = sB[(k + lk) * LDS_LD + wc + li];
        const T b1 = sB[(k + lk) * LDS_LD + wc + 16 + li];
        acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
        acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
        acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
        acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
    }
}

// accumulators of the 4 waves -> LDS tile sC[row + col*65]
template <typename T>
__device__ inline void tile_stage(T *sC, typename Acc<T>::type (&acc)[2][2], int lane, int w) {
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
                sC[(wr + bi * 16 + mfma_row(T(0), lk, rr)) + (wc + bj * 16 + li) * LDT] = acc[bi][bj][rr];
}

// Rows below the pivot block: L21 = F21 (L11^-1)^T D^-1 as one MFMA product
// per 64-row tile (L11^-1 is stored in the pivot block).
// row tile `tile` below the pivot block at t0 of front d in period n, by the
// whole 256-thread workgroup; sA, sB [NB * LDS_LD] and Ds [NB] in LDS
template <typename T>
__device__ inline void trsm_core(const FactorArgs<T> &fa, const FrontDesc &d, int n, int tile, int t0, int pe,
                                 int win, T *sA, T *sB, T *Ds) {
    typedef typename Acc<T>::type acc_t;
    const int tid = threadIdx.x;
    const int nb = min(NB, d.c - t0), m = d.m;
    const int mr = win == 3 ? min(pe, d.c) : m;  // rows below mr are left to k_panel_trsm
    const int R0 = t0 + nb + tile * 64;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    {
        // clamped addresses, all loads issued before the first use
        const int row = tid & 63, kk = tid >> 6;
        const T *Pa = P + min(R0 + row, mr - 1) + (int64_t)t0 * m;
        const T *Pb = P + (t0 + min(row, nb - 1)) + (int64_t)t0 * m;
        T va[16], vb[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int kc = min(kk + 4 * j, nb - 1);
            va[j] = Pa[(int64_t)kc * m];
            vb[j] = Pb[(int64_t)kc * m];
        }
        const T dv = P[(t0 + min(row, nb - 1)) + (int64_t)(t0 + min(row, nb - 1)) * m];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k = kk + 4 * j;
            sA[k * LDS_LD + row] = (k < nb && R0 + row < mr) ? va[j] : T(0);
            // B[q = row][k] = (L11^-1)[row][k]
            sB[k * LDS_LD + row] = (row < nb && k < nb) ? (k < row ? vb[j] : (k == row ? T(1) : T(0))) : T(0);
        }
        if (tid < NB) Ds[tid] = tid < nb ? dv : T(1);
    }
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6;
    acc_t acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
    tile_mma<T>(sA, sB, acc, lane, w);
    __syncthreads();
    T *sC = sA;
    tile_stage<T>(sC, acc, lane, w);
    __syncthreads();
    const int row = tid & 63;
    const int r = R0 + row;
    if (r < mr)
        for (int q = tid >> 6; q < nb; q += 4) P[r + (int64_t)(t0 + q) * m] = sC[row + q * LDT] / Ds[q];
}

template <typename T>
__global__ __launch_bounds__(256) void k_trsm(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fl,
                                              const int32_t *pre, int nf, int t0, int pe, int win) {
    __shared__ T sA[NB * LDS_LD];
    __shared__ T sB[NB * LDS_LD];
    __shared__ T Ds[NB];
    chain_priority();
    const int fi = find_front(pre, nf, blockIdx.x);
    trsm_core<T>(fa, sd[fl[fi]], blockIdx.y, blockIdx.x - pre[fi], t0, pe, win, sA, sB, Ds);
}

// Rows below a factored sub-panel (columns [t0, cend), cend = min(pe, c), at
// most 4 pivot blocks of 64) of every listed front and period: L21 = A21 L11^-T D^-1 for the rows [cend, m),
// one 64-row tile per workgroup. For column block b of the sub-panel,
//   V_b = A21_b - sum_{c<b} L21_c D_c L_bc^T,   L21_b = V_b X_b^T D_b^-1,
// with L_bc the factored diagonal block's sub-block and X_b the stored
// inverse of its unit lower 64x64 diagonal block b: the per-block triangular
// solves and in-panel updates of the rows below, done for one row tile at a
// time (one launch per sub-panel instead of two per pivot block). The tile's
// finished blocks L21_c stay in registers (accumulator layout) and pass
// through LDS as MFMA operands.
template <typename T>
__device__ inline void acc_to_kmajor(T *sA, const typename Acc<T>::type (&acc)[2][2], const T *scale, int lane,
                                     int w) {
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int r = wr + bi * 16 + mfma_row(T(0), lk, rr), k = wc + bj * 16 + li;
                sA[k * LDS_LD + r] = acc[bi][bj][rr] * scale[k];
            }
}

template <typename T>
__global__ __launch_bounds__(256) void k_panel_trsm(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fl,
                                                    const int32_t *pre, int nf, int t0, int pe) {
    typedef typename Acc<T>::type acc_t;
    __shared__ T sA[NB * LDS_LD];
    __shared__ T sB[NB * LDS_LD];
    __shared__ T sD[4 * NB];
    chain_priority();
    const int fi = find_front(pre, nf, blockIdx.x);
    const FrontDesc d = sd[fl[fi]];
    const int n = blockIdx.y, tid = threadIdx.x;
    const int m = d.m, cend = min(pe, d.c), W = cend - t0;
    const int R0 = cend + (blockIdx.x - pre[fi]) * 64;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    const int lane = tid & 63, w = tid >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32, li = lane & 15, lk = lane >> 4;
    const int row = tid & 63, kk = tid >> 6;
    for (int k = tid; k < 4 * NB; k += 256) sD[k] = k < W ? P[(t0 + k) + (int64_t)(t0 + k) * m] : T(1);
    const int rowc = min(R0 + row, m - 1);  // clamped row of this thread's loads
    acc_t Lr[4][2][2];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) Lr[b][bi][bj] = acc_t{0, 0, 0, 0};
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int cb = t0 + 64 * b;
        if (cb < cend) {
            const int nbb = min(64, cend - cb);
            acc_t acc[2][2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
            // acc = sum_{c<b} L21_c D_c L_bc^T (blocks c < b are full 64 wide)
#pragma unroll
            for (int c = 0; c < b; ++c) {
                T vb[16];
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    vb[j] = P[(cb + min(row, nbb - 1)) + (int64_t)(t0 + 64 * c + kk + 4 * j) * m];
                acc_to_kmajor<T>(sA, Lr[c], sD + 64 * c, lane, w);
#pragma unroll
                for (int j = 0; j < 16; ++j) sB[(kk + 4 * j) * LDS_LD + row] = row < nbb ? vb[j] : T(0);
                __syncthreads();
                tile_mma<T>(sA, sB, acc, lane, w);
                __syncthreads();
            }
            // V = A21_b - acc, k-major in sA; X_b^T operand in sB
            {
                T va[16], vx[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int k = min(kk + 4 * j, nbb - 1);
                    va[j] = P[rowc + (int64_t)(cb + k) * m];
                    vx[j] = P[(cb + min(row, nbb - 1)) + (int64_t)(cb + k) * m];
                }
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int k = kk + 4 * j;
                    sA[k * LDS_LD + row] = (k < nbb && R0 + row < m) ? va[j] : T(0);
                    // sB[k][q] = X_b(q, k): unit lower, stored strictly below the diagonal
                    sB[k * LDS_LD + row] = (row < nbb && k < nbb) ? (k < row ? vx[j] : (k == row ? T(1) : T(0))) : T(0);
                }
            }
            __syncthreads();
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int r = wr + bi * 16 + mfma_row(T(0), lk, rr), k = wc + bj * 16 + li;
                        sA[k * LDS_LD + r] -= acc[bi][bj][rr];
                    }
            __syncthreads();
            acc_t res[2][2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) res[bi][bj] = acc_t{0, 0, 0, 0};
            tile_mma<T>(sA, sB, res, lane, w);
            // L21_b = V X_b^T D_b^-1
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int q = wc + bj * 16 + li;
                        Lr[b][bi][bj][rr] = res[bi][bj][rr] / sD[64 * b + q];
                    }
            __syncthreads();
            // coalesced store through LDS
            tile_stage<T>(sA, Lr[b], lane, w);
            __syncthreads();
            if (R0 + row < m)
                for (int q = kk; q < nbb; q += 4) P[(R0 + row) + (int64_t)(cb + q) * m] = sA[row + q * LDT];
            __syncthreads();
        }
    }
}

// algorithmic work of one trailing-update launch on a front (see kkt.h)
void update_work(int t0, int pe, int c, int m, int win, double *flops, double *bytes) {
    const UpdGeom g = upd_geom(3, t0, pe, c, m, win);
    const double lo = g.lo, qhi = g.qhi, K = g.K;
    if (qhi <= lo || K <= 0) { *flops = 0.0; *bytes = 0.0; return; }
    const double entries = (qhi - lo) * m - (lo + qhi - 1.0) * (qhi - lo) * 0.5;
    *flops = 2.0 * K * entries;
    *bytes = 16.0 * entries + 8.0 * K * ((m - lo) + (qhi - lo));
}

// tile (ti, tj) of a trapezoid: column tiles tj < Tc, row tiles ti in [tj, Tr)
__device__ inline void trap_decode(int t, int Tr, int &ti, int &tj) {
    int j = (int)floor(((2.0 * Tr + 1.0) - sqrt((2.0 * Tr + 1.0) * (2.0 * Tr + 1.0) - 8.0 * t)) * 0.5);
    if (j < 0) j = 0;
    while (j > 0 && j * Tr - j * (j - 1) / 2 > t) --j;
    while ((j + 1) * Tr - (j + 1) * j / 2 <= t) ++j;
    tj = j;
    ti = j + (t - (j * Tr - j * (j - 1) / 2));
}

// F(r, q) -= sum_k L(r, k) d_k L(q, k) for r >= q in the region of upd_geom:
// one 64x64 tile per workgroup, K in chunks of 64, FP64/FP32 MFMA 16x16x4,
// coalesced read-modify-write of the target through an LDS stage.
// tile `tile` of an update of front d in period n, by the whole 256-thread
// workgroup; sA, sB [NB * LDS_LD] in LDS
template <typename T>
__device__ inline void update_core(const FactorArgs<T> &fa, const FrontDesc &d, int n, int tile, int kind, int t0,
                                   int pe, int win, T *sA, T *sB) {
    typedef typename Acc<T>::type acc_t;
    const int tid = threadIdx.x;
    const int m = d.m, c = d.c;
    const UpdGeom g = upd_geom(kind, t0, pe, c, m, win);
    const int mr = (kind == 2 && win == 3) ? g.qhi : m;  // rows below mr are left to k_panel_trsm
    const int Tr = (mr - g.lo + 63) / 64;
    int ti, tj;
    trap_decode(tile, Tr, ti, tj);
    const int R0 = g.lo + 64 * ti, Q0 = g.lo + 64 * tj;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    T *Ub = fa.U + (int64_t)n * fa.Ustride + d.Uoff;
    const int lane = tid & 63, w = tid >> 6;
    acc_t acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
    const int row = tid & 63, kk = tid >> 6;
    const bool arow = R0 + row < m, brow = Q0 + row < m;
    const T *Pa = P + min(R0 + row, m - 1), *Pb = P + min(Q0 + row, m - 1);
    for (int kc = 0; kc < g.K; kc += NB) {
        const int kn = min(NB, g.K - kc);
        T ra[16], rb[16], rd[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k = min(kk + 4 * j, kn - 1);
            const int col = t0 + kc + k;
            ra[j] = Pa[(int64_t)col * m];
            rb[j] = Pb[(int64_t)col * m];
            rd[j] = P[col + (int64_t)col * m];
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k = kk + 4 * j;
            const bool ok = k < kn;
            sA[k * LDS_LD + row] = (ok && arow) ? ra[j] * rd[j] : T(0);
            sB[k * LDS_LD + row] = (ok && brow) ? rb[j] : T(0);
        }
        __syncthreads();
        tile_mma<T>(sA, sB, acc, lane, w);
        __syncthreads();
    }
    T *sC = sA;
    tile_stage<T>(sC, acc, lane, w);
    __syncthreads();
    rmw_sub_row<T, 16>(P, Ub, m, c, R0 + row, Q0, kk, 4, g.qhi, sC + row, LDT, mr);
}

template <typename T>
__global__ __launch_bounds__(256) void k_update(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fl,
                                                const int32_t *pre, int nf, int kind, int t0, int pe, int win) {
    __shared__ T sA[NB * LDS_LD];
    __shared__ T sB[NB * LDS_LD];
    chain_priority();
    const int fi = find_front(pre, nf, blockIdx.x);
    update_core<T>(fa, sd[fl[fi]], blockIdx.y, blockIdx.x - pre[fi], kind, t0, pe, win, sA, sB);
}

// Trailing update after an outer panel (kind 3) on 128x128 tiles: four waves
// of 64x64 (4x4 MFMA 16x16x4 blocks each). No LDS and no barrier in the main
// loop: every lane loads its own MFMA operands (rows of the panel, one K step
// of 4 per slot) with buffer loads into a ring of UPF register slots, so each
// wave runs on its own and the loads of later steps are in flight while the
// current one is multiplied. Buffer loads (intrinsic calls) keep the ring: a
// plain load feeding a loop-carried value is folded into the next iteration.
// Columns past the panel's K read as zero through the buffer's range check.
// The epilogue goes through LDS in four 32-column quarters for a coalesced
// read-modify-write of the target.
constexpr int BT = BIG_TILE;  // tile edge
constexpr int UPF = 3;       // K steps in flight per lane

template <typename T>
__global__ __launch_bounds__(256, 2) void k_update_big(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fl,
                                                       const int32_t *pre, int nf, int t0, int pe, int win) {
    typedef typename Acc<T>::type acc_t;
    __shared__ T sC[32 * (BT + 1)];
    __shared__ T sD[MAX_OUTER_W + 4 * UPF];
    const int fi = find_front(pre, nf, blockIdx.x);
    const FrontDesc d = sd[fl[fi]];
    const int n = blockIdx.y, tid = threadIdx.x;
    const int m = d.m, c = d.c;
    const UpdGeom g = upd_geom(3, t0, pe, c, m, win);
    const int Tr = (m - g.lo + BT - 1) / BT;
    int ti, tj;
    if (nf == 1 && gridDim.y == 1) trap_decode_xcd(blockIdx.x, Tr, (g.qhi - g.lo + BT - 1) / BT, ti, tj);
    else trap_decode(blockIdx.x - pre[fi], Tr, ti, tj);
    const int R0 = g.lo + BT * ti, Q0 = g.lo + BT * tj;
    T *P = fa.L + (int64_t)n * fa.Lstride + d.Loff;
    T *Ub = fa.U + (int64_t)n * fa.Ustride + d.Uoff;
    const int lane = tid & 63, w = tid >> 6;
    const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
    const int li = lane & 15, lk = lane >> 4;
    acc_t acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
    // pivots D of the K range (K <= MAX_OUTER_W), zero past K
    const int nks = (g.K + 3) / 4;                     // K steps of 4
    const int nkp = ((nks + UPF - 1) / UPF) * UPF;     // padded to the ring
    for (int k = tid; k < 4 * nkp; k += 256) sD[k] = k < g.K ? P[(t0 + k) + (int64_t)(t0 + k) * m] : T(0);
    __syncthreads();
    // the panel's K columns as one buffer; lane offsets of its four A rows
    // and four B rows (rows past the front clamped) in column lk
    const BufRes rs = make_bufres(P + (int64_t)t0 * m, (int64_t)g.K * m * (int64_t)sizeof(T));
    int oa[4], ob[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        oa[x] = (int)sizeof(T) * (min(R0 + wr + 16 * x + li, m - 1) + lk * m);
        ob[x] = (int)sizeof(T) * (min(Q0 + wc + 16 * x + li, m - 1) + lk * m);
    }
    const int step = (int)sizeof(T) * 4 * m;
    T ra[UPF][4], rb[UPF][4];
    auto load = [&](int slot, int ks) {
        const int co = step * ks;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            ra[slot][x] = buf_load(rs, oa[x] + co, T(0));
            rb[slot][x] = buf_load(rs, ob[x] + co, T(0));
        }
    };
#pragma unroll
    for (int sl = 0; sl < UPF - 1; ++sl) load(sl, sl);
    for (int ks0 = 0; ks0 < nkp; ks0 += UPF) {
#pragma unroll
        for (int sl = 0; sl < UPF; ++sl) {
            const int ks = ks0 + sl;
            load((sl + UPF - 1) % UPF, ks + UPF - 1);
            const T dk = sD[4 * ks + lk];
            T a[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) a[x] = ra[sl][x] * dk;
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma16x16x4(a[bi], rb[sl][bj], acc[bi][bj]);
        }
    }
    const int lrow = tid & (BT - 1), lkk = tid >> 7;
    // epilogue: four 32-column quarters through LDS (128 x 32 stage, ld 129)
#pragma unroll
    for (int qt = 0; qt < 4; ++qt) {
        if ((w & 1) == (qt >> 1)) {
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr)
                        sC[(wr + 16 * bi + mfma_row(T(0), lk, rr)) + (16 * bb + li) * (BT + 1)] =
                            acc[bi][2 * (qt & 1) + bb][rr];
        }
        __syncthreads();
        rmw_sub_row<T, 16>(P, Ub, m, c, R0 + lrow, Q0 + 32 * qt, lkk, 2, g.qhi, sC + lrow, BT + 1);
        __syncthreads();
    }
}

// In-place inverse of the unit lower 256x256 diagonal block of a factor
// (after the panel holding it is complete), from the inverses of its 64x64
// diagonal sub-blocks: for every sub-block column j and row i > j,
//   X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj     (X_jj unit lower, stored below
// its diagonal), processed column by column so that every L_ik still needed
// is intact. Products on MFMA through the 64x64 tile helpers. blockIdx.x
// picks the front, blockIdx.y the diagonal block, blockIdx.z the period.
template <typename T>
__global__ __launch_bounds__(256) void k_inv256(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fl, int j0) {
    typedef typename Acc<T>::type acc_t;
    __shared__ T sA[NB * LDS_LD];
    __shared__ T sB[NB * LDS_LD];
    const FrontDesc d = sd[fl[blockIdx.x]];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m = d.m;
    j0 += INV_W * blockIdx.y;  // one diagonal block per blockIdx.y
    if (j0 >= d.c) return;
    const int nbw = min(INV_W, d.c - j0);
    const int nsb = (nbw + 63) / 64;
    T *P = fa.L + (int64_t)blockIdx.z * fa.Lstride + d.Loff;
    const int row = tid & 63, kk = tid >> 6;
    // load a 64x64 sub-block (rows r0.., cols c0..) as sX[k][r] = M[r][k]
    // (transposed, "A" operand) or sX[k][q] = M[k][q] ("B" operand); unit
    // lower when diag.
    auto load = [&](T *sX, int r0, int c0, bool asA, bool diag) {
        // clamped addresses, all 16 loads issued before the first use
        const int lim = j0 + nbw - 1;
        T val[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k = kk + 4 * j;
            const int a = asA ? row : k, b = asA ? k : row;
            val[j] = P[(int64_t)min(r0 + a, lim) + (int64_t)min(c0 + b, lim) * m];
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k = kk + 4 * j;
            const int a = asA ? row : k, b = asA ? k : row;
            const bool in = r0 + a <= lim && c0 + b <= lim;
            T v = in ? val[j] : T(0);
            if (diag) v = a > b ? v : (a == b ? T(1) : T(0));
            sX[k * LDS_LD + row] = v;
        }
    };
    acc_t acc[2][2];
    for (int j = 0; j + 1 < nsb; ++j) {
        for (int i = j + 1; i < nsb; ++i) {
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
            for (int k = j; k < i; ++k) {
                __syncthreads();
                load(sA, j0 + 64 * i, j0 + 64 * k, true, false);        // L_ik
                load(sB, j0 + 64 * k, j0 + 64 * j, false, k == j);      // X_kj
                __syncthreads();
                tile_mma<T>(sA, sB, acc, lane, w);
            }
            // T -> sB as a "B" operand (sB[k][q] = T[k][q]), X_ii -> sA
            __syncthreads();
            T *sC = sB;
            {
                const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
                const int li = lane & 15, lk = lane >> 4;
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr)
                            sC[(wr + bi * 16 + mfma_row(T(0), lk, rr)) * LDS_LD + (wc + bj * 16 + li)] = acc[bi][bj][rr];
            }
            load(sA, j0 + 64 * i, j0 + 64 * i, true, true);             // X_ii
            __syncthreads();
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
            tile_mma<T>(sA, sB, acc, lane, w);
            __syncthreads();
            tile_stage<T>(sA, acc, lane, w);
            __syncthreads();
            const int r = j0 + 64 * i + row;
            if (r < j0 + nbw)
                for (int q = kk; q < 64; q += 4) {
                    const int cq = j0 + 64 * j + q;
                    P[(int64_t)r + (int64_t)cq * m] = -sA[row + q * LDT];
                }
        }
    }
}

// Copy of the inverted INV_W window of a wide front (strictly below its
// diagonal) into the window's strict upper triangle, transposed, so that the
// backward solve reads X^T with the same row-wise products as the forward
// solve reads X. The upper triangle of a front's pivot block holds nothing
// else. 64x64 tiles through LDS: blockIdx.x the front, blockIdx.y the
// window, blockIdx.z the period.
template <typename T>
__global__ __launch_bounds__(256) void k_win_transpose(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fl) {
    __shared__ T tile[64 * 65];
    const FrontDesc d = sd[fl[blockIdx.x]];
    const int j0 = INV_W * blockIdx.y;
    if (j0 >= d.c) return;
    const int nbw = min(INV_W, d.c - j0), nsb = (nbw + 63) / 64;
    const int m = d.m;
    T *P = fa.L + (int64_t)blockIdx.z * fa.Lstride + d.Loff + j0 + (int64_t)j0 * m;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int kb = 0; kb < nsb; ++kb)
        for (int qb = 0; qb <= kb; ++qb) {
            // tile rows 64 kb + a, columns 64 qb + q (a lane, q over the waves)
            const int r = min(64 * kb + lane, nbw - 1);
            for (int q = w; q < 64; q += 4) tile[lane + q * 65] = P[r + (int64_t)min(64 * qb + q, nbw - 1) * m];
            __syncthreads();
            // written transposed: row 64 qb + lane, column 64 kb + a
            const int i = 64 * qb + lane;
            for (int a = w; a < 64; a += 4) {
                const int col = 64 * kb + a;
                if (i < nbw && col < nbw && col > i) P[i + (int64_t)col * m] = tile[a + lane * 65];
            }
            __syncthreads();
        }
}

// Inverse of the unit lower 2W block [ja, ja + 2W) of a dense factor from
// the inverses Xa, Xb of its two W-wide diagonal blocks (stored below their
// diagonals): X = [Xa 0; Xba Xb] with Xba = -Xb Lba Xa, in two launches of
// 64x64 tiles: mode 0 forms T = Lba Xa into `tmp` (ld W), mode 1 writes -Xb T
// in place of Lba. Lba is no longer needed by the factorisation once the
// panel's own updates are done. W is INV_W or 2 INV_W; blockIdx.y picks the
// 2W block (ja = j0 + 2W blockIdx.y, its own W x W staging in tmp).
__device__ inline void load_tile64(double *sX, const double *base, int64_t ld, int r0, int c0, int rlim, int clim,
                                   bool asA, bool diag, int row, int kk) {
    // sX[k][r] = M[r0 + r][c0 + k] ("A" operand, transposed) or
    // sX[k][q] = M[r0 + k][c0 + q] ("B" operand); rows >= rlim and columns
    // >= clim read as zero; unit lower (upper part zero) when diag
    double val[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int k = kk + 4 * j;
        const int a = asA ? row : k, b = asA ? k : row;
        val[j] = base[(int64_t)min(r0 + a, rlim - 1) + (int64_t)min(c0 + b, clim - 1) * ld];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int k = kk + 4 * j;
        const int a = asA ? row : k, b = asA ? k : row;
        const bool in = r0 + a < rlim && c0 + b < clim;
        double v = in ? val[j] : 0.0;
        if (diag) v = a > b ? v : (a == b ? 1.0 : 0.0);
        sX[k * LDS_LD + row] = v;
    }
}

__global__ __launch_bounds__(256) void k_inv_combine(FactorArgs<double> fa, const FrontDesc *sd, const int32_t *fl,
                                                     int j0, int mode, double *tmp, int W) {
    typedef Acc<double>::type acc_t;
    __shared__ double sA[NB * LDS_LD];
    __shared__ double sB[NB * LDS_LD];
    const FrontDesc d = sd[fl[0]];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int row = tid & 63, kk = tid >> 6;
    const int m = d.m;
    const int ja = j0 + 2 * W * blockIdx.y, jb = ja + W;
    tmp += (int64_t)W * W * blockIdx.y;
    const int nbw_b = min(W, d.c - jb);
    const int ti = blockIdx.x / (W / 64), tj = blockIdx.x % (W / 64);
    if (nbw_b <= 64 * ti) return;  // no second block, or a tile row past its end
    double *P = fa.L + d.Loff;
    acc_t acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
    if (mode == 0) {
        // T_ij = sum_{k >= j} Lba_ik Xa_kj
        for (int k = tj; k < W / 64; ++k) {
            __syncthreads();
            load_tile64(sA, P, m, jb + 64 * ti, ja + 64 * k, jb + nbw_b, jb, true, false, row, kk);
            load_tile64(sB, P, m, ja + 64 * k, ja + 64 * tj, jb, jb, false, k == tj, row, kk);
            __syncthreads();
            tile_mma<double>(sA, sB, acc, lane, w);
        }
    } else {
        // Xba_ij = -sum_{k <= i} Xb_ik T_kj
        for (int k = 0; k <= ti; ++k) {
            __syncthreads();
            load_tile64(sA, P, m, jb + 64 * ti, jb + 64 * k, jb + nbw_b, jb + nbw_b, true, k == ti, row, kk);
            load_tile64(sB, tmp, W, 64 * k, 64 * tj, nbw_b, W, false, false, row, kk);
            __syncthreads();
            tile_mma<double>(sA, sB, acc, lane, w);
        }
    }
    __syncthreads();
    tile_stage<double>(sA, acc, lane, w);
    __syncthreads();
    const int r = 64 * ti + row;
    if (r < nbw_b)
        for (int q = kk; q < 64; q += 4) {
            const double v = sA[row + q * LDT];
            if (mode == 0) tmp[r + (int64_t)(64 * tj + q) * W] = v;
            else P[(int64_t)(jb + r) + (int64_t)(ja + 64 * tj + q) * m] = -v;
        }
}

void launch_inv256(FactorArgs<double> fa, const FrontDesc *sd, const int32_t *fl, int j0, hipStream_t st) {
    hipLaunchKernelGGL(k_inv256<double>, dim3(1), dim3(256), 0, st, fa, sd, fl, j0);
}

template <typename T>
void launch_window_inverses(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *fronts, int nfront, int maxc,
                            int64_t N, hipStream_t st) {
    if (nfront <= 0 || maxc <= 0) return;
    const dim3 g(nfront, (unsigned)((maxc + INV_W - 1) / INV_W), (unsigned)N);
    hipLaunchKernelGGL(k_inv256<T>, g, dim3(256), 0, st, fa, sd, fronts, 0);
    hipLaunchKernelGGL(k_win_transpose<T>, g, dim3(256), 0, st, fa, sd, fronts);
}

void launch_inv_combine(FactorArgs<double> fa, const FrontDesc *sd, const int32_t *fl, int j0, int c, double *tmp,
                        hipStream_t st) {
    const int nbw_b = std::min(INV_W, c - (j0 + INV_W));
    if (nbw_b <= 0) return;
    const int tiles = ((nbw_b + 63) / 64) * (INV_W / 64);
    for (int mode = 0; mode < 2; ++mode)
        hipLaunchKernelGGL(k_inv_combine, dim3(tiles), dim3(256), 0, st, fa, sd, fl, j0, mode, tmp, INV_W);
}

void launch_inverses_all(FactorArgs<double> fa, const FrontDesc *sd, const int32_t *fl, int c, double *tmp,
                         hipStream_t st) {
    if (c <= 0) return;
    hipLaunchKernelGGL(k_inv256<double>, dim3(1, (unsigned)((c + INV_W - 1) / INV_W)), dim3(256), 0, st, fa, sd, fl,
                       0);
    // 2 INV_W blocks from pairs of INV_W ones, then DENSE_INV_W blocks
    for (int W = INV_W; 2 * W <= DENSE_INV_W && c > W; W *= 2) {
        const int pairs = (c + 2 * W - 1) / (2 * W);
        for (int mode = 0; mode < 2; ++mode)
            hipLaunchKernelGGL(k_inv_combine, dim3((W / 64) * (W / 64), (unsigned)pairs), dim3(256), 0, st, fa, sd,
                               fl, 0, mode, tmp, W);
    }
}

// Structured Schur elimination (section 4.3): G = W Linv for one front, W the
// N_s x N_s block below its pivot block (rows ns.., ld m) and Linv the
// inverse of the unit lower pivot block stored strictly below its diagonal
// (ld m); G (ld ns) and its transpose GT (ld ns) are written out. 64x64 tiles:
//   G[I][Q] = sum_{K >= Q} W[I][K] Linv[K][Q]   (Linv[Q][Q] unit lower)
__global__ __launch_bounds__(256) void k_struct_g(const double *F, int m, int ns, double *G, double *GT) {
    typedef Acc<double>::type acc_t;
    __shared__ double sA[NB * LDS_LD];
    __shared__ double sB[NB * LDS_LD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int row = tid & 63, kk = tid >> 6;
    const int nt = (ns + 63) / 64;
    const int ti = blockIdx.x / nt, tq = blockIdx.x % nt;
    acc_t acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
    for (int k = tq; k < nt; ++k) {
        __syncthreads();
        load_tile64(sA, F, m, ns + 64 * ti, 64 * k, m, ns, true, false, row, kk);   // W[I][K]
        load_tile64(sB, F, m, 64 * k, 64 * tq, ns, ns, false, k == tq, row, kk);   // Linv[K][Q]
        __syncthreads();
        tile_mma<double>(sA, sB, acc, lane, w);
    }
    __syncthreads();
    tile_stage<double>(sA, acc, lane, w);
    __syncthreads();
    const int i = 64 * ti + row;
    if (i < ns)
        for (int c = kk; c < 64; c += 4) {
            const int q = 64 * tq + c;
            if (q < ns) {
                const double v = sA[row + c * LDT];
                G[i + (int64_t)q * ns] = v;
                GT[q + (int64_t)i * ns] = v;
            }
        }
}

void launch_struct_g(const double *F, int m, int ns, double *G, double *GT, hipStream_t st) {
    const int nt = (ns + 63) / 64;
    hipLaunchKernelGGL(k_struct_g, dim3((unsigned)(nt * nt)), dim3(256), 0, st, F, m, ns, G, GT);
}

// Pairs of block columns of the structured factor (the solves take the
// recurrences two columns per step): for pair p (columns 2p, 2p + 1)
//   M_p = (I - G_{2p+1}) (I - G_{2p}) = I - G_{2p} - G_{2p+1} + G_{2p+1} G_{2p}
// and its transpose; G_{N-1} = 0 (the last column has no block below).
// 64x64 tiles, grid (tiles, pairs).
__global__ __launch_bounds__(256) void k_struct_pair(const double *G, int ns, int N, double *M, double *MT) {
    typedef Acc<double>::type acc_t;
    __shared__ double sA[NB * LDS_LD];
    __shared__ double sB[NB * LDS_LD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int row = tid & 63, kk = tid >> 6;
    const int nt = (ns + 63) / 64;
    const int ti = blockIdx.x / nt, tq = blockIdx.x % nt, pr = blockIdx.y;
    const int64_t nn = (int64_t)ns * ns;
    const double *G0 = G + (int64_t)(2 * pr) * nn;
    const bool has1 = 2 * pr + 1 <= N - 2;
    const double *G1 = G + (int64_t)(2 * pr + 1) * nn;
    acc_t acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = acc_t{0, 0, 0, 0};
    if (has1)
        for (int k = 0; k < nt; ++k) {
            __syncthreads();
            load_tile64(sA, G1, ns, 64 * ti, 64 * k, ns, ns, true, false, row, kk);   // G_{2p+1}[I][K]
            load_tile64(sB, G0, ns, 64 * k, 64 * tq, ns, ns, false, false, row, kk);  // G_{2p}[K][Q]
            __syncthreads();
            tile_mma<double>(sA, sB, acc, lane, w);
        }
    __syncthreads();
    tile_stage<double>(sA, acc, lane, w);
    __syncthreads();
    const int i = 64 * ti + row;
    if (i < ns)
        for (int c = kk; c < 64; c += 4) {
            const int q = 64 * tq + c;
            if (q < ns) {
                const int64_t at = i + (int64_t)q * ns;
                const double v = (i == q ? 1.0 : 0.0) - G0[at] - (has1 ? G1[at] : 0.0) + sA[row + c * LDT];
                M[(int64_t)pr * nn + at] = v;
                MT[(int64_t)pr * nn + q + (int64_t)i * ns] = v;
            }
        }
}

void launch_struct_pair(const double *G, int ns, int N, double *M, double *MT, hipStream_t st) {
    const int nt = (ns + 63) / 64;
    hipLaunchKernelGGL(k_struct_pair, dim3((unsigned)(nt * nt), (unsigned)(N / 2)), dim3(256), 0, st, G, ns, N, M, MT);
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
void launch_small_fronts(FactorArgs<T> fa, const FrontDesc *sd, const int32_t *tasks, const int *ncls, int64_t N,
                         const TreeArgs &tr, hipStream_t st) {
    // tasks: the fronts of at most 16, then 32, then 64 rows (ncls[0..2] of each)
    if (ncls[0] > 0)
        hipLaunchKernelGGL((k_small_front<T, 16>), dim3(ncls[0], (unsigned)N), dim3(64), 0, st, fa, sd, tasks,
                           tr.cptr, tr.clist, tr.relptr, tr.rel);
    if (ncls[1] > 0)
        hipLaunchKernelGGL((k_small_front<T, 32>), dim3(ncls[1], (unsigned)N), dim3(64), 0, st, fa, sd,
                           tasks + ncls[0], tr.cptr, tr.clist, tr.relptr, tr.rel);
    if (ncls[2] > 0)
        hipLaunchKernelGGL((k_small_front<T, 64>), dim3(ncls[2], (unsigned)N), dim3(64), 0, st, fa, sd,
                           tasks + ncls[0] + ncls[1], tr.cptr, tr.clist, tr.relptr, tr.rel);
}

template <typename T>
void launch_extend_add(FactorArgs<T> fa, const FrontDesc *sd, const EaTask *tasks, int ntasks, int64_t N,
                       const TreeArgs &tr, hipStream_t st) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_extend_add<T>, dim3(ntasks, (unsigned)N), dim3(256), 0, st, fa, sd, tasks,
                       (const int32_t *)tasks, tr.relptr, tr.rel);
}

template <typename T>
void launch_step(FactorArgs<T> fa, const FrontDesc *sd, const StepDev &s, int64_t N, hipStream_t st) {
    if (s.nf <= 0 || (s.kind != 0 && s.ntasks <= 0)) return;
    switch (s.kind) {
        case 0:
            hipLaunchKernelGGL(k_diag<T>, dim3(s.nf, (unsigned)N), dim3(256), 0, st, fa, sd, s.fl, s.t0);
            break;
        case 1:
            hipLaunchKernelGGL(k_trsm<T>, dim3(s.ntasks, (unsigned)N), dim3(256), 0, st, fa, sd, s.fl, s.pre, s.nf,
                               s.t0, s.pe, s.win);
            break;
        case 7:
            hipLaunchKernelGGL(k_panel_trsm<T>, dim3(s.ntasks, (unsigned)N), dim3(256), 0, st, fa, sd, s.fl, s.pre,
                               s.nf, s.t0, s.pe);
            break;

        case 4:
            hipLaunchKernelGGL(k_update_big<T>, dim3(s.ntasks, (unsigned)N), dim3(256), 0, st, fa, sd, s.fl, s.pre,
                               s.nf, s.t0, s.pe, s.win);
            break;
        default:
            hipLaunchKernelGGL(k_update<T>, dim3(s.ntasks, (unsigned)N), dim3(256), 0, st, fa, sd, s.fl, s.pre,
                               s.nf, s.kind, s.t0, s.pe, s.win);
    }
}

#define KKT_INST(T)                                                                                        \
    template void launch_zero<T>(T *, int64_t, hipStream_t);                                              \
    template void launch_scatter<T>(const ScatterArgs &, FactorArgs<T>, int64_t, hipStream_t);            \
    template void launch_small_fronts<T>(FactorArgs<T>, const FrontDesc *, const int32_t *, const int *, int64_t, \
                                         const TreeArgs &, hipStream_t);                                  \
    template void launch_extend_add<T>(FactorArgs<T>, const FrontDesc *, const EaTask *, int, int64_t,    \
                                       const TreeArgs &, hipStream_t);                                    \
    template void launch_step<T>(FactorArgs<T>, const FrontDesc *, const StepDev &, int64_t, hipStream_t); \
    template void launch_window_inverses<T>(FactorArgs<T>, const FrontDesc *, const int32_t *, int, int, int64_t, \
                                            hipStream_t);
KKT_INST(double)
KKT_INST(float)
template void launch_zero<int64_t>(int64_t *, int64_t, hipStream_t);
template void launch_zero<int>(int *, int64_t, hipStream_t);

}  // namespace kkt
