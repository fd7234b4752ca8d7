// FP64 residual r = b - K x on the arrowhead blocks (refinement, section 2.1)
// with the MPOPF border of Eq. B12N, and the norms that steer refinement.
//
// A true residual (b given) is evaluated with compensated sums: every product
// a x is split exactly into p + e (p = fl(a x), e = fma(a, x, -p)), every
// addition into s + e (Knuth's TwoSum), and the error terms are summed
// separately, so r is as accurate as if the sums ran in twice the working
// precision and then were rounded once (Ogita, Rump and Oishi, "Accurate sum
// and dot product", SIAM J. Sci. Comput. 26, 2005: Sum2 / Dot2). A residual
// summed in plain FP64 carries an error of order eps || |K||x| + |b| ||, which
// on late-IPM barrier ranges is larger than the residual of the correctly
// rounded solution itself; the compensated one resolves it. K x alone (the
// Krylov products) is summed plainly.
#include "device.hpp"
#include "kernels.hpp"

namespace kkt {

// inclusive scan of buf[0..255] over the workgroup (Hillis-Steele)
__device__ inline void block_scan256(double *buf, int tid) {
    for (int off = 1; off < 256; off <<= 1) {
        double v = buf[tid];
        if (tid >= off) v += buf[tid - off];
        __syncthreads();
        buf[tid] = v;
        __syncthreads();
    }
}


// s + e = a + b exactly (Knuth's TwoSum; no branch on the magnitudes)
__device__ inline void two_sum(double a, double b, double &s, double &e) {
#pragma clang fp contract(off)
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) -= a x: the product split exactly by fma, the difference by
// TwoSum, both error terms accumulated in lo (one Dot2 step)
__device__ inline void dot2_sub(double &hi, double &lo, double a, double x) {
#pragma clang fp contract(off)
    const double p = a * x;
    const double pe = fma(a, x, -p);
    double s, e;
    two_sum(hi, -p, s, e);
    hi = s;
    lo += e - pe;
}

// (hi, lo) += (bh, bl), renormalised so that |lo| <= ulp(hi) / 2
__device__ inline void dd_add(double &hi, double &lo, double bh, double bl) {
#pragma clang fp contract(off)
    double s, e;
    two_sum(hi, bh, s, e);
    e += lo + bl;
    hi = s + e;
    lo = e - (hi - s);
}

// inclusive scan of the pairs (bh, bl)[0..255] over the workgroup
__device__ inline void block_scan256_dd(double *bh, double *bl, int tid) {
    for (int off = 1; off < 256; off <<= 1) {
        double h = bh[tid], l = bl[tid];
        if (tid >= off) dd_add(h, l, bh[tid - off], bl[tid - off]);
        __syncthreads();
        bh[tid] = h;
        bl[tid] = l;
        __syncthreads();
    }
}

// Border rows, one workgroup per (storage unit s, right-hand side k), one
// thread per period m (chunks of 256 periods with carries):
//   r_g[m] = b_C[m] - C x_g[m] - C_1 x_m - sum_{n<m} C_0 x_n   (Eq. B12N)
// and the suffix sums sg[n] = sum_{m>n} x_g[m] used by the period rows. The
// sums over periods are workgroup scans. With COMP (a true residual) every
// sum is compensated, the scans run on (hi, lo) pairs and the suffix sums are
// stored as pairs (sg, sg + N Ns nrhs). With norms: the largest componentwise
// error |r_i|/(|K||x| + |b|)_i goes to norms[4k + 2] and the workgroup's sum
// of (|K||x| + |b|)_i^2 to bpart[k Ns + s].
template <bool COMP>
__global__ __launch_bounds__(256) void k_res_border(ResidualArgs ra, const double *b, const double *x, double *r,
                                                    double *sg, double *norms, double *bpart) {
    __shared__ double sc[256], sl[256], sa[256];
    __shared__ double wred[4];
    double ab2 = 0.0;  // this thread's sum of (|K||x| + |b|)_row^2
    const int64_t s = blockIdx.x;
    const int k = blockIdx.y, tid = threadIdx.x;
    const int64_t ng = ra.N * ra.Ns;
    const double *xk = x + (int64_t)k * ra.ntot;
    const double *xg = xk + ra.N * ra.nA;
    const int64_t c1a = ra.c1p[s], c1b = ra.c1p[s + 1], c0a = ra.c0p[s], c0b = ra.c0p[s + 1];
    double carry = 0.0, carry_lo = 0.0, carry_abs = 0.0, wmax = 0.0;
    for (int64_t m0 = 0; m0 < ra.N; m0 += 256) {
        const int64_t m = m0 + tid;
        const bool on = m < ra.N;
        const int64_t mc = on ? m : ra.N - 1;
        const int64_t g = mc * ra.Ns + s;
        const double *xm = xk + mc * ra.nA;
        const double bc = b ? b[(int64_t)k * ra.ntot + ra.N * ra.nA + g] : 0.0;
        double acc = bc, lo = 0.0, ab = fabs(bc);
        if (ra.corner) {
            if constexpr (COMP) dot2_sub(acc, lo, ra.corner[g], xg[g]);
            else acc -= ra.corner[g] * xg[g];
            ab += fabs(ra.corner[g] * xg[g]);
        }
        for (int64_t e = c1a; e < c1b; ++e) {
            if constexpr (COMP) dot2_sub(acc, lo, ra.C1v[e], xm[ra.c1i[e]]);
            else acc -= ra.C1v[e] * xm[ra.c1i[e]];
            ab += fabs(ra.C1v[e] * xm[ra.c1i[e]]);
        }
        // this period's C_0 x_m, negated (so that the scans add)
        double c0 = 0.0, c0lo = 0.0, a0 = 0.0;
        for (int64_t e = c0a; e < c0b; ++e) {
            if constexpr (COMP) dot2_sub(c0, c0lo, ra.C0v[e], xm[ra.c0i[e]]);
            else c0 -= ra.C0v[e] * xm[ra.c0i[e]];
            a0 += fabs(ra.C0v[e] * xm[ra.c0i[e]]);
        }
        sc[tid] = on ? c0 : 0.0;
        sl[tid] = on ? c0lo : 0.0;
        sa[tid] = on ? a0 : 0.0;
        __syncthreads();
        if constexpr (COMP) block_scan256_dd(sc, sl, tid);
        else block_scan256(sc, tid);
        block_scan256(sa, tid);
        // exclusive sums over the earlier periods
        if constexpr (COMP) {
            dd_add(acc, lo, carry, carry_lo);
            if (tid > 0) dd_add(acc, lo, sc[tid - 1], sl[tid - 1]);
            acc += lo;
        } else {
            acc += carry + (tid > 0 ? sc[tid - 1] : 0.0);
        }
        ab += carry_abs + (tid > 0 ? sa[tid - 1] : 0.0);
        if (on) {
            r[(int64_t)k * ra.ntot + ra.N * ra.nA + g] = b ? acc : -acc;
            if (ab > 0.0) wmax = fmax(wmax, fabs(acc) / ab);
            else if (acc != 0.0) wmax = INFINITY;
            ab2 += ab * ab;
        }
        if constexpr (COMP) dd_add(carry, carry_lo, sc[255], sl[255]);
        else carry += sc[255];
        carry_abs += sa[255];
        __syncthreads();
    }
    // suffix sums of x_g over the periods, from the last chunk back
    double scarry = 0.0, scarry_lo = 0.0;
    const int64_t nch = (ra.N + 255) / 256;
    for (int64_t ch = nch - 1; ch >= 0; --ch) {
        const int64_t m = ch * 256 + (255 - tid);  // reversed: thread 0 holds the last period
        const bool on = m < ra.N;
        sc[tid] = on ? xg[m * ra.Ns + s] : 0.0;
        sl[tid] = 0.0;
        __syncthreads();
        if constexpr (COMP) block_scan256_dd(sc, sl, tid);
        else block_scan256(sc, tid);
        if (on) {
            const int64_t o = (int64_t)k * ng + m * ra.Ns + s;
            if constexpr (COMP) {
                double h = scarry, l = scarry_lo;
                if (tid > 0) dd_add(h, l, sc[tid - 1], sl[tid - 1]);
                sg[o] = h;
                sg[ng * ra.nrhs + o] = l;
            } else {
                sg[o] = scarry + (tid > 0 ? sc[tid - 1] : 0.0);
            }
        }
        if constexpr (COMP) dd_add(scarry, scarry_lo, sc[255], sl[255]);
        else scarry += sc[255];
        __syncthreads();
    }
    if (norms) {
        wmax = wave_max(wmax);
        if ((tid & 63) == 0) wred[tid >> 6] = wmax;
        __syncthreads();
        if (tid == 0) atomic_max_nonneg(norms + 4 * k + 2, fmax(fmax(wred[0], wred[1]), fmax(wred[2], wred[3])));
        // fixed-order tree sum of the rows' (|K||x| + |b|)^2 for the floor norm
        sc[tid] = ab2;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h) sc[tid] += sc[tid + h];
            __syncthreads();
        }
        if (tid == 0) bpart[(int64_t)k * ra.Ns + s] = sc[0];
    }
}

// Period rows, one wavefront per 64-row slice of K's sliced ELLPACK, lane l
// holding row i = 64 s + l (all right-hand sides of a pass together):
//   r_n = b_n - (A_n + shifts) x_n - C_1^T x_g[n] - C_0^T sg[n]
// The slice's column indices and values are read coalesced, RES_B entries
// per row at a time (padding entries carry a zero value and the row's own
// column). With COMP the sums are compensated and sg is a (hi, lo) pair.
constexpr int RES_B = 8;
template <int RBT, bool COMP>
__global__ __launch_bounds__(256) void k_res_periods(ResidualArgs ra, const double *b, const double *x, double *r,
                                                     const double *sg, double *wpart) {
    __shared__ double wred[4 * RBT], ared[4 * RBT];
    const int tid = threadIdx.x, lane = tid & 63;
    const int64_t nsl = (ra.nA + 63) / 64;
    int bx, n;
    period_task(bx, n);
    const int64_t sl = min((int64_t)bx * 4 + (tid >> 6), nsl - 1);
    const bool slice_on = (int64_t)bx * 4 + (tid >> 6) < nsl;
    const int64_t i = 64 * sl + lane;
    const bool on = slice_on && i < ra.nA;
    const int64_t ic = on ? i : ra.nA - 1;
    const int64_t ng = ra.N * ra.Ns;
    const int64_t p0 = ra.sl_off[sl];
    const int w = (int)((ra.sl_off[sl + 1] - p0) / 64);
    const int32_t *cis = ra.sl_ci + p0 + lane;
    const double *avs = ra.Asell + (int64_t)n * ra.nnz_sell + p0 + lane;
    for (int k0 = 0; k0 < ra.nrhs; k0 += RBT) {
        const int nr = (int)min((int64_t)RBT, ra.nrhs - k0);
        const double *xn[RBT];
        double acc[RBT], lo[RBT], ab[RBT];
#pragma unroll
        for (int q = 0; q < RBT; ++q) {
            const int kk = k0 + min(q, nr - 1);
            xn[q] = x + (int64_t)kk * ra.ntot + (int64_t)n * ra.nA;
            acc[q] = b ? b[(int64_t)kk * ra.ntot + (int64_t)n * ra.nA + ic] : 0.0;
            lo[q] = 0.0;
            ab[q] = fabs(acc[q]);
        }
        for (int u0 = 0; u0 < w; u0 += RES_B) {
            int32_t j[RES_B];
            double a[RES_B], xv[RES_B][RBT];
#pragma unroll
            for (int u = 0; u < RES_B; ++u) {
                const int uu = min(u0 + u, w - 1);
                j[u] = cis[64 * uu];
                a[u] = avs[64 * uu];
            }
#pragma unroll
            for (int u = 0; u < RES_B; ++u)
#pragma unroll
                for (int q = 0; q < RBT; ++q) xv[u][q] = xn[q][j[u]];
#pragma unroll
            for (int u = 0; u < RES_B; ++u) {
                const double au = u0 + u < w ? a[u] : 0.0;
#pragma unroll
                for (int q = 0; q < RBT; ++q) {
                    if constexpr (COMP) dot2_sub(acc[q], lo[q], au, xv[u][q]);
                    else acc[q] -= au * xv[u][q];
                    ab[q] += fabs(au * xv[u][q]);
                }
            }
        }
        const int64_t t1a = on ? ra.c1tp[ic] : 0, t1b = on ? ra.c1tp[ic + 1] : 0;
        for (int64_t e = t1a; e < t1b; ++e) {
            const double cv = ra.C1v[ra.c1tk[e]];
            const int64_t gi = (int64_t)n * ra.Ns + ra.c1ts[e];
#pragma unroll
            for (int q = 0; q < RBT; ++q) {
                const double xq = x[(int64_t)(k0 + min(q, nr - 1)) * ra.ntot + ra.N * ra.nA + gi];
                if constexpr (COMP) dot2_sub(acc[q], lo[q], cv, xq);
                else acc[q] -= cv * xq;
                ab[q] += fabs(cv * xq);
            }
        }
        const int64_t t0a = on ? ra.c0tp[ic] : 0, t0b = on ? ra.c0tp[ic + 1] : 0;
        for (int64_t e = t0a; e < t0b; ++e) {
            const double cv = ra.C0v[ra.c0tk[e]];
            const int64_t gi = (int64_t)n * ra.Ns + ra.c0ts[e];
#pragma unroll
            for (int q = 0; q < RBT; ++q) {
                const int64_t o = (int64_t)(k0 + min(q, nr - 1)) * ng + gi;
                const double sq = sg[o];
                if constexpr (COMP) {
                    dot2_sub(acc[q], lo[q], cv, sq);
                    lo[q] -= cv * sg[ng * ra.nrhs + o];
                } else {
                    acc[q] -= cv * sq;
                }
                ab[q] += fabs(cv * sq);
            }
        }
        double wq[RBT], aq[RBT];
#pragma unroll
        for (int q = 0; q < RBT; ++q) {
            if constexpr (COMP) acc[q] += lo[q];
            wq[q] = 0.0;
            aq[q] = 0.0;
            if (on && q < nr) {
                r[(int64_t)(k0 + q) * ra.ntot + (int64_t)n * ra.nA + i] = b ? acc[q] : -acc[q];
                if (ab[q] > 0.0) wq[q] = fabs(acc[q]) / ab[q];
                else if (acc[q] != 0.0) wq[q] = INFINITY;
                aq[q] = ab[q] * ab[q];
            }
        }
        if (wpart) {
            // per workgroup: the largest componentwise error and the sum of
            // (|K||x| + |b|)_i^2, both reduced in a fixed order
            const int64_t nw = (int64_t)gridDim.x * gridDim.y;
            double *apart = wpart + ra.nrhs * nw;
#pragma unroll
            for (int q = 0; q < RBT; ++q) {
                const double wm = wave_max(wq[q]), as = wave_sum(aq[q]);
                if (lane == 0) {
                    wred[q * 4 + (tid >> 6)] = wm;
                    ared[q * 4 + (tid >> 6)] = as;
                }
            }
            __syncthreads();
            if (tid < nr) {
                const int64_t o = (int64_t)(k0 + tid) * nw + (int64_t)n * gridDim.x + bx;
                wpart[o] = fmax(fmax(wred[tid * 4 + 0], wred[tid * 4 + 1]), fmax(wred[tid * 4 + 2], wred[tid * 4 + 3]));
                apart[o] = (ared[tid * 4 + 0] + ared[tid * 4 + 1]) + (ared[tid * 4 + 2] + ared[tid * 4 + 3]);
            }
            __syncthreads();
        }
    }
}

// values of every period in the sliced layout, shifts on the diagonal
__global__ __launch_bounds__(64) void k_sell_values(const double *A, int64_t nnzA, int64_t nA, int64_t n_primal,
                                                    const int64_t *sl_off, const int32_t *sl_ci,
                                                    const int32_t *sl_vi, int64_t nnz_sell, double dw, double dc,
                                                    double *Asell) {
    const int64_t sl = blockIdx.x;
    const int n = blockIdx.y, lane = threadIdx.x;
    const int64_t i = 64 * sl + lane;
    const int64_t p0 = sl_off[sl];
    const int w = (int)((sl_off[sl + 1] - p0) / 64);
    const double shift = i < n_primal ? dw : -dc;
    const double *An = A + (int64_t)n * nnzA;
    double *out = Asell + (int64_t)n * nnz_sell + p0 + lane;
    for (int u = 0; u < w; ++u) {
        const int32_t v = sl_vi[p0 + 64 * u + lane];
        const int32_t c = sl_ci[p0 + 64 * u + lane];
        out[64 * u] = v >= 0 ? An[v] + (c == i ? shift : 0.0) : 0.0;
    }
}

void launch_sell_values(const double *A, int64_t nnzA, int64_t N, int64_t nA, int64_t n_primal,
                        const int64_t *sl_off, const int32_t *sl_ci, const int32_t *sl_vi, int64_t nnz_sell,
                        double dw, double dc, double *Asell, hipStream_t st) {
    hipLaunchKernelGGL(k_sell_values, dim3((unsigned)((nA + 63) / 64), (unsigned)N), dim3(64), 0, st, A, nnzA, nA,
                       n_primal, sl_off, sl_ci, sl_vi, nnz_sell, dw, dc, Asell);
}

// deterministic two-stage sums of r^2 and b^2 per right-hand side
constexpr int NPART = 512;
__global__ __launch_bounds__(256) void k_norm_partial(const double *r, const double *b, int64_t ntot,
                                                      double *part) {
    __shared__ double s1[256], s2[256];
    const int p = blockIdx.x, k = blockIdx.y;
    const int64_t chunk = (ntot + NPART - 1) / NPART;
    const int64_t lo = p * chunk, hi = min(ntot, lo + chunk);
    double a = 0.0, c = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        double rv = r[(int64_t)k * ntot + i], bv = b[(int64_t)k * ntot + i];
        a += rv * rv;
        c += bv * bv;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) { s1[threadIdx.x] += s1[threadIdx.x + s]; s2[threadIdx.x] += s2[threadIdx.x + s]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[((int64_t)k * NPART + p) * 2 + 0] = s1[0];
        part[((int64_t)k * NPART + p) * 2 + 1] = s2[0];
    }
}

// norms[4k + 0..3] = ||r_k||_2, ||b_k||_2, max_i |r_i|/(|K||x| + |b|)_i and
// || |K||x_k| + |b_k| ||_2 (the scale of the rounding error of r itself)
__global__ __launch_bounds__(256) void k_norm_final(const double *part, const double *wpart, int64_t nw,
                                                    const double *bpart, int64_t nb, int64_t nrhs, double *norms) {
    __shared__ double s1[256], s2[256], s3[256], s4[256];
    const int k = blockIdx.x;
    const double *apart = wpart + nrhs * nw;
    double a = 0.0, c = 0.0, w = 0.0, f = 0.0;
    for (int p = threadIdx.x; p < NPART; p += 256) {
        a += part[((int64_t)k * NPART + p) * 2 + 0];
        c += part[((int64_t)k * NPART + p) * 2 + 1];
    }
    for (int64_t p = threadIdx.x; p < nw; p += 256) {
        w = fmax(w, wpart[(int64_t)k * nw + p]);
        f += apart[(int64_t)k * nw + p];
    }
    for (int64_t p = threadIdx.x; p < nb; p += 256) f += bpart[(int64_t)k * nb + p];
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = c;
    s3[threadIdx.x] = w;
    s4[threadIdx.x] = f;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            s1[threadIdx.x] += s1[threadIdx.x + s];
            s2[threadIdx.x] += s2[threadIdx.x + s];
            s3[threadIdx.x] = fmax(s3[threadIdx.x], s3[threadIdx.x + s]);
            s4[threadIdx.x] += s4[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        norms[4 * k + 0] = sqrt(s1[0]);
        norms[4 * k + 1] = sqrt(s2[0]);
        norms[4 * k + 2] = fmax(norms[4 * k + 2], s3[0]);
        norms[4 * k + 3] = sqrt(s4[0]);
    }
}

__global__ void k_zero_norms(double *norms, int nrhs) {
    int i = threadIdx.x;
    if (i < 4 * nrhs) norms[i] = 0.0;
}

int64_t residual_work(int64_t N, int64_t nA, int64_t Ns, int64_t nrhs) {
    // sg (hi and lo), norm partials, per-workgroup max and floor partials,
    // border partials
    return 2 * std::max<int64_t>(N * Ns * nrhs, 1) + 2 * NPART * nrhs + 2 * ((nA + 255) / 256) * N * nrhs + Ns * nrhs +
           8;
}

template <bool COMP>
static void launch_res_periods(const ResidualArgs &ra, const double *b, const double *x, double *r, const double *sg,
                               double *wpart, hipStream_t st) {
    const dim3 grid((unsigned)(((ra.nA + 63) / 64 + 3) / 4), (unsigned)ra.N);  // four 64-row slices per workgroup
    if (ra.nrhs >= 3) hipLaunchKernelGGL((k_res_periods<4, COMP>), grid, dim3(256), 0, st, ra, b, x, r, sg, wpart);
    else if (ra.nrhs == 2) hipLaunchKernelGGL((k_res_periods<2, COMP>), grid, dim3(256), 0, st, ra, b, x, r, sg, wpart);
    else hipLaunchKernelGGL((k_res_periods<1, COMP>), grid, dim3(256), 0, st, ra, b, x, r, sg, wpart);
}

// work must hold residual_work() doubles; r = b - K x compensated
void launch_residual(const ResidualArgs &ra, const double *b, const double *x, double *r, double *work,
                     double *norms, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_norms, dim3(1), dim3(256), 0, st, norms, (int)ra.nrhs);
    double *sg = work;
    double *part = work + 2 * std::max<int64_t>(ra.N * ra.Ns * ra.nrhs, 1);
    double *wpart = part + 2 * NPART * ra.nrhs;
    const int64_t nw = ((ra.nA + 255) / 256) * ra.N;
    double *bpart = wpart + 2 * nw * ra.nrhs;
    if (ra.Ns > 0)
        hipLaunchKernelGGL(k_res_border<true>, dim3((unsigned)ra.Ns, (unsigned)ra.nrhs), dim3(256), 0, st, ra, b, x,
                           r, sg, norms, bpart);
    launch_res_periods<true>(ra, b, x, r, sg, wpart, st);
    hipLaunchKernelGGL(k_norm_partial, dim3(NPART, (unsigned)ra.nrhs), dim3(256), 0, st, r, b, ra.ntot, part);
    hipLaunchKernelGGL(k_norm_final, dim3((unsigned)ra.nrhs), dim3(256), 0, st, part, wpart, nw, bpart, ra.Ns,
                       ra.nrhs, norms);
}

// y = K x (no norms, plain sums)
void launch_matvec(const ResidualArgs &ra, const double *x, double *y, double *work, hipStream_t st) {
    double *sg = work;
    if (ra.Ns > 0)
        hipLaunchKernelGGL(k_res_border<false>, dim3((unsigned)ra.Ns, (unsigned)ra.nrhs), dim3(256), 0, st, ra,
                           (const double *)nullptr, x, y, sg, (double *)nullptr, (double *)nullptr);
    launch_res_periods<false>(ra, nullptr, x, y, sg, nullptr, st);
}

__global__ void k_axpy(double *x, const double *dx, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += dx[i];
}

void launch_axpy(double *x, const double *dx, int64_t n, hipStream_t st) {
    int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)blocks), dim3(256), 0, st, x, dx, n);
}

}  // namespace kkt
