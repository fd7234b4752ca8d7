// FP64 residual r = b - K x on the arrowhead blocks (refinement, section 2.1)
// with the MPOPF border of Eq. B12N, and the norms that steer refinement.
#include "device.hpp"
#include "kernels.hpp"

namespace kkt {

// border rows: r_g[m] = b_C[m] - C x_g[m] - C_1 x_m - sum_{n<m} C_0 x_n ; also
// the suffix sums sg[n] = sum_{m>n} x_g[m] used by the period rows.
__global__ void k_res_border(ResidualArgs ra, const double *b, const double *x, double *r, double *sg,
                             double *norms) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (s >= ra.Ns) return;
    const int64_t ng = ra.N * ra.Ns;
    const double *xk = x + (int64_t)k * ra.ntot;
    const double *xg = xk + ra.N * ra.nA;
    double acc0 = 0.0, abs0 = 0.0, wmax = 0.0;
    for (int64_t m = 0; m < ra.N; ++m) {
        const int64_t g = m * ra.Ns + s;
        const double *xm = xk + m * ra.nA;
        double bc = b ? b[(int64_t)k * ra.ntot + ra.N * ra.nA + g] : 0.0;
        double acc = bc, ab = fabs(bc);
        if (ra.corner) { double t = ra.corner[g] * xg[g]; acc -= t; ab += fabs(t); }
        for (int64_t e = ra.c1p[s]; e < ra.c1p[s + 1]; ++e) {
            double t = ra.C1v[e] * xm[ra.c1i[e]];
            acc -= t;
            ab += fabs(t);
        }
        acc -= acc0;
        ab += abs0;
        r[(int64_t)k * ra.ntot + ra.N * ra.nA + g] = b ? acc : -acc;
        if (ab > 0.0) wmax = fmax(wmax, fabs(acc) / ab);
        else if (acc != 0.0) wmax = INFINITY;
        for (int64_t e = ra.c0p[s]; e < ra.c0p[s + 1]; ++e) {
            double t = ra.C0v[e] * xm[ra.c0i[e]];
            acc0 += t;
            abs0 += fabs(t);
        }
    }
    double acc = 0.0;
    for (int64_t n = ra.N - 1; n >= 0; --n) {
        sg[(int64_t)k * ng + n * ra.Ns + s] = acc;
        acc += xg[n * ra.Ns + s];
    }
    if (norms) atomic_max_nonneg(norms + 4 * k + 2, wmax);
}

__global__ __launch_bounds__(256) void k_res_periods(ResidualArgs ra, const double *b, const double *x, double *r,
                                                     const double *sg, double *wpart) {
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int n = blockIdx.y;
    const int64_t ng = ra.N * ra.Ns;
    const int64_t e0 = i < ra.nA ? ra.rp[i] : 0, e1 = i < ra.nA ? ra.rp[i + 1] : 0;
    const double *An = ra.A + (int64_t)n * ra.nnz;
    for (int k = 0; k < ra.nrhs; ++k) {
        double w = 0.0;
        if (i < ra.nA) {
            const double *xk = x + (int64_t)k * ra.ntot;
            const double *xn = xk + (int64_t)n * ra.nA;
            const double *xg = xk + ra.N * ra.nA;
            const int64_t row = (int64_t)k * ra.ntot + (int64_t)n * ra.nA + i;
            double acc = b ? b[row] : 0.0, ab = fabs(acc);
#pragma unroll 4
            for (int64_t e = e0; e < e1; ++e) {
                const int32_t j = ra.ci[e];
                double a = An[ra.vi[e]];
                if (j == i) a += i < ra.n_primal ? ra.dw : -ra.dc;
                const double t = a * xn[j];
                acc -= t;
                ab += fabs(t);
            }
            for (int64_t e = ra.c1tp[i]; e < ra.c1tp[i + 1]; ++e) {
                const double t = ra.C1v[ra.c1tk[e]] * xg[(int64_t)n * ra.Ns + ra.c1ts[e]];
                acc -= t;
                ab += fabs(t);
            }
            for (int64_t e = ra.c0tp[i]; e < ra.c0tp[i + 1]; ++e) {
                const double t = ra.C0v[ra.c0tk[e]] * sg[(int64_t)k * ng + (int64_t)n * ra.Ns + ra.c0ts[e]];
                acc -= t;
                ab += fabs(t);
            }
            r[row] = b ? acc : -acc;
            if (ab > 0.0) w = fabs(acc) / ab;
            else if (acc != 0.0) w = INFINITY;
        }
        red[threadIdx.x] = w;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0 && wpart)
            wpart[(int64_t)k * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
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

__global__ __launch_bounds__(256) void k_norm_final(const double *part, const double *wpart, int64_t nw,
                                                    double *norms) {
    __shared__ double s1[256], s2[256], s3[256];
    const int k = blockIdx.x;
    double a = 0.0, c = 0.0, w = 0.0;
    for (int p = threadIdx.x; p < NPART; p += 256) {
        a += part[((int64_t)k * NPART + p) * 2 + 0];
        c += part[((int64_t)k * NPART + p) * 2 + 1];
    }
    for (int64_t p = threadIdx.x; p < nw; p += 256) w = fmax(w, wpart[(int64_t)k * nw + p]);
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = c;
    s3[threadIdx.x] = w;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            s1[threadIdx.x] += s1[threadIdx.x + s];
            s2[threadIdx.x] += s2[threadIdx.x + s];
            s3[threadIdx.x] = fmax(s3[threadIdx.x], s3[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        norms[4 * k + 0] = sqrt(s1[0]);
        norms[4 * k + 1] = sqrt(s2[0]);
        norms[4 * k + 2] = fmax(norms[4 * k + 2], s3[0]);
    }
}

__global__ void k_zero_norms(double *norms, int nrhs) {
    int i = threadIdx.x;
    if (i < 4 * nrhs) norms[i] = 0.0;
}

int64_t residual_work(int64_t N, int64_t nA, int64_t Ns, int64_t nrhs) {
    return N * Ns * nrhs + 2 * NPART * nrhs + ((nA + 255) / 256) * N * nrhs + 8;
}

// work must hold residual_work() doubles
void launch_residual(const ResidualArgs &ra, const double *b, const double *x, double *r, double *work,
                     double *norms, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_norms, dim3(1), dim3(256), 0, st, norms, (int)ra.nrhs);
    double *sg = work;
    double *part = work + std::max<int64_t>(ra.N * ra.Ns * ra.nrhs, 1);
    double *wpart = part + 2 * NPART * ra.nrhs;
    const int64_t nw = ((ra.nA + 255) / 256) * ra.N;
    if (ra.Ns > 0)
        hipLaunchKernelGGL(k_res_border, dim3((unsigned)((ra.Ns + 127) / 128), (unsigned)ra.nrhs), dim3(128), 0, st,
                           ra, b, x, r, sg, norms);
    hipLaunchKernelGGL(k_res_periods, dim3((unsigned)((ra.nA + 255) / 256), (unsigned)ra.N), dim3(256), 0, st, ra, b,
                       x, r, sg, wpart);
    hipLaunchKernelGGL(k_norm_partial, dim3(NPART, (unsigned)ra.nrhs), dim3(256), 0, st, r, b, ra.ntot, part);
    hipLaunchKernelGGL(k_norm_final, dim3((unsigned)ra.nrhs), dim3(256), 0, st, part, wpart, nw, norms);
}

// y = K x (no norms)
void launch_matvec(const ResidualArgs &ra, const double *x, double *y, double *work, hipStream_t st) {
    double *sg = work;
    if (ra.Ns > 0)
        hipLaunchKernelGGL(k_res_border, dim3((unsigned)((ra.Ns + 127) / 128), (unsigned)ra.nrhs), dim3(128), 0, st,
                           ra, (const double *)nullptr, x, y, sg, (double *)nullptr);
    hipLaunchKernelGGL(k_res_periods, dim3((unsigned)((ra.nA + 255) / 256), (unsigned)ra.N), dim3(256), 0, st, ra,
                       (const double *)nullptr, x, y, sg, (double *)nullptr);
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
