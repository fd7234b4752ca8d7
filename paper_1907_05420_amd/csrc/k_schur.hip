// Assembly of the dense Schur complement from the per-period local blocks
// (Algorithm 1 steps 3-6; section 4.3, Eqs. LocalSchurBs, GlobalSchur).
//
// With S_n := -B_n A_n^-1 B_n^T and S = C + sum_n S_n, block (m, m') (Ns x Ns,
// m >= m', periods 0-based) of S is
//     m == m':  C_mm + S_11,m + sum_{n<m} S_00,n
//     m >  m':  S_10,m' + sum_{n<m'} S_00,n
// so every block below the diagonal of a block column is the same matrix.
// The local blocks S_bar_n = [[S_11, S_10^T], [S_10, S_00]] are the update
// matrix of the border node of period n (lower triangle, ld 2Ns).
#include "device.hpp"
#include "kernels.hpp"

namespace kkt {

template <typename T>
__device__ inline double sbar_at(const T *Sb, int64_t nb, int64_t i, int64_t j) {  // symmetric read
    return i >= j ? (double)Sb[i + j * nb] : (double)Sb[j + i * nb];
}

template <typename T>
__global__ void k_schur_prefix(const T *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns, double *prefix) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Ns * Ns) return;
    const int64_t i = idx % Ns, j = idx / Ns, nb = 2 * Ns;
    double acc = 0.0;
    for (int64_t m = 0; m < N; ++m) {
        prefix[m * Ns * Ns + idx] = acc;
        acc += sbar_at(U + m * Ustride + uoff, nb, Ns + i, Ns + j);
    }
    prefix[N * Ns * Ns + idx] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_schur_assemble(const T *U, int64_t Ustride, int64_t uoff, int64_t N,
                                                        int64_t Ns, const double *prefix, const double *corner,
                                                        double *S, double *tau_s, double eps, double *amax_s,
                                                        int mirror) {
    const int64_t ng = N * Ns, nb = 2 * Ns;
    const int64_t R = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t Q = blockIdx.y;
    if (R >= ng || (R < Q && !mirror)) return;
    const int64_t r = R >= Q ? R : Q, q = R >= Q ? Q : R;
    const int64_t m = r / Ns, i = r % Ns, mp = q / Ns, j = q % Ns;
    double v;
    if (m == mp) {
        v = sbar_at(U + m * Ustride + uoff, nb, i, j) + prefix[m * Ns * Ns + i + j * Ns];
        if (i == j && corner) v += corner[r];
    } else {
        v = sbar_at(U + mp * Ustride + uoff, nb, Ns + i, j) + prefix[mp * Ns * Ns + i + j * Ns];
    }
    S[R + Q * ng] = v;
    if (R == Q) {
        // the diagonal sets the thresholds; for a definite S max|s_ij| = max|s_ii|
        if (tau_s) tau_s[R] = eps * fabs(v);
        if (amax_s) atomic_max_nonneg(amax_s, fabs(v));
    }
}

template <typename T>
__global__ void k_copy_sbar(const T *U, int64_t Ustride, int64_t uoff, int64_t nb, double *out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = blockIdx.y;
    if (idx >= nb * nb) return;
    const int64_t i = idx % nb, j = idx / nb;
    out[n * nb * nb + idx] = sbar_at(U + n * Ustride + uoff, nb, i, j);
}

// Copy the strict lower triangle of the factor of S into the strict upper
// triangle (U[q][i] = L[i][q]), one 64x64 tile per workgroup through LDS.
__global__ __launch_bounds__(256) void k_mirror_lower(double *S, int64_t ng, int nt) {
    __shared__ double T[64 * 65];
    // blockIdx.x enumerates the lower tiles (I >= J) row by row
    const int64_t t = blockIdx.x;
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int64_t J = t - I * (I + 1) / 2;
    if (I >= nt) return;
    const int64_t r0 = I * 64, c0 = J * 64;
    const int nr = (int)min((int64_t)64, ng - r0), nc = (int)min((int64_t)64, ng - c0);
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 64 * 64; idx += 256) {
        const int a = idx & 63, q = idx >> 6;
        if (a < nr && q < nc) T[a + q * 65] = S[(r0 + a) + (c0 + q) * ng];
    }
    __syncthreads();
    // U[c0 + q][r0 + a] = L[r0 + a][c0 + q]: write down the columns of U
    for (int idx = tid; idx < 64 * 64; idx += 256) {
        const int q = idx & 63, a = idx >> 6;
        if (a < nr && q < nc && (I > J || q < a)) S[(c0 + q) + (r0 + a) * ng] = T[a + q * 65];
    }
}

void launch_mirror_lower(double *S, int64_t ng, hipStream_t st) {
    const int nt = (int)((ng + 63) / 64);
    const int64_t ntiles = (int64_t)nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_mirror_lower, dim3((unsigned)ntiles), dim3(256), 0, st, S, ng, nt);
}

void launch_schur_prefix(const void *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns, int precision,
                         double *prefix, hipStream_t st) {
    unsigned g = (unsigned)((Ns * Ns + 255) / 256);
    if (precision == 1)
        hipLaunchKernelGGL(k_schur_prefix<float>, dim3(g), dim3(256), 0, st, (const float *)U, Ustride, uoff, N, Ns,
                           prefix);
    else
        hipLaunchKernelGGL(k_schur_prefix<double>, dim3(g), dim3(256), 0, st, (const double *)U, Ustride, uoff, N,
                           Ns, prefix);
}

void launch_schur_assemble(const void *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns, int precision,
                           const double *prefix, const double *corner, double *S, double *tau_s, double eps,
                           double *amax_s, int mirror, hipStream_t st) {
    const int64_t ng = N * Ns;
    dim3 g((unsigned)((ng + 255) / 256), (unsigned)ng);
    if (precision == 1)
        hipLaunchKernelGGL(k_schur_assemble<float>, g, dim3(256), 0, st, (const float *)U, Ustride, uoff, N, Ns,
                           prefix, corner, S, tau_s, eps, amax_s, mirror);
    else
        hipLaunchKernelGGL(k_schur_assemble<double>, g, dim3(256), 0, st, (const double *)U, Ustride, uoff, N, Ns,
                           prefix, corner, S, tau_s, eps, amax_s, mirror);
}

void launch_copy_sbar(const void *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t nb, int precision,
                      double *out, hipStream_t st) {
    dim3 g((unsigned)((nb * nb + 255) / 256), (unsigned)N);
    if (precision == 1)
        hipLaunchKernelGGL(k_copy_sbar<float>, g, dim3(256), 0, st, (const float *)U, Ustride, uoff, nb, out);
    else
        hipLaunchKernelGGL(k_copy_sbar<double>, g, dim3(256), 0, st, (const double *)U, Ustride, uoff, nb, out);
}

}  // namespace kkt
