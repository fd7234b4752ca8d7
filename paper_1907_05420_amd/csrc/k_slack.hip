// Slack elimination around the arrowhead solve (section 2.1): a slack s_j
// of period n enters its flow row i = lam_row[j] of A_n through -1 and has
// the diagonal L_s = S^-1 Y, so eliminating it (Eq. SCOPFhessianReduced)
// subtracts 1/L_s from A_n's diagonal entry (i, i) and adds r_j / L_s to the
// right-hand side of row i; afterwards L_s s_j = r_j + x_i (Eq.
// SCOPFslackReduction). One thread per (slack, period); HBM-bound.
#include "device.hpp"
#include "kernels.hpp"

namespace kkt {

__global__ void k_slack_reduce(const double *Ls, const double *rs, int64_t ns, int64_t N, int64_t nrhs,
                               const int32_t *lam_row, const int64_t *dpos, int64_t nnzA, int64_t nA, int64_t ntot,
                               double *A_out, double *b_out, int *flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns * N) return;
    const int64_t n = t / ns, j = t % ns;
    const double l = Ls[t];
    if (!(l > 0.0) || !isfinite(l)) {
        atomicOr(flag, 1);
        return;
    }
    const double inv = 1.0 / l;
    A_out[n * nnzA + dpos[j]] -= inv;
    const int64_t row = n * nA + lam_row[j];
    for (int64_t k = 0; k < nrhs; ++k) b_out[k * ntot + row] += rs[k * N * ns + t] / l;
}

__global__ void k_slack_recover(const double *Ls, const double *rs, int64_t ns, int64_t N, int64_t nrhs,
                                const int32_t *lam_row, int64_t nA, int64_t ntot, const double *x, double *s_out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns * N) return;
    const int64_t n = t / ns, j = t % ns;
    const int64_t row = n * nA + lam_row[j];
    for (int64_t k = 0; k < nrhs; ++k) s_out[k * N * ns + t] = (rs[k * N * ns + t] + x[k * ntot + row]) / Ls[t];
}

void launch_slack_reduce(const double *Ls, const double *rs, int64_t ns, int64_t N, int64_t nrhs,
                         const int32_t *lam_row, const int64_t *dpos, int64_t nnzA, int64_t nA, int64_t ntot,
                         double *A_out, double *b_out, int *flag, hipStream_t st) {
    const int64_t n = ns * N;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_slack_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Ls, rs, ns, N, nrhs,
                       lam_row, dpos, nnzA, nA, ntot, A_out, b_out, flag);
}

void launch_slack_recover(const double *Ls, const double *rs, int64_t ns, int64_t N, int64_t nrhs,
                          const int32_t *lam_row, int64_t nA, int64_t ntot, const double *x, double *s_out,
                          hipStream_t st) {
    const int64_t n = ns * N;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_slack_recover, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Ls, rs, ns, N, nrhs,
                       lam_row, nA, ntot, x, s_out);
}

}  // namespace kkt
