// Reductions and vector combinations for the flexible GMRES refinement
// (FP64, deterministic reduction order).
#include "device.hpp"
#include "footprint.hpp"
#include "kernels.hpp"

namespace kkt {

constexpr int KP = KRYLOV_PART;

// part[(k * nv + i) * KP + p] = sum over chunk p of W_k . V_i,k
__global__ __launch_bounds__(256) void k_dots_partial(const double *W, const double *V, int nv, int64_t nrhs,
                                                      int64_t n, double *part) {
    __shared__ double red[256];
    const int p = blockIdx.x, k = blockIdx.y, i = blockIdx.z;
    const int64_t chunk = (n + KP - 1) / KP;
    const int64_t lo = p * chunk, hi = min(n, lo + chunk);
    const double *w = W + (int64_t)k * n, *v = V + ((int64_t)i * nrhs + k) * n;
    double a = 0.0;
    for (int64_t j = lo + threadIdx.x; j < hi; j += 256) a += w[j] * v[j];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[((int64_t)k * nv + i) * KP + p] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_partial(const double *part, int nv, double *h, int ldh) {
    __shared__ double red[256];
    const int k = blockIdx.x, i = blockIdx.y;
    double a = 0.0;
    for (int p = threadIdx.x; p < KP; p += 256) a += part[((int64_t)k * nv + i) * KP + p];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[(int64_t)k * ldh + i] = red[0];
}

__global__ void k_combine(double *W, const double *V, int nv, int64_t nrhs, int64_t n, const double *h, int ldh,
                          double sign) {
    const int k = blockIdx.y;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int i = 0; i < nv; ++i) a += h[(int64_t)k * ldh + i] * V[((int64_t)i * nrhs + k) * n + j];
        W[(int64_t)k * n + j] += sign * a;
    }
}

__global__ void k_scale_by(double *W, int64_t n, const double *nrm) {
    const int k = blockIdx.y;
    const double s = nrm[k] > 0.0 ? 1.0 / nrm[k] : 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        W[(int64_t)k * n + j] *= s;
}

__global__ void k_sqrt_inplace(double *h, int nrhs) {
    const int k = threadIdx.x;
    if (k < nrhs) h[k] = sqrt(h[k]);
}

void launch_dots(const double *W, const double *V, int nv, int64_t nrhs, int64_t n, double *part, double *h, int ldh,
                 hipStream_t st) {
    if (nv <= 0) return;
    hipLaunchKernelGGL(k_dots_partial, dim3(KP, (unsigned)nrhs, (unsigned)nv), dim3(256), 0, st, W, V, nv, nrhs, n,
                       part);
    hipLaunchKernelGGL(k_sum_partial, dim3((unsigned)nrhs, (unsigned)nv), dim3(256), 0, st, part, nv, h, ldh);
}

void launch_combine(double *W, const double *V, int nv, int64_t nrhs, int64_t n, const double *h, int ldh, double sign,
                    hipStream_t st) {
    if (nv <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_combine, dim3(g, (unsigned)nrhs), dim3(256), 0, st, W, V, nv, nrhs, n, h, ldh, sign);
}

void launch_norm(double *W, int64_t nrhs, int64_t n, double *part, double *nrm, int normalize, hipStream_t st) {
    // <W, W> through the dot kernels with V = W, nv = 1
    hipLaunchKernelGGL(k_dots_partial, dim3(KP, (unsigned)nrhs, 1), dim3(256), 0, st, W, W, 1, nrhs, n, part);
    hipLaunchKernelGGL(k_sum_partial, dim3((unsigned)nrhs, 1), dim3(256), 0, st, part, 1, nrm, 1);
    hipLaunchKernelGGL(k_sqrt_inplace, dim3(1), dim3(64), 0, st, nrm, (int)nrhs);
    if (normalize) {
        const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
        hipLaunchKernelGGL(k_scale_by, dim3(g, (unsigned)nrhs), dim3(256), 0, st, W, n, nrm);
    }
}

}  // namespace kkt
