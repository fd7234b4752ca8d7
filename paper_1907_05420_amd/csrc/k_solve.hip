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

template <typename T>
__global__ __launch_bounds__(256) void k_fwd(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *tasks,
                                             TreeArgs tr, SolveArgs sa) {
    extern __shared__ double v[];
    const int s = tasks[blockIdx.x];
    const int n = blockIdx.y, tid = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    const T *P = L + (int64_t)n * Lstride + d.Loff;
    const int32_t *R = tr.rows + tr.rowptr[s];
    for (int k = 0; k < sa.nrhs; ++k) {
        double *x = sa.xp + ((int64_t)n * sa.nrhs + k) * sa.nv;
        double *U = sa.uv + ((int64_t)n * sa.nrhs + k) * sa.usz;
        for (int i = tid; i < m; i += 256) v[i] = i < c ? x[R[i]] : 0.0;
        __syncthreads();
        for (int q = tr.cptr[s]; q < tr.cptr[s + 1]; ++q) {
            const int ch = tr.clist[q];
            const int uc = sd[ch].m - sd[ch].c;
            const int32_t *rl = tr.rel + tr.relptr[ch];
            const double *uch = U + tr.relptr[ch];
            for (int i = tid; i < uc; i += 256) v[rl[i]] += uch[i];
            __syncthreads();
        }
        for (int k0 = 0; k0 < c; k0 += 64) {
            const int nb = min(64, c - k0);
            for (int j = 0; j < nb; ++j) {
                const double yj = v[k0 + j];
                const int i = k0 + j + 1 + tid;
                if (i < k0 + nb) v[i] -= (double)P[i + (int64_t)(k0 + j) * m] * yj;
                __syncthreads();
            }
            for (int i = k0 + nb + tid; i < m; i += 256) {
                double acc = 0.0;
                for (int j = 0; j < nb; ++j) acc += (double)P[i + (int64_t)(k0 + j) * m] * v[k0 + j];
                v[i] -= acc;
            }
            __syncthreads();
        }
        for (int i = tid; i < m; i += 256) {
            if (i < c) x[R[i]] = v[i];
            else U[tr.relptr[s] + (i - c)] = v[i];
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bwd(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *tasks,
                                             TreeArgs tr, SolveArgs sa) {
    extern __shared__ double v[];
    const int s = tasks[blockIdx.x];
    const int n = blockIdx.y, tid = threadIdx.x;
    const FrontDesc d = sd[s];
    const int m = d.m, c = d.c;
    if (c == 0) return;
    const T *P = L + (int64_t)n * Lstride + d.Loff;
    const int32_t *R = tr.rows + tr.rowptr[s];
    for (int k = 0; k < sa.nrhs; ++k) {
        double *x = sa.xp + ((int64_t)n * sa.nrhs + k) * sa.nv;
        for (int i = tid; i < m; i += 256) v[i] = i < c ? x[R[i]] / (double)P[i + (int64_t)i * m] : x[R[i]];
        __syncthreads();
        for (int q = tid; q < c; q += 256) {
            double acc = 0.0;
            const T *col = P + (int64_t)q * m;
            for (int i = c; i < m; ++i) acc += (double)col[i] * v[i];
            v[q] -= acc;
        }
        __syncthreads();
        for (int kb = ((c - 1) / 64) * 64; kb >= 0; kb -= 64) {
            const int nb = min(64, c - kb);
            for (int j = nb - 1; j >= 0; --j) {
                const double xj = v[kb + j];
                const int q = kb + tid;
                if (q < kb + j) v[q] -= (double)P[(kb + j) + (int64_t)q * m] * xj;
                __syncthreads();
            }
            for (int q = tid; q < kb; q += 256) {
                double acc = 0.0;
                const T *col = P + (int64_t)q * m;
                for (int j = 0; j < nb; ++j) acc += (double)col[kb + j] * v[kb + j];
                v[q] -= acc;
            }
            __syncthreads();
        }
        for (int i = tid; i < c; i += 256) x[R[i]] = v[i];
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

// ---- dense Schur factor solves (unit lower L, D on the diagonal) ------------
constexpr int DNB = 64;

// forward step for rows [j0, j0+nb): every workgroup solves the block
// redundantly, workgroup 0 stores it; each workgroup then updates 256 rows below.
__global__ __launch_bounds__(256) void k_dense_fwd(const double *S, int64_t ng, double *v, double *y, int nrhs,
                                                   int64_t j0) {
    __shared__ double Lb[DNB * 65];
    __shared__ double yb[DNB * 4];
    const int tid = threadIdx.x;
    const int nb = (int)min((int64_t)DNB, ng - j0);
    for (int idx = tid; idx < nb * nb; idx += 256) {
        int i = idx % nb, q = idx / nb;
        Lb[i + q * 65] = S[(j0 + i) + (j0 + q) * ng];
    }
    for (int idx = tid; idx < nb * nrhs; idx += 256) {
        int i = idx % nb, k = idx / nb;
        yb[i + k * DNB] = v[(int64_t)k * ng + j0 + i];
    }
    __syncthreads();
    if (tid < nrhs) {
        double *yy = yb + tid * DNB;
        for (int j = 0; j < nb; ++j)
            for (int i = j + 1; i < nb; ++i) yy[i] -= Lb[i + j * 65] * yy[j];
    }
    __syncthreads();
    if (blockIdx.x == 0)
        for (int idx = tid; idx < nb * nrhs; idx += 256) {
            int i = idx % nb, k = idx / nb;
            y[(int64_t)k * ng + j0 + i] = yb[i + k * DNB];
        }
    const int64_t i = j0 + nb + (int64_t)blockIdx.x * 256 + tid;
    if (i >= ng) return;
    for (int k = 0; k < nrhs; ++k) {
        double acc = 0.0;
        for (int j = 0; j < nb; ++j) acc += S[i + (j0 + j) * ng] * yb[j + k * DNB];
        v[(int64_t)k * ng + i] -= acc;
    }
}

__global__ void k_div_diag(const double *S, int64_t ng, const double *y, double *z, int nrhs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng) return;
    const double dd = S[i + i * ng];
    for (int k = 0; k < nrhs; ++k) z[(int64_t)k * ng + i] = y[(int64_t)k * ng + i] / dd;
}

// backward step for rows [j0, j0+nb): solve L_jj^T x_j = z_j redundantly,
// then each workgroup updates z of 256 columns q < j0.
__global__ __launch_bounds__(256) void k_dense_bwd(const double *S, int64_t ng, double *z, double *x, int nrhs,
                                                   int64_t j0) {
    __shared__ double Lb[DNB * 65];
    __shared__ double xb[DNB * 4];
    const int tid = threadIdx.x;
    const int nb = (int)min((int64_t)DNB, ng - j0);
    for (int idx = tid; idx < nb * nb; idx += 256) {
        int i = idx % nb, q = idx / nb;
        Lb[i + q * 65] = S[(j0 + i) + (j0 + q) * ng];
    }
    for (int idx = tid; idx < nb * nrhs; idx += 256) {
        int i = idx % nb, k = idx / nb;
        xb[i + k * DNB] = z[(int64_t)k * ng + j0 + i];
    }
    __syncthreads();
    if (tid < nrhs) {
        double *xx = xb + tid * DNB;
        for (int j = nb - 1; j >= 0; --j)
            for (int q = 0; q < j; ++q) xx[q] -= Lb[j + q * 65] * xx[j];
    }
    __syncthreads();
    if (blockIdx.x == 0)
        for (int idx = tid; idx < nb * nrhs; idx += 256) {
            int i = idx % nb, k = idx / nb;
            x[(int64_t)k * ng + j0 + i] = xb[i + k * DNB];
        }
    const int64_t q = (int64_t)blockIdx.x * 256 + tid;
    if (q >= j0) return;
    for (int k = 0; k < nrhs; ++k) {
        double acc = 0.0;
        for (int j = 0; j < nb; ++j) acc += S[(j0 + j) + q * ng] * xb[j + k * DNB];
        z[(int64_t)k * ng + q] -= acc;
    }
}

// ---- launchers ---------------------------------------------------------------
template <typename T>
void launch_gather_rhs(const double *b, int64_t ntot, int64_t nA, const int32_t *perm, SolveArgs sa,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_gather_rhs<T>, dim3((unsigned)((sa.nv + 255) / 256), (unsigned)sa.N, (unsigned)sa.nrhs),
                       dim3(256), 0, st, b, ntot, nA, perm, sa);
}

template <typename T>
void launch_fwd_level(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *tasks, int ntasks, int maxm,
                      const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_fwd<T>, dim3(ntasks, (unsigned)sa.N), dim3(256), sizeof(double) * maxm, st, L, Lstride,
                       sd, tasks, tr, sa);
}

template <typename T>
void launch_bwd_level(const T *L, int64_t Lstride, const FrontDesc *sd, const int32_t *tasks, int ntasks, int maxm,
                      const TreeArgs &tr, SolveArgs sa, hipStream_t st) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(k_bwd<T>, dim3(ntasks, (unsigned)sa.N), dim3(256), sizeof(double) * maxm, st, L, Lstride,
                       sd, tasks, tr, sa);
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
    for (int64_t j0 = 0; j0 < ng; j0 += DNB) {
        int64_t below = ng - j0 - DNB;
        unsigned g = below > 0 ? (unsigned)((below + 255) / 256) : 1u;
        hipLaunchKernelGGL(k_dense_fwd, dim3(g), dim3(256), 0, st, S, ng, v, y, (int)nrhs, j0);
    }
}

void launch_dense_bwd(const double *S, int64_t ng, double *z, double *x, int64_t nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_div_diag, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, S, ng, z, z, (int)nrhs);
    for (int64_t j0 = ((ng - 1) / DNB) * DNB; j0 >= 0; j0 -= DNB) {
        unsigned g = j0 > 0 ? (unsigned)((j0 + 255) / 256) : 1u;
        hipLaunchKernelGGL(k_dense_bwd, dim3(g), dim3(256), 0, st, S, ng, z, x, (int)nrhs, j0);
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
