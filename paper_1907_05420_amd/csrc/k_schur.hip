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
#include <algorithm>

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
                                                        int mirror, int64_t q0) {
    const int64_t ng = N * Ns, nb = 2 * Ns;
    const int64_t R = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t Q = q0 + blockIdx.y;
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

// The diagonal entries of S alone (the same sums as k_schur_assemble's), for
// the pivot thresholds: lets the factorisation's first panel start before
// the rest of S is assembled.
template <typename T>
__global__ __launch_bounds__(256) void k_schur_diag(const T *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns,
                                                    const double *prefix, const double *corner, double *tau_s,
                                                    double eps, double *amax_s) {
    const int64_t ng = N * Ns, nb = 2 * Ns;
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= ng) return;
    const int64_t m = r / Ns, i = r % Ns;
    double v = sbar_at(U + m * Ustride + uoff, nb, i, i) + prefix[m * Ns * Ns + i + i * Ns];
    if (corner) v += corner[r];
    tau_s[r] = eps * fabs(v);
    atomic_max_nonneg(amax_s, fabs(v));
}

template <typename T>
__global__ void k_copy_sbar(const T *U, int64_t Ustride, int64_t uoff, int64_t nb, double *out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = blockIdx.y;
    if (idx >= nb * nb) return;
    const int64_t i = idx % nb, j = idx / nb;
    out[n * nb * nb + idx] = sbar_at(U + n * Ustride + uoff, nb, i, j);
}

// ---- structured Schur (section 4.3, Eq. GlobalSchur) ------------------------
// Block column j (0-based) of S has the diagonal block S_d[j] = C_jj + S_11,j +
// P_j and, in every row block below it, S_o[j] = S_10,j + P_j (P_j = sum of
// S_00,n over n < j). Block elimination keeps that structure: with U_0 = 0,
//   A_j = S_d[j] - U_j,  B_j = S_o[j] - U_j,  U_j+1 = U_j + B_j A_j^-1 B_j^T.
// Each step is one front [A_j; B_j] (ld 2 Ns, Ns for the last block column)
// with Ns pivots whose update matrix is -B_j A_j^-1 B_j^T.

// pivot thresholds eps |S_ii| and max |S_ii| from the diagonal of S
template <typename T>
__global__ void k_struct_tau(const T *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns, const double *prefix,
                             const double *corner, double *tau_s, double eps, double *amax_s) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N * Ns) return;
    const int64_t m = r / Ns, i = r % Ns;
    double v = sbar_at(U + m * Ustride + uoff, 2 * Ns, i, i) + prefix[m * Ns * Ns + i + i * Ns];
    if (corner) v += corner[r];
    tau_s[r] = eps * fabs(v);
    atomic_max_nonneg(amax_s, fabs(v));
}

template <typename T>
__global__ void k_struct_front(const T *U, int64_t Ustride, int64_t uoff, int64_t Ns, int64_t j, int last,
                               const double *prefix, const double *corner, const double *Uprev,
                               const double *Ubprev, double *Uout, double *F, double *Ubz) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // row of the front
    const int64_t q = blockIdx.y;                                        // pivot column
    const int64_t mj = last ? Ns : 2 * Ns;
    const T *Sb = U + j * Ustride + uoff;
    const double *Pj = prefix + j * Ns * Ns;
    // U_j = U_{j-1} + B A^-1 B^T of the previous column; the update block of
    // that column's front holds -(B A^-1 B^T), lower triangle
    auto u_at = [&](int64_t i) {
        return Uprev[i + q * Ns] - (i >= q ? Ubprev[i + q * Ns] : Ubprev[q + i * Ns]);
    };
    if (r < mj) {
        double v = 0.0;
        if (r < Ns) {
            const double u = u_at(r);
            Uout[r + q * Ns] = u;
            if (r >= q) {
                v = sbar_at(Sb, 2 * Ns, r, q) + Pj[r + q * Ns] - u;
                if (r == q && corner) v += corner[j * Ns + r];
            }
        } else {
            const int64_t i = r - Ns;
            v = sbar_at(Sb, 2 * Ns, Ns + i, q) + Pj[i + q * Ns] - u_at(i);
        }
        F[r + q * mj] = v;
    }
    if (!last && r < Ns) Ubz[r + q * Ns] = 0.0;
}

// Solves with the structured factor. With Linv_j the inverse of front j's
// unit lower pivot block, D_j its pivots, W_j its block below and G_j =
// W_j Linv_j, the block factor of S is unit lower with L_j on the diagonal
// and W_j (the front's rows below its pivots) in every block of column j
// below it; the forward substitution carries s_j = sum_{k<j} W_k z_k:
//   s_j+1 = s_j + G_j (bh_j - s_j),  z_j = Linv_j (bh_j - s_j),  w_j = z_j / D_j
// and the backward one t_j = sum_{m>j} x_m:
//   a_j = Linv_j^T w_j,  x_j = a_j - G_j^T t_j,  t_j-1 = t_j + x_j.
// The recurrences on s and t are one N_s x N_s product per block column (one
// workgroup walks them); everything else is per block column and parallel.
constexpr int SC_T = 1024;  // threads of the recurrence kernels
constexpr int SC_R = 4;     // right-hand sides per pass
constexpr int SC_B = 40;    // loads in flight per thread in a chain product

// y[i] (+)= sum_q M[i + q ld] x[q] for i < Ns, all threads of the workgroup:
// thread (i, g) sums over its share of q, partial sums reduced through red
__device__ __forceinline__ void sc_matvec(const double *M, int64_t ld, int Ns, const double *x, double *red, double *acc_out,
                                 int nr, int tid) {
    const int G = max(1, min(16, SC_T / max(Ns, 1)));
    const int i = tid % Ns, g = tid / Ns;
    const bool on = tid < G * Ns;
    double acc[SC_R] = {0.0, 0.0, 0.0, 0.0};
    if (on) {
        const int q0 = (int)((int64_t)Ns * g / G), q1 = (int)((int64_t)Ns * (g + 1) / G);
        // batches of SC_B: at N_s = 200 (5 groups of 40 columns) all of a
        // step's loads are in flight together
        for (int qb = q0; qb < q1; qb += SC_B) {
            double mv[SC_B];
#pragma unroll
            for (int u = 0; u < SC_B; ++u) mv[u] = M[i + (int64_t)min(qb + u, q1 - 1) * ld];
#pragma unroll
            for (int u = 0; u < SC_B; ++u) {
                const int q = min(qb + u, q1 - 1);
                const double a = qb + u < q1 ? mv[u] : 0.0;
#pragma unroll
                for (int r = 0; r < SC_R; ++r) acc[r] += a * x[q * SC_R + r];
            }
        }
#pragma unroll
        for (int r = 0; r < SC_R; ++r) red[(g * Ns + i) * SC_R + r] = acc[r];
    }
    __syncthreads();
    for (int idx = tid; idx < Ns * nr; idx += SC_T) {
        const int ii = idx / nr, r = idx % nr;
        double t = 0.0;
        for (int gg = 0; gg < G; ++gg) t += red[(gg * Ns + ii) * SC_R + r];
        acc_out[ii * SC_R + r] = t;
    }
    __syncthreads();
}

// forward recurrence: s_all[j] = s_j for every block column (nrhs <= SC_R)
__global__ __launch_bounds__(SC_T) void k_struct_fwd_chain(const double *G, int64_t N, int Ns, const double *bh,
                                                           int64_t ng, double *s_all, int nrhs) {
    extern __shared__ double sm[];
    double *s = sm, *v = sm + (int64_t)Ns * SC_R, *p = v + (int64_t)Ns * SC_R, *red = p + (int64_t)Ns * SC_R;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < Ns * SC_R; idx += SC_T) s[idx] = 0.0;
    __syncthreads();
    for (int64_t j = 0; j < N; ++j) {
        for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
            const int i = idx / nrhs, r = idx % nrhs;
            s_all[((int64_t)r * N + j) * Ns + i] = s[i * SC_R + r];
            v[i * SC_R + r] = bh[(int64_t)r * ng + j * Ns + i] - s[i * SC_R + r];
        }
        __syncthreads();
        if (j + 1 == N) break;
        sc_matvec(G + j * Ns * Ns, Ns, Ns, v, red, p, nrhs, tid);
        for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
            const int i = idx / nrhs, r = idx % nrhs;
            s[i * SC_R + r] += p[i * SC_R + r];
        }
        __syncthreads();
    }
}

// backward recurrence: x_j = a_j - G_j^T t_j (a_all holds a_j), into xg
__global__ __launch_bounds__(SC_T) void k_struct_bwd_chain(const double *GT, int64_t N, int Ns, const double *a_all,
                                                           double *xg, int64_t ng, int nrhs) {
    extern __shared__ double sm[];
    double *t = sm, *p = sm + (int64_t)Ns * SC_R, *red = p + (int64_t)Ns * SC_R;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < Ns * SC_R; idx += SC_T) t[idx] = 0.0;
    __syncthreads();
    for (int64_t j = N - 1; j >= 0; --j) {
        if (j + 1 < N) sc_matvec(GT + j * Ns * Ns, Ns, Ns, t, red, p, nrhs, tid);
        for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
            const int i = idx / nrhs, r = idx % nrhs;
            const double x = a_all[((int64_t)r * N + j) * Ns + i] - (j + 1 < N ? p[i * SC_R + r] : 0.0);
            xg[(int64_t)r * ng + j * Ns + i] = x;
            t[i * SC_R + r] += x;
        }
        __syncthreads();
    }
}

// per block column j (workgroup j): z = Linv_j (bh_j - s_j), w = z / D_j,
// a_j = Linv_j^T w, written to a_all. Linv_j lives below the diagonal of front
// j's pivot block (ld mj), D_j on its diagonal.
__global__ __launch_bounds__(256) void k_struct_blocks(const double *F, int64_t N, int Ns, const double *bh,
                                                       int64_t ng, const double *s_all, double *a_all, int nrhs) {
    extern __shared__ double sm[];
    double *v = sm, *w = sm + (int64_t)Ns * SC_R;
    const int64_t j = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t mj = j + 1 < N ? 2 * (int64_t)Ns : Ns;
    const double *Fj = F + j * 2 * (int64_t)Ns * Ns;
    for (int idx = tid; idx < Ns * SC_R; idx += 256) {
        const int i = idx / SC_R, r = idx % SC_R;
        v[idx] = r < nrhs ? bh[(int64_t)r * ng + j * Ns + i] - s_all[((int64_t)r * N + j) * Ns + i] : 0.0;
    }
    __syncthreads();
    // w_i = (v_i + sum_{q<i} Linv[i][q] v_q) / D_i, thread per row
    for (int i = tid; i < Ns; i += 256) {
        double acc[SC_R];
#pragma unroll
        for (int r = 0; r < SC_R; ++r) acc[r] = v[i * SC_R + r];
        for (int q = 0; q < i; ++q) {
            const double l = Fj[i + q * mj];
#pragma unroll
            for (int r = 0; r < SC_R; ++r) acc[r] += l * v[q * SC_R + r];
        }
        const double dinv = 1.0 / Fj[i + (int64_t)i * mj];
#pragma unroll
        for (int r = 0; r < SC_R; ++r) w[i * SC_R + r] = acc[r] * dinv;
    }
    __syncthreads();
    // a_q = w_q + sum_{i>q} Linv[i][q] w_i: one wavefront per column q, lanes over i
    const int lane = tid & 63, wv = tid >> 6;
    for (int q = wv; q < Ns; q += 4) {
        double acc[SC_R] = {0.0, 0.0, 0.0, 0.0};
        for (int i = q + 1 + lane; i < Ns; i += 64) {
            const double l = Fj[i + (int64_t)q * mj];
#pragma unroll
            for (int r = 0; r < SC_R; ++r) acc[r] += l * w[i * SC_R + r];
        }
#pragma unroll
        for (int r = 0; r < SC_R; ++r)
            for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off);
        if (lane == 0)
            for (int r = 0; r < nrhs; ++r) a_all[((int64_t)r * N + j) * Ns + q] = w[q * SC_R + r] + acc[r];
    }
}

void launch_struct_tau(const void *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns, int precision,
                       const double *prefix, const double *corner, double *tau_s, double eps, double *amax_s,
                       hipStream_t st) {
    const int64_t ng = N * Ns;
    const unsigned g = (unsigned)((ng + 255) / 256);
    if (precision == 1)
        hipLaunchKernelGGL(k_struct_tau<float>, dim3(g), dim3(256), 0, st, (const float *)U, Ustride, uoff, N, Ns,
                           prefix, corner, tau_s, eps, amax_s);
    else
        hipLaunchKernelGGL(k_struct_tau<double>, dim3(g), dim3(256), 0, st, (const double *)U, Ustride, uoff, N, Ns,
                           prefix, corner, tau_s, eps, amax_s);
}

void launch_struct_front(const void *U, int64_t Ustride, int64_t uoff, int64_t Ns, int64_t j, int last, int precision,
                         const double *prefix, const double *corner, const double *Uprev, const double *Ubprev,
                         double *Uout, double *F, double *Ubz, hipStream_t st) {
    const int64_t mj = last ? Ns : 2 * Ns;
    const dim3 g((unsigned)((mj + 255) / 256), (unsigned)Ns);
    if (precision == 1)
        hipLaunchKernelGGL(k_struct_front<float>, g, dim3(256), 0, st, (const float *)U, Ustride, uoff, Ns, j, last,
                           prefix, corner, Uprev, Ubprev, Uout, F, Ubz);
    else
        hipLaunchKernelGGL(k_struct_front<double>, g, dim3(256), 0, st, (const double *)U, Ustride, uoff, Ns, j,
                           last, prefix, corner, Uprev, Ubprev, Uout, F, Ubz);
}

// ---- the recurrences two block columns per step (N even) --------------------
// Both recurrences are affine, s_{j+1} = (I - G_j) s_j + G_j bh_j and
// t_{j-1} = (I - G_j^T) t_j + a_j, so two steps fold into one with
// M_p = (I - G_{2p+1})(I - G_{2p}) (formed at factorisation):
//   s_{2p+2} = M_p s_{2p} + c_p,       c_p = y + G_{2p+1}(bh_{2p+1} - y), y = G_{2p} bh_{2p}
//   t_{2p-1} = M_p^T t_{2p+1} + e_p,   e_p = a_{2p+1} - G_{2p}^T a_{2p+1} + a_{2p}
// The off-chain terms c_p, e_p and the values at the columns in between,
//   s_{2p+1} = s_{2p} + G_{2p}(bh_{2p} - s_{2p}),
//   x_{2p+1} = a_{2p+1} - G_{2p+1}^T t_{2p+1},  t_{2p} = t_{2p+1} + x_{2p+1},
//   x_{2p} = a_{2p} - G_{2p}^T t_{2p},
// are per pair and parallel; only N/2 dependent products remain per chain.

// The per-pair kernels run SC_T threads and take their products with
// sc_matvec (red: its reduction buffer after x, y, z in LDS).
// workgroup p: c_p (into c_all [SC_R][N/2][Ns])
__global__ __launch_bounds__(SC_T) void k_pair_fwd_c(const double *G, int64_t N, int Ns, const double *bh, int64_t ng,
                                                    double *c_all, int nrhs) {
    extern __shared__ double sm[];
    double *x = sm, *y = sm + (int64_t)Ns * SC_R, *z = y + (int64_t)Ns * SC_R, *red = z + (int64_t)Ns * SC_R;
    const int64_t p = blockIdx.x, P = N / 2, nn = (int64_t)Ns * Ns;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < Ns * SC_R; idx += SC_T) {
        const int i = idx / SC_R, r = idx % SC_R;
        x[idx] = r < nrhs ? bh[(int64_t)r * ng + 2 * p * Ns + i] : 0.0;
    }
    __syncthreads();
    sc_matvec(G + 2 * p * nn, Ns, Ns, x, red, y, nrhs, tid);
    __syncthreads();
    const bool has1 = 2 * p + 1 <= N - 2;
    for (int idx = tid; idx < Ns * SC_R; idx += SC_T) {
        const int i = idx / SC_R, r = idx % SC_R;
        z[idx] = r < nrhs ? bh[(int64_t)r * ng + (2 * p + 1) * Ns + i] - y[idx] : 0.0;
    }
    __syncthreads();
    if (has1) sc_matvec(G + (2 * p + 1) * nn, Ns, Ns, z, red, x, nrhs, tid);
    __syncthreads();
    for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
        const int i = idx / nrhs, r = idx % nrhs;
        c_all[((int64_t)r * P + p) * Ns + i] = y[i * SC_R + r] + (has1 ? x[i * SC_R + r] : 0.0);
    }
}

// one workgroup: s_{2p} for every pair into s_all [SC_R][N][Ns]
__global__ __launch_bounds__(SC_T) void k_pair_fwd_chain(const double *M, int64_t N, int Ns, const double *c_all,
                                                         double *s_all, int nrhs) {
    extern __shared__ double sm[];
    double *s = sm, *pv = sm + (int64_t)Ns * SC_R, *red = pv + (int64_t)Ns * SC_R;
    const int tid = threadIdx.x;
    const int64_t P = N / 2, nn = (int64_t)Ns * Ns;
    for (int idx = tid; idx < Ns * SC_R; idx += SC_T) s[idx] = 0.0;
    __syncthreads();
    for (int64_t p = 0; p < P; ++p) {
        for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
            const int i = idx / nrhs, r = idx % nrhs;
            s_all[((int64_t)r * N + 2 * p) * Ns + i] = s[i * SC_R + r];
        }
        __syncthreads();
        if (p + 1 == P) break;
        sc_matvec(M + p * nn, Ns, Ns, s, red, pv, nrhs, tid);
        for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
            const int i = idx / nrhs, r = idx % nrhs;
            s[i * SC_R + r] = pv[i * SC_R + r] + c_all[((int64_t)r * P + p) * Ns + i];
        }
        __syncthreads();
    }
}

// workgroup p: s_{2p+1} = s_{2p} + G_{2p}(bh_{2p} - s_{2p})
__global__ __launch_bounds__(SC_T) void k_pair_fwd_fill(const double *G, int64_t N, int Ns, const double *bh, int64_t ng,
                                                       double *s_all, int nrhs) {
    extern __shared__ double sm[];
    double *x = sm, *y = sm + (int64_t)Ns * SC_R, *red = y + 2 * (int64_t)Ns * SC_R;
    const int64_t p = blockIdx.x, nn = (int64_t)Ns * Ns;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < Ns * SC_R; idx += SC_T) {
        const int i = idx / SC_R, r = idx % SC_R;
        x[idx] = r < nrhs ? bh[(int64_t)r * ng + 2 * p * Ns + i] - s_all[((int64_t)r * N + 2 * p) * Ns + i] : 0.0;
    }
    __syncthreads();
    sc_matvec(G + 2 * p * nn, Ns, Ns, x, red, y, nrhs, tid);
    __syncthreads();
    for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
        const int i = idx / nrhs, r = idx % nrhs;
        s_all[((int64_t)r * N + 2 * p + 1) * Ns + i] = s_all[((int64_t)r * N + 2 * p) * Ns + i] + y[i * SC_R + r];
    }
}

// workgroup p - 1 (p >= 1): e_p = a_{2p+1} - G_{2p}^T a_{2p+1} + a_{2p}
__global__ __launch_bounds__(SC_T) void k_pair_bwd_e(const double *GT, int64_t N, int Ns, const double *a_all,
                                                    double *e_all, int nrhs) {
    extern __shared__ double sm[];
    double *x = sm, *y = sm + (int64_t)Ns * SC_R, *red = y + 2 * (int64_t)Ns * SC_R;
    const int64_t p = blockIdx.x + 1, P = N / 2, nn = (int64_t)Ns * Ns;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < Ns * SC_R; idx += SC_T) {
        const int i = idx / SC_R, r = idx % SC_R;
        x[idx] = r < nrhs ? a_all[((int64_t)r * N + 2 * p + 1) * Ns + i] : 0.0;
    }
    __syncthreads();
    sc_matvec(GT + 2 * p * nn, Ns, Ns, x, red, y, nrhs, tid);
    __syncthreads();
    for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
        const int i = idx / nrhs, r = idx % nrhs;
        e_all[((int64_t)r * P + p) * Ns + i] =
            x[i * SC_R + r] - y[i * SC_R + r] + a_all[((int64_t)r * N + 2 * p) * Ns + i];
    }
}

// one workgroup: t_{N-1} = 0 and t_{2p-1} for p = N/2 - 1 .. 1 into t_all
__global__ __launch_bounds__(SC_T) void k_pair_bwd_chain(const double *MT, int64_t N, int Ns, const double *e_all,
                                                         double *t_all, int nrhs) {
    extern __shared__ double sm[];
    double *t = sm, *pv = sm + (int64_t)Ns * SC_R, *red = pv + (int64_t)Ns * SC_R;
    const int tid = threadIdx.x;
    const int64_t P = N / 2, nn = (int64_t)Ns * Ns;
    for (int idx = tid; idx < Ns * SC_R; idx += SC_T) t[idx] = 0.0;
    for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
        const int i = idx / nrhs, r = idx % nrhs;
        t_all[((int64_t)r * N + N - 1) * Ns + i] = 0.0;
    }
    __syncthreads();
    for (int64_t p = P - 1; p >= 1; --p) {
        sc_matvec(MT + p * nn, Ns, Ns, t, red, pv, nrhs, tid);
        for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
            const int i = idx / nrhs, r = idx % nrhs;
            const double v = pv[i * SC_R + r] + e_all[((int64_t)r * P + p) * Ns + i];
            t[i * SC_R + r] = v;
            t_all[((int64_t)r * N + 2 * p - 1) * Ns + i] = v;
        }
        __syncthreads();
    }
}

// workgroup p: x_{2p+1}, t_{2p}, x_{2p} into xg
__global__ __launch_bounds__(SC_T) void k_pair_bwd_fill(const double *GT, int64_t N, int Ns, const double *a_all,
                                                       const double *t_all, double *xg, int64_t ng, int nrhs) {
    extern __shared__ double sm[];
    double *x = sm, *y = sm + (int64_t)Ns * SC_R, *red = y + 2 * (int64_t)Ns * SC_R;
    const int64_t p = blockIdx.x, nn = (int64_t)Ns * Ns;
    const int tid = threadIdx.x;
    const bool has1 = 2 * p + 1 <= N - 2;
    for (int idx = tid; idx < Ns * SC_R; idx += SC_T) {
        const int i = idx / SC_R, r = idx % SC_R;
        x[idx] = r < nrhs ? t_all[((int64_t)r * N + 2 * p + 1) * Ns + i] : 0.0;
    }
    __syncthreads();
    if (has1) sc_matvec(GT + (2 * p + 1) * nn, Ns, Ns, x, red, y, nrhs, tid);
    __syncthreads();
    // x_{2p+1} = a_{2p+1} - G_{2p+1}^T t_{2p+1}; t_{2p} = t_{2p+1} + x_{2p+1} (into x)
    for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
        const int i = idx / nrhs, r = idx % nrhs;
        const double x1 = a_all[((int64_t)r * N + 2 * p + 1) * Ns + i] - (has1 ? y[i * SC_R + r] : 0.0);
        xg[(int64_t)r * ng + (2 * p + 1) * Ns + i] = x1;
        x[i * SC_R + r] += x1;
    }
    __syncthreads();
    sc_matvec(GT + 2 * p * nn, Ns, Ns, x, red, y, nrhs, tid);
    __syncthreads();
    for (int idx = tid; idx < Ns * nrhs; idx += SC_T) {
        const int i = idx / nrhs, r = idx % nrhs;
        xg[(int64_t)r * ng + 2 * p * Ns + i] = a_all[((int64_t)r * N + 2 * p) * Ns + i] - y[i * SC_R + r];
    }
}

bool struct_pairs(int64_t N) { return N >= 4 && N % 2 == 0; }

// bh [nrhs][ng] -> xg [nrhs][ng]; sa, aa: [SC_R][N][Ns] workspace
void launch_struct_solve(const double *F, const double *G, const double *GT, const double *M, const double *MT,
                         int64_t N, int64_t Ns, const double *bh, double *xg, double *sa, double *aa, double *ce,
                         int64_t nrhs, hipStream_t st) {
    const int64_t ng = N * Ns;
    if (struct_pairs(N)) {
        const int Gm = std::max(1, std::min(16, SC_T / (int)std::max<int64_t>(Ns, 1)));
        const size_t lds_c = sizeof(double) * ((size_t)2 * Ns * SC_R + (size_t)Gm * Ns * SC_R);
        const size_t lds_w = sizeof(double) * ((size_t)3 * Ns * SC_R + (size_t)Gm * Ns * SC_R);
        const size_t lds_k = sizeof(double) * ((size_t)2 * Ns * SC_R);
        if (lds_c > 64 * 1024) {
            (void)hipFuncSetAttribute((const void *)k_pair_fwd_chain, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds_c);
            (void)hipFuncSetAttribute((const void *)k_pair_bwd_chain, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds_c);
        }
        if (lds_k > 64 * 1024)
            (void)hipFuncSetAttribute((const void *)k_struct_blocks, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds_k);
        if (lds_w > 64 * 1024)
            for (const void *kf : {(const void *)k_pair_fwd_c, (const void *)k_pair_fwd_fill,
                                   (const void *)k_pair_bwd_e, (const void *)k_pair_bwd_fill})
                (void)hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_w);
        const unsigned P = (unsigned)(N / 2);
        for (int64_t k0 = 0; k0 < nrhs; k0 += SC_R) {
            const int nr = (int)std::min<int64_t>(SC_R, nrhs - k0);
            hipLaunchKernelGGL(k_pair_fwd_c, dim3(P), dim3(SC_T), lds_w, st, G, N, (int)Ns, bh + k0 * ng, ng, ce, nr);
            hipLaunchKernelGGL(k_pair_fwd_chain, dim3(1), dim3(SC_T), lds_c, st, M, N, (int)Ns, (const double *)ce, sa,
                               nr);
            hipLaunchKernelGGL(k_pair_fwd_fill, dim3(P), dim3(SC_T), lds_w, st, G, N, (int)Ns, bh + k0 * ng, ng, sa, nr);
            hipLaunchKernelGGL(k_struct_blocks, dim3((unsigned)N), dim3(256), lds_k, st, F, N, (int)Ns, bh + k0 * ng,
                               ng, (const double *)sa, aa, nr);
            hipLaunchKernelGGL(k_pair_bwd_e, dim3(P - 1), dim3(SC_T), lds_w, st, GT, N, (int)Ns, (const double *)aa, ce,
                               nr);
            hipLaunchKernelGGL(k_pair_bwd_chain, dim3(1), dim3(SC_T), lds_c, st, MT, N, (int)Ns, (const double *)ce, sa,
                               nr);
            hipLaunchKernelGGL(k_pair_bwd_fill, dim3(P), dim3(SC_T), lds_w, st, GT, N, (int)Ns, (const double *)aa,
                               (const double *)sa, xg + k0 * ng, ng, nr);
        }
        return;
    }
    const int Gm = std::max(1, std::min(16, SC_T / (int)std::max<int64_t>(Ns, 1)));
    const size_t lds_f = sizeof(double) * ((size_t)3 * Ns * SC_R + (size_t)Gm * Ns * SC_R);
    const size_t lds_b = sizeof(double) * ((size_t)2 * Ns * SC_R + (size_t)Gm * Ns * SC_R);
    const size_t lds_k = sizeof(double) * ((size_t)2 * Ns * SC_R);
    if (lds_f > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)k_struct_fwd_chain, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds_f);
    if (lds_b > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)k_struct_bwd_chain, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds_b);
    if (lds_k > 64 * 1024)
        (void)hipFuncSetAttribute((const void *)k_struct_blocks, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds_k);
    for (int64_t k0 = 0; k0 < nrhs; k0 += SC_R) {
        const int nr = (int)std::min<int64_t>(SC_R, nrhs - k0);
        hipLaunchKernelGGL(k_struct_fwd_chain, dim3(1), dim3(SC_T), lds_f, st, G, N, (int)Ns, bh + k0 * ng, ng, sa,
                           nr);
        hipLaunchKernelGGL(k_struct_blocks, dim3((unsigned)N), dim3(256), lds_k, st, F, N, (int)Ns, bh + k0 * ng, ng,
                           (const double *)sa, aa, nr);
        hipLaunchKernelGGL(k_struct_bwd_chain, dim3(1), dim3(SC_T), lds_b, st, GT, N, (int)Ns, (const double *)aa,
                           xg + k0 * ng, ng, nr);
    }
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
                           double *amax_s, int mirror, hipStream_t st, int64_t q0, int64_t q1) {
    const int64_t ng = N * Ns;
    if (q1 < 0 || q1 > ng) q1 = ng;
    if (q1 <= q0) return;
    const dim3 gg((unsigned)((ng + 255) / 256), (unsigned)(q1 - q0));  // columns [q0, q1)
    if (precision == 1)
        hipLaunchKernelGGL(k_schur_assemble<float>, gg, dim3(256), 0, st, (const float *)U, Ustride, uoff, N, Ns,
                           prefix, corner, S, tau_s, eps, amax_s, mirror, q0);
    else
        hipLaunchKernelGGL(k_schur_assemble<double>, gg, dim3(256), 0, st, (const double *)U, Ustride, uoff, N, Ns,
                           prefix, corner, S, tau_s, eps, amax_s, mirror, q0);
}

void launch_schur_diag(const void *U, int64_t Ustride, int64_t uoff, int64_t N, int64_t Ns, int precision,
                       const double *prefix, const double *corner, double *tau_s, double eps, double *amax_s,
                       hipStream_t st) {
    const int64_t ng = N * Ns;
    const dim3 g((unsigned)((ng + 255) / 256));
    if (precision == 1)
        hipLaunchKernelGGL(k_schur_diag<float>, g, dim3(256), 0, st, (const float *)U, Ustride, uoff, N, Ns, prefix,
                           corner, tau_s, eps, amax_s);
    else
        hipLaunchKernelGGL(k_schur_diag<double>, g, dim3(256), 0, st, (const double *)U, Ustride, uoff, N, Ns,
                           prefix, corner, tau_s, eps, amax_s);
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
