// Launch geometry and global addresses of the triangular solves with the
// dense Schur factor (host and device; the host side serves the tests of
// their address ranges). The factor is column-major with leading dimension
// ng; vectors are [nrhs][ng]. Every address below is computed from clamped
// indices, so that a load issued for a lane past the end of a ragged block
// stays inside the factor; such lanes' values are masked afterwards.
#pragma once
#include <cstdint>

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#endif

namespace kkt {

constexpr int DENSE_BLOCK = 1024;  // width of the factor's inverted diagonal blocks
constexpr int DS_RB = 4;           // right-hand sides per pass of a kernel

__host__ __device__ inline int64_t ds_min(int64_t a, int64_t b) { return a < b ? a : b; }
__host__ __device__ inline int64_t ds_max(int64_t a, int64_t b) { return a > b ? a : b; }

// Forward product below a block, out[row0 + i] -= sum_q S[row0 + i, col0 + q]
// w[q] (i < nrow, q < ncol <= DENSE_BLOCK): 512 threads per workgroup,
// GV_R rows by GV_G groups of 64 columns.
constexpr int GV_G = DENSE_BLOCK / 64;
constexpr int GV_R = 512 / GV_G;
// factor entry u (< 64) of thread tid in workgroup blk
__host__ __device__ inline int64_t gemv_s_addr(int64_t ng, int64_t row0, int64_t nrow, int64_t col0, int ncol,
                                               int64_t blk, int tid, int u) {
    const int64_t i = blk * GV_R + tid % GV_R;
    const int qa = 64 * (tid / GV_R);
    const int ncq = (int)ds_max(1, ds_min(64, ncol - qa));
    return row0 + ds_min(i, nrow - 1) + (col0 + ds_min(qa, ncol - 1) + ds_min(u, ncq - 1)) * ng;
}

// Forward in-block product out[j0 + i] = in[j0 + i] + sum_{q < i} X[i][q]
// in[j0 + q] (i < nbw): 256 threads, 16 rows by 16 groups of BK_C columns.
constexpr int BK_C = DENSE_BLOCK / 16;
__host__ __device__ inline int64_t blk_s_addr(int64_t ng, int64_t j0, int nbw, int64_t blk, int tid, int u) {
    const int64_t i = blk * 16 + (tid & 15);
    const int64_t q0 = ds_min((int64_t)BK_C * (tid >> 4), nbw - 1);
    return j0 + ds_min(i, nbw - 1) + (j0 + q0 + ds_min(u, nbw - 1 - q0)) * ng;
}

// Backward products with the transpose, as dot products down the columns:
// 4 waves per workgroup, TD_CPW outputs per wave, DENSE_BLOCK / 64 terms per
// lane; output i of the launch reads S[row0 .. row0 + nq, col0 + i].
constexpr int TD_CPW = 2;
__host__ __device__ inline int64_t tdot_s_addr(int64_t ng, int64_t row0, int nq, int64_t col0, int ncols, int64_t blk,
                                               int wave, int c, int lane, int k) {
    const int64_t i0 = (blk * 4 + wave) * TD_CPW;
    return row0 + ds_min(lane + 64 * k, nq - 1) + (col0 + ds_min(i0 + c, ncols - 1)) * ng;
}

// workgroups of each launch
__host__ __device__ inline int64_t gemv_grid(int64_t nrow) { return (nrow + GV_R - 1) / GV_R; }
__host__ __device__ inline int64_t blk_grid(int nbw) { return (nbw + 15) / 16; }
__host__ __device__ inline int64_t tdot_grid(int64_t ncols) { return (ncols + 4 * TD_CPW - 1) / (4 * TD_CPW); }

}  // namespace kkt
