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

// The forward in-block product out[j0 + i] = in[j0 + i] + sum_{q < i}
// X[i][q] in[j0 + q] (i < nbw) takes the same geometry and addresses with
// row0 = col0 = j0, nrow = ncol = nbw; a column group loads only if it has a
// column left of the row's diagonal (64 g < i).
__host__ __device__ inline bool gemv_tri_used(int64_t blk, int tid) {
    return 64 * (tid / GV_R) < blk * GV_R + tid % GV_R;
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
__host__ __device__ inline int64_t tdot_grid(int64_t ncols) { return (ncols + 4 * TD_CPW - 1) / (4 * TD_CPW); }

// One launch per block step joins a product below or above a block with the
// next block's in-block product. Forward step after block [j0, j1): row
// workgroups 0 .. gemv_grid(ng - j1) - 1 (the first gemv_grid(nbw1) of them
// cover the next block [j1, j1 + nbw1)), then gemv_grid(nbw1) workgroups of
// the next block's in-block product. Backward step before block [j0 - DB,
// j0): the product with block [j0, ..) over the columns [0, j0) in reverse
// order of workgroups (workgroup b takes tdot block tdot_grid(j0) - 1 - b, so
// the first tdot_grid(DB) of them cover the columns of block [j0 - DB, j0)),
// then tdot_grid(DB) workgroups of that block's in-block product.
__host__ __device__ inline int64_t fwd_step_grid(int64_t ng, int64_t j1) {
    return gemv_grid(ng - j1) + gemv_grid(ds_min(DENSE_BLOCK, ng - j1));
}
__host__ __device__ inline int64_t bwd_step_grid(int64_t j0) {
    return tdot_grid(j0) + tdot_grid(DENSE_BLOCK);
}

}  // namespace kkt
