// Shared device-side declarations: task descriptors, MFMA wrappers, atomics.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "ea_plan.hpp"

namespace kkt {

// A dense front of one supernode in the per-period storage: a column-major
// panel (m x c, ld m) holding the pivot columns, followed conceptually by the
// update block U (u x u, ld u, u = m - c) holding rows/columns >= c.
// Front-local element (r, q), r >= q, lives in the panel when q < c, else in U.
struct FrontDesc {
    int64_t Loff;   // panel offset inside one period's factor storage
    int64_t Uoff;   // update block offset inside one period's update storage
    int32_t m, c;   // rows, pivots
    int32_t piv0;   // global pivot index of panel column 0 (new order)
    int32_t sn;     // supernode id
};

struct TileTask {   // one 64x64 tile of a trailing update of front `f`
    int32_t f, ti, tj, pad;
};

struct RowTask {    // up to 256 consecutive rows [r0, ...) of front `f`
    int32_t f, r0;
};


// Factor-wide pointers handed to every factor kernel.
template <typename T>
struct FactorArgs {
    T *L;               // [N][Lstride]
    T *U;               // [N][Ustride]
    int64_t Lstride, Ustride;
    const double *tau;  // [N][tstride] per-pivot threshold eps*|a_kk| (0: use eps*amax)
    int64_t tstride;
    const double *amax; // [N] max |a_ij| of each matrix
    const int8_t *sign; // [npiv] expected sign for an exactly zero pivot, or null (-1)
    int64_t *cnt;       // [N][4] (n_pos, n_neg, n_zero, n_perturbed)
    double eps;
};

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma16x16x4(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma16x16x4(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Output row of accumulator register rr held by a lane in row group lk
// (lane / 16) of a 16x16x4 MFMA; the column is lane % 16. FP64: rows
// lk, lk+4, lk+8, lk+12; FP32: rows 4*lk .. 4*lk+3 (checked on gfx950).
__device__ inline int mfma_row(double, int lk, int rr) { return lk + 4 * rr; }
__device__ inline int mfma_row(float, int lk, int rr) { return 4 * lk + rr; }

// Raw buffer access (stride 0): loads at byte offsets past `bytes` return
// zero. Word 3 of the descriptor selects 32-bit data without swizzling.
typedef __amdgpu_buffer_rsrc_t BufRes;
__device__ inline BufRes make_bufres(const void *base, int64_t bytes) {
    const int nr = bytes < 0x7fffffff ? (int)bytes : 0x7fffffff;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, nr, 0x00020000);
}
__device__ inline double buf_load(BufRes r, int off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ inline float buf_load(BufRes r, int off, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Task and period of a workgroup of a (tasks, periods) grid, dealt so that
// every workgroup of one period runs on the same XCD: the dispatcher hands
// workgroups to the 8 XCDs round-robin in launch order (x fastest), so the
// launch index L goes to XCD L % 8, and period n takes the indices with
// L % 8 == n % 8. A period's vectors are then cached in one XCD's L2. Plain
// order when the period count is not a multiple of 8.
__device__ inline void period_task(int &task, int &n) {
    const int gx = (int)gridDim.x, np = (int)gridDim.y;
    if (np % 8 == 0) {
        const int L = (int)blockIdx.x + gx * (int)blockIdx.y;
        const int s = L >> 3;
        n = 8 * (s / gx) + (L & 7);
        task = s % gx;
    } else {
        task = (int)blockIdx.x;
        n = (int)blockIdx.y;
    }
}

__device__ inline double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// butterfly sum over the wavefront (the same order on every run)
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <typename T> struct Acc;
template <> struct Acc<double> { typedef v4d type; };
template <> struct Acc<float> { typedef v4f type; };

// max of non-negative doubles through their bit patterns (order preserving)
__device__ inline void atomic_max_nonneg(double *addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

}  // namespace kkt
