// emb_common.h -- cross-lane helpers for gfx950 wavefronts (64 lanes).
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

namespace dp {

// Value of `v` from the lane selected by the DPP control word CTRL
// (quad_perm 0x00-0xFF, row_mirror 0x140, row_half_mirror 0x141, ...),
// all rows and banks enabled.
template <int CTRL>
__device__ inline float dpp_f(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                                 0xF, 0xF, false));
}

template <int CTRL>
__device__ inline double dpp_d(double v)
{
    int2 p = __builtin_bit_cast(int2, v);
    p.x = __builtin_amdgcn_update_dpp(0, p.x, CTRL, 0xF, 0xF, false);
    p.y = __builtin_amdgcn_update_dpp(0, p.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, p);
}

// Writes x as a GEMM operand element (row, col) of a matrix with ncols
// logical columns: as is for FP64/FP32, as the [hi | hi | lo] split for BF16.
__device__ inline void store_op(double *p, long row, int col, int ncols, double x)
{
    p[row * ncols + col] = x;
}
__device__ inline void store_op(float *p, long row, int col, int ncols, double x)
{
    p[row * ncols + col] = (float)x;
}
__device__ inline void store_op(__bf16 *p, long row, int col, int ncols, double x)
{
    float f = (float)x;
    __bf16 hi = (__bf16)f;
    __bf16 lo = (__bf16)(f - (float)hi);
    __bf16 *r = p + row * 3 * ncols;
    r[col] = hi;
    r[ncols + col] = hi;
    r[2 * ncols + col] = lo;
}

}  // namespace dp
