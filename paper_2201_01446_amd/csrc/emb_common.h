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

}  // namespace dp
