// fit_common.h -- MFMA fragments, precision conversions and the epilogue
// tanh shared by the fitting-net GEMM (gemm.hip) and the fused fitting tail
// (fit.hip).
#pragma once

#include "dp_internal.h"
#include "tanh64.h"

#include <type_traits>

namespace dp {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef double d2v __attribute__((ext_vector_type(2)));
// 16 raw bytes as a native vector (HIP's uint4 struct defeats register promotion)
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

namespace {

template <typename TA> struct MMT;
template <> struct MMT<double> { using acc = double; using accv = d4v; static constexpr int VEC = 2; };
template <> struct MMT<float> { using acc = float; using accv = f4v; static constexpr int VEC = 4; };
template <> struct MMT<__bf16> { using acc = float; using accv = f4v; static constexpr int VEC = 8; };

// One K-group (4 lanes-groups x VEC elements) of MFMA on 16-byte fragments.
// For the 4-deep FP32/FP64 instructions the VEC elements of a fragment feed
// VEC instructions; lane group q then holds k = q*VEC + v of the group in the
// v-th one, the same mapping for A and B, so the group's sum is complete.
__device__ inline void mfma_frag(const u4v &a, const u4v &b, d4v &c)
{
    d2v x = __builtin_bit_cast(d2v, a), y = __builtin_bit_cast(d2v, b);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(x[0], y[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(x[1], y[1], c, 0, 0, 0);
}
__device__ inline void mfma_frag_f32(const u4v &a, const u4v &b, f4v &c)
{
    f4v x = __builtin_bit_cast(f4v, a), y = __builtin_bit_cast(f4v, b);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[0], y[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[1], y[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[2], y[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x[3], y[3], c, 0, 0, 0);
}
__device__ inline void mfma_frag_bf16(const u4v &a, const u4v &b, f4v &c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b),
                                                c, 0, 0, 0);
}

template <typename TA, typename AV>
__device__ inline void mfma_any(const u4v &a, const u4v &b, AV &c)
{
    if constexpr (std::is_same<TA, double>::value) mfma_frag(a, b, c);
    else if constexpr (std::is_same<TA, float>::value) mfma_frag_f32(a, b, c);
    else mfma_frag_bf16(a, b, c);
}

template <typename T> __device__ inline T to(float v);
template <> __device__ inline float to<float>(float v) { return v; }
template <> __device__ inline double to<double>(float v) { return v; }
template <> __device__ inline __bf16 to<__bf16>(float v) { return (__bf16)v; }
template <typename T> __device__ inline T tod(double v);
template <> __device__ inline float tod<float>(double v) { return (float)v; }
template <> __device__ inline double tod<double>(double v) { return v; }
template <> __device__ inline __bf16 tod<__bf16>(double v) { return (__bf16)(float)v; }

__device__ inline float tanh_r(float v) { return tanhf(v); }
__device__ inline double tanh_r(double v) { return tanh_f64(v); }

// tanh of an epilogue: native, or from the second-order table on [0, 8)
// (odd extension, 1 beyond 8), read in the epilogue's precision.
__device__ inline float tanh_e(float x, const float *tab)
{
    if (!tab) return tanhf(x);
    float ax = fabsf(x);
    if (ax >= 8.f) return copysignf(1.f, x);
    int k = (int)(ax * (kTanhN / 8.f));
    k = k < kTanhN - 1 ? k : kTanhN - 1;
    float t = ax - k * (8.f / kTanhN);
    float4 a = *reinterpret_cast<const float4 *>(tab + 4 * k);
    float y = fmaf(t, fmaf(t, a.z, a.y), a.x);
    return copysignf(y, x);
}
__device__ inline double tanh_e(double x, const double *tab)
{
    if (!tab) return tanh_f64(x);
    double ax = fabs(x);
    if (ax >= 8.0) return copysign(1.0, x);
    int k = (int)(ax * (kTanhN / 8.0));
    k = k < kTanhN - 1 ? k : kTanhN - 1;
    double t = ax - k * (8.0 / kTanhN);
    const double *a = tab + 4 * k;
    double y = fma(t, fma(t, a[2], a[1]), a[0]);
    return copysign(y, x);
}
// The table an epilogue of result type TR takes (NULL: native tanh).
__device__ inline const float *tanh_table_for(const Epi &e, float) { return e.tanh_tab; }
__device__ inline const double *tanh_table_for(const Epi &e, double) { return e.tanh_tab64; }

}  // namespace

}  // namespace dp
