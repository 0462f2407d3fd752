// emb.hip -- fused environment matrix, tabulated embedding and R^T G
// contraction (forward), and its hand-written adjoint down to forces and the
// virial (backward), on gfx950.
//
// What is computed per atom i (paper Sec. 2.1, Eqs. 1-5; Sec. 3.2-3.4):
//   for every neighbor j with r = |r_ij| < rcut (the sel nearest at most):
//     s = w(r)/r, R_j = s (1, x/r, y/r, z/r)                      (Eq. 1)
//     G_j = f_theta(s): the M quintics of s's table interval      (Sec. 3.2)
//   T = desc_scale * sum_j R_j^T G_j   (4 x M), D = T<^T T (M< x M)  (Eq. 2)
// G is never stored: each lane evaluates its columns of G_j in registers and
// folds them into T at once (the kernel fusion of Sec. 3.3/3.4.1).  Padded
// neighbors do not exist here: the loop runs over the n_i real neighbors only
// (the redundancy removal of Sec. 3.4.2; with unnormalised R the padded rows
// would contribute exact zeros).
//
// Work distribution (one 64-lane wavefront per atom):
//   lanes are split into NG groups of GL = 128/CPL lanes; lane l of a group
//   owns the CPL columns eta = l + GL*c.  Group g walks the g-th contiguous
//   chunk of the distance-sorted neighbor list, so consecutive neighbors
//   mostly share a table interval and the lane keeps that interval's
//   coefficients in registers, reloading only when the interval changes.
//   Neighbor data is staged once in LDS and read as group-uniform
//   broadcasts.  The forward needs no cross-lane traffic inside the loop;
//   partial T's of the groups are summed once at the end.
//
// Backward (the adjoint of the same fused step, G recomputed from the
// table): with dT = dE/dT (4 x M) per atom,
//   dE/dR_jk  = desc_scale * sum_eta dT_k,eta G_j,eta
//   dE/ds_j  += desc_scale * sum_eta (sum_k dT_k,eta R_jk) G'_j,eta
//   g_ij = dE_i/dr_ij by the chain rule through Eq. 1,
//   F_i += g_ij, F_j -= g_ij (FP64 atomics), W_i -= r_ij (x) g_ij.
// The sums over eta are reduced across the lanes of a group with DPP row
// operations (quad_perm, row_half_mirror, row_mirror).

#include "dp_internal.h"
#include "emb_common.h"
#include "env.h"

#include <type_traits>

namespace dp {

namespace {

// Coefficients of CPL columns of interval th into registers.
template <typename real, int CPL, int GL>
__device__ inline void load_coef(const real *tab, int th, int l, real (&a)[CPL][6]);

template <>
__device__ inline void load_coef<float, 8, 16>(const float *tab, int th, int l, float (&a)[8][6])
{
#pragma unroll
    for (int c = 0; c < 8; c++) {
        const float4 *p = reinterpret_cast<const float4 *>(tab + ((long)th * kM + l + 16 * c) * 8);
        float4 u = p[0], v = p[1];
        a[c][0] = u.x; a[c][1] = u.y; a[c][2] = u.z; a[c][3] = u.w; a[c][4] = v.x; a[c][5] = v.y;
    }
}

template <>
__device__ inline void load_coef<float, 4, 32>(const float *tab, int th, int l, float (&a)[4][6])
{
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const float4 *p = reinterpret_cast<const float4 *>(tab + ((long)th * kM + l + 32 * c) * 8);
        float4 u = p[0], v = p[1];
        a[c][0] = u.x; a[c][1] = u.y; a[c][2] = u.z; a[c][3] = u.w; a[c][4] = v.x; a[c][5] = v.y;
    }
}

template <>
__device__ inline void load_coef<double, 4, 32>(const double *tab, int th, int l, double (&a)[4][6])
{
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const double2 *p = reinterpret_cast<const double2 *>(tab + ((long)th * kM + l + 32 * c) * 6);
        double2 u = p[0], v = p[1], w = p[2];
        a[c][0] = u.x; a[c][1] = u.y; a[c][2] = v.x; a[c][3] = v.y; a[c][4] = w.x; a[c][5] = w.y;
    }
}

template <>
__device__ inline void load_coef<double, 2, 64>(const double *tab, int th, int l, double (&a)[2][6])
{
#pragma unroll
    for (int c = 0; c < 2; c++) {
        const double2 *p = reinterpret_cast<const double2 *>(tab + ((long)th * kM + l + 64 * c) * 6);
        double2 u = p[0], v = p[1], w = p[2];
        a[c][0] = u.x; a[c][1] = u.y; a[c][2] = v.x; a[c][3] = v.y; a[c][4] = w.x; a[c][5] = w.y;
    }
}

template <typename real>
__device__ inline real horner(const real (&a)[6], real t)
{
    return fma(fma(fma(fma(fma(a[5], t, a[4]), t, a[3]), t, a[2]), t, a[1]), t, a[0]);
}

template <typename real>
__device__ inline void horner2(const real (&a)[6], real t, real &f, real &fp)
{
    real p = a[5], q = a[5];
    p = fma(p, t, a[4]);
    q = fma(q, t, p);
    p = fma(p, t, a[3]);
    q = fma(q, t, p);
    p = fma(p, t, a[2]);
    q = fma(q, t, p);
    p = fma(p, t, a[1]);
    q = fma(q, t, p);
    f = fma(p, t, a[0]);
    fp = q;
}

// Sum over the GL lanes of a group, result in every lane of the group.
template <int GL>
__device__ inline float group_sum(float v)
{
    v += dpp_f<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);   // row_half_mirror
    v += dpp_f<0x140>(v);   // row_mirror
    if (GL >= 32) v += __shfl_xor(v, 16);
    if (GL >= 64) v += __shfl_xor(v, 32);
    return v;
}

template <int GL>
__device__ inline double group_sum(double v)
{
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    if (GL >= 32) v += __shfl_xor(v, 16);
    if (GL >= 64) v += __shfl_xor(v, 32);
    return v;
}

template <typename T> __device__ inline T cvt(float v);
template <> __device__ inline float cvt<float>(float v) { return v; }
template <> __device__ inline double cvt<double>(float v) { return v; }
template <> __device__ inline __hip_bfloat16 cvt<__hip_bfloat16>(float v) { return __float2bfloat16(v); }
template <typename T> __device__ inline T cvtd(double v);
template <> __device__ inline double cvtd<double>(double v) { return v; }
template <> __device__ inline float cvtd<float>(double v) { return (float)v; }
template <> __device__ inline __hip_bfloat16 cvtd<__hip_bfloat16>(double v) { return __float2bfloat16((float)v); }

// -------------------------------------------------------------- forward
template <typename real, typename TD, int CPL>
__global__ void __launch_bounds__(256) k_emb_fwd(int natoms, EnvArgs A, const real *__restrict__ tab,
                                                 real sigma, real *__restrict__ T_out,
                                                 TD *__restrict__ D_out, int *__restrict__ nnei_out)
{
    constexpr int GL = kM / CPL, NG = 64 / GL;
    HIP_DYNAMIC_SHARED(uint4, smem_raw)   // 16-byte aligned
    char *smem = reinterpret_cast<char *>(smem_raw);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = blockIdx.x * (blockDim.x >> 6) + wave;
    real *Tl;
    NbrLDS<real> L = carve<real>(smem + wave * lds_bytes_per_wave<real>(A.sel, false), A.sel, false, Tl);
    bool live = i < natoms;
    int nn = 0, n_in = 0, oob = 0;
    if (live) nn = build_env<real, false>(i, A, L, lane, n_in, oob);
    __syncthreads();
    if (!live) return;
    record_flags<real>(A, lane, n_in, oob);
    if (nnei_out && lane == 0) nnei_out[i] = nn;

    int g = lane / GL, l = lane % GL;
    int chunk = (nn + NG - 1) / NG;
    int beg = g * chunk, end = min(nn, beg + chunk);
    real acc[4][CPL];
#pragma unroll
    for (int c = 0; c < CPL; c++) acc[0][c] = acc[1][c] = acc[2][c] = acc[3][c] = 0;
    real a[CPL][6];
    int cur = -1;
    for (int k = beg; k < end; k++) {
        int th = L.I[k].x & ~kOobBit;
        real t = L.P[k].x;
        V4<real> R = L.R[k];
        if (th != cur) {
            load_coef<real, CPL, GL>(tab, th, l, a);
            cur = th;
        }
#pragma unroll
        for (int c = 0; c < CPL; c++) {
            real f = horner<real>(a[c], t);
            acc[0][c] = fma(R.x, f, acc[0][c]);
            acc[1][c] = fma(R.y, f, acc[1][c]);
            acc[2][c] = fma(R.z, f, acc[2][c]);
            acc[3][c] = fma(R.w, f, acc[3][c]);
        }
    }
    // sum the groups' partial T
#pragma unroll
    for (int off = GL; off < 64; off <<= 1)
#pragma unroll
        for (int c = 0; c < CPL; c++)
#pragma unroll
            for (int k = 0; k < 4; k++) acc[k][c] += __shfl_xor(acc[k][c], off);
    if (g == 0) {
#pragma unroll
        for (int c = 0; c < CPL; c++)
#pragma unroll
            for (int k = 0; k < 4; k++) {
                real v = sigma * acc[k][c];
                Tl[k * kM + l + GL * c] = v;
                T_out[(long)i * 4 * kM + k * kM + l + GL * c] = v;
            }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // D[a][b] = sum_k T[k][a] T[k][b], a < M<
    for (int o = lane; o < kDdim; o += 64) {
        int aa = o >> 7, bb = o & (kM - 1);
        real v = Tl[aa] * Tl[bb];
        v = fma(Tl[kM + aa], Tl[kM + bb], v);
        v = fma(Tl[2 * kM + aa], Tl[2 * kM + bb], v);
        v = fma(Tl[3 * kM + aa], Tl[3 * kM + bb], v);
        store_op(D_out, i, o, kDdim, (double)v);
    }
}

// ------------------------------------------------------------- backward
template <typename real, int CPL>
__global__ void __launch_bounds__(256) k_emb_bwd(int natoms, EnvArgs A, const real *__restrict__ tab,
                                                 real sigma, const real *__restrict__ dT,
                                                 double *__restrict__ force, double *__restrict__ w_atom)
{
    constexpr int GL = kM / CPL, NG = 64 / GL;
    HIP_DYNAMIC_SHARED(uint4, smem_raw)   // 16-byte aligned
    char *smem = reinterpret_cast<char *>(smem_raw);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = blockIdx.x * (blockDim.x >> 6) + wave;
    real *Tl;
    NbrLDS<real> L = carve<real>(smem + wave * lds_bytes_per_wave<real>(A.sel, true), A.sel, true, Tl);
    bool live = i < natoms;
    int nn = 0, n_in = 0, oob = 0;
    if (live) nn = build_env<real, true>(i, A, L, lane, n_in, oob);
    __syncthreads();
    if (!live) return;

    int g = lane / GL, l = lane % GL;
    real dt[4][CPL];
#pragma unroll
    for (int c = 0; c < CPL; c++)
#pragma unroll
        for (int k = 0; k < 4; k++) dt[k][c] = sigma * dT[(long)i * 4 * kM + k * kM + l + GL * c];
    int chunk = (nn + NG - 1) / NG;
    int beg = g * chunk, end = min(nn, beg + chunk);
    real a[CPL][6];
    int cur = -1;
    real Fi0 = 0, Fi1 = 0, Fi2 = 0;
    real W[9];
#pragma unroll
    for (int q = 0; q < 9; q++) W[q] = 0;
    for (int k = beg; k < end; k++) {
        int2 I = L.I[k];
        V4<real> P = L.P[k];
        V4<real> R = L.R[k];
        int th = I.x & ~kOobBit;
        if (th != cur) {
            load_coef<real, CPL, GL>(tab, th, l, a);
            cur = th;
        }
        real dR0 = 0, dR1 = 0, dR2 = 0, dR3 = 0, dsG = 0;
#pragma unroll
        for (int c = 0; c < CPL; c++) {
            real f, fp;
            horner2<real>(a[c], P.x, f, fp);
            dR0 = fma(dt[0][c], f, dR0);
            dR1 = fma(dt[1][c], f, dR1);
            dR2 = fma(dt[2][c], f, dR2);
            dR3 = fma(dt[3][c], f, dR3);
            real av = dt[0][c] * R.x;
            av = fma(dt[1][c], R.y, av);
            av = fma(dt[2][c], R.z, av);
            av = fma(dt[3][c], R.w, av);
            dsG = fma(av, fp, dsG);
        }
        dR0 = group_sum<GL>(dR0);
        dR1 = group_sum<GL>(dR1);
        dR2 = group_sum<GL>(dR2);
        dR3 = group_sum<GL>(dR3);
        dsG = group_sum<GL>(dsG);
        if (I.x & kOobBit) dsG = 0;
        if (l == 0) {
            V4<real> d = L.Dv[k];
            real rinv = P.z, s = P.w, sp = P.y;
            real h0 = d.x * rinv, h1 = d.y * rinv, h2 = d.z * rinv;
            // R = s (1, h): dE/ds collects dR0 + dR.h; dE/dh = s dR[1..3]
            real dEds = dsG + dR0 + dR1 * h0 + dR2 * h1 + dR3 * h2;
            real u0 = s * dR1, u1 = s * dR2, u2 = s * dR3;
            real udh = u0 * h0 + u1 * h1 + u2 * h2;
            real c0 = dEds * sp;
            real g0 = c0 * h0 + (u0 - udh * h0) * rinv;
            real g1 = c0 * h1 + (u1 - udh * h1) * rinv;
            real g2 = c0 * h2 + (u2 - udh * h2) * rinv;
            int j = I.y;
            unsafeAtomicAdd(&force[3 * j], -(double)g0);
            unsafeAtomicAdd(&force[3 * j + 1], -(double)g1);
            unsafeAtomicAdd(&force[3 * j + 2], -(double)g2);
            Fi0 += g0;
            Fi1 += g1;
            Fi2 += g2;
            W[0] -= d.x * g0; W[1] -= d.x * g1; W[2] -= d.x * g2;
            W[3] -= d.y * g0; W[4] -= d.y * g1; W[5] -= d.y * g2;
            W[6] -= d.z * g0; W[7] -= d.z * g1; W[8] -= d.z * g2;
        }
    }
    // group leaders hold partials, other lanes zeros: sum over the wave
    for (int off = 32; off > 0; off >>= 1) {
        Fi0 += __shfl_xor(Fi0, off);
        Fi1 += __shfl_xor(Fi1, off);
        Fi2 += __shfl_xor(Fi2, off);
#pragma unroll
        for (int q = 0; q < 9; q++) W[q] += __shfl_xor(W[q], off);
    }
    if (lane == 0) {
        unsafeAtomicAdd(&force[3 * i], (double)Fi0);
        unsafeAtomicAdd(&force[3 * i + 1], (double)Fi1);
        unsafeAtomicAdd(&force[3 * i + 2], (double)Fi2);
    }
    if (lane < 9) {
        real v = W[0];
#pragma unroll
        for (int q = 1; q < 9; q++) v = lane == q ? W[q] : v;
        w_atom[(long)i * 9 + lane] = (double)v;
    }
}

}  // namespace

// ---------------------------------------------------------- launchers
template <typename real, typename TD, int CPL>
static void launch_fwd_t(const dp_model *m, const dp_nlist *nl, int n, const double *x, void *T,
                         void *D, int *nnei, hipStream_t st)
{
    EnvArgs A = make_env_args(m, nl, x);
    const real *tab = std::is_same<real, double>::value ? (const real *)m->tab64 : (const real *)m->tab32;
    int wpb = 4;
    size_t lds = (size_t)wpb * lds_bytes_per_wave<real>(A.sel, false);
    hipLaunchKernelGGL((k_emb_fwd<real, TD, CPL>), dim3(div_up(n, wpb)), dim3(64 * wpb), lds, st, n, A,
                       tab, (real)m->cfg.desc_scale, (real *)T, (TD *)D, nnei);
}

template <typename real, int CPL>
static void launch_bwd_t(const dp_model *m, const dp_nlist *nl, int n, const double *x,
                         const void *dT, double *force, double *w_atom, hipStream_t st)
{
    EnvArgs A = make_env_args(m, nl, x);
    const real *tab = std::is_same<real, double>::value ? (const real *)m->tab64 : (const real *)m->tab32;
    int wpb = 4;
    size_t lds = (size_t)wpb * lds_bytes_per_wave<real>(A.sel, true);
    hipLaunchKernelGGL((k_emb_bwd<real, CPL>), dim3(div_up(n, wpb)), dim3(64 * wpb), lds, st, n, A, tab,
                       (real)m->cfg.desc_scale, (const real *)dT, force, w_atom);
}

void launch_emb_fwd(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision,
                    void *T, void *D, int *nnei, hipStream_t st)
{
    if (precision == DP_FP64) launch_fwd_t<double, double, 4>(m, nl, n, x, T, D, nnei, st);
    else if (precision == DP_FP32) launch_fwd_t<float, float, 8>(m, nl, n, x, T, D, nnei, st);
    else launch_fwd_t<float, __bf16, 8>(m, nl, n, x, T, D, nnei, st);
}

void launch_emb_bwd(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision,
                    const void *dT, double *force, double *w_atom, hipStream_t st)
{
    if (precision == DP_FP64) launch_bwd_t<double, 4>(m, nl, n, x, dT, force, w_atom, st);
    else launch_bwd_t<float, 8>(m, nl, n, x, dT, force, w_atom, st);
}

}  // namespace dp
