// fit.hip -- fitting net on MFMA, its input gradient, and the per-atom
// glue kernels of the force step (gfx950).
//
// Fitting net (paper Sec. 2.1): y1 = tanh(D V1 + c1); y2 = y1 + tanh(y1 V2 + c2);
// y3 = y2 + tanh(y2 V3 + c3); E_i = y3 . w4 + b4 (shortcuts between the
// equal-width layers, linear output).  Its input gradient for the forces:
//   dz3 = w4 (1 - t3^2);  dy2 = w4 + dz3 V3^T;  dz2 = dy2 (1 - t2^2);
//   dy1 = dy2 + dz2 V2^T; dz1 = dy1 (1 - y1^2); dD = dz1 V1^T,
// with t_k the tanh outputs.  Every product is the dense GEMM
// C[M x N] = A[M x K] B[N x K]^T (both operands K-contiguous), done by one
// MFMA kernel whose epilogue applies bias, tanh, shortcut or tanh' in
// registers.  Widths are padded to 256 with zero weights and biases, so the
// padded columns stay exactly zero.
//
// Then dT (dE/dT from dE/dD through D = T<^T T), the per-atom energy, and
// deterministic FP64 sums of the energy and virial.

#include "dp_internal.h"
#include "emb_common.h"

#include <type_traits>

namespace dp {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

namespace {

template <typename TA> struct MMT;
template <> struct MMT<double> { using acc = double; using accv = d4v; static constexpr int VEC = 2; };
template <> struct MMT<float> { using acc = float; using accv = f4v; static constexpr int VEC = 4; };
template <> struct MMT<__bf16> { using acc = float; using accv = f4v; static constexpr int VEC = 8; };

// One K-group (4 lanes-groups x VEC elements) of MFMA on 16-byte fragments.
// For the 4-deep FP32/FP64 instructions the VEC elements of a fragment feed
// VEC instructions; lane group q then holds k = q*VEC + v of the group in the
// v-th one, the same mapping for A and B, so the group's sum is complete.
__device__ inline void mfma_frag(const uint4 &a, const uint4 &b, d4v &c)
{
    double2 x = __builtin_bit_cast(double2, a), y = __builtin_bit_cast(double2, b);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, y.y, c, 0, 0, 0);
}
__device__ inline void mfma_frag_f32(const uint4 &a, const uint4 &b, f4v &c)
{
    float4 x = __builtin_bit_cast(float4, a), y = __builtin_bit_cast(float4, b);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, y.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, y.y, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, y.z, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, y.w, c, 0, 0, 0);
}
__device__ inline void mfma_frag_bf16(const uint4 &a, const uint4 &b, f4v &c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b),
                                                c, 0, 0, 0);
}

template <typename TA, typename AV>
__device__ inline void mfma_any(const uint4 &a, const uint4 &b, AV &c)
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
__device__ inline double tanh_r(double v) { return tanh(v); }

}  // namespace

namespace {

constexpr int BM = 64, BN = 64, ROWB = 144;   // tile rows/cols, LDS row pitch (bytes)

template <typename TA, typename TR, int EPI>
__global__ void __launch_bounds__(256) k_gemm_nt(int M, int N, int K, const TA *__restrict__ A,
                                                 const TA *__restrict__ Bt, Epi e)
{
    using accv = typename MMT<TA>::accv;
    constexpr int VEC = MMT<TA>::VEC;
    constexpr int BK = 128 / sizeof(TA);   // 128 bytes of K per row and stage
    __shared__ __align__(16) char As[2][BM * ROWB];
    __shared__ __align__(16) char Bs[2][BN * ROWB];
    int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int row0 = blockIdx.y * BM, col0 = blockIdx.x * BN;
    int wr = wave >> 1, wc = wave & 1;
    int m = lane & 15, q = lane >> 4;

    // global -> LDS: 2 x 16 bytes of A and of B per thread and stage
    int lr[2], lc[2];
    for (int r = 0; r < 2; r++) {
        int c = tid + 256 * r;
        lr[r] = c >> 3;
        lc[r] = c & 7;
    }
    const char *Ag = reinterpret_cast<const char *>(A) + (long)row0 * K * sizeof(TA);
    const char *Bg = reinterpret_cast<const char *>(Bt) + (long)col0 * K * sizeof(TA);
    long ldb = (long)K * sizeof(TA);
    uint4 ra[2], rb[2];
    auto gload = [&](int kt) {
        for (int r = 0; r < 2; r++) {
            ra[r] = *reinterpret_cast<const uint4 *>(Ag + lr[r] * ldb + kt * 128 + lc[r] * 16);
            rb[r] = *reinterpret_cast<const uint4 *>(Bg + lr[r] * ldb + kt * 128 + lc[r] * 16);
        }
    };
    auto sstore = [&](int buf) {
        for (int r = 0; r < 2; r++) {
            *reinterpret_cast<uint4 *>(&As[buf][lr[r] * ROWB + lc[r] * 16]) = ra[r];
            *reinterpret_cast<uint4 *>(&Bs[buf][lr[r] * ROWB + lc[r] * 16]) = rb[r];
        }
    };
    accv acc[2][2];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) acc[a][b] = accv{0, 0, 0, 0};

    int KT = K / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < KT; kt++) {
        int buf = kt & 1;
        if (kt + 1 < KT) gload(kt + 1);
#pragma unroll
        for (int kg = 0; kg < 2; kg++) {
            int off = kg * 64 + q * 16;   // bytes: group kg of 4*VEC elements, lane group q
            uint4 fa[2], fb[2];
            for (int t = 0; t < 2; t++) {
                fa[t] = *reinterpret_cast<const uint4 *>(&As[buf][(wr * 32 + t * 16 + m) * ROWB + off]);
                fb[t] = *reinterpret_cast<const uint4 *>(&Bs[buf][(wc * 32 + t * 16 + m) * ROWB + off]);
            }
            for (int a = 0; a < 2; a++)
                for (int b = 0; b < 2; b++) mfma_any<TA>(fa[a], fb[b], acc[a][b]);
        }
        if (kt + 1 < KT) sstore(buf ^ 1);
        __syncthreads();
    }
    (void)VEC;

    // epilogue: acc[a][b][i] is C[row][col] with col = wc*32 + b*16 + m and
    // row = wr*32 + a*16 + r, where r = 4q + i for the FP32-accumulating
    // instructions and r = 4i + q for v_mfma_f64_16x16x4f64 (lane layouts
    // measured on gfx950)
    const TR *bias = (const TR *)e.bias;
    constexpr bool kF64 = std::is_same<TA, double>::value;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int i = 0; i < 4; i++) {
                int gm = row0 + wr * 32 + a * 16 + (kF64 ? 4 * i + q : 4 * q + i);
                int gn = col0 + wc * 32 + b * 16 + m;
                if (gm >= M) continue;
                long idx = (long)gm * N + gn;
                TR v = (TR)acc[a][b][i];
                if constexpr (EPI == EPI_LIN) {
                    ((TR *)e.out_r)[idx] = v;
                } else if constexpr (EPI == EPI_T1) {
                    TR y = tanh_r(v + bias[gn]);
                    ((TR *)e.out_r)[idx] = y;
                    if (e.out_o) store_op((TA *)e.out_o, gm, gn, N, (double)y);
                } else if constexpr (EPI == EPI_T2) {
                    TR t = tanh_r(v + bias[gn]);
                    TR y = ((const TR *)e.res)[idx] + t;
                    ((TR *)e.out_t)[idx] = t;
                    ((TR *)e.out_r)[idx] = y;
                    if (e.out_o) store_op((TA *)e.out_o, gm, gn, N, (double)y);
                } else if constexpr (EPI == EPI_T3) {
                    ((TR *)e.out_t)[idx] = tanh_r(v + bias[gn]);
                } else if constexpr (EPI == EPI_EMB) {
                    TR t = tanh_r(v + bias[gn]);
                    ((TR *)e.out_t)[idx] = t;
                    ((TR *)e.out_r)[idx] = ((const TR *)e.res)[(long)gm * e.resw + gn % e.resw] + t;
                } else if constexpr (EPI == EPI_FOLD) {
                    if (gn < e.half) {
                        const TR *res = (const TR *)e.res;
                        long r0 = (long)gm * 2 * e.half + gn, o = (long)gm * e.half + gn;
                        TR dy = res[r0] + res[r0 + e.half] + v;
                        TR t = ((const TR *)e.tt)[o];
                        store_op((TA *)e.out_o, gm, gn, e.half, (double)(dy * ((TR)1 - t * t)));
                    }
                } else {
                    TR dy = (e.resv ? ((const TR *)e.resv)[gn] : ((const TR *)e.res)[idx]) + v;
                    if (e.out_r) ((TR *)e.out_r)[idx] = dy;
                    TR t = ((const TR *)e.tt)[idx];
                    store_op((TA *)e.out_o, gm, gn, N, (double)(dy * ((TR)1 - t * t)));
                }
            }
}

// E_i = (y2 + t3) . w4 + b4 and dz3 = w4 (1 - t3^2): one wave per atom.
template <typename TA, typename TR>
__global__ void __launch_bounds__(256) k_energy(int n, const TR *__restrict__ y2, const TR *__restrict__ t3,
                                                const TR *__restrict__ w4, double b4,
                                                double *__restrict__ e_atom, TA *__restrict__ dz3)
{
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = blockIdx.x * 4 + wave;
    if (i >= n) return;
    TR acc = 0;
    for (int c = lane; c < kFitPad; c += 64) {
        long idx = (long)i * kFitPad + c;
        TR t = t3[idx];
        acc += (y2[idx] + t) * w4[c];
        if (dz3) store_op(dz3, i, c, kFitPad, (double)(w4[c] * ((TR)1 - t * t)));
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) e_atom[i] = (double)acc + b4;
}

// dT[k][c] = sum_{a<M<} dD[a][c] T[k][a] + [c<M<] sum_b dD[c][b] T[k][b]
// (D[a][b] = sum_k T[k][a] T[k][b]); one wave per atom.
template <typename TR>
__global__ void __launch_bounds__(256) k_dT(int n, const TR *__restrict__ dD, const TR *__restrict__ T,
                                            TR *__restrict__ dT)
{
    __shared__ TR Ts[4][4 * kM];
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = blockIdx.x * 4 + wave;
    if (i < n)
        for (int o = lane; o < 4 * kM; o += 64) Ts[wave][o] = T[(long)i * 4 * kM + o];
    __syncthreads();
    if (i >= n) return;
    const TR *dd = dD + (long)i * kDdim;
    const TR *Tw = Ts[wave];
    for (int o = lane; o < 4 * kM; o += 64) {
        int k = o >> 7, c = o & (kM - 1);
        TR v = 0;
        for (int a = 0; a < kMlt; a++) v += dd[a * kM + c] * Tw[k * kM + a];
        if (c < kMlt)
            for (int b = 0; b < kM; b++) v += dd[c * kM + b] * Tw[k * kM + b];
        dT[(long)i * 4 * kM + o] = v;
    }
}

// Deterministic sums: per block a fixed slice, then one block over blocks.
constexpr int kRedBlocks = 256;

__global__ void __launch_bounds__(256) k_reduce_partial(int n, const double *__restrict__ e_atom,
                                                        const double *__restrict__ w_atom,
                                                        double *__restrict__ part)
{
    __shared__ double sh[256][11];
    int per = (n + gridDim.x - 1) / gridDim.x;
    int beg = blockIdx.x * per, end = min(n, beg + per);
    double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = beg + threadIdx.x; i < end; i += 256) {
        v[0] += e_atom[i];
        if (w_atom)
            for (int q = 0; q < 9; q++) v[1 + q] += w_atom[(long)i * 9 + q];
    }
    for (int q = 0; q < 10; q++) sh[threadIdx.x][q] = v[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int q = 0; q < 10; q++) sh[threadIdx.x][q] += sh[threadIdx.x + s][q];
        __syncthreads();
    }
    if (threadIdx.x < 10) part[blockIdx.x * 10 + threadIdx.x] = sh[0][threadIdx.x];
}

__global__ void __launch_bounds__(64) k_reduce_final(int nblk, const double *__restrict__ part,
                                                     double *energy, double *virial)
{
    int q = threadIdx.x;
    if (q >= 10) return;
    double s = 0;
    for (int b = 0; b < nblk; b++) s += part[b * 10 + q];
    if (q == 0) {
        if (energy) *energy = s;
    } else if (virial) {
        virial[q - 1] = s;
    }
}

template <typename T>
__global__ void k_to_double(long n, const T *__restrict__ a, double *__restrict__ b)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)(float)a[i];
}
template <>
__global__ void k_to_double<double>(long n, const double *__restrict__ a, double *__restrict__ b)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

template <typename T>
__global__ void k_op_to_double(long n, int ncols, const T *__restrict__ a, double *__restrict__ b)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    long row = i / ncols;
    int col = (int)(i % ncols);
    if constexpr (std::is_same<T, __bf16>::value)
        b[i] = (double)(float)a[row * 3 * ncols + col] + (double)(float)a[row * 3 * ncols + 2 * ncols + col];
    else
        b[i] = (double)a[i];
}

__global__ void k_fill_zero(double *p, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_fill_zero_u32(unsigned *p, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

// ----------------------------------------------------------- launchers
template <typename TA, typename TR>
void launch_gemm(int epi, int M, int N, int K, const TA *A, const TA *Bt, const Epi &e, hipStream_t st)
{
    dim3 grid(N / BN, div_up(M, BM));
    switch (epi) {
    case EPI_LIN: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_LIN>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    case EPI_T1: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_T1>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    case EPI_T2: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_T2>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    case EPI_T3: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_T3>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    case EPI_EMB: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_EMB>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    case EPI_FOLD: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_FOLD>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    default: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_BWD>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    }
}
template void launch_gemm<double, double>(int, int, int, int, const double *, const double *, const Epi &, hipStream_t);
template void launch_gemm<float, float>(int, int, int, int, const float *, const float *, const Epi &, hipStream_t);
template void launch_gemm<__bf16, float>(int, int, int, int, const __bf16 *, const __bf16 *, const Epi &, hipStream_t);

template <typename TA, typename TR>
void launch_energy(int n, const TR *y2, const TR *t3, const TR *w4, double b4, double *e_atom, TA *dz3,
                   hipStream_t st)
{
    hipLaunchKernelGGL((k_energy<TA, TR>), dim3(div_up(n, 4)), dim3(256), 0, st, n, y2, t3, w4, b4, e_atom, dz3);
}
template void launch_energy<double, double>(int, const double *, const double *, const double *, double, double *, double *, hipStream_t);
template void launch_energy<float, float>(int, const float *, const float *, const float *, double, double *, float *, hipStream_t);
template void launch_energy<__bf16, float>(int, const float *, const float *, const float *, double, double *, __bf16 *, hipStream_t);

template <typename TR>
void launch_dT(int n, const TR *dD, const TR *T, TR *dT, hipStream_t st)
{
    hipLaunchKernelGGL((k_dT<TR>), dim3(div_up(n, 4)), dim3(256), 0, st, n, dD, T, dT);
}
template void launch_dT<double>(int, const double *, const double *, double *, hipStream_t);
template void launch_dT<float>(int, const float *, const float *, float *, hipStream_t);

void launch_reduce(int n, const double *e_atom, const double *w_atom, double *part, double *energy,
                   double *virial, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_partial, dim3(kRedBlocks), dim3(256), 0, st, n, e_atom, w_atom, part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, st, kRedBlocks, part, energy, virial);
}

template <typename T>
void launch_to_double(long n, const T *a, double *b, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL((k_to_double<T>), dim3(div_up(n, 256)), dim3(256), 0, st, n, a, b);
}
template void launch_to_double<double>(long, const double *, double *, hipStream_t);
template void launch_to_double<float>(long, const float *, double *, hipStream_t);
template void launch_to_double<__bf16>(long, const __bf16 *, double *, hipStream_t);

template <typename T>
void launch_op_to_double(int n, int ncols, const T *a, double *b, hipStream_t st)
{
    long tot = (long)n * ncols;
    if (tot > 0) hipLaunchKernelGGL((k_op_to_double<T>), dim3(div_up(tot, 256)), dim3(256), 0, st, tot, ncols, a, b);
}
template void launch_op_to_double<double>(int, int, const double *, double *, hipStream_t);
template void launch_op_to_double<float>(int, int, const float *, double *, hipStream_t);
template void launch_op_to_double<__bf16>(int, int, const __bf16 *, double *, hipStream_t);

void launch_fill_zero(double *p, long n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_zero, dim3(div_up(n, 256)), dim3(256), 0, st, p, n);
}

void launch_fill_zero_bytes(void *p, size_t nbytes, hipStream_t st)
{
    long n = (long)(nbytes / 4);
    if (n > 0) hipLaunchKernelGGL(k_fill_zero_u32, dim3(div_up(n, 256)), dim3(256), 0, st, (unsigned *)p, n);
}

}  // namespace dp
