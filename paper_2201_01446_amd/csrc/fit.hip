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
__device__ inline double tanh_r(double v) { return tanh(v); }

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
    if (!tab) return tanh(x);
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

namespace {

constexpr int ROWB = 144;   // LDS row pitch (bytes): 128 bytes of K + 16 of padding

typedef __bf16 bf4v __attribute__((ext_vector_type(4)));

// Four consecutive GEMM-operand elements (row gm, columns gn..gn+3) as FP32
// or as the BF16 [hi | hi | lo] split.
__device__ inline void store_op4(float *p, long gm, int gn, int N, f4v y)
{
    *reinterpret_cast<f4v *>(p + gm * N + gn) = y;
}
__device__ inline void store_op4(__bf16 *p, long gm, int gn, int N, f4v y)
{
    bf4v hi, lo;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        hi[j] = (__bf16)y[j];
        lo[j] = (__bf16)(y[j] - (float)hi[j]);
    }
    __bf16 *r = p + gm * 3 * N;
    *reinterpret_cast<bf4v *>(r + gn) = hi;
    *reinterpret_cast<bf4v *>(r + N + gn) = hi;
    *reinterpret_cast<bf4v *>(r + 2 * N + gn) = lo;
}

// The epilogue of an FP32-accumulating GEMM on C[gm][gn..gn+3] (see Epi).
template <typename TA, int EPI>
__device__ inline void epi4(const Epi &e, const float *bias, const float *resv, f4v v, int gm, int gn, int N)
{
    long idx = (long)gm * N + gn;
    auto ld = [&](const void *p) { return *reinterpret_cast<const f4v *>((const float *)p + idx); };
    auto st = [&](void *p, f4v x) { *reinterpret_cast<f4v *>((float *)p + idx) = x; };
    if constexpr (EPI == EPI_LIN) {
        st(e.out_r, v);
    } else if constexpr (EPI == EPI_BWD) {
        f4v dy = (resv ? *reinterpret_cast<const f4v *>(resv + gn) : ld(e.res)) + v;
        if (e.out_r) st(e.out_r, dy);
        f4v t = ld(e.tt), o;
#pragma unroll
        for (int j = 0; j < 4; j++) o[j] = dy[j] * (1.f - t[j] * t[j]);
        store_op4((TA *)e.out_o, gm, gn, N, o);
    } else {
        f4v b = *reinterpret_cast<const f4v *>(bias + gn), t;
#pragma unroll
        for (int j = 0; j < 4; j++) t[j] = tanh_e(v[j] + b[j], e.tanh_tab);
        if constexpr (EPI == EPI_T1) {
            st(e.out_r, t);
            if (e.out_o) store_op4((TA *)e.out_o, gm, gn, N, t);
        } else if constexpr (EPI == EPI_T2) {
            f4v y = ld(e.res) + t;
            st(e.out_t, t);
            st(e.out_r, y);
            if (e.out_o) store_op4((TA *)e.out_o, gm, gn, N, y);
        } else {
            st(e.out_t, t);
        }
    }
}

// N 16-byte chunks of a stage held by one thread: chunk r of thread tid is
// row (tid + 256 r) / 8, byte column 16 ((tid + 256 r) mod 8) of the tile.
template <int N>
struct Stage {
    u4v v;
    Stage<N - 1> rest;
    __device__ __attribute__((always_inline)) void load(const char *g, long ld, int kt, int tid)
    {
        int c = tid + 256 * (N - 1);
        v = *reinterpret_cast<const u4v *>(g + (c >> 3) * ld + kt * 128 + (c & 7) * 16);
        rest.load(g, ld, kt, tid);
    }
    __device__ __attribute__((always_inline)) void store(char *lds, int tid) const
    {
        int c = tid + 256 * (N - 1);
        *reinterpret_cast<u4v *>(lds + (c >> 3) * ROWB + (c & 7) * 16) = v;
        rest.store(lds, tid);
    }
};
template <>
struct Stage<0> {
    __device__ inline void load(const char *, long, int, int) {}
    __device__ inline void store(char *, int) const {}
};

// C[M x N] = A[M x K] Bt[N x K]^T with the epilogue EPI.  Block: 4 waves in a
// 2 x 2 arrangement, each wave TM x TN MFMA tiles of 16 x 16, so the block
// tile is BM = 32 TM by BN = 32 TN.  K advances 128 bytes per stage through a
// double-buffered LDS copy (16-byte global loads staged in registers).  The
// grid is 1-D: tile t goes to block (t mod 8) * (T / 8) + t / 8 order, i.e.
// consecutive tiles (the column tiles of one row tile first) land on the same
// XCD, whose L2 then serves the shared A rows.
template <typename TA, typename TR, int EPI, int TM, int TN>
__global__ void __launch_bounds__(256) k_gemm_nt(int M, int N, int K, const TA *__restrict__ A,
                                                 const TA *__restrict__ Bt, Epi e)
{
    using accv = typename MMT<TA>::accv;
    constexpr int BM = 32 * TM, BN = 32 * TN;
    constexpr int BK = 128 / sizeof(TA);   // elements of K per row and stage
    constexpr int LA = BM * 8 / 256, LB = BN * 8 / 256;   // 16-byte chunks per thread
    // one LDS block: the double-buffered A and B stages, reused by the
    // epilogue to stage the C tile
    __shared__ __align__(16) char smem[2 * BM * ROWB + 2 * BN * ROWB];
    char (*As)[BM * ROWB] = reinterpret_cast<char (*)[BM * ROWB]>(smem);
    char (*Bs)[BN * ROWB] = reinterpret_cast<char (*)[BN * ROWB]>(smem + 2 * BM * ROWB);
    int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // XCD-aware tile order
    int ntn = N / BN, ntm = (M + BM - 1) / BM;
    int ntiles = ntn * ntm;
    int pid = blockIdx.x;
    int per = (ntiles + 7) / 8;
    int tile = (pid % 8) * per + pid / 8;
    if (tile >= ntiles) return;
    int row0 = (tile / ntn) * BM, col0 = (tile % ntn) * BN;
    int wr = wave >> 1, wc = wave & 1;
    int m = lane & 15, q = lane >> 4;
    // rows grouped by atom type: the tile's group selects the weights
    int ty = 0;
    for (int g = 1; g < e.ntr; g++) ty += row0 >= e.trow[g] ? 1 : 0;
    Bt += ty * e.bstride;

    const char *Ag = reinterpret_cast<const char *>(A) + (long)row0 * K * sizeof(TA);
    const char *Bg = reinterpret_cast<const char *>(Bt) + (long)col0 * K * sizeof(TA);
    long ld = (long)K * sizeof(TA);
    // register staging of the next stage (all indices compile-time)
    Stage<LA> ra;
    Stage<LB> rb;
    accv acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; a++)
#pragma unroll
        for (int b = 0; b < TN; b++) acc[a][b] = accv{0, 0, 0, 0};

    int KT = K / BK;
    ra.load(Ag, ld, 0, tid);
    rb.load(Bg, ld, 0, tid);
    ra.store(As[0], tid);
    rb.store(Bs[0], tid);
    __syncthreads();
    for (int kt = 0; kt < KT; kt++) {
        int buf = kt & 1;
        if (kt + 1 < KT) {
            ra.load(Ag, ld, kt + 1, tid);
            rb.load(Bg, ld, kt + 1, tid);
        }
#pragma unroll
        for (int kg = 0; kg < 2; kg++) {
            int off = kg * 64 + q * 16;   // bytes: group kg of 4*VEC elements, lane group q
            u4v fa[TM], fb[TN];
#pragma unroll
            for (int t = 0; t < TM; t++)
                fa[t] = *reinterpret_cast<const u4v *>(&As[buf][(wr * 16 * TM + t * 16 + m) * ROWB + off]);
#pragma unroll
            for (int t = 0; t < TN; t++)
                fb[t] = *reinterpret_cast<const u4v *>(&Bs[buf][(wc * 16 * TN + t * 16 + m) * ROWB + off]);
#pragma unroll
            for (int a = 0; a < TM; a++)
#pragma unroll
                for (int b = 0; b < TN; b++) mfma_any<TA>(fa[a], fb[b], acc[a][b]);
        }
        if (kt + 1 < KT) {
            ra.store(As[buf ^ 1], tid);
            rb.store(Bs[buf ^ 1], tid);
        }
        __syncthreads();
    }

    // FP32-accumulating tiles of the fitting net: C goes through LDS so that
    // the epilogue reads its operands and writes its results as whole rows
    // of 16-byte accesses
    constexpr bool kStaged = !std::is_same<TA, double>::value && TM == 4 && TN == 4 &&
                             (EPI == EPI_LIN || EPI == EPI_T1 || EPI == EPI_T2 || EPI == EPI_T3 || EPI == EPI_BWD);
    if constexpr (kStaged) {
        constexpr int CP = BN + 4;   // staged row pitch (floats)
        static_assert(BM * CP * 4 <= 2 * BM * ROWB + 2 * BN * ROWB, "C tile must fit the stage buffers");
        float *Cs = reinterpret_cast<float *>(smem);
        // (the main loop ends with a barrier: every wave is done with As / Bs)
#pragma unroll
        for (int a = 0; a < TM; a++)
#pragma unroll
            for (int b = 0; b < TN; b++)
#pragma unroll
                for (int i = 0; i < 4; i++)
                    Cs[(wr * 16 * TM + a * 16 + 4 * q + i) * CP + wc * 16 * TN + b * 16 + m] = acc[a][b][i];
        __syncthreads();
        const float *bias4 = e.bias ? (const float *)e.bias + ty * e.vstride : nullptr;
        const float *resv4 = e.resv ? (const float *)e.resv + ty * e.vstride : nullptr;
        constexpr int CH = BN / 4;               // 16-byte chunks per row
        constexpr int NCH = BM * CH / 256;       // chunks per thread
#pragma unroll 4
        for (int r = 0; r < NCH; r++) {
            int k = tid + 256 * r;
            int row = k / CH, c4 = (k % CH) * 4;
            int gm = row0 + row, gn = col0 + c4;
            if (gm >= M) continue;
            f4v v = *reinterpret_cast<const f4v *>(&Cs[row * CP + c4]);
            epi4<TA, EPI>(e, bias4, resv4, v, gm, gn, N);
        }
        return;
    }

    // epilogue: acc[a][b][i] is C[row][col] with col = wc*16TN + b*16 + m and
    // row = wr*16TM + a*16 + r, where r = 4q + i for the FP32-accumulating
    // instructions and r = 4i + q for v_mfma_f64_16x16x4f64 (lane layouts
    // measured on gfx950)
    const TR *bias = e.bias ? (const TR *)e.bias + ty * e.vstride : nullptr;
    const TR *resv = e.resv ? (const TR *)e.resv + ty * e.vstride : nullptr;
    constexpr bool kF64 = std::is_same<TA, double>::value;
#pragma unroll
    for (int a = 0; a < TM; a++)
#pragma unroll
        for (int b = 0; b < TN; b++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                int gm = row0 + wr * 16 * TM + a * 16 + (kF64 ? 4 * i + q : 4 * q + i);
                int gn = col0 + wc * 16 * TN + b * 16 + m;
                if (gm >= M) continue;
                long idx = (long)gm * N + gn;
                TR v = (TR)acc[a][b][i];
                if constexpr (EPI == EPI_LIN) {
                    ((TR *)e.out_r)[idx] = v;
                } else if constexpr (EPI == EPI_T1) {
                    TR y = tanh_e(v + bias[gn], tanh_table_for(e, TR()));
                    ((TR *)e.out_r)[idx] = y;
                    if (e.out_o) store_op((TA *)e.out_o, gm, gn, N, (double)y);
                } else if constexpr (EPI == EPI_T2) {
                    TR t = tanh_e(v + bias[gn], tanh_table_for(e, TR()));
                    TR y = ((const TR *)e.res)[idx] + t;
                    ((TR *)e.out_t)[idx] = t;
                    ((TR *)e.out_r)[idx] = y;
                    if (e.out_o) store_op((TA *)e.out_o, gm, gn, N, (double)y);
                } else if constexpr (EPI == EPI_T3) {
                    ((TR *)e.out_t)[idx] = tanh_e(v + bias[gn], tanh_table_for(e, TR()));
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
                    TR dy = (resv ? resv[gn] : ((const TR *)e.res)[idx]) + v;
                    if (e.out_r) ((TR *)e.out_r)[idx] = dy;
                    TR t = ((const TR *)e.tt)[idx];
                    store_op((TA *)e.out_o, gm, gn, N, (double)(dy * ((TR)1 - t * t)));
                }
            }
}

// E_i = (y2 + t3) . w4 + b4 and dz3 = w4 (1 - t3^2): one wave per row.
// Several types: w4 and b4 of the row's type group, E to the row's atom
// (pad rows only get dz3, which nothing reads back).
template <typename TA, typename TR>
__global__ void __launch_bounds__(256) k_energy(int rows, const TR *__restrict__ y2, const TR *__restrict__ t3,
                                                const TR *__restrict__ w4_all, RowTypes rt,
                                                double *__restrict__ e_atom, TA *__restrict__ dz3)
{
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = blockIdx.x * 4 + wave;
    if (i >= rows) return;
    int ty = 0;
    for (int g = 1; g < rt.ntr; g++) ty += i >= rt.trow[g] ? 1 : 0;
    const TR *w4 = w4_all + ty * kFitB;
    TR acc = 0;
    for (int c = lane; c < kFitPad; c += 64) {
        long idx = (long)i * kFitPad + c;
        TR t = t3[idx];
        acc += (y2[idx] + t) * w4[c];
        if (dz3) store_op(dz3, i, c, kFitPad, (double)(w4[c] * ((TR)1 - t * t)));
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    int atom = rt.ratom ? rt.ratom[i] : i;
    if (lane == 0 && atom >= 0) e_atom[atom] = (double)acc + rt.b4[ty];
}

// ------------------------------------------------ fused fitting-net tail
// The four 256-wide products of a force step and the energy, per tile of
// kTailBM rows, in one kernel (FP64 and FP32):
//   t2 = tanh(y1 V2 + c2), y2 = y1 + t2;   t3 = tanh(y2 V3 + c3);
//   E_i = (y2 + t3) . w4 + b4,  dz3 = w4 (1 - t3^2);
//   dy2 = w4 + dz3 V3^T, dz2 = dy2 (1 - t2^2);   dy1 = dy2 + dz2 V2^T,
//   dz1 = dy1 (1 - y1^2).
// The tile's current operand (y1, then y2, dz3, dz2) lives in LDS and each
// product's result in registers; t2 and dy2 wait in scratch arrays for the
// product that needs them (read back by the lane that wrote them).  Each
// element of the operand is read back and overwritten in place by the lane
// whose accumulator holds it.  Eight waves: wave w owns rows 16 (w mod 2)
// .. +16 and columns 64 (w / 2) .. +64 (four 16 x 16 MFMA tiles), so two
// blocks give four waves per SIMD (measured faster than four waves per
// block: FP64 1.34 -> 1.32 ms, FP32 0.63 -> 0.58 ms on 108,000 atoms).  B (the
// weights, K-contiguous) streams from L2 in chunks of 64 bytes of K, one
// chunk ahead in registers, through one LDS buffer (FP64: two barriers per
// chunk) or two (FP32: one).  Two blocks share a CU, so one block's
// epilogues and barriers overlap the other's products.  Neither LDS array is
// padded (two FP64 blocks take all 160 KB): 16-byte granules are
// XOR-swizzled by row so that the 16 rows a fragment read touches fall in
// distinct banks.
constexpr int kTailBM = 32;
constexpr int kTailThreads = 512;
constexpr int kTailCG = kTailThreads / 64 / 2;   // column groups (waves per 16 rows)
constexpr int kTailCT = 16 / kTailCG;            // 16 x 16 column tiles per wave
constexpr int kTailBChunk = kFitPad * 64;   // bytes of one staged weight chunk

template <typename T>
struct Tail {
    static constexpr int ROWB = kFitPad * (int)sizeof(T);   // operand row (bytes)
    static constexpr int NC = ROWB / 64;                    // 64-byte chunks of K per product
    static constexpr int NB = sizeof(T) == 8 ? 1 : 2;       // weight buffers
    static constexpr int LDS = kTailBM * ROWB + NB * kTailBChunk;
};

// Byte offset of granule g (16 bytes) of operand row r: granules are
// permuted within each aligned group of 16 by r mod 16.
__device__ inline int tail_a_off(int r, int rowb, int byte)
{
    return r * rowb + ((((byte >> 4) ^ (r & 15)) << 4) | (byte & 15));
}
// Byte offset of granule g (0..3) of weight row c within a staged chunk: the
// four granules of a row permuted by (c / 4) mod 4.
__device__ inline int tail_b_off(int c, int g) { return c * 64 + ((g ^ ((c >> 2) & 3)) << 4); }

// Rows of the tile (one center type per tile, as the row groups are padded
// to 128 rows) and where each row's energy goes.
struct TailArgs {
    int ntr = 0;
    int trow[kMaxTypes + 1] = {0, 0, 0, 0, 0};
    long bstride = 0;   // one type's 256 x 256 weight matrix
    int vstride = 0;    // one type's block of vectors (kFitB)
    const int *ratom = nullptr;   // several types: row -> atom (-1: pad)
    int nlive = 0;                // one type: rows below this are atoms
    double b4[kMaxTypes] = {0, 0, 0, 0};
    const void *tanh_tab = nullptr;   // table of the result type, or NULL (native tanh)
};

constexpr int kTailPieces = kTailBChunk / 16 / kTailThreads;   // 16-byte pieces of a chunk per thread

template <typename T>
__device__ inline void tail_load_chunk(u4v (&pf)[kTailPieces], const T *__restrict__ Bt, int kc, int tid)
{
    // 256 weight rows x 64 bytes: 1024 pieces of 16 bytes
#pragma unroll
    for (int r = 0; r < kTailPieces; r++) {
        int idx = tid + kTailThreads * r;
        int col = idx >> 2, part = idx & 3;
        pf[r] = *reinterpret_cast<const u4v *>(reinterpret_cast<const char *>(Bt + (long)col * kFitPad) + kc * 64 +
                                               part * 16);
    }
}

__device__ inline void tail_store_chunk(char *Bbuf, const u4v (&pf)[kTailPieces], int tid)
{
#pragma unroll
    for (int r = 0; r < kTailPieces; r++) {
        int idx = tid + kTailThreads * r;
        *reinterpret_cast<u4v *>(Bbuf + tail_b_off(idx >> 2, idx & 3)) = pf[r];
    }
}

template <typename T>
__device__ inline void tail_chunk_mfma(const char *As, const char *Bc, typename MMT<T>::accv (&acc)[kTailCT], int kc, int ar,
                                       int ch, int m, int q)
{
    u4v a = *reinterpret_cast<const u4v *>(As + tail_a_off(ar, Tail<T>::ROWB, kc * 64 + q * 16));
#pragma unroll
    for (int ct = 0; ct < kTailCT; ct++) {
        u4v b = *reinterpret_cast<const u4v *>(Bc + tail_b_off(ch * 16 * kTailCT + ct * 16 + m, q));
        mfma_any<T>(a, b, acc[ct]);
    }
}

// acc[ct] = (the tile's operand in As) x Bt^T for this wave's rows and its
// eight column tiles, over K = 256.  Enters after a barrier that follows the
// last writes of As and the last reads of Bs; leaves after one that follows
// the last reads of both.
template <typename T>
__device__ inline void tail_gemm(const char *As, char *Bs, const T *__restrict__ Bt,
                                 typename MMT<T>::accv (&acc)[kTailCT], int tid, int rg, int ch, int m, int q)
{
    using accv = typename MMT<T>::accv;
    constexpr int NC = Tail<T>::NC;
#pragma unroll
    for (int t = 0; t < kTailCT; t++) acc[t] = accv{0, 0, 0, 0};
    const int ar = rg * 16 + m;
    u4v pf[kTailPieces];
    tail_load_chunk<T>(pf, Bt, 0, tid);
    if constexpr (Tail<T>::NB == 1) {
        // one buffer: the chunk in registers goes in once every wave is done
        // with the previous one
#pragma unroll 2
        for (int kc = 0; kc < NC; kc++) {
            if (kc > 0) __syncthreads();
            tail_store_chunk(Bs, pf, tid);
            __syncthreads();
            if (kc + 1 < NC) tail_load_chunk<T>(pf, Bt, kc + 1, tid);
            tail_chunk_mfma<T>(As, Bs, acc, kc, ar, ch, m, q);
        }
    } else {
        // two buffers: the next chunk goes into the one read in the previous
        // iteration (before its barrier)
        tail_store_chunk(Bs, pf, tid);
        tail_load_chunk<T>(pf, Bt, 1, tid);
        __syncthreads();
#pragma unroll 2
        for (int kc = 0; kc < NC; kc++) {
            tail_chunk_mfma<T>(As, Bs + (kc & 1) * kTailBChunk, acc, kc, ar, ch, m, q);
            if (kc + 1 < NC) {
                tail_store_chunk(Bs + ((kc + 1) & 1) * kTailBChunk, pf, tid);
                if (kc + 2 < NC) tail_load_chunk<T>(pf, Bt, kc + 2, tid);
            }
            __syncthreads();
        }
    }
    if constexpr (Tail<T>::NB == 1) __syncthreads();
}

template <typename T, bool TAB>
__global__ void __launch_bounds__(kTailThreads, kTailThreads / 128) k_fit_tail(const T *__restrict__ y1, const T *__restrict__ V2t,
                                                                const T *__restrict__ V3t, const T *__restrict__ V3,
                                                                const T *__restrict__ V2, const T *__restrict__ fb,
                                                                TailArgs ta, double *__restrict__ e_atom,
                                                                T *__restrict__ dz1, T *__restrict__ t2s,
                                                                T *__restrict__ dy2s)
{
    using accv = typename MMT<T>::accv;
    constexpr int ROWB = Tail<T>::ROWB;
    constexpr bool kF64 = std::is_same<T, double>::value;
    __shared__ __align__(16) char smem[Tail<T>::LDS];
    char *As = smem;
    char *Bs = smem + kTailBM * ROWB;
    // the energy's per-half row partials [2][kTailBM], in the weight buffers
    // while no product runs
    double *Ep = reinterpret_cast<double *>(Bs);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int rg = wave & 1, ch = wave >> 1, m = lane & 15, q = lane >> 4;   // ch: column group
    const long row0 = (long)blockIdx.x * kTailBM;
    int ty = 0;
    for (int g = 1; g < ta.ntr; g++) ty += row0 >= ta.trow[g] ? 1 : 0;
    const long wo = ty * ta.bstride;
    const T *c2 = fb + ty * ta.vstride + kFitPad, *c3 = c2 + kFitPad, *w4 = c3 + kFitPad;
    // the table switch is a template parameter, so the epilogues' elements
    // are free of branches and interleave
    const T *tab = TAB ? reinterpret_cast<const T *>(ta.tanh_tab) : nullptr;

    // the y1 tile into the operand buffer (16-byte granules)
    constexpr int PR = ROWB / 16;
    for (int k = tid; k < kTailBM * PR; k += kTailThreads) {
        int r = k / PR, c = k % PR;
        *reinterpret_cast<u4v *>(As + tail_a_off(r, ROWB, c * 16)) =
            *reinterpret_cast<const u4v *>(reinterpret_cast<const char *>(y1 + (row0 + r) * kFitPad) + c * 16);
    }
    __syncthreads();
    // element (ct, i) of this lane: tile row and column (MFMA result layouts
    // measured on gfx950: FP64 row 4i + q, FP32 row 4q + i; column m)
    auto erow = [&](int i) { return rg * 16 + (kF64 ? 4 * i + q : 4 * q + i); };
    auto ecol = [&](int ct) { return ch * 16 * kTailCT + ct * 16 + m; };
    auto el = [&](int ct, int i) -> T & {
        return *reinterpret_cast<T *>(As + tail_a_off(erow(i), ROWB, ecol(ct) * (int)sizeof(T)));
    };

    // t2 (from the first product to the third) and dy2 (third to fourth)
    // wait in the scratch arrays t2s and dy2s, each element written and read
    // back by the same lane (registers are taken by the accumulators)
    auto gel = [&](T *p, int ct, int i) -> T & { return p[(row0 + erow(i)) * kFitPad + ecol(ct)]; };
    accv acc[kTailCT];
    // y2 = y1 + tanh(y1 V2 + c2)
    tail_gemm<T>(As, Bs, V2t + wo, acc, tid, rg, ch, m, q);
#pragma unroll
    for (int ct = 0; ct < kTailCT; ct++) {
        T b = c2[ecol(ct)];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            T t = tanh_e((T)acc[ct][i] + b, tab);
            gel(t2s, ct, i) = t;
            el(ct, i) += t;
        }
    }
    __syncthreads();
    // t3 = tanh(y2 V3 + c3); E = (y2 + t3) . w4 + b4; dz3 = w4 (1 - t3^2)
    tail_gemm<T>(As, Bs, V3t + wo, acc, tid, rg, ch, m, q);
    T es[4] = {0, 0, 0, 0};
#pragma unroll
    for (int ct = 0; ct < kTailCT; ct++) {
        T b = c3[ecol(ct)], w = w4[ecol(ct)];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            T t = tanh_e((T)acc[ct][i] + b, tab);
            T &o = el(ct, i);
            es[i] += (o + t) * w;
            o = w * ((T)1 - t * t);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) es[i] += __shfl_xor(es[i], off);   // the 16 columns of a tile row
        if (m == 0) Ep[ch * kTailBM + erow(i)] = (double)es[i];
    }
    __syncthreads();
    if (tid < kTailBM) {
        long row = row0 + tid;
        int atom = ta.ratom ? ta.ratom[row] : (row < ta.nlive ? (int)row : -1);
        T e = (T)Ep[tid];
#pragma unroll
        for (int g = 1; g < kTailCG; g++) e += (T)Ep[g * kTailBM + tid];
        if (atom >= 0) e_atom[atom] = (double)e + ta.b4[ty];
    }
    __syncthreads();
    // dy2 = w4 + dz3 V3^T; dz2 = dy2 (1 - t2^2)
    tail_gemm<T>(As, Bs, V3 + wo, acc, tid, rg, ch, m, q);
#pragma unroll
    for (int ct = 0; ct < kTailCT; ct++) {
        T w = w4[ecol(ct)];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            T dy = w + (T)acc[ct][i];
            T t = gel(t2s, ct, i);
            gel(dy2s, ct, i) = dy;
            el(ct, i) = dy * ((T)1 - t * t);
        }
    }
    __syncthreads();
    // dy1 = dy2 + dz2 V2^T; dz1 = dy1 (1 - y1^2), written out through LDS
    tail_gemm<T>(As, Bs, V2 + wo, acc, tid, rg, ch, m, q);
#pragma unroll
    for (int ct = 0; ct < kTailCT; ct++) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            T y = y1[(row0 + erow(i)) * kFitPad + ecol(ct)];
            el(ct, i) = (gel(dy2s, ct, i) + (T)acc[ct][i]) * ((T)1 - y * y);
        }
    }
    __syncthreads();
    for (int k = tid; k < kTailBM * PR; k += kTailThreads) {
        int r = k / PR, c = k % PR;
        *reinterpret_cast<u4v *>(reinterpret_cast<char *>(dz1 + (row0 + r) * kFitPad) + c * 16) =
            *reinterpret_cast<const u4v *>(As + tail_a_off(r, ROWB, c * 16));
    }
}

// dT[k][c] = sum_{a<M<} dD[a][c] T[k][a] + [c<M<] sum_b dD[c][b] T[k][b]
// (D[a][b] = sum_k T[k][a] T[k][b]); one wave per atom.  The atom's dD
// (M< x M) and T (4 x M) are staged in LDS with rows padded by one element,
// so the row-wise dot products of the second term are free of bank
// conflicts; every lane then does the same amount of work.
template <typename TR>
__global__ void __launch_bounds__(256) k_dT(int n, const TR *__restrict__ dD, const TR *__restrict__ T,
                                            TR *__restrict__ dT)
{
    constexpr int P = kM + 1;   // padded row pitch
    __shared__ TR sD[4][kMlt * P];
    __shared__ TR sT[4][4 * P];
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = blockIdx.x * 4 + wave;
    bool live = i < n;
    if (live) {
        const TR *dd = dD + (long)i * kDdim;
        for (int o = lane; o < kDdim; o += 64) sD[wave][(o >> 7) * P + (o & (kM - 1))] = dd[o];
        const TR *tt = T + (long)i * 4 * kM;
        for (int o = lane; o < 4 * kM; o += 64) sT[wave][(o >> 7) * P + (o & (kM - 1))] = tt[o];
    }
    __syncthreads();
    if (!live) return;
    const TR *D = sD[wave], *Tw = sT[wave];
    // first term: lane owns columns c = lane and lane + 64, all four k
    TR acc[4][2];
    for (int k = 0; k < 4; k++) acc[k][0] = acc[k][1] = 0;
    for (int a = 0; a < kMlt; a++) {
        TR d0 = D[a * P + lane], d1 = D[a * P + lane + 64];
        for (int k = 0; k < 4; k++) {
            TR t = Tw[k * P + a];
            acc[k][0] += d0 * t;
            acc[k][1] += d1 * t;
        }
    }
    // second term: lane owns (c, k) = (lane / 4, lane % 4), c < M<
    int c2 = lane >> 2, k2 = lane & 3;
    TR s2 = 0;
    for (int b = 0; b < kM; b++) s2 += D[c2 * P + b] * Tw[k2 * P + b];
    TR *out = dT + (long)i * 4 * kM;
    for (int k = 0; k < 4; k++) {
        out[k * kM + lane + 64] = acc[k][1];
        // columns < M< also receive the second term (held by lane 4c + k)
        TR extra = __shfl(s2, (lane & 15) * 4 + k);
        out[k * kM + lane] = acc[k][0] + (lane < kMlt ? extra : (TR)0);
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

// Sum of the kRedBlocks partials: one per thread, then a tree in LDS
// (a fixed order).
__global__ void __launch_bounds__(256) k_reduce_final(int nblk, const double *__restrict__ part,
                                                      double *energy, double *virial, int *flags)
{
    __shared__ double sh[256][11];
    int t = threadIdx.x;
    for (int q = 0; q < 10; q++) sh[t][q] = t < nblk ? part[t * 10 + q] : 0.0;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
            for (int q = 0; q < 10; q++) sh[t][q] += sh[t + s][q];
        __syncthreads();
    }
    if (t == 0 && energy) *energy = sh[0][0];
    if (t >= 1 && t < 10 && virial) virial[t - 1] = sh[0][t];
    if (t < 10 && !isfinite(sh[0][t])) atomicOr(&flags[kFlagNonFinite], 1);
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
__global__ void k_op_to_double(long n, int ncols, const T *__restrict__ a, const int *__restrict__ rowmap,
                               double *__restrict__ b)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    long atom = i / ncols;
    long row = rowmap ? rowmap[atom] : atom;
    int col = (int)(i % ncols);
    if constexpr (std::is_same<T, __bf16>::value)
        b[i] = (double)(float)a[row * 3 * ncols + col] + (double)(float)a[row * 3 * ncols + 2 * ncols + col];
    else
        b[i] = (double)a[row * ncols + col];
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
template <typename TA, typename TR, int TM, int TN>
static void launch_gemm_t(int epi, int M, int N, int K, const TA *A, const TA *Bt, const Epi &e, hipStream_t st)
{
    constexpr int BM = 32 * TM, BN = 32 * TN;
    int ntiles = (N / BN) * div_up(M, BM);
    dim3 grid(8 * div_up(ntiles, 8));
    switch (epi) {
    case EPI_LIN: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_LIN, TM, TN>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    case EPI_T1: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_T1, TM, TN>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    case EPI_T2: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_T2, TM, TN>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    case EPI_T3: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_T3, TM, TN>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    case EPI_EMB: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_EMB, TM, TN>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    case EPI_FOLD: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_FOLD, TM, TN>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    default: hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_BWD, TM, TN>), grid, dim3(256), 0, st, M, N, K, A, Bt, e); break;
    }
}

// Tile choice: 128 x 128 when M and N allow it (M padded to 128 rows), else
// 64 x 64.  FP64 takes 64 x 64 tiles for the first fitting layer and its
// input gradient too: four blocks (16 waves) per CU instead of two, and
// many more tiles for the last round (measured on 108,000 atoms: first layer
// 2.35 ms with 64 x 128 tiles, 2.65 with 128 x 128, 2.11 with 64 x 64); the
// FP32 ones keep 128 x 128 and their LDS-staged epilogue.
template <typename TA, typename TR>
void launch_gemm(int epi, int M, int N, int K, const TA *A, const TA *Bt, const Epi &e, hipStream_t st)
{
    if (std::is_same<TA, double>::value && (N == kFitPad || N == kDdim) && M % 64 == 0)
        launch_gemm_t<TA, TR, 2, 2>(epi, M, N, K, A, Bt, e, st);
    else if (N % 128 == 0 && M % 128 == 0) launch_gemm_t<TA, TR, 4, 4>(epi, M, N, K, A, Bt, e, st);
    else launch_gemm_t<TA, TR, 2, 2>(epi, M, N, K, A, Bt, e, st);
}
template void launch_gemm<double, double>(int, int, int, int, const double *, const double *, const Epi &, hipStream_t);
template void launch_gemm<float, float>(int, int, int, int, const float *, const float *, const Epi &, hipStream_t);
template void launch_gemm<__bf16, float>(int, int, int, int, const __bf16 *, const __bf16 *, const Epi &, hipStream_t);

template <typename TA, typename TR>
void launch_energy(int rows, const TR *y2, const TR *t3, const TR *w4, const RowTypes &rt, double *e_atom, TA *dz3,
                   hipStream_t st)
{
    hipLaunchKernelGGL((k_energy<TA, TR>), dim3(div_up(rows, 4)), dim3(256), 0, st, rows, y2, t3, w4, rt, e_atom,
                       dz3);
}
template void launch_energy<double, double>(int, const double *, const double *, const double *, const RowTypes &, double *, double *, hipStream_t);
template void launch_energy<float, float>(int, const float *, const float *, const float *, const RowTypes &, double *, float *, hipStream_t);
template void launch_energy<__bf16, float>(int, const float *, const float *, const float *, const RowTypes &, double *, __bf16 *, hipStream_t);

template <typename T>
void launch_fit_tail(int rows, const T *y1, const FitWeights &fw, const T *fb, const TailLaunch &tl, double *e_atom,
                     T *dz1, T *t2s, T *dy2s, hipStream_t st)
{
    TailArgs ta;
    ta.ntr = tl.ntr;
    for (int t = 0; t <= kMaxTypes; t++) ta.trow[t] = tl.trow[t];
    for (int t = 0; t < kMaxTypes; t++) ta.b4[t] = tl.b4[t];
    ta.bstride = (long)kFitPad * kFitPad;
    ta.vstride = kFitB;
    ta.ratom = tl.ratom;
    ta.nlive = tl.nlive;
    ta.tanh_tab = tl.tanh_tab;
    if (tl.tanh_tab)
        hipLaunchKernelGGL((k_fit_tail<T, true>), dim3(rows / kTailBM), dim3(kTailThreads), 0, st, y1,
                           (const T *)fw.V2t, (const T *)fw.V3t, (const T *)fw.V3, (const T *)fw.V2, fb, ta, e_atom,
                           dz1, t2s, dy2s);
    else
        hipLaunchKernelGGL((k_fit_tail<T, false>), dim3(rows / kTailBM), dim3(kTailThreads), 0, st, y1,
                           (const T *)fw.V2t, (const T *)fw.V3t, (const T *)fw.V3, (const T *)fw.V2, fb, ta, e_atom,
                           dz1, t2s, dy2s);
}
template void launch_fit_tail<double>(int, const double *, const FitWeights &, const double *, const TailLaunch &,
                                      double *, double *, double *, double *, hipStream_t);
template void launch_fit_tail<float>(int, const float *, const FitWeights &, const float *, const TailLaunch &,
                                     double *, float *, float *, float *, hipStream_t);

template <typename TR>
void launch_dT(int n, const TR *dD, const TR *T, TR *dT, hipStream_t st)
{
    hipLaunchKernelGGL((k_dT<TR>), dim3(div_up(n, 4)), dim3(256), 0, st, n, dD, T, dT);
}
template void launch_dT<double>(int, const double *, const double *, double *, hipStream_t);
template void launch_dT<float>(int, const float *, const float *, float *, hipStream_t);

void launch_reduce(int n, const double *e_atom, const double *w_atom, double *part, double *energy,
                   double *virial, int *flags, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce_partial, dim3(kRedBlocks), dim3(256), 0, st, n, e_atom, w_atom, part);
    static_assert(kRedBlocks <= 256, "one partial per thread");
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, kRedBlocks, part, energy, virial, flags);
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
void launch_op_to_double(int n, int ncols, const T *a, const int *row, double *b, hipStream_t st)
{
    long tot = (long)n * ncols;
    if (tot > 0)
        hipLaunchKernelGGL((k_op_to_double<T>), dim3(div_up(tot, 256)), dim3(256), 0, st, tot, ncols, a, row, b);
}
template void launch_op_to_double<double>(int, int, const double *, const int *, double *, hipStream_t);
template void launch_op_to_double<float>(int, int, const float *, const int *, double *, hipStream_t);
template void launch_op_to_double<__bf16>(int, int, const __bf16 *, const int *, double *, hipStream_t);

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
