// gemm.hip -- the fitting net's dense products on MFMA (gfx950).
//
// Every product of the fitting net (and of the plain path's embedding net) is
// C[M x N] = A[M x K] B[N x K]^T with both operands K-contiguous, done by one
// MFMA kernel whose epilogue applies bias, tanh, shortcut or tanh' in
// registers (the layer formulas are listed at the top of fit.hip).
//
// This translation unit is compiled with the MFMA results kept in ordinary
// VGPRs (the build passes -amdgpu-mfma-vgpr-form): with accumulation
// registers the compiler copied the FP64 accumulators out and back on every
// K stage of the tanh-epilogue kernels (first fitting layer 2.12 -> 1.92 ms
// on 108,000 atoms without the copies).

#include "dp_internal.h"
#include "emb_common.h"
#include "fit_common.h"

#include <type_traits>

namespace dp {

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

// Four elements of T (one column) as a native vector.
template <typename T> struct TV4;
template <> struct TV4<double> { using type = d4v; };
template <> struct TV4<float> { using type = f4v; };
template <> struct TV4<__bf16> { using type = f4v; };

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
//
// DT (first fitting layer, FP32 / FP64): A is the descriptor D = T<^T T
// (Eq. 2) of each row's atom, formed from T as each K stage is staged
// instead of read from a stored D.  K then runs in the order
// k' = b M< + a (a < M<, b < M), which the weights' copy V1tp follows, so a
// stage covers whole columns b of D: a thread keeps the T<[k][a] of its
// chunk's a in registers for the whole loop and loads the four T[k][b] of
// each stage as one vector (T is stored by column: (T_0b, .., T_3b)).  Each
// element is summed as the embedding kernel sums D (k = 0..3, fused
// multiply-adds from zero), so both forms are bit-equal.
template <typename TA, typename TR, int EPI, int TM, int TN, bool DT = false>
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

    const long ld = (long)(e.kld > 0 ? e.kld : K) * sizeof(TA);   // row length (bytes)
    const char *Ag = DT ? nullptr : reinterpret_cast<const char *>(A) + (long)row0 * ld;
    const char *Bg = reinterpret_cast<const char *>(Bt) + (long)col0 * ld;
    // register staging of the next stage (all indices compile-time)
    Stage<LA> ra;
    Stage<LB> rb;
    accv acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; a++)
#pragma unroll
        for (int b = 0; b < TN; b++) acc[a][b] = accv{0, 0, 0, 0};

    // K in whole stages, or ending in half a stage (K a multiple of BK / 2:
    // the last stage is staged whole, its second half unused)
    const int KT = (K + BK - 1) / BK;
    const int kg_last = K % BK ? 1 : 2;   // K groups of the last stage
    // DT: chunk rr of this thread is row (tid / 8) + 32 rr of the tile and
    // elements VEC (tid mod 8) .. + VEC of the stage, i.e. a = that mod M<
    // and one b per stage; rows without an atom (padding) get D = 0
    constexpr int VEC = 16 / (int)sizeof(TA);
    constexpr int NL = DT ? LA : 1;
    using TV = typename TV4<TA>::type;
    const TV *Trow[NL];
    TA tl[NL][4][VEC], tb[NL][4];
    const int pa = tid & 7;
    if constexpr (DT) {
        const TV *Tg = reinterpret_cast<const TV *>(e.dt_T);
#pragma unroll
        for (int rr = 0; rr < LA; rr++) {
            int gm = row0 + (tid >> 3) + 32 * rr;
            int atom = e.dt_ratom ? e.dt_ratom[gm] : (gm < e.dt_nlive ? gm : -1);
            Trow[rr] = Tg + (long)(atom >= 0 ? atom : 0) * kM;
#pragma unroll
            for (int v = 0; v < VEC; v++) {
                TV t = Trow[rr][(pa * VEC) % kMlt + v];
#pragma unroll
                for (int k = 0; k < 4; k++) tl[rr][k][v] = atom >= 0 ? t[k] : (TA)0;
            }
        }
    }
    // A of stage kt into registers, and from there into an LDS buffer
    auto a_load = [&](int kt) {
        if constexpr (DT) {
            const int b = (kt * BK + pa * VEC) / kMlt;
#pragma unroll
            for (int rr = 0; rr < LA; rr++) {
                TV t = Trow[rr][b];
#pragma unroll
                for (int k = 0; k < 4; k++) tb[rr][k] = t[k];
            }
        } else {
            ra.load(Ag, ld, kt, tid);
        }
    };
    auto a_store = [&](char *as) {
        if constexpr (DT) {
#pragma unroll
            for (int rr = 0; rr < LA; rr++) {
                TA d[VEC];
#pragma unroll
                for (int v = 0; v < VEC; v++) {
                    TA x = (TA)0;
#pragma unroll
                    for (int k = 0; k < 4; k++) x = fma(tl[rr][k][v], tb[rr][k], x);
                    d[v] = x;
                }
                u4v w;
                __builtin_memcpy(&w, d, 16);
                int c = tid + 256 * rr;
                *reinterpret_cast<u4v *>(as + (c >> 3) * ROWB + (c & 7) * 16) = w;
            }
        } else {
            ra.store(as, tid);
        }
    };
    a_load(0);
    rb.load(Bg, ld, 0, tid);
    a_store(As[0]);
    rb.store(Bs[0], tid);
    __syncthreads();
    for (int kt = 0; kt < KT; kt++) {
        int buf = kt & 1;
        if (kt + 1 < KT) {
            a_load(kt + 1);
            rb.load(Bg, ld, kt + 1, tid);
        }
#pragma unroll
        for (int kg = 0; kg < 2; kg++) {
            if (kt == KT - 1 && kg >= kg_last) break;
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
            a_store(As[buf ^ 1]);
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
template <typename TA, typename TR>
void launch_gemm_dt(int M, int N, const TA *Bt, const Epi &e, hipStream_t st)
{
    // FP64: 64 x 64 tiles (as launch_gemm takes for the first layer); FP32: 128 x 128
    constexpr int TM = std::is_same<TA, double>::value ? 2 : 4, TN = TM;
    constexpr int BM = 32 * TM, BN = 32 * TN;
    int ntiles = (N / BN) * div_up(M, BM);
    hipLaunchKernelGGL((k_gemm_nt<TA, TR, EPI_T1, TM, TN, true>), dim3(8 * div_up(ntiles, 8)), dim3(256), 0, st, M, N,
                       kDdim, (const TA *)nullptr, Bt, e);
}
template void launch_gemm_dt<double, double>(int, int, const double *, const Epi &, hipStream_t);
template void launch_gemm_dt<float, float>(int, int, const float *, const Epi &, hipStream_t);

template void launch_gemm<double, double>(int, int, int, int, const double *, const double *, const Epi &, hipStream_t);
template void launch_gemm<float, float>(int, int, int, int, const float *, const float *, const Epi &, hipStream_t);
template void launch_gemm<__bf16, float>(int, int, int, int, const __bf16 *, const __bf16 *, const Epi &, hipStream_t);

}  // namespace dp
