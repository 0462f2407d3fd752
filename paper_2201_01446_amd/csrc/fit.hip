// fit.hip -- fitting net on MFMA, its input gradient, and the per-atom
// glue kernels of the force step (gfx950).
//
// Fitting net (paper Sec. 2.1): y1 = tanh(D V1 + c1); y2 = y1 + tanh(y1 V2 + c2);
// y3 = y2 + tanh(y2 V3 + c3); E_i = y3 . w4 + b4 (shortcuts between the
// equal-width layers, linear output).  Its input gradient for the forces:
//   dz3 = w4 (1 - t3^2);  dy2 = w4 + dz3 V3^T;  dz2 = dy2 (1 - t2^2);
//   dy1 = dy2 + dz2 V2^T; dz1 = dy1 (1 - y1^2); dD = dz1 V1^T,
// with t_k the tanh outputs.  The first layer and dD are products of the
// GEMM in gemm.hip; the 256-wide layers, the energy and their gradients down
// to dz1 are fused here (k_fit_tail), with k_energy for the mixed-precision
// mode, whose 256-wide layers are GEMMs too.  Widths are padded to 256 with
// zero weights and biases, so the padded columns stay exactly zero.
//
// Then dT (dE/dT from dE/dD through D = T<^T T), the per-atom energy, and
// deterministic FP64 sums of the energy and virial.

#include "dp_internal.h"
#include "emb_common.h"
#include "fit_common.h"

#include <type_traits>

namespace dp {

namespace {

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
    int nc = 0;                       // chunks of K per product (the net's width; the rest is zero padding)
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
// kTailCT column tiles, over K = 256.  Enters after a barrier that follows the
// last writes of As and the last reads of Bs; leaves after one that follows
// the last reads of both.
template <typename T>
__device__ inline void tail_gemm(const char *As, char *Bs, const T *__restrict__ Bt,
                                 typename MMT<T>::accv (&acc)[kTailCT], int tid, int rg, int ch, int m, int q, int NC)
{
    using accv = typename MMT<T>::accv;
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
    tail_gemm<T>(As, Bs, V2t + wo, acc, tid, rg, ch, m, q, ta.nc);
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
    tail_gemm<T>(As, Bs, V3t + wo, acc, tid, rg, ch, m, q, ta.nc);
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
    tail_gemm<T>(As, Bs, V3 + wo, acc, tid, rg, ch, m, q, ta.nc);
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
    tail_gemm<T>(As, Bs, V2 + wo, acc, tid, rg, ch, m, q, ta.nc);
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
__global__ void k_tcol_to_double(long n, const T *__restrict__ a, double *__restrict__ b)
{
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;   // output element (i, k, c)
    if (idx >= n) return;
    long i = idx / (4 * kM);
    int k = (int)(idx / kM % 4), c = (int)(idx % kM);
    b[idx] = (double)a[(i * kM + c) * 4 + k];
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
    // K: the net's width in 64-byte chunks (the weights are zero past it)
    ta.nc = std::min(Tail<T>::NC, div_up(tl.width * (int)sizeof(T), 64));
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
void launch_tcol_to_double(int n, const T *a, double *b, hipStream_t st)
{
    long tot = (long)n * 4 * kM;
    if (tot > 0) hipLaunchKernelGGL((k_tcol_to_double<T>), dim3(div_up(tot, 256)), dim3(256), 0, st, tot, a, b);
}
template void launch_tcol_to_double<double>(int, const double *, double *, hipStream_t);
template void launch_tcol_to_double<float>(int, const float *, double *, hipStream_t);

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
