// plain.hip -- the untabulated force step: the embedding net evaluated layer
// by layer over sel padded rows per atom, with every activation stored in
// HBM, as in the baseline the paper compresses (Sec. 2.2, Fig. 1e: the
// embedding matrix G, N_a x N_m x M, is materialised; padded rows are
// computed).  It is the speed denominator of the compressed path.
//
// Rows are (atom i, slot k < sel).  Forward:
//   k_plain_env      s, R, r_ij, ds/dr, 1/r per row (zeros, j = -1 when padded)
//   k_plain_l0       h0 = tanh(s W0 + b0)                         (Eq. 4)
//   GEMM (EPI_EMB)   h1 = [h0, h0] + tanh(h0 W1 + b1)             (Eq. 5)
//   GEMM (EPI_EMB)   G  = [h1, h1] + tanh(h1 W2 + b2)
//   k_plain_contract T = desc_scale R^T G, D = T<^T T             (Eq. 2)
// then the fitting net shared with the compressed path, and backward:
//   k_plain_dG       dG = desc_scale R dT; dz2 = dG (1 - t2^2); fold [x, x]
//   GEMM (EPI_BWD)   dh1 = fold(dG) + dz2 W2^T; dz1 = dh1 (1 - t1^2)
//   GEMM (EPI_FOLD)  dh0 = fold(dh1) + dz1 W1^T; dz0 = dh0 (1 - h0^2)
//   k_plain_force    dE/ds = dz0 . W0 + dR . u; g_ij; forces, virial

#include "dp_internal.h"
#include "emb_common.h"
#include "env.h"
#include "tanh64.h"

#include <type_traits>

namespace dp {

namespace {

template <typename real>
__device__ inline real tanh_p(real v);
template <> __device__ inline float tanh_p<float>(float v) { return tanhf(v); }
template <> __device__ inline double tanh_p<double>(double v) { return tanh_f64(v); }

template <typename T> __device__ inline T cvd(double v);
template <> __device__ inline double cvd<double>(double v) { return v; }
template <> __device__ inline float cvd<float>(double v) { return (float)v; }
template <> __device__ inline __bf16 cvd<__bf16>(double v) { return (__bf16)(float)v; }

template <typename real>
__global__ void __launch_bounds__(256) k_plain_env(int natoms, EnvArgs A, real *__restrict__ s_out,
                                                   V4<real> *__restrict__ R_out, V4<real> *__restrict__ P_out,
                                                   V4<real> *__restrict__ D_out, int *__restrict__ j_out,
                                                   int *__restrict__ nnei_out)
{
    HIP_DYNAMIC_SHARED(uint4, smem_raw)
    char *smem = reinterpret_cast<char *>(smem_raw);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = blockIdx.x * (blockDim.x >> 6) + wave;
    NbrLDS<real> L = carve<real>(smem + wave * nbr_lds_bytes<real>(A.sel, ENV_PLAIN), A.sel, ENV_PLAIN);
    bool live = i < natoms;
    int nn = 0, n_in = 0, over = 0, oob = 0;
    if (live) nn = build_env<real, ENV_PLAIN, false>(i, A, L, lane, n_in, over, oob);
    __syncthreads();
    if (!live) return;
    record_flags<real>(A, lane, n_in, over, 0);
    if (nnei_out && lane == 0) nnei_out[i] = nn;
    for (int k = lane; k < A.sel; k += 64) {
        long row = (long)i * A.sel + k;
        if (k < nn) {
            V4<real> P = L.P[k];
            s_out[row] = P.w;
            R_out[row] = L.R[k];
            P_out[row] = P;
            D_out[row] = L.Dv[k];
            j_out[row] = L.j[k];
        } else {
            // a padded row: s = 0 and R = 0, still evaluated by the net
            s_out[row] = 0;
            R_out[row] = V4<real>{0, 0, 0, 0};
            P_out[row] = V4<real>{0, 0, 0, 0};
            D_out[row] = V4<real>{0, 0, 0, 0};
            j_out[row] = -1;
        }
    }
}

template <typename real>
__global__ void k_plain_l0(long rows, const real *__restrict__ s, const real *__restrict__ W0,
                           const real *__restrict__ b0, real *__restrict__ h0)
{
    long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (id >= rows * 32) return;
    long row = id >> 5;
    int a = (int)(id & 31);
    h0[id] = tanh_p<real>(s[row] * W0[a] + b0[a]);
}

// T = sig R^T G over the sel rows of an atom, then D; one wave per atom,
// lane owns columns lane and lane + 64.
template <typename real, typename TD>
__global__ void __launch_bounds__(256) k_plain_contract(int natoms, int sel, real sigma,
                                                        const V4<real> *__restrict__ R,
                                                        const real *__restrict__ G, real *__restrict__ T_out,
                                                        TD *__restrict__ D_out)
{
    __shared__ real Ts[4][4 * kM];
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = blockIdx.x * 4 + wave;
    bool live = i < natoms;
    real acc[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    if (live) {
        for (int k = 0; k < sel; k++) {
            long row = (long)i * sel + k;
            V4<real> r = R[row];
            real g0 = G[row * kM + lane], g1 = G[row * kM + lane + 64];
            acc[0][0] = fma(r.x, g0, acc[0][0]);
            acc[1][0] = fma(r.y, g0, acc[1][0]);
            acc[2][0] = fma(r.z, g0, acc[2][0]);
            acc[3][0] = fma(r.w, g0, acc[3][0]);
            acc[0][1] = fma(r.x, g1, acc[0][1]);
            acc[1][1] = fma(r.y, g1, acc[1][1]);
            acc[2][1] = fma(r.z, g1, acc[2][1]);
            acc[3][1] = fma(r.w, g1, acc[3][1]);
        }
        for (int k = 0; k < 4; k++)
            for (int c = 0; c < 2; c++) {
                real v = sigma * acc[k][c];
                Ts[wave][k * kM + lane + 64 * c] = v;
                T_out[(long)i * 4 * kM + k * kM + lane + 64 * c] = v;
            }
    }
    __syncthreads();
    if (!live) return;
    const real *Tl = Ts[wave];
    for (int o = lane; o < kDdim; o += 64) {
        int aa = o >> 7, bb = o & (kM - 1);
        real v = Tl[aa] * Tl[bb];
        v = fma(Tl[kM + aa], Tl[kM + bb], v);
        v = fma(Tl[2 * kM + aa], Tl[2 * kM + bb], v);
        v = fma(Tl[3 * kM + aa], Tl[3 * kM + bb], v);
        store_op(D_out, i, o, kDdim, (double)v);
    }
}

// dG = sig R dT (row x 128); dz2 = dG (1 - t2^2) in place of t2; fold of the
// [h1, h1] shortcut: dGf[c] = dG[c] + dG[c + 64] in place of h1.
template <typename real>
__global__ void k_plain_dG(long rows, int sel, real sigma, const V4<real> *__restrict__ R,
                           const real *__restrict__ dT, real *__restrict__ t2dz2, real *__restrict__ h1dGf)
{
    long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (id >= rows * 64) return;
    long row = id >> 6;
    int c = (int)(id & 63);
    long atom = row / sel;
    V4<real> r = R[row];
    const real *d = dT + atom * 4 * kM;
    real g0 = sigma * (d[c] * r.x + d[kM + c] * r.y + d[2 * kM + c] * r.z + d[3 * kM + c] * r.w);
    int c2 = c + 64;
    real g1 = sigma * (d[c2] * r.x + d[kM + c2] * r.y + d[2 * kM + c2] * r.z + d[3 * kM + c2] * r.w);
    real t0 = t2dz2[row * kM + c], t1 = t2dz2[row * kM + c2];
    t2dz2[row * kM + c] = g0 * ((real)1 - t0 * t0);
    t2dz2[row * kM + c2] = g1 * ((real)1 - t1 * t1);
    h1dGf[row * 64 + c] = g0 + g1;
}

// Tabulated but unfused (the intermediate rung between the plain and the
// fused paths): G and G' = dG/ds of every row, padded rows included, written
// to memory from the table (Sec. 3.2), one thread per (row, column).
template <typename real>
__device__ inline void tab_coef(const real *tab, int th, int c, real (&a)[6])
{
    const real *p = tab + ((long)th * kM + c) * 6;
    for (int e = 0; e < 6; e++) a[e] = p[e];
}

template <typename real>
__global__ void k_tab_eval(long rows, EnvArgs A, const real *__restrict__ tab, const real *__restrict__ s,
                           real *__restrict__ G, real *__restrict__ Gp)
{
    long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (id >= rows * kM) return;
    long row = id >> 7;
    int c = (int)(id & (kM - 1));
    int th;
    real t;
    int oob = table_interval<real>(A, s[row], th, t);
    real a[6];
    tab_coef<real>(tab, th & ~kOobBit, c, a);
    real f = a[5], fp = a[5];
    for (int e = 4; e >= 1; e--) {
        f = fma(f, t, a[e]);
        fp = fma(fp, t, f);
    }
    f = fma(f, t, a[0]);
    G[id] = f;
    Gp[id] = oob ? (real)0 : fp;
}

// dE/ds through the tabulated G: sum_c (sig sum_k R_k dT[k][c]) G'[c]; one
// wave per row, lanes over columns.
template <typename real>
__global__ void __launch_bounds__(256) k_tab_dsG(long rows, int sel, real sigma, const V4<real> *__restrict__ R,
                                                 const real *__restrict__ dT, const real *__restrict__ Gp,
                                                 real *__restrict__ dsG)
{
    long row = blockIdx.x * 4L + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (row >= rows) return;
    long atom = row / sel;
    V4<real> r = R[row];
    const real *d = dT + atom * 4 * kM;
    real acc = 0;
    for (int c = lane; c < kM; c += 64) {
        real g = d[c] * r.x + d[kM + c] * r.y + d[2 * kM + c] * r.z + d[3 * kM + c] * r.w;
        acc = fma(sigma * g, Gp[row * kM + c], acc);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) dsG[row] = acc;
}

// Per atom (block), per row (thread): dE/ds through G (dz0 . W0, or the
// row's dsG in the tabulated rung) and through R (dR . u), then
// g_ij = dE_i/dr_ij; forces by atomics, virial per atom.
template <typename real>
__global__ void __launch_bounds__(256) k_plain_force(int natoms, int sel, real sigma,
                                                     const V4<real> *__restrict__ R,
                                                     const V4<real> *__restrict__ P,
                                                     const V4<real> *__restrict__ Dv, const int *__restrict__ jrow,
                                                     const real *__restrict__ G, const real *__restrict__ dz0,
                                                     const real *__restrict__ W0, const real *__restrict__ dsG_row,
                                                     const real *__restrict__ dT,
                                                     double *__restrict__ force, double *__restrict__ w_atom)
{
    __shared__ real dTs[4 * kM];
    __shared__ double red[256][12];
    int i = blockIdx.x, k = threadIdx.x;
    for (int o = k; o < 4 * kM; o += blockDim.x) dTs[o] = sigma * dT[(long)i * 4 * kM + o];
    __syncthreads();
    double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (k < sel) {
        long row = (long)i * sel + k;
        int j = jrow[row];
        if (j >= 0) {
            real dsG = 0;
            if (dsG_row) dsG = dsG_row[row];
            else
                for (int a = 0; a < 32; a++) dsG = fma(dz0[row * 32 + a], W0[a], dsG);
            real dR0 = 0, dR1 = 0, dR2 = 0, dR3 = 0;
            const real *g = G + row * kM;
            for (int e = 0; e < kM; e++) {
                real gv = g[e];
                dR0 = fma(dTs[e], gv, dR0);
                dR1 = fma(dTs[kM + e], gv, dR1);
                dR2 = fma(dTs[2 * kM + e], gv, dR2);
                dR3 = fma(dTs[3 * kM + e], gv, dR3);
            }
            V4<real> p = P[row], d = Dv[row];
            real rinv = p.z, s = p.w, sp = p.y;
            real h0 = d.x * rinv, h1 = d.y * rinv, h2 = d.z * rinv;
            real dEds = dsG + dR0 + dR1 * h0 + dR2 * h1 + dR3 * h2;
            real u0 = s * dR1, u1 = s * dR2, u2 = s * dR3;
            real udh = u0 * h0 + u1 * h1 + u2 * h2;
            real c0 = dEds * sp;
            real g0 = c0 * h0 + (u0 - udh * h0) * rinv;
            real g1 = c0 * h1 + (u1 - udh * h1) * rinv;
            real g2 = c0 * h2 + (u2 - udh * h2) * rinv;
            unsafeAtomicAdd(&force[3 * j], -(double)g0);
            unsafeAtomicAdd(&force[3 * j + 1], -(double)g1);
            unsafeAtomicAdd(&force[3 * j + 2], -(double)g2);
            acc[0] = g0; acc[1] = g1; acc[2] = g2;
            acc[3] = -d.x * g0; acc[4] = -d.x * g1; acc[5] = -d.x * g2;
            acc[6] = -d.y * g0; acc[7] = -d.y * g1; acc[8] = -d.y * g2;
            acc[9] = -d.z * g0; acc[10] = -d.z * g1; acc[11] = -d.z * g2;
        }
    }
    for (int q = 0; q < 12; q++) red[k][q] = acc[q];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (k < st)
            for (int q = 0; q < 12; q++) red[k][q] += red[k + st][q];
        __syncthreads();
    }
    if (k < 3) unsafeAtomicAdd(&force[3 * i + k], red[0][k]);
    if (k >= 3 && k < 12) w_atom[(long)i * 9 + k - 3] = red[0][k];
}

template <typename real>
struct PlainWS {
    real *s, *h0, *h1, *t1, *G, *t2;
    V4<real> *R, *P, *Dv;
    int *j;
};

template <typename real>
size_t plain_bytes(long rows)
{
    auto al = [](size_t b) { return (size_t)round_up((long)b, 256); };
    return al(rows * sizeof(real)) + al(rows * 32 * sizeof(real)) + 2 * al(rows * 64 * sizeof(real)) +
           2 * al(rows * kM * sizeof(real)) + 3 * al(rows * sizeof(V4<real>)) + al(rows * sizeof(int));
}

template <typename real>
PlainWS<real> plain_carve(void *base, long rows)
{
    char *p = (char *)base;
    auto take = [&](size_t b) {
        void *q = p;
        p += round_up((long)b, 256);
        return q;
    };
    PlainWS<real> w;
    w.s = (real *)take(rows * sizeof(real));
    w.h0 = (real *)take(rows * 32 * sizeof(real));
    w.h1 = (real *)take(rows * 64 * sizeof(real));
    w.t1 = (real *)take(rows * 64 * sizeof(real));
    w.G = (real *)take(rows * kM * sizeof(real));
    w.t2 = (real *)take(rows * kM * sizeof(real));
    w.R = (V4<real> *)take(rows * sizeof(V4<real>));
    w.P = (V4<real> *)take(rows * sizeof(V4<real>));
    w.Dv = (V4<real> *)take(rows * sizeof(V4<real>));
    w.j = (int *)take(rows * sizeof(int));
    return w;
}

}  // namespace

// Embedding weights in the GEMM layouts: W1t [64][32], W2t [128][64],
// W2 [64][128], W1p [64][64] (W1 with zero rows 32..63), W0, b0, b1, b2.
template <typename real>
struct EmbW {
    const real *W1t, *W2t, *W2, *W1p, *W0, *b0, *b1, *b2;
};

template <typename real>
static EmbW<real> emb_weights(const dp_model *m)
{
    const real *p = (const real *)(std::is_same<real, double>::value ? m->embg64 : m->embg32);
    EmbW<real> w;
    w.W1t = p;
    w.W2t = w.W1t + 64 * 32;
    w.W2 = w.W2t + 128 * 64;
    w.W1p = w.W2 + 64 * 128;
    w.W0 = w.W1p + 64 * 64;
    w.b0 = w.W0 + 32;
    w.b1 = w.b0 + 32;
    w.b2 = w.b1 + 64;
    return w;
}

template <typename real>
dp_status plain_ensure(dp_nlist *nl, long rows)
{
    size_t need = plain_bytes<real>(round_up(rows, kRowPad));
    if (nl->ws_plain_bytes >= need) return DP_OK;
    if (nl->ws_plain) DP_HIP(hipFree(nl->ws_plain));
    nl->ws_plain = nullptr;
    nl->ws_plain_bytes = 0;
    if (hipMalloc(&nl->ws_plain, need) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DP_ERR_OOM, "plain-path workspace allocation failed");
    }
    nl->ws_plain_bytes = need;
    DP_HIP(hipMemset(nl->ws_plain, 0, need));
    return DP_OK;
}

// Forward of the embedding stage: T (real) and D (TD) for every atom.
// tabulated: G from the table (materialised) instead of the network.
template <typename real, typename TD>
dp_status plain_forward(const dp_model *m, dp_nlist *nl, int n, const double *x, void *T, void *D, int *nnei,
                        hipStream_t st, bool tabulated)
{
    int sel = m->cfg.sel;
    long rows = (long)n * sel, rows_p = round_up(rows, kRowPad);
    dp_status s = plain_ensure<real>(nl, rows);
    if (s != DP_OK) return s;
    PlainWS<real> w = plain_carve<real>(nl->ws_plain, rows_p);
    EmbW<real> ew = emb_weights<real>(m);
    EnvArgs A = make_env_args(m, nl, x);
    int wpb = lds_wpb(nbr_lds_bytes<real>(A.sel, ENV_PLAIN));
    size_t lds = (size_t)wpb * nbr_lds_bytes<real>(A.sel, ENV_PLAIN);
    DP_TIMED("plain_env", st,
             hipLaunchKernelGGL((k_plain_env<real>), dim3(div_up(n, wpb)), dim3(64 * wpb), lds, st, n, A, w.s, w.R,
                                w.P, w.Dv, w.j, nnei));
    if (tabulated) {
        // G and G' (in t2) of every row from the table
        const real *tab = std::is_same<real, double>::value ? (const real *)m->tab64 : (const real *)m->tab32;
        DP_TIMED("tab_eval", st,
                 hipLaunchKernelGGL((k_tab_eval<real>), dim3(div_up(rows * kM, 256)), dim3(256), 0, st, rows, A, tab,
                                    w.s, w.G, w.t2));
    } else {
        DP_TIMED("plain_l0", st,
                 hipLaunchKernelGGL((k_plain_l0<real>), dim3(div_up(rows * 32, 256)), dim3(256), 0, st, rows, w.s,
                                    ew.W0, ew.b0, w.h0));
        Epi e{};
        e = Epi{ew.b1, w.h0, nullptr, nullptr, w.h1, nullptr, w.t1, 32, 0};
        DP_TIMED("plain_gemm", st, launch_gemm<real, real>(EPI_EMB, (int)rows_p, 64, 32, w.h0, ew.W1t, e, st));
        e = Epi{ew.b2, w.h1, nullptr, nullptr, w.G, nullptr, w.t2, 64, 0};
        DP_TIMED("plain_gemm", st, launch_gemm<real, real>(EPI_EMB, (int)rows_p, kM, 64, w.h1, ew.W2t, e, st));
    }
    DP_TIMED("plain_contract", st,
             hipLaunchKernelGGL((k_plain_contract<real, TD>), dim3(div_up(n, 4)), dim3(256), 0, st, n, sel,
                                (real)m->cfg.desc_scale, w.R, w.G, (real *)T, (TD *)D));
    return step_check("plain_forward", st);
}

template <typename real>
dp_status plain_backward(const dp_model *m, dp_nlist *nl, int n, const void *dT, double *force, double *w_atom,
                         hipStream_t st, bool tabulated)
{
    int sel = m->cfg.sel;
    long rows = (long)n * sel, rows_p = round_up(rows, kRowPad);
    PlainWS<real> w = plain_carve<real>(nl->ws_plain, rows_p);
    EmbW<real> ew = emb_weights<real>(m);
    real sig = (real)m->cfg.desc_scale;
    if (tabulated) {
        // dE/ds of every row through the tabulated G' (into s), then the forces
        DP_TIMED("tab_dsG", st,
                 hipLaunchKernelGGL((k_tab_dsG<real>), dim3(div_up(rows, 4)), dim3(256), 0, st, rows, sel, sig, w.R,
                                    (const real *)dT, w.t2, w.s));
        launch_fill_zero(force, 3L * n, st);
        DP_TIMED("plain_force", st,
                 hipLaunchKernelGGL((k_plain_force<real>), dim3(n), dim3(256), 0, st, n, sel, sig, w.R, w.P, w.Dv,
                                    w.j, w.G, (const real *)nullptr, ew.W0, (const real *)w.s, (const real *)dT, force,
                                    w_atom));
        return step_check("tab_backward", st);
    }
    DP_TIMED("plain_dG", st,
             hipLaunchKernelGGL((k_plain_dG<real>), dim3(div_up(rows * 64, 256)), dim3(256), 0, st, rows, sel, sig, w.R,
                                (const real *)dT, w.t2, w.h1));
    Epi e{};
    // dh1 = fold(dG) + dz2 W2^T (into h1), dz1 = dh1 (1 - t1^2) (into t1)
    e = Epi{nullptr, w.h1, nullptr, w.t1, w.h1, w.t1, nullptr, 0, 0};
    DP_TIMED("plain_gemm", st, launch_gemm<real, real>(EPI_BWD, (int)rows_p, 64, kM, w.t2, ew.W2, e, st));
    // dh0 = fold(dh1) + dz1 W1^T, dz0 = dh0 (1 - h0^2) (into h0)
    e = Epi{nullptr, w.h1, nullptr, w.h0, nullptr, w.h0, nullptr, 0, 32};
    DP_TIMED("plain_gemm", st, launch_gemm<real, real>(EPI_FOLD, (int)rows_p, 64, 64, w.t1, ew.W1p, e, st));
    launch_fill_zero(force, 3L * n, st);
    DP_TIMED("plain_force", st,
             hipLaunchKernelGGL((k_plain_force<real>), dim3(n), dim3(256), 0, st, n, sel, sig, w.R, w.P, w.Dv, w.j,
                                w.G, w.h0, ew.W0, (const real *)nullptr, (const real *)dT, force, w_atom));
    return step_check("plain_backward", st);
}

template dp_status plain_forward<double, double>(const dp_model *, dp_nlist *, int, const double *, void *, void *,
                                                 int *, hipStream_t, bool);
template dp_status plain_forward<float, float>(const dp_model *, dp_nlist *, int, const double *, void *, void *,
                                               int *, hipStream_t, bool);
template dp_status plain_forward<float, __bf16>(const dp_model *, dp_nlist *, int, const double *, void *, void *,
                                                int *, hipStream_t, bool);
template dp_status plain_backward<double>(const dp_model *, dp_nlist *, int, const void *, double *, double *,
                                          hipStream_t, bool);
template dp_status plain_backward<float>(const dp_model *, dp_nlist *, int, const void *, double *, double *,
                                         hipStream_t, bool);

}  // namespace dp
