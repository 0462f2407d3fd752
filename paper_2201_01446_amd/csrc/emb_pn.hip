// emb_pn.hip -- the per-neighbor form of the fused embedding step, for the
// ablation ladder of the optimizations (paper Sec. 3.3-3.4 and its
// step-by-step evaluation of them).
//
// Same result as emb.hip (Eqs. 1-5 with the tabulated G of Sec. 3.2), but
// evaluated the way the paper's fused kernel does it: every column of G_j is
// evaluated for every neighbor j and folded into T at once (Sec. 3.4.1),
// and, in the backward, dE/dR_j and dE/ds_j are summed over the columns for
// every neighbor.  With `padded` set, the loops also run over the rows past
// the real neighbors up to sel (R = 0, s = 0), i.e. without the redundancy
// removal of Sec. 3.4.2; their contribution is exactly zero.
//
// One 64-lane wavefront per atom: lanes split into NG groups of GL = 128/CPL
// lanes; lane l of a group owns the CPL columns eta = l + GL c.  Group g walks
// the g-th contiguous chunk of the distance-sorted list and keeps the
// current interval's coefficients in registers, reloading them when the
// interval changes.  Sums over the columns (backward) use DPP row operations.
// The neighbor records, the pair-gradient slots and the force gather are
// those of the default path.

#include "dp_internal.h"
#include "emb_common.h"
#include "env.h"

#include <type_traits>

namespace dp {

namespace {

__device__ inline void pn_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Coefficients of the CPL columns l + GL c of interval th.
template <typename real, int CPL, int GL>
__device__ inline void pn_coef(const real *tab, int th, int l, real (&a)[CPL][6])
{
#pragma unroll
    for (int c = 0; c < CPL; c++) {
        if (sizeof(real) == 4) {
            const float2 *p =
                reinterpret_cast<const float2 *>(reinterpret_cast<const float *>(tab) + ((long)th * kM + l + GL * c) * 6);
            float2 u = p[0], v = p[1], w = p[2];
            a[c][0] = u.x; a[c][1] = u.y; a[c][2] = v.x; a[c][3] = v.y; a[c][4] = w.x; a[c][5] = w.y;
        } else {
            const double2 *p =
                reinterpret_cast<const double2 *>(reinterpret_cast<const double *>(tab) + ((long)th * kM + l + GL * c) * 6);
            double2 u = p[0], v = p[1], w = p[2];
            a[c][0] = u.x; a[c][1] = u.y; a[c][2] = v.x; a[c][3] = v.y; a[c][4] = w.x; a[c][5] = w.y;
        }
    }
}

template <typename real>
__device__ inline real pn_horner(const real (&a)[6], real t)
{
    return fma(fma(fma(fma(fma(a[5], t, a[4]), t, a[3]), t, a[2]), t, a[1]), t, a[0]);
}

template <typename real>
__device__ inline void pn_horner2(const real (&a)[6], real t, real &f, real &fp)
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

template <int GL>
__device__ inline float pn_group_sum(float v)
{
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    if (GL >= 32) v += __shfl_xor(v, 16);
    if (GL >= 64) v += __shfl_xor(v, 32);
    return v;
}
template <int GL>
__device__ inline double pn_group_sum(double v)
{
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    if (GL >= 32) v += __shfl_xor(v, 16);
    if (GL >= 64) v += __shfl_xor(v, 32);
    return v;
}

// Rows [nn, sel) as padding: R = 0, s = 0 (interval 0, offset 0).
template <typename real>
__device__ inline void pad_rows(NbrLDS<real> L, int nn, int sel, int lane)
{
    for (int k = nn + lane; k < sel; k += 64) {
        if (L.R) L.R[k] = V4<real>{0, 0, 0, 0};
        L.t[k] = 0;
        L.th[k] = 0;
    }
    pn_wave_sync();
}

template <typename real>
constexpr int pn_fwd_lds_bytes(int sel)
{
    return nbr_lds_bytes<real>(sel, ENV_FWD) + 4 * kM * (int)sizeof(real);
}

template <typename real, typename TD, int CPL>
__global__ void __launch_bounds__(256) k_emb_fwd_pn(int natoms, EnvArgs A, const real *__restrict__ tab,
                                                    real sigma, real *__restrict__ T_out, TD *__restrict__ D_out,
                                                    int padded, int *__restrict__ nnei_out)
{
    constexpr int GL = kM / CPL, NG = 64 / GL;
    HIP_DYNAMIC_SHARED(uint4, smem_raw)
    char *base = reinterpret_cast<char *>(smem_raw);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = xcd_item(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave;
    base += wave * pn_fwd_lds_bytes<real>(A.sel);
    NbrLDS<real> L = carve<real>(base, A.sel, ENV_FWD);
    real *Tl = reinterpret_cast<real *>(base + nbr_lds_bytes<real>(A.sel, ENV_FWD));
    bool live = i < natoms;
    int nn = 0, n_in = 0, over = 0, oob = 0;
    if (live) nn = build_env<real, ENV_FWD>(i, A, L, lane, n_in, over, oob);
    __syncthreads();
    if (!live) return;
    int nrow = nn;
    if (padded) {
        pad_rows<real>(L, nn, A.sel, lane);
        nrow = A.sel;
    }
    int g = lane / GL, l = lane % GL;
    int chunk = (nrow + NG - 1) / NG;
    int beg = g * chunk, end = min(nrow, beg + chunk);
    real acc[4][CPL];
#pragma unroll
    for (int c = 0; c < CPL; c++) acc[0][c] = acc[1][c] = acc[2][c] = acc[3][c] = 0;
    real a[CPL][6];
    int cur = -1;
    for (int k = beg; k < end; k++) {
        int th = L.th[k] & ~kOobBit;
        real t = L.t[k];
        V4<real> R = L.R[k];
        if (th != cur) {
            pn_coef<real, CPL, GL>(tab, th, l, a);
            cur = th;
        }
#pragma unroll
        for (int c = 0; c < CPL; c++) {
            real f = pn_horner<real>(a[c], t);
            acc[0][c] = fma(R.x, f, acc[0][c]);
            acc[1][c] = fma(R.y, f, acc[1][c]);
            acc[2][c] = fma(R.z, f, acc[2][c]);
            acc[3][c] = fma(R.w, f, acc[3][c]);
        }
    }
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
    pn_wave_sync();
    for (int o = lane; o < kDdim; o += 64) {
        int aa = o >> 7, bb = o & (kM - 1);
        real v = Tl[aa] * Tl[bb];
        v = fma(Tl[kM + aa], Tl[kM + bb], v);
        v = fma(Tl[2 * kM + aa], Tl[2 * kM + bb], v);
        v = fma(Tl[3 * kM + aa], Tl[3 * kM + bb], v);
        store_op(D_out, fit_row(A, i), o, kDdim, (double)v);
    }
    if (nnei_out && lane == 0) nnei_out[i] = nn;
    record_flags<real>(A, lane, n_in, over, oob);
}

template <typename real, int CPL>
__global__ void __launch_bounds__(256) k_emb_bwd_pn(int natoms, EnvArgs A, const real *__restrict__ tab,
                                                    real sigma, const real *__restrict__ T,
                                                    const real *__restrict__ dD, int padded,
                                                    double *__restrict__ force, double *__restrict__ w_atom)
{
    constexpr int GL = kM / CPL, NG = 64 / GL;
    HIP_DYNAMIC_SHARED(uint4, smem_raw)
    char *base = reinterpret_cast<char *>(smem_raw);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = xcd_item(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave;
    base += wave * nbr_lds_bytes<real>(A.sel, ENV_BWDR);
    NbrLDS<real> L = carve<real>(base, A.sel, ENV_BWDR);
    bool live = i < natoms;
    int nn = 0;
    if (live) nn = load_env<real, ENV_BWDR>(i, A, L, lane);
    __syncthreads();
    if (!live) return;
    int g = lane / GL, l = lane % GL;
    // dE/dT through D = T<^T T (Eq. 2), held per lane for its CPL columns
    // (group g takes the rows a of dD in [g APG, (g+1) APG); see emb.hip)
    constexpr int APG = kMlt / NG;
    const real *Ti = T + (long)i * 4 * kM;
    const real *dDi = dD + fit_row(A, i) * kDdim;
    real dt[4][CPL], tc[4][CPL];
#pragma unroll
    for (int c = 0; c < CPL; c++)
#pragma unroll
        for (int k = 0; k < 4; k++) {
            tc[k][c] = Ti[k * kM + l + GL * c];
            dt[k][c] = 0;
        }
#pragma unroll
    for (int qa = 0; qa < APG; qa++) {
        int a0 = g * APG + qa;
        real ta[4], s2[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            ta[k] = Ti[k * kM + a0];
            s2[k] = 0;
        }
#pragma unroll
        for (int c = 0; c < CPL; c++) {
            real v = dDi[a0 * kM + l + GL * c];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                dt[k][c] = fma(v, ta[k], dt[k][c]);
                s2[k] = fma(v, tc[k][c], s2[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            s2[k] = pn_group_sum<GL>(s2[k]);
            dt[k][0] += l == a0 ? s2[k] : (real)0;
        }
    }
#pragma unroll
    for (int off = GL; off < 64; off <<= 1)
#pragma unroll
        for (int c = 0; c < CPL; c++)
#pragma unroll
            for (int k = 0; k < 4; k++) dt[k][c] += __shfl_xor(dt[k][c], off);
#pragma unroll
    for (int c = 0; c < CPL; c++)
#pragma unroll
        for (int k = 0; k < 4; k++) dt[k][c] *= sigma;
    int nrow = nn;
    if (padded) {
        pad_rows<real>(L, nn, A.sel, lane);
        nrow = A.sel;
    }
    int chunk = (nrow + NG - 1) / NG;
    int beg = g * chunk, end = min(nrow, beg + chunk);
    real a[CPL][6];
    int cur = -1;
    for (int k = beg; k < end; k++) {
        int th = L.th[k];
        real t = L.t[k];
        V4<real> R = L.R[k];
        if ((th & ~kOobBit) != cur) {
            cur = th & ~kOobBit;
            pn_coef<real, CPL, GL>(tab, cur, l, a);
        }
        real dR0 = 0, dR1 = 0, dR2 = 0, dR3 = 0, dsG = 0;
#pragma unroll
        for (int c = 0; c < CPL; c++) {
            real f, fp;
            pn_horner2<real>(a[c], t, f, fp);
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
        dR0 = pn_group_sum<GL>(dR0);
        dR1 = pn_group_sum<GL>(dR1);
        dR2 = pn_group_sum<GL>(dR2);
        dR3 = pn_group_sum<GL>(dR3);
        dsG = pn_group_sum<GL>(dsG);
        // R_j and t_j are not read again: park the neighbor's sums in their place
        if (l == 0 && k < nn) {
            L.R[k] = V4<real>{dR0, dR1, dR2, dR3};
            L.t[k] = (th & kOobBit) ? (real)0 : dsG;
        }
    }
    pn_wave_sync();
    // chain rule through Eq. 1, one real neighbor per lane
    real Fi0 = 0, Fi1 = 0, Fi2 = 0;
    real W[9];
#pragma unroll
    for (int r = 0; r < 9; r++) W[r] = 0;
    for (int k = lane; k < nn; k += 64) {
        V4<real> dR = L.R[k], d = L.Dv[k];
        int slot = L.j[k];
        real dsG = L.t[k], rinv, s, sp;
        env_geom<real>(A, d, rinv, s, sp);
        real h0 = d.x * rinv, h1 = d.y * rinv, h2 = d.z * rinv;
        real dEds = dsG + dR.x + dR.y * h0 + dR.z * h1 + dR.w * h2;
        real u0 = s * dR.y, u1 = s * dR.z, u2 = s * dR.w;
        real udh = u0 * h0 + u1 * h1 + u2 * h2;
        real c0 = dEds * sp;
        real g0 = c0 * h0 + (u0 - udh * h0) * rinv;
        real g1 = c0 * h1 + (u1 - udh * h1) * rinv;
        real g2 = c0 * h2 + (u2 - udh * h2) * rinv;
        put_pg<real>(A.pg, A.cap, i, slot, g0, g1, g2);
        Fi0 += g0;
        Fi1 += g1;
        Fi2 += g2;
        W[0] -= d.x * g0; W[1] -= d.x * g1; W[2] -= d.x * g2;
        W[3] -= d.y * g0; W[4] -= d.y * g1; W[5] -= d.y * g2;
        W[6] -= d.z * g0; W[7] -= d.z * g1; W[8] -= d.z * g2;
    }
    for (int off = 32; off > 0; off >>= 1) {
        Fi0 += __shfl_xor(Fi0, off);
        Fi1 += __shfl_xor(Fi1, off);
        Fi2 += __shfl_xor(Fi2, off);
#pragma unroll
        for (int r = 0; r < 9; r++) W[r] += __shfl_xor(W[r], off);
    }
    if (lane == 0) {
        force[3 * i] = (double)Fi0;
        force[3 * i + 1] = (double)Fi1;
        force[3 * i + 2] = (double)Fi2;
    }
    if (lane < 9) {
        real v = W[0];
#pragma unroll
        for (int r = 1; r < 9; r++) v = lane == r ? W[r] : v;
        w_atom[(long)i * 9 + lane] = (double)v;
    }
}

}  // namespace

template <typename real, typename TD, int CPL>
static void launch_fwd_pn_t(const dp_model *m, const dp_nlist *nl, int n, const double *x, void *T, void *D,
                            void *rec, int *rcnt, bool padded, int *nnei, hipStream_t st)
{
    EnvArgs A = make_env_args(m, nl, x);
    A.rec = rec;
    A.rcnt = rcnt;
    A.pg = nl->pg;
    const real *tab = std::is_same<real, double>::value ? (const real *)m->tab64 : (const real *)m->tab32;
    int wpb = lds_wpb(pn_fwd_lds_bytes<real>(A.sel));
    size_t lds = (size_t)wpb * pn_fwd_lds_bytes<real>(A.sel);
    hipLaunchKernelGGL((k_emb_fwd_pn<real, TD, CPL>), dim3(xcd_grid(div_up(n, wpb))), dim3(64 * wpb), lds, st, n,
                       A, tab, (real)m->cfg.desc_scale, (real *)T, (TD *)D, padded ? 1 : 0, nnei);
}

template <typename real, int CPL>
static void launch_bwd_pn_t(const dp_model *m, const dp_nlist *nl, int n, const double *x, const void *T,
                            const void *dD, const void *rec, const int *rcnt, bool padded, double *force,
                            double *w_atom, hipStream_t st)
{
    EnvArgs A = make_env_args(m, nl, x);
    A.rec = const_cast<void *>(rec);
    A.rcnt = const_cast<int *>(rcnt);
    A.pg = nl->pg;
    const real *tab = std::is_same<real, double>::value ? (const real *)m->tab64 : (const real *)m->tab32;
    int wpb = lds_wpb(nbr_lds_bytes<real>(A.sel, ENV_BWDR));
    size_t lds = (size_t)wpb * nbr_lds_bytes<real>(A.sel, ENV_BWDR);
    hipLaunchKernelGGL((k_emb_bwd_pn<real, CPL>), dim3(xcd_grid(div_up(n, wpb))), dim3(64 * wpb), lds, st, n, A,
                       tab, (real)m->cfg.desc_scale, (const real *)T, (const real *)dD, padded ? 1 : 0, force, w_atom);
}

void launch_emb_fwd_pn(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision, void *T,
                       void *D, void *rec, int *rcnt, bool padded, int *nnei, hipStream_t st)
{
    if (precision == DP_FP64) launch_fwd_pn_t<double, double, 4>(m, nl, n, x, T, D, rec, rcnt, padded, nnei, st);
    else if (precision == DP_FP32) launch_fwd_pn_t<float, float, 8>(m, nl, n, x, T, D, rec, rcnt, padded, nnei, st);
    else launch_fwd_pn_t<float, __bf16, 8>(m, nl, n, x, T, D, rec, rcnt, padded, nnei, st);
}

void launch_emb_bwd_pn(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision, const void *T,
                       const void *dD, const void *rec, const int *rcnt, bool padded, double *force, double *w_atom,
                       hipStream_t st)
{
    if (precision == DP_FP64) launch_bwd_pn_t<double, 4>(m, nl, n, x, T, dD, rec, rcnt, padded, force, w_atom, st);
    else launch_bwd_pn_t<float, 8>(m, nl, n, x, T, dD, rec, rcnt, padded, force, w_atom, st);
}

}  // namespace dp
