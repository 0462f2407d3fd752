// emb.hip -- fused environment matrix, tabulated embedding and R^T G
// contraction (forward), and its hand-written adjoint down to forces and the
// virial (backward), on gfx950.
//
// What is computed per atom i (paper Sec. 2.1, Eqs. 1-5; Sec. 3.2-3.4):
//   for every neighbor j with r = |r_ij| < rcut (the sel nearest at most):
//     s = w(r)/r, R_j = s (1, x/r, y/r, z/r)                      (Eq. 1)
//     G_j = f_theta(s): the M quintics of s's table interval      (Sec. 3.2)
//   T = desc_scale * sum_j R_j^T G_j   (4 x M), D = T<^T T (M< x M)  (Eq. 2)
// G is never stored (the kernel fusion of Sec. 3.3/3.4.1) and only the n_i
// real neighbors are visited (the redundancy removal of Sec. 3.4.2; with
// unnormalised R the padded rows would contribute exact zeros).
//
// Interval-moment form of the contraction.  In table interval theta the
// embedding is G_eta(s) = sum_e a[theta][eta][e] t^e with t = s - x_theta, so
// for the neighbors j whose s falls in theta
//   sum_j R_jk G_j,eta = sum_e a[theta][eta][e] M[theta][k][e],
//   M[theta][k][e] = sum_{j in theta} R_jk t_j^e      (4 x 6 moments).
// The neighbor list is sorted by distance and s decreases with r, so the
// neighbors of one interval form consecutive runs ("segments"; about 20 per
// atom in copper against about 178 neighbors).  The forward therefore forms
// 24 moments per neighbor and then 24 FMA per (segment, column), instead of
// 9 FMA per (neighbor, column).  The backward does the same on the other
// side: with dT = dE/dT (desc_scale applied),
//   dE/dR_jk  = sum_eta dT_k,eta G_j,eta = sum_e B[theta][k][e] t_j^e,
//   B[theta][k][e] = sum_eta dT_k,eta a[theta][eta][e],
//   dE/ds_j  += sum_k R_jk d/dt (sum_e B[theta][k][e] t^e) at t_j,
// so each segment costs 24 FMA per column once, and each neighbor two
// quintics per k.  Then g_ij = dE_i/dr_ij by the chain rule through Eq. 1:
// F_i = sum_j g_ij is written directly and W_i -= r_ij (x) g_ij; each g_ij is
// stored at its candidate slot, and a gather after the kernel subtracts from
// F_j the g_ij of every atom i that lists j (no atomics, a fixed order).
// Neighbors clamped to the table end form their own segment and get G' = 0.
// A run split because atoms moved since the list was sorted gives two
// segments of the same interval.  In the forward, such duplicates within a
// round of segments share one representative (the first of the round with
// that interval), which alone is contracted, with the sum of their moments
// (the backward's B, computed by the segments' quads in parallel, gains
// nothing from sharing).
//
// Work distribution (one 64-lane wavefront per atom, neighbor data in LDS):
//   moments and B: quad q of the wave owns one segment per round; for the
//   moments lane l of the quad takes environment column k = l of every
//   neighbor of the segment, for B the four lanes split the 128 columns and
//   their partial sums meet in two DPP steps;
//   contraction into T: each lane owns columns eta = lane and lane + 64;
//   per-neighbor tail of the backward: each lane owns neighbors.

#include "dp_internal.h"
#include "emb_common.h"
#include "env.h"

#include <type_traits>

namespace dp {

namespace {

constexpr int kSegRound = 16;   // segments per round: one per quad of the wave

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The 6 coefficients of column c of interval th (24 bytes, 8-byte aligned).
__device__ inline void coef_col(const float *tab, int th, int c, float (&a)[6])
{
    const float2 *p = reinterpret_cast<const float2 *>(tab + ((long)th * kM + c) * 6);
    float2 u = p[0], v = p[1], w = p[2];
    a[0] = u.x; a[1] = u.y; a[2] = v.x; a[3] = v.y; a[4] = w.x; a[5] = w.y;
}
__device__ inline void coef_col(const double *tab, int th, int c, double (&a)[6])
{
    const double2 *p = reinterpret_cast<const double2 *>(tab + ((long)th * kM + c) * 6);
    double2 u = p[0], v = p[1], w = p[2];
    a[0] = u.x; a[1] = u.y; a[2] = v.x; a[3] = v.y; a[4] = w.x; a[5] = w.y;
}

// f = sum_e a[e] t^e and its derivative.
template <typename real>
__device__ inline void horner2(const real *a, real t, real &f, real &fp)
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

__device__ inline float quad_sum(float v)
{
    v += dpp_f<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);   // quad_perm [2,3,0,1]
    return v;
}
__device__ inline double quad_sum(double v)
{
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    return v;
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

// One DPP move of a float or a double.
template <int CTRL>
__device__ inline float dpp_any(float v) { return dpp_f<CTRL>(v); }
template <int CTRL>
__device__ inline double dpp_any(double v) { return dpp_d<CTRL>(v); }

// Representatives of the ns segments of a round starting at s0: lane u < ns
// returns the first segment v <= u of the round with the same table interval
// (the clamp bit aside); other lanes return themselves.
template <typename real>
__device__ inline int round_reps(const NbrLDS<real> &L, const int *seg, int s0, int ns, int lane)
{
    int thu = lane < ns ? (L.th[seg[s0 + lane]] & ~kOobBit) : -1;
    int rep = lane;
    for (int v = 0; v < ns; v++) {
        int thv = __shfl(thu, v);
        if (v < lane && thv == thu && rep == lane) rep = v;
    }
    return rep;
}

// Starts of the runs of equal interval in the neighbor list: seg[0..nseg-1],
// seg[nseg] = nn.  Returns nseg (uniform over the wave).  X > 0: a run longer
// than X is cut into pieces of X neighbors (and a last shorter one), which
// become segments of their own; nruns then receives the number of whole runs.
template <typename real, int X = 0>
__device__ int find_segments(const NbrLDS<real> &L, int nn, int lane, int *seg, int *nruns = nullptr)
{
    int nseg = 0, runs = 0;
    int open = 0;   // start of the run that continues into the next chunk
    for (int base = 0; base < nn; base += 64) {
        int k = base + lane;
        bool head = k < nn && (k == 0 || L.th[k] != L.th[k - 1]);
        if (X > 0) {
            unsigned long long hm = __ballot(head);
            runs += __popcll(hm);
            unsigned long long upto = hm & ((2ull << lane) - 1ull);   // run heads at lanes <= lane
            int start = upto ? base + 63 - __builtin_clzll(upto) : open;
            head = head || (k < nn && (k - start) % X == 0);
            if (hm) open = base + 63 - __builtin_clzll(hm);
        }
        unsigned long long m = __ballot(head);
        if (head) seg[nseg + __popcll(m & ((1ull << lane) - 1ull))] = k;
        nseg += __popcll(m);
    }
    if (lane == 0) seg[nseg] = nn;
    if (nruns) *nruns = X > 0 ? runs : nseg;
    wave_sync();
    return nseg;
}

// Longest segment of the forward: its moments take one quad as many steps as
// the segment has neighbors, and a round waits for its longest segment, so
// long runs (a whole neighbor shell can share one table interval) are cut;
// the pieces share an interval, and the round's representatives merge them
// again before the contraction.
constexpr int kFwdMaxRun = 16;

constexpr int seg_bytes(int sel) { return ((sel + 1) * 4 + 15) / 16 * 16; }

// Per-wave LDS of the forward: neighbor arrays, the moments of one round of
// segments, segment starts; T (4 x M) for the descriptor at the end takes
// the slice's start once those are dead.
template <typename real>
constexpr int fwd_lds_bytes(int sel)
{
    constexpr int al = (int)sizeof(V4<real>);   // keeps every wave's slice aligned
    int b = nbr_lds_bytes<real>(sel, ENV_FWD) + kSegRound * 24 * (int)sizeof(real) + seg_bytes(sel);
    int t = 4 * kM * (int)sizeof(real);
    return ((b > t ? b : t) + al - 1) / al * al;
}

// Per-wave LDS of the backward: neighbor arrays, dT as (dT_0c, .., dT_3c)
// per column c, B of one round of segments, segment starts.
template <typename real>
constexpr int bwd_lds_bytes(int sel)
{
    constexpr int al = (int)sizeof(V4<real>);
    return (nbr_lds_bytes<real>(sel, ENV_BWD) + kM * (int)sizeof(V4<real>) + kSegRound * 24 * (int)sizeof(real) +
            seg_bytes(sel) + al - 1) / al * al;
}

// -------------------------------------------------------------- forward
template <typename real, typename TD>
__global__ void __launch_bounds__(256) k_emb_fwd(int natoms, EnvArgs A, const real *__restrict__ tab,
                                                 real sigma, real *__restrict__ T_out,
                                                 TD *__restrict__ D_out, int *__restrict__ nnei_out,
                                                 int *__restrict__ nseg_out)
{
    HIP_DYNAMIC_SHARED(uint4, smem_raw)   // 16-byte aligned
    char *base = reinterpret_cast<char *>(smem_raw);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = xcd_item(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave;
    base += wave * fwd_lds_bytes<real>(A.sel);
    NbrLDS<real> L = carve<real>(base, A.sel, ENV_FWD);
    char *p = base + nbr_lds_bytes<real>(A.sel, ENV_FWD);
    real *Tl = reinterpret_cast<real *>(base);   // 4 x M, after the rounds
    real *Ms = reinterpret_cast<real *>(p);   // kSegRound x 24
    p += kSegRound * 24 * sizeof(real);
    int *seg = reinterpret_cast<int *>(p);
    bool live = i < natoms;
    int nn = 0, n_in = 0, over = 0, oob = 0;
    if (live) nn = build_env<real, ENV_FWD>(i, A, L, lane, n_in, over, oob);
    __syncthreads();
    if (!live) return;
    int nruns = 0;
    int nseg = find_segments<real, kFwdMaxRun>(L, nn, lane, seg, &nruns);

    int q = lane >> 2, ql = lane & 3;
    real T0[4] = {0, 0, 0, 0}, T1[4] = {0, 0, 0, 0};   // columns lane, lane + 64
    for (int s0 = 0; s0 < nseg; s0 += kSegRound) {
        int ns = min(kSegRound, nseg - s0);
        // moments of segment s0 + q: lane ql of the quad sums column k = ql
        // of R over the segment's neighbors, in list order
        if (q < ns) {
            real Mk[6] = {0, 0, 0, 0, 0, 0};
            int e1 = seg[s0 + q + 1];
            for (int k = seg[s0 + q]; k < e1; k++) {
                real t = L.t[k];
                real r = reinterpret_cast<const real *>(&L.R[k])[ql];
                real pw = 1;
#pragma unroll
                for (int e = 0; e < 6; e++) {
                    Mk[e] = fma(r, pw, Mk[e]);
                    pw *= t;
                }
            }
#pragma unroll
            for (int e = 0; e < 6; e++) Ms[q * 24 + ql * 6 + e] = Mk[e];
        }
        // segments of the round that share an interval: the representative
        // takes the others' moments (in segment order), and only it is contracted
        const int rep = round_reps(L, seg, s0, ns, lane);
        const unsigned long long reps = __ballot(lane < ns && rep == lane);
        if (reps != ((1ull << ns) - 1ull)) {
            wave_sync();
            const bool qrep = q < ns && __shfl(rep, q) == q;   // quad q holds a representative
            real add[6] = {0, 0, 0, 0, 0, 0};
            for (int u = 0; u < ns; u++) {
                int ru = __shfl(rep, u);
                if (qrep && ru == q && u != q) {
#pragma unroll
                    for (int e = 0; e < 6; e++) add[e] += Ms[u * 24 + ql * 6 + e];
                }
            }
            if (qrep) {
#pragma unroll
                for (int e = 0; e < 6; e++) Ms[q * 24 + ql * 6 + e] += add[e];
            }
        }
        wave_sync();
        // T[k][c] += sum_e a[theta][c][e] M[k][e], lanes over columns; the
        // coefficients of up to four representatives are requested before any is used
        for (unsigned long long left = reps; left;) {
            int us[4];
            int nu = 0;
#pragma unroll
            for (int u = 0; u < 4; u++) {
                us[u] = left ? __builtin_ctzll(left) : -1;
                if (left) {
                    left &= left - 1;
                    nu++;
                }
            }
            real a0[4][6], a1[4][6];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (u < nu) {
                    int th = L.th[seg[s0 + us[u]]] & ~kOobBit;
                    coef_col(tab, th, lane, a0[u]);
                    coef_col(tab, th, lane + 64, a1[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (u < nu) {
                    const real *m = Ms + us[u] * 24;
#pragma unroll
                    for (int k = 0; k < 4; k++)
#pragma unroll
                        for (int e = 0; e < 6; e++) {
                            real mv = m[k * 6 + e];
                            T0[k] = fma(mv, a0[u][e], T0[k]);
                            T1[k] = fma(mv, a1[u][e], T1[k]);
                        }
                }
            }
        }
        wave_sync();   // Ms is rewritten by the next round (and the arrays give way to T)
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        T0[k] *= sigma;
        T1[k] *= sigma;
        Tl[k * kM + lane] = T0[k];
        Tl[k * kM + lane + 64] = T1[k];
    }
    // T out by column: (T_0c, T_1c, T_2c, T_3c) for c < M, one vector store per column
    V4<real> *T4 = reinterpret_cast<V4<real> *>(T_out) + (long)i * kM;
    T4[lane] = V4<real>{T0[0], T0[1], T0[2], T0[3]};
    T4[lane + 64] = V4<real>{T1[0], T1[1], T1[2], T1[3]};
    wave_sync();
    // D[a][b] = sum_k T[k][a] T[k][b], a < M<: lane owns b = lane, lane + 64;
    // the row of the atom in the fitting net's operand (grouped by type).
    // No D_out: the first fitting layer forms D from T itself.
    const long drow = fit_row(A, i);
#pragma unroll 4
    for (int a = 0; a < (D_out ? kMlt : 0); a++) {
        real d0 = 0, d1 = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            real ta = Tl[k * kM + a];
            d0 = fma(ta, T0[k], d0);
            d1 = fma(ta, T1[k], d1);
        }
        store_op(D_out, drow, a * kM + lane, kDdim, (double)d0);
        store_op(D_out, drow, a * kM + lane + 64, kDdim, (double)d1);
    }
    // counters last: nothing in this kernel waits for these atomics
    if (nnei_out && lane == 0) nnei_out[i] = nn;
    if (nseg_out && lane == 0) nseg_out[i] = nruns;
    record_flags<real>(A, lane, n_in, over, oob);
}

// ------------------------------------------------------------- backward
// B[k][e] = sum_c dT[k][c] a[theta][c][e] for the ns segments of a round
// starting at s0, 2^lg lanes per segment (lg = 2 in a full round; the last
// round's segments get more): segment s0 + (lane >> lg), its lanes taking
// columns c = 2^lg m + (lane mod 2^lg), then summed over the group, whose
// first lane stores B at Bs[(lane >> lg) * 24].  FULL: lg = 2 known at
// compile time.
template <typename real, bool FULL>
__device__ inline void round_B(const NbrLDS<real> &L, const int *seg, int s0, int ns, int lg,
                               const real *__restrict__ tab, const V4<real> *dTl, real *Bs, int lane)
{
    if (FULL) lg = 2;
    const int G = 1 << lg, q = lane >> lg, ql = lane & (G - 1);
    real B[4][6];
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
        for (int e = 0; e < 6; e++) B[k][e] = 0;
    if (q < ns) {
        int th = L.th[seg[s0 + q]] & ~kOobBit;
        // full rounds: in FP64 every coefficient load of the segment in flight
        // at once, in FP32 four (measured fastest for each); wider groups: two
        constexpr int kLoadsInFlight = !FULL ? 2 : sizeof(real) == 8 ? kM / 4 : 4;
#pragma unroll kLoadsInFlight
        for (int m = 0; m < (kM >> lg); m++) {
            int c = (m << lg) + ql;
            V4<real> d = dTl[c];
            real a[6];
            coef_col(tab, th, c, a);
#pragma unroll
            for (int e = 0; e < 6; e++) {
                B[0][e] = fma(d.x, a[e], B[0][e]);
                B[1][e] = fma(d.y, a[e], B[1][e]);
                B[2][e] = fma(d.z, a[e], B[2][e]);
                B[3][e] = fma(d.w, a[e], B[3][e]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
        for (int e = 0; e < 6; e++) B[k][e] = quad_sum(B[k][e]);
    if (!FULL) {
        // the rest of the group (wave-uniform steps): within 8 and 16 lanes by
        // DPP mirrors, then across rows
        if (lg >= 3) {
#pragma unroll
            for (int k = 0; k < 4; k++)
#pragma unroll
                for (int e = 0; e < 6; e++) B[k][e] += dpp_any<0x141>(B[k][e]);
        }
        if (lg >= 4) {
#pragma unroll
            for (int k = 0; k < 4; k++)
#pragma unroll
                for (int e = 0; e < 6; e++) B[k][e] += dpp_any<0x140>(B[k][e]);
        }
        for (int off = 16; off < G; off <<= 1) {
#pragma unroll
            for (int k = 0; k < 4; k++)
#pragma unroll
                for (int e = 0; e < 6; e++) B[k][e] += __shfl_xor(B[k][e], off);
        }
    }
    if (q < ns && ql == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
            for (int e = 0; e < 6; e++) Bs[q * 24 + k * 6 + e] = B[k][e];
    }
}

// CPL: columns per lane in the dE/dT prologue (lanes in NG groups of GL).
template <typename real, int CPL>
__global__ void __launch_bounds__(256) k_emb_bwd(int natoms, EnvArgs A, const real *__restrict__ tab,
                                                 real sigma, const real *__restrict__ T,
                                                 const real *__restrict__ dD, double *__restrict__ force,
                                                 double *__restrict__ w_atom)
{
    constexpr int GL = kM / CPL, NG = 64 / GL;
    HIP_DYNAMIC_SHARED(uint4, smem_raw)   // 16-byte aligned
    char *base = reinterpret_cast<char *>(smem_raw);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int i = xcd_item(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave;
    base += wave * bwd_lds_bytes<real>(A.sel);
    NbrLDS<real> L = carve<real>(base, A.sel, ENV_BWD);
    char *p = base + nbr_lds_bytes<real>(A.sel, ENV_BWD);
    V4<real> *dTl = reinterpret_cast<V4<real> *>(p);   // per column
    p += kM * sizeof(V4<real>);
    real *Bs = reinterpret_cast<real *>(p);             // kSegRound x 24
    p += kSegRound * 24 * sizeof(real);
    int *seg = reinterpret_cast<int *>(p);
    bool live = i < natoms;
    // this lane's part of dE/dD (see below) into registers first: its loads
    // stream from HBM while the neighbor scan runs
    constexpr int APG = kMlt / NG;
    const int g = lane / GL, l = lane % GL;
    real dv[APG][CPL];
    if (live) {
        const real *dDi = dD + fit_row(A, i) * kDdim;
#pragma unroll
        for (int qa = 0; qa < APG; qa++)
#pragma unroll
            for (int c = 0; c < CPL; c++) dv[qa][c] = dDi[(g * APG + qa) * kM + l + GL * c];
    }
    int nn = 0;
    if (live) nn = load_env<real>(i, A, L, lane);
    __syncthreads();
    if (!live) return;

    // dE/dT from dE/dD through D = T<^T T (Eq. 2; T already carries desc_scale):
    //   dT[k][b] = sum_{a<M<} dD[a][b] T[k][a] + [b<M<] sum_c dD[b][c] T[k][c].
    // Group g takes the rows a of dD in [g APG, (g+1) APG), each lane its CPL
    // columns b = l + GL c; the second term's sum over c is a group
    // reduction, added at the lane that owns column b = a; the groups'
    // partials are then summed and group 0 parks dT in LDS.
    {
        const V4<real> *Ti = reinterpret_cast<const V4<real> *>(T) + (long)i * kM;   // T by column
        real dt[4][CPL], tc[4][CPL];
#pragma unroll
        for (int c = 0; c < CPL; c++) {
            V4<real> t = Ti[l + GL * c];
            tc[0][c] = t.x;
            tc[1][c] = t.y;
            tc[2][c] = t.z;
            tc[3][c] = t.w;
#pragma unroll
            for (int k = 0; k < 4; k++) dt[k][c] = 0;
        }
#pragma unroll
        for (int qa = 0; qa < APG; qa++) {
            int a0 = g * APG + qa;
            real ta[4], s2[4];
            V4<real> t = Ti[a0];
            ta[0] = t.x;
            ta[1] = t.y;
            ta[2] = t.z;
            ta[3] = t.w;
#pragma unroll
            for (int k = 0; k < 4; k++) s2[k] = 0;
#pragma unroll
            for (int c = 0; c < CPL; c++) {
                real v = dv[qa][c];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    dt[k][c] = fma(v, ta[k], dt[k][c]);
                    s2[k] = fma(v, tc[k][c], s2[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < 4; k++) {
                s2[k] = group_sum<GL>(s2[k]);
                dt[k][0] += l == a0 ? s2[k] : (real)0;
            }
        }
#pragma unroll
        for (int off = GL; off < 64; off <<= 1)
#pragma unroll
            for (int c = 0; c < CPL; c++)
#pragma unroll
                for (int k = 0; k < 4; k++) dt[k][c] += __shfl_xor(dt[k][c], off);
        if (g == 0) {
#pragma unroll
            for (int c = 0; c < CPL; c++)
                dTl[l + GL * c] = V4<real>{sigma * dt[0][c], sigma * dt[1][c], sigma * dt[2][c], sigma * dt[3][c]};
        }
    }
    int nseg = find_segments(L, nn, lane, seg);   // its wave barrier also publishes dT

    real Fi0 = 0, Fi1 = 0, Fi2 = 0;
    real W[9];
#pragma unroll
    for (int r = 0; r < 9; r++) W[r] = 0;
    for (int s0 = 0; s0 < nseg; s0 += kSegRound) {
        int ns = min(kSegRound, nseg - s0);
        // B of the round's segments: four lanes per segment in a full round;
        // a round of at most 8, 4, 2 or 1 segments (the last one) gives each
        // 8, 16, 32 or 64 lanes, so its lanes still share the columns
        if (ns > 8) round_B<real, true>(L, seg, s0, ns, 2, tab, dTl, Bs, lane);
        else round_B<real, false>(L, seg, s0, ns, ns > 4 ? 3 : ns > 2 ? 4 : ns > 1 ? 5 : 6, tab, dTl, Bs, lane);
        wave_sync();
        // the neighbors of these segments, one per lane: dE/dR_j and dE/ds_j
        // from B, then the chain rule through Eq. 1 and the scatter
        int kb = seg[s0], ke = seg[s0 + ns];
        int cur = -1;   // segment (relative to s0) of the last neighbor before this chunk
        for (int b0 = kb; b0 < ke; b0 += 64) {
            int k = b0 + lane;
            bool in = k < ke;
            bool head = in && (k == kb || L.th[k] != L.th[k - 1]);
            unsigned long long hm = __ballot(head);
            int sidx = cur + __popcll(hm & ((2ull << lane) - 1ull));   // heads up to and including k
            cur += __popcll(hm);
            if (!in) continue;
            int th = L.th[k];
            real t = L.t[k];
            V4<real> d = L.Dv[k];
            int slot = L.j[k];
            const real *b = Bs + sidx * 24;
            real dR[4], Q[4];
#pragma unroll
            for (int kk = 0; kk < 4; kk++) horner2<real>(b + kk * 6, t, dR[kk], Q[kk]);
            real rinv, s, sp;
            env_geom<real>(A, d, rinv, s, sp);
            real h0 = d.x * rinv, h1 = d.y * rinv, h2 = d.z * rinv;
            // dE/ds through G: sum_k R_k dB_k/dt with R = s (1, h); no G' past the table end
            real dsG = (th & kOobBit) ? (real)0 : s * (Q[0] + Q[1] * h0 + Q[2] * h1 + Q[3] * h2);
            // R = s (1, h): dE/ds collects dR0 + dR.h; dE/dh = s dR[1..3]
            real dEds = dsG + dR[0] + dR[1] * h0 + dR[2] * h1 + dR[3] * h2;
            real u0 = s * dR[1], u1 = s * dR[2], u2 = s * dR[3];
            real udh = u0 * h0 + u1 * h1 + u2 * h2;
            real c0 = dEds * sp;
            real g0 = c0 * h0 + (u0 - udh * h0) * rinv;
            real g1 = c0 * h1 + (u1 - udh * h1) * rinv;
            real g2 = c0 * h2 + (u2 - udh * h2) * rinv;
            // dE_i/dr_ij, gathered into F_j after the kernel (no atomics)
            put_pg<real>(A.pg, A.cap, i, slot, g0, g1, g2);
            Fi0 += g0;
            Fi1 += g1;
            Fi2 += g2;
            W[0] -= d.x * g0; W[1] -= d.x * g1; W[2] -= d.x * g2;
            W[3] -= d.y * g0; W[4] -= d.y * g1; W[5] -= d.y * g2;
            W[6] -= d.z * g0; W[7] -= d.z * g1; W[8] -= d.z * g2;
        }
        wave_sync();   // Bs is rewritten by the next round
    }
    for (int off = 32; off > 0; off >>= 1) {
        Fi0 += __shfl_xor(Fi0, off);
        Fi1 += __shfl_xor(Fi1, off);
        Fi2 += __shfl_xor(Fi2, off);
#pragma unroll
        for (int r = 0; r < 9; r++) W[r] += __shfl_xor(W[r], off);
    }
    if (lane == 0) {   // the gather then subtracts the neighbors' dE_j/dr_ji
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

// ---------------------------------------------------------- launchers
template <typename real, typename TD>
static void launch_fwd_t(const dp_model *m, const dp_nlist *nl, int n, const double *x, void *T,
                         void *D, void *rec, int *rcnt, int *nnei, int *nseg, hipStream_t st)
{
    EnvArgs A = make_env_args(m, nl, x);
    A.rec = rec;
    A.rcnt = rcnt;
    A.pg = nl->pg;
    const real *tab = std::is_same<real, double>::value ? (const real *)m->tab64 : (const real *)m->tab32;
    int wpb = lds_wpb(fwd_lds_bytes<real>(A.sel));
    size_t lds = (size_t)wpb * fwd_lds_bytes<real>(A.sel);
    hipLaunchKernelGGL((k_emb_fwd<real, TD>), dim3(xcd_grid(div_up(n, wpb))), dim3(64 * wpb), lds, st, n, A, tab,
                       (real)m->cfg.desc_scale, (real *)T, (TD *)D, nnei, nseg);
}

template <typename real, int CPL>
static void launch_bwd_t(const dp_model *m, const dp_nlist *nl, int n, const double *x, const void *T,
                         const void *dD, const void *rec, const int *rcnt, double *force, double *w_atom,
                         hipStream_t st)
{
    EnvArgs A = make_env_args(m, nl, x);
    A.rec = const_cast<void *>(rec);
    A.rcnt = const_cast<int *>(rcnt);
    A.pg = nl->pg;
    const real *tab = std::is_same<real, double>::value ? (const real *)m->tab64 : (const real *)m->tab32;
    int wpb = lds_wpb(bwd_lds_bytes<real>(A.sel));
    size_t lds = (size_t)wpb * bwd_lds_bytes<real>(A.sel);
    hipLaunchKernelGGL((k_emb_bwd<real, CPL>), dim3(xcd_grid(div_up(n, wpb))), dim3(64 * wpb), lds, st, n, A, tab,
                       (real)m->cfg.desc_scale, (const real *)T, (const real *)dD, force, w_atom);
}

void launch_emb_fwd(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision,
                    void *T, void *D, void *rec, int *rcnt, int *nnei, int *nseg, hipStream_t st)
{
    if (precision == DP_FP64) launch_fwd_t<double, double>(m, nl, n, x, T, D, rec, rcnt, nnei, nseg, st);
    else if (precision == DP_FP32) launch_fwd_t<float, float>(m, nl, n, x, T, D, rec, rcnt, nnei, nseg, st);
    else launch_fwd_t<float, __bf16>(m, nl, n, x, T, D, rec, rcnt, nnei, nseg, st);
}

void launch_emb_bwd(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision,
                    const void *T, const void *dD, const void *rec, const int *rcnt, double *force,
                    double *w_atom, hipStream_t st)
{
    if (precision == DP_FP64) launch_bwd_t<double, 4>(m, nl, n, x, T, dD, rec, rcnt, force, w_atom, st);
    else launch_bwd_t<float, 8>(m, nl, n, x, T, dD, rec, rcnt, force, w_atom, st);
}

}  // namespace dp
