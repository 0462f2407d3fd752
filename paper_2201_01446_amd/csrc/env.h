// env.h -- the environment-matrix stage shared by the compressed and the
// plain paths: filter the skin list to r < rcut, keep the sel nearest (with
// several atom types: the sel_t nearest of each neighbor type), and form
// s = w(r)/r, R = s (1, x/r, y/r, z/r) (paper Eq. 1) and, for the table, the
// interval of s and the offset from its left node (Sec. 3.2).  Tables of the
// types sit back to back, so a neighbor of type t in interval theta reads
// global interval t n_int + theta; runs of equal global interval then never
// mix types.
#pragma once

#include "dp_internal.h"

namespace dp {

template <typename real>
struct alignas(sizeof(real) * 4) V4 {
    real x, y, z, w;
};

struct EnvArgs {
    const double *x;
    const int *cnt, *nei, *shift;
    int cap, sel;
    double L0, L1, L2;
    const double *atomL;   // per-atom box edges (3 per atom) of a batch of cells, or NULL
    double rc2;
    // gate
    double rs, rc;
    int switch_kind;
    // table
    int n_fine, n_tail;
    double h, s_max, h_tail, tail_max;
    int *flags;
    // compacted neighbors of the forward (r_ij and the candidate slot, sel
    // entries per atom) and their count, written by the forward, read back by
    // the backward; or NULL
    void *rec;
    int *rcnt;
    // per candidate slot dE_i/dr_ij (3 reals; cap slots per atom): the
    // backward writes the kept ones; the forward zeroes those within rcut
    // that a neighbor limit cut off (slots beyond rcut are never read)
    void *pg;
    // several atom types: per-type limits, the candidates of each type per
    // atom (the list is grouped by type), one type's interval count
    int ntypes;
    int sel_t[kMaxTypes];
    const int *tcnt;
    int n_int;
    // fitting-net row of each atom (NULL: the atom index)
    const int *row;
    // early end of the scan: per atom and type the prefix of candidates whose
    // build distance is <= rcut + margin, the largest displacement since the
    // build (FP64 bits); NULL: every candidate is scanned
    const int *inner;
    const unsigned long long *disp;
    double margin;
};

__device__ inline long fit_row(const EnvArgs &A, int i) { return A.row ? A.row[i] : i; }

// Angstrom of slack in the early end of the candidate scan (far above the
// rounding of an FP32 distance of a few tens of Angstrom).
constexpr double kScanSlack = 1e-3;

// Kept-neighbor count of an atom as the forward records it: bit 30 set when a
// neighbor limit cut off some within rcut.
constexpr int kTruncBit = 1 << 30;

// Displacement r_ij = x_j - x_i + shift and whether |r_ij| < rcut: the one
// test of every kernel that decides membership (so all decide alike).
__device__ inline bool within_cut(const double *x, int j, double xi0, double xi1, double xi2, int s, double L0,
                                  double L1, double L2, double rc2, double &d0, double &d1, double &d2)
{
    d0 = (x[3 * j] - xi0) + (int)(signed char)(s & 0xFF) * L0;
    d1 = (x[3 * j + 1] - xi1) + (int)(signed char)((s >> 8) & 0xFF) * L1;
    d2 = (x[3 * j + 2] - xi2) + (int)(signed char)((s >> 16) & 0xFF) * L2;
    return d0 * d0 + d1 * d1 + d2 * d2 < rc2;
}

// What a kernel keeps per neighbor in its LDS slice.
enum EnvMode {
    ENV_FWD = 0,    // R_j, t_j, interval
    ENV_BWD = 1,    // r_ij, t_j, interval, candidate slot (R_j is recomputed from r_ij)
    ENV_PLAIN = 2,  // R_j, r_ij, (t, ds/dr, 1/r, s), interval, j for the untabulated path
    ENV_BWDR = 3    // r_ij, R_j, t_j, interval, candidate slot (per-neighbor backward)
};

// Per-wave LDS slice (arrays of sel entries; V4 arrays first for alignment).
template <typename real>
struct NbrLDS {
    V4<real> *R;   // R_j (ENV_FWD, ENV_PLAIN); holds r_ij and the type during the scan
    V4<real> *Dv;  // r_ij and the neighbor's type (ENV_BWD, ENV_PLAIN, ENV_BWDR)
    V4<real> *P;   // t, ds/dr, 1/r, s (ENV_PLAIN)
    real *t;       // offset of s_j from its interval's left node
    int *th;       // table interval (bit 30: s past the table end)
    int *j;        // neighbor index j (ENV_PLAIN) or its candidate slot (ENV_BWD)
};

template <typename real>
__device__ inline void gate(const EnvArgs &A, real r, real &w, real &dw)
{
    real rs = (real)A.rs, rc = (real)A.rc;
    if (r < rs) { w = 1; dw = 0; return; }
    if (r >= rc) { w = 0; dw = 0; return; }
    real L = rc - rs;
    real u = (r - rs) / L;
    if (A.switch_kind == 1) {
        const real pi = (real)3.141592653589793;
        w = (real)0.5 * cos(pi * u) + (real)0.5;
        dw = (real)-0.5 * pi * sin(pi * u) / L;
    } else {
        real u2 = u * u, u3 = u2 * u;
        w = (real)1 + u3 * ((real)-10 + u * ((real)15 - (real)6 * u));
        dw = u2 * ((real)-30 + u * ((real)60 - (real)30 * u)) / L;
    }
    // both gates lie in [0, 1]; near rcut the polynomial can round to a tiny
    // negative value, which would give s < 0 and an interval index below 0
    w = w < (real)0 ? (real)0 : w;
}

constexpr int kOobBit = 1 << 30;

// 1/r, s = w(r)/r and ds/dr of one neighbor displacement d.
template <typename real>
__device__ inline void env_geom(const EnvArgs &A, const V4<real> &d, real &rinv, real &s, real &sp)
{
    real r = sqrt(d.x * d.x + d.y * d.y + d.z * d.z);
    real w, dw;
    gate<real>(A, r, w, dw);
    rinv = (real)1 / r;
    s = w * rinv;
    sp = dw * rinv - s * rinv;
}

__device__ inline int s8(int v, int sh) { return (int)(signed char)((v >> sh) & 0xFF); }

// Rank of an image shift among equal distances to the same atom j: the
// signed components compared in the order x, y, z (so (-1,0,0) precedes
// (0,-1,0), which precedes (0,0,1)).  Returned as one integer that orders
// like that lexicographic comparison.
__device__ inline int shift_order(int s)
{
    return ((s8(s, 0) + 128) << 16) | ((s8(s, 8) + 128) << 8) | (s8(s, 16) + 128);
}

// Table interval of s (left-closed) and the offset t from its left node;
// returns 1 when s lies past the table end: then s is clamped there (G is
// constant, G' = 0) and bit 30 of th tells the backward to drop G'.
template <typename real>
__device__ inline int table_interval(const EnvArgs &A, real s, int &th, real &t)
{
    if (s < (real)A.s_max) {
        int q = (int)floor(s / (real)A.h);
        q = q > 0 ? q : 0;
        th = q < A.n_fine - 1 ? q : A.n_fine - 1;
        t = s - (real)th * (real)A.h;
        return 0;
    }
    if (A.n_tail > 0 && s < (real)A.tail_max) {
        int q = (int)floor((s - (real)A.s_max) / (real)A.h_tail);
        q = q > 0 ? q : 0;
        q = q < A.n_tail - 1 ? q : A.n_tail - 1;
        th = A.n_fine + q;
        t = s - ((real)A.s_max + (real)q * (real)A.h_tail);
        return 0;
    }
    th = (A.n_fine + A.n_tail - 1) | kOobBit;
    t = (real)(A.n_tail > 0 ? A.h_tail : A.h);
    return 1;
}

// Record of one compacted neighbor: r_ij and its candidate slot c (< 2^24)
// with the neighbor's type in bits 24..25 (an int carried in the bits of a
// float, or exactly as a double).
__device__ inline int record_slot(float w) { return __builtin_bit_cast(int, w); }
__device__ inline int record_slot(double w) { return (int)w; }
__device__ inline int slot_code(int c, int ty) { return c | (ty << 24); }
template <typename real>
__device__ inline void put_record(const EnvArgs &A, int i, int pos, double d0, double d1, double d2, int c)
{
    V4<real> *rec = reinterpret_cast<V4<real> *>(A.rec) + (long)i * A.sel + pos;
    if (sizeof(real) == 4)
        *reinterpret_cast<V4<float> *>(rec) =
            V4<float>{(float)d0, (float)d1, (float)d2, __builtin_bit_cast(float, c)};
    else
        *reinterpret_cast<V4<double> *>(rec) = V4<double>{d0, d1, d2, (double)c};
}
// Pair gradient slot of candidate c of atom i: 4 floats (one 16-byte
// access) or 3 doubles.
template <typename real>
__device__ inline real *pg_slot(void *pg, int cap, long i, int c)
{
    return reinterpret_cast<real *>(pg) + ((long)i * cap + c) * (sizeof(real) == 4 ? 4 : 3);
}
template <typename real>
__device__ inline void put_pg(void *pg, int cap, long i, int c, real g0, real g1, real g2)
{
    real *g = pg_slot<real>(pg, cap, i, c);
    if (sizeof(real) == 4) {
        *reinterpret_cast<V4<float> *>(g) = V4<float>{(float)g0, (float)g1, (float)g2, 0.f};
    } else {
        g[0] = g0;
        g[1] = g1;
        g[2] = g2;
    }
}
// Zero pair gradient for candidate slot c of atom i (not kept this step).
template <typename real>
__device__ inline void zero_pg(const EnvArgs &A, int i, int c)
{
    put_pg<real>(A.pg, A.cap, i, c, (real)0, (real)0, (real)0);
}

// Per neighbor k < nn of the slice: s, R_j, the table interval and offset
// (and what MODE keeps); returns this lane's count of look-ups past the table.
template <typename real, int MODE, bool TAB>
__device__ int finish_env(const EnvArgs &A, NbrLDS<real> L, int nn, int lane)
{
    int oob = 0;
    for (int k = lane; k < nn; k += 64) {
        V4<real> d = (MODE == ENV_BWD || MODE == ENV_BWDR) ? L.Dv[k] : L.R[k];
        real rinv, s, sp;
        env_geom<real>(A, d, rinv, s, sp);
        int th = 0;
        real t = 0;
        if (TAB) {
            oob += table_interval<real>(A, s, th, t);
            th += (int)d.w * A.n_int;   // the neighbor type's table (d.w holds the type)
        }
        if (MODE != ENV_BWD) L.R[k] = V4<real>{s, s * d.x * rinv, s * d.y * rinv, s * d.z * rinv};
        L.t[k] = t;
        L.th[k] = th;
        if (MODE == ENV_PLAIN) {
            L.Dv[k] = d;
            L.P[k] = V4<real>{t, sp, rinv, s};
        }
    }
    return oob;
}

// The candidates [c0, c0 + ct) of atom i (one neighbor type ty): those
// within rcut, the lim nearest, go to LDS positions base, base + 1, ...
// Returns how many lie within rcut.
template <typename real, int MODE>
__device__ int scan_candidates(int i, const EnvArgs &A, NbrLDS<real> L, int lane, int c0, int ct, int lim,
                               int base, int ty, double xi0, double xi1, double xi2, double L0, double L1,
                               double L2)
{
    const int *nei = A.nei + (long)i * A.cap;
    const int *shf = A.shift + (long)i * A.cap;
    const real rty = (real)ty;
    int n_in = 0;
    // four chunks of 64 candidates per pass: the index, shift and position
    // loads of all of them are in flight together (the ~218 candidates of a
    // copper atom's scan prefix in one pass)
    constexpr int NCH = 4;
    for (int b = 0; b < ct; b += 64 * NCH) {
        int kk[NCH], jj[NCH], ss[NCH];
        bool ll[NCH], inn[NCH];
        double dd[NCH][3];
#pragma unroll
        for (int h = 0; h < NCH; h++) {
            kk[h] = c0 + b + 64 * h + lane;
            ll[h] = b + 64 * h + lane < ct;
            jj[h] = ll[h] ? nei[kk[h]] : 0;
            ss[h] = ll[h] ? shf[kk[h]] : 0;
        }
#pragma unroll
        for (int h = 0; h < NCH; h++) {
            dd[h][0] = dd[h][1] = dd[h][2] = 0;
            inn[h] = ll[h] && within_cut(A.x, jj[h], xi0, xi1, xi2, ss[h], L0, L1, L2, A.rc2, dd[h][0], dd[h][1],
                                         dd[h][2]);
        }
#pragma unroll
        for (int h = 0; h < NCH; h++) {
            const bool in = inn[h];
            const double d0 = dd[h][0], d1 = dd[h][1], d2 = dd[h][2];
            unsigned long long mask = __ballot(in);
            int q = n_in + __popcll(mask & ((1ull << lane) - 1ull));
            if (in && q < lim) {
                int pos = base + q;
                (MODE == ENV_BWD ? L.Dv : L.R)[pos] = V4<real>{(real)d0, (real)d1, (real)d2, rty};
                if (MODE != ENV_FWD) L.j[pos] = jj[h];
                if (MODE == ENV_FWD && A.rec) put_record<real>(A, i, pos, d0, d1, d2, slot_code(kk[h], ty));
            }
            n_in += __popcll(mask);
        }
    }
    if (n_in > lim) {
        // keep the lim nearest by (r^2, j, image shift x, y, z); ranks are a
        // permutation
        for (int k = c0 + lane; k < c0 + ct; k += 64) {
            int j = nei[k], s = shf[k];
            double d0, d1, d2;
            if (!within_cut(A.x, j, xi0, xi1, xi2, s, L0, L1, L2, A.rc2, d0, d1, d2)) continue;
            double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            int so = shift_order(s);
            int rank = 0;
            for (int q = c0; q < c0 + ct; q++) {
                int jq = nei[q], sq = shf[q];
                double e0, e1, e2;
                if (!within_cut(A.x, jq, xi0, xi1, xi2, sq, L0, L1, L2, A.rc2, e0, e1, e2)) continue;
                double rq = e0 * e0 + e1 * e1 + e2 * e2;
                bool less = rq < r2 || (rq == r2 && (jq < j || (jq == j && shift_order(sq) < so)));
                rank += less ? 1 : 0;
            }
            if (rank < lim) {
                int pos = base + rank;
                (MODE == ENV_BWD ? L.Dv : L.R)[pos] = V4<real>{(real)d0, (real)d1, (real)d2, rty};
                if (MODE != ENV_FWD) L.j[pos] = j;
                if (MODE == ENV_FWD && A.rec) put_record<real>(A, i, pos, d0, d1, d2, slot_code(k, ty));
            } else if (MODE == ENV_FWD && A.pg) {
                zero_pg<real>(A, i, k);   // within rcut but beyond the lim nearest
            }
        }
    }
    return n_in;
}

// Neighbors of atom i within rcut, the sel nearest (of each type the sel_t
// nearest), into LDS, grouped by type; returns their number (uniform over
// the wave).  n_in_out: neighbors within rcut; over_out: 1 when a limit cut
// some off; oob_out: table look-ups past the end.
template <typename real, int MODE, bool TAB = true>
__device__ int build_env(int i, const EnvArgs &A, NbrLDS<real> L, int lane, int &n_in_out, int &over_out,
                         int &oob_out)
{
    int nc = A.cnt[i];
    double xi0 = A.x[3 * i], xi1 = A.x[3 * i + 1], xi2 = A.x[3 * i + 2];
    double L0 = A.L0, L1 = A.L1, L2 = A.L2;
    if (A.atomL) {
        L0 = A.atomL[3 * i];
        L1 = A.atomL[3 * i + 1];
        L2 = A.atomL[3 * i + 2];
    }
    // A candidate past the prefix was farther than rcut + margin at build;
    // both atoms moved at most disp since, so it is now farther than
    // rcut + margin - 2 disp, and beyond rcut while 2 disp + slack <= margin
    // (the slack covers the FP32 rounding of the stored distance).
    bool prefix = false;
    if (A.inner) prefix = 2.0 * __longlong_as_double((long long)*A.disp) + kScanSlack <= A.margin;
    int nn = 0, n_in = 0, over = 0;
    if (A.ntypes <= 1) {
        if (prefix) nc = A.inner[(long)i * kMaxTypes];
        n_in = scan_candidates<real, MODE>(i, A, L, lane, 0, nc, A.sel, 0, 0, xi0, xi1, xi2, L0, L1, L2);
        nn = n_in < A.sel ? n_in : A.sel;
        over = n_in > A.sel;
    } else {
        int c0 = 0;
        for (int ty = 0; ty < A.ntypes; ty++) {
            int ct = A.tcnt[(long)i * kMaxTypes + ty];
            int cs = prefix ? A.inner[(long)i * kMaxTypes + ty] : ct;
            int lim = A.sel_t[ty];
            int m = scan_candidates<real, MODE>(i, A, L, lane, c0, cs, lim, nn, ty, xi0, xi1, xi2, L0, L1, L2);
            nn += m < lim ? m : lim;
            n_in += m;
            over |= m > lim;
            c0 += ct;
        }
    }
    if (MODE == ENV_FWD && A.rec && lane == 0) A.rcnt[i] = nn | (over ? kTruncBit : 0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    oob_out = finish_env<real, MODE, TAB>(A, L, nn, lane);
    n_in_out = n_in;
    over_out = over;
    return nn;
}

// The backward's neighbors of atom i: read back the forward's records (no
// scan of the skin list), then the same per-neighbor quantities.
template <typename real, int MODE = ENV_BWD>
__device__ int load_env(int i, const EnvArgs &A, NbrLDS<real> L, int lane)
{
    int nn = A.rcnt[i] & ~kTruncBit;
    const V4<real> *rec = reinterpret_cast<const V4<real> *>(A.rec) + (long)i * A.sel;
    // four records per lane in flight
    for (int k0 = 0; k0 < nn; k0 += 256) {
        V4<real> r[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            int k = k0 + 64 * u + lane;
            if (k < nn) r[u] = rec[k];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            int k = k0 + 64 * u + lane;
            if (k < nn) {
                int code = record_slot(r[u].w);
                L.Dv[k] = V4<real>{r[u].x, r[u].y, r[u].z, (real)(code >> 24)};
                L.j[k] = code & 0xFFFFFF;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    finish_env<real, MODE, true>(A, L, nn, lane);
    return nn;
}

template <typename real>
__device__ inline void record_flags(const EnvArgs &A, int lane, int n_in, int over, int oob)
{
    // wave-wide sum of oob
    for (int off = 32; off > 0; off >>= 1) oob += __shfl_xor(oob, off);
    if (lane == 0) {
        // the maximum only grows: an atomic only when this atom would raise
        // the value read (one address shared by every wave of the launch, so
        // an atomic per wave would serialise them)
        int seen = __hip_atomic_load(&A.flags[kFlagMaxNei], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (n_in > seen) atomicMax(&A.flags[kFlagMaxNei], n_in);
        if (over) atomicAdd(&A.flags[kFlagSelOverflow], 1);
        if (oob) atomicAdd(&A.flags[kFlagTableOob], oob);
    }
}

// Bytes of the per-neighbor arrays of one wave's slice (a multiple of the
// V4 size, so slices and what follows them stay aligned).
template <typename real>
constexpr int nbr_lds_bytes(int sel, int mode)
{
    int v4 = mode == ENV_PLAIN ? 3 : (mode == ENV_BWDR ? 2 : 1);
    int ints = mode == ENV_FWD ? 1 : 2;
    int b = sel * (v4 * (int)sizeof(V4<real>) + (int)sizeof(real) + ints * 4);
    constexpr int al = (int)sizeof(V4<real>);
    return (b + al - 1) / al * al;
}

template <typename real>
__device__ NbrLDS<real> carve(char *base, int sel, int mode)
{
    NbrLDS<real> L;
    V4<real> *v = reinterpret_cast<V4<real> *>(base);
    L.R = mode != ENV_BWD ? v : nullptr;
    if (mode != ENV_BWD) v += sel;
    L.Dv = mode != ENV_FWD ? v : nullptr;
    if (mode != ENV_FWD) v += sel;
    L.P = mode == ENV_PLAIN ? v : nullptr;
    if (mode == ENV_PLAIN) v += sel;
    L.t = reinterpret_cast<real *>(v);
    L.th = reinterpret_cast<int *>(L.t + sel);
    L.j = mode != ENV_FWD ? L.th + sel : nullptr;
    return L;
}

inline EnvArgs make_env_args(const dp_model *m, const dp_nlist *nl, const double *x)
{
    EnvArgs A;
    A.x = x;
    A.cnt = nl->cnt;
    A.nei = nl->nei;
    A.shift = nl->shift;
    A.cap = nl->cap;
    A.sel = m->cfg.sel;
    A.L0 = nl->L[0];
    A.L1 = nl->L[1];
    A.L2 = nl->L[2];
    A.atomL = nl->atomL;
    A.rc2 = m->cfg.rcut * m->cfg.rcut;
    A.rs = m->cfg.rcut_smth;
    A.rc = m->cfg.rcut;
    A.switch_kind = m->cfg.switch_kind;
    A.n_fine = m->tab.n_fine;
    A.n_tail = m->tab.n_tail;
    A.h = m->tab.h;
    A.s_max = m->tab.s_max;
    A.h_tail = m->tab.h_tail;
    A.tail_max = m->tab.tail_max;
    A.flags = nl->flags;
    A.rec = nullptr;
    A.rcnt = nullptr;
    A.pg = nullptr;
    A.ntypes = nl->ntypes;
    for (int t = 0; t < kMaxTypes; t++) A.sel_t[t] = t < m->cfg.ntypes ? m->cfg.sel_t[t] : 0;
    A.tcnt = nl->ntypes > 1 ? nl->tcnt : nullptr;
    A.n_int = m->tab.n_int();
    // the prefixes were taken at the build's cut-off: another model's reads everything
    A.inner = (nl->x0 && m->cfg.rcut == nl->rcut_build) ? nl->inner : nullptr;
    A.disp = nl->disp;
    A.margin = nl->margin;
    A.row = nl->ntypes > 1 ? nl->row : nullptr;
    return A;
}

}  // namespace dp
