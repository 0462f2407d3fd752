// env.h -- the environment-matrix stage shared by the compressed and the
// plain paths: filter the skin list to r < rcut, keep the sel nearest, and
// form s = w(r)/r, R = s (1, x/r, y/r, z/r) (paper Eq. 1) and, for the
// table, the interval of s and the offset from its left node (Sec. 3.2).
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
};

// Per-wave LDS slice.
template <typename real>
struct NbrLDS {
    V4<real> *R;   // R_j (4 environment columns); holds r_ij during the scan
    V4<real> *P;   // t (table offset), ds/dr, 1/r, s
    V4<real> *Dv;  // r_ij (backward only)
    int2 *I;       // table interval, neighbor index j
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

__device__ inline int s8(int v, int sh) { return (int)(signed char)((v >> sh) & 0xFF); }

// Neighbors of atom i within rcut, the sel nearest, into LDS; returns their
// number (uniform over the wave).  *oob counts table look-ups past the end.
template <typename real, bool BWD, bool TAB = true>
__device__ int build_env(int i, const EnvArgs &A, NbrLDS<real> L, int lane, int &n_in_out,
                         int &oob_out)
{
    int nc = A.cnt[i];
    const int *nei = A.nei + (long)i * A.cap;
    const int *shf = A.shift + (long)i * A.cap;
    double xi0 = A.x[3 * i], xi1 = A.x[3 * i + 1], xi2 = A.x[3 * i + 2];
    double L0 = A.L0, L1 = A.L1, L2 = A.L2;
    if (A.atomL) {
        L0 = A.atomL[3 * i];
        L1 = A.atomL[3 * i + 1];
        L2 = A.atomL[3 * i + 2];
    }
    int n_in = 0;
    for (int base = 0; base < nc; base += 64) {
        int k = base + lane;
        bool in = false;
        double d0 = 0, d1 = 0, d2 = 0;
        int j = 0;
        if (k < nc) {
            j = nei[k];
            int s = shf[k];
            d0 = (A.x[3 * j] - xi0) + s8(s, 0) * L0;
            d1 = (A.x[3 * j + 1] - xi1) + s8(s, 8) * L1;
            d2 = (A.x[3 * j + 2] - xi2) + s8(s, 16) * L2;
            in = d0 * d0 + d1 * d1 + d2 * d2 < A.rc2;
        }
        unsigned long long mask = __ballot(in);
        int pos = n_in + __popcll(mask & ((1ull << lane) - 1ull));
        if (in && pos < A.sel) {
            L.R[pos] = V4<real>{(real)d0, (real)d1, (real)d2, (real)0};
            L.I[pos] = make_int2(0, j);
        }
        n_in += __popcll(mask);
    }
    if (n_in > A.sel) {
        // keep the sel nearest by (r^2, j, image); ranks are a permutation
        for (int k = lane; k < nc; k += 64) {
            int j = nei[k], s = shf[k];
            double d0 = (A.x[3 * j] - xi0) + s8(s, 0) * L0;
            double d1 = (A.x[3 * j + 1] - xi1) + s8(s, 8) * L1;
            double d2 = (A.x[3 * j + 2] - xi2) + s8(s, 16) * L2;
            double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (!(r2 < A.rc2)) continue;
            int rank = 0;
            for (int q = 0; q < nc; q++) {
                int jq = nei[q], sq = shf[q];
                double e0 = (A.x[3 * jq] - xi0) + s8(sq, 0) * L0;
                double e1 = (A.x[3 * jq + 1] - xi1) + s8(sq, 8) * L1;
                double e2 = (A.x[3 * jq + 2] - xi2) + s8(sq, 16) * L2;
                double rq = e0 * e0 + e1 * e1 + e2 * e2;
                if (!(rq < A.rc2)) continue;
                bool less = rq < r2 || (rq == r2 && (jq < j || (jq == j && sq < s)));
                rank += less ? 1 : 0;
            }
            if (rank < A.sel) {
                L.R[rank] = V4<real>{(real)d0, (real)d1, (real)d2, (real)0};
                L.I[rank] = make_int2(0, j);
            }
        }
    }
    int nn = n_in < A.sel ? n_in : A.sel;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int oob = 0;
    for (int k = lane; k < nn; k += 64) {
        V4<real> d = L.R[k];
        real r = sqrt(d.x * d.x + d.y * d.y + d.z * d.z);
        real w, dw;
        gate<real>(A, r, w, dw);
        real rinv = (real)1 / r;
        real s = w * rinv;
        real sp = dw * rinv - s * rinv;
        // table interval of s (left-closed) and offset from its left node
        int th = 0;
        real t = 0;
        if (!TAB) {
        } else if (s < (real)A.s_max) {
            int q = (int)floor(s / (real)A.h);
            q = q > 0 ? q : 0;
            th = q < A.n_fine - 1 ? q : A.n_fine - 1;
            t = s - (real)th * (real)A.h;
        } else if (A.n_tail > 0 && s < (real)A.tail_max) {
            int q = (int)floor((s - (real)A.s_max) / (real)A.h_tail);
            q = q > 0 ? q : 0;
            q = q < A.n_tail - 1 ? q : A.n_tail - 1;
            th = A.n_fine + q;
            t = s - ((real)A.s_max + (real)q * (real)A.h_tail);
        } else {
            // clamped to the table end: G is constant there, so G' = 0
            // (flag bit 30 on the interval tells the backward to drop G')
            th = (A.n_fine + A.n_tail - 1) | kOobBit;
            t = (real)(A.n_tail > 0 ? A.h_tail : A.h);
            oob++;
        }
        L.R[k] = V4<real>{s, s * d.x * rinv, s * d.y * rinv, s * d.z * rinv};
        L.P[k] = V4<real>{t, sp, rinv, s};
        if (BWD) L.Dv[k] = d;
        L.I[k].x = th;
    }
    n_in_out = n_in;
    oob_out = oob;
    return nn;
}

template <typename real>
__device__ inline void record_flags(const EnvArgs &A, int lane, int n_in, int oob)
{
    // wave-wide sum of oob
    for (int off = 32; off > 0; off >>= 1) oob += __shfl_xor(oob, off);
    if (lane == 0) {
        atomicMax(&A.flags[kFlagMaxNei], n_in);
        if (n_in > A.sel) atomicAdd(&A.flags[kFlagSelOverflow], 1);
        if (oob) atomicAdd(&A.flags[kFlagTableOob], oob);
    }
}

template <typename real>
constexpr int lds_bytes_per_wave(int sel, bool bwd)
{
    return sel * (int)(sizeof(V4<real>) * (bwd ? 3 : 2) + sizeof(int2)) +
           (bwd ? 0 : 4 * kM * (int)sizeof(real));
}

template <typename real>
__device__ NbrLDS<real> carve(char *base, int sel, bool bwd, real *&Tl)
{
    NbrLDS<real> L;
    L.R = reinterpret_cast<V4<real> *>(base);
    L.P = L.R + sel;
    L.Dv = bwd ? L.P + sel : nullptr;
    L.I = reinterpret_cast<int2 *>(bwd ? L.Dv + sel : L.P + sel);
    Tl = reinterpret_cast<real *>(L.I + sel);
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
    return A;
}

}  // namespace dp
