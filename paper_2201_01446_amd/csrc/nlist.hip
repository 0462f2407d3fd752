// nlist.hip -- neighbor list with a skin on gfx950.
//
// L_Rc(i) of the paper (Sec. 2.1) is built here with a buffer of `skin`
// beyond R_c (the MD protocol of the physical-systems section uses 2 A), so
// that the per-step kernels only filter the stored candidates by the current
// distance.  For each atom the candidates are all (j, periodic image) within
// rcut + skin, sorted by distance; the sort makes neighbors that fall into
// the same table interval consecutive, which the fused kernels exploit.
//
// With several atom types the candidates are grouped by the neighbor's type
// (nearest first within a type) and their number per type is kept, so that
// the per-type limits and tables apply to contiguous runs.
//
// Periodic boxes: atoms are wrapped into the box and binned into a grid of
// nc >= 1 cells per edge with edge >= (rcut + skin)/2.  An atom scans the
// cell offsets -R..R (R <= 2) per axis; an offset that leaves the grid maps to
// the wrapped cell and an image shift, so boxes smaller than the cut-off
// sphere see several images of the same atom (and of the atom itself).
// Each candidate stores j and the image shift n with r_ij = x_j - x_i + n L in
// the caller's (unwrapped) coordinates.

#include "dp_internal.h"
#include "env.h"

#include <cmath>
#include <cstdio>

namespace dp {

namespace {

__device__ inline int pack_shift(int a, int b, int c)
{
    return (a & 0xFF) | ((b & 0xFF) << 8) | ((c & 0xFF) << 16);
}

// 64-bit sort key: type (2 bits), distance (31 bits: the bits of a
// non-negative float, which order like unsigned integers), atom index (24
// bits), image code (7 bits, 5 values per axis).
__device__ inline unsigned long long make_key(int ty, float r, int j, int code)
{
    return ((unsigned long long)(unsigned)ty << 62) | ((unsigned long long)__float_as_uint(r) << 31) |
           ((unsigned long long)(unsigned)j << 7) | (unsigned)code;
}
__device__ inline int key_type(unsigned long long k) { return (int)(k >> 62); }

__global__ void k_zero_int(int *p, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Wrap every atom into the box, record its image index and cell, and store
// it (wrapped position, index, type) in its cell's slot.
__global__ void k_bin(int n, const double *__restrict__ x, const int *__restrict__ types,
                      const int *__restrict__ key_types, double Lx, double Ly, double Lz, int ncx, int ncy,
                      int ncz, int cellcap, double *__restrict__ wpos, int *__restrict__ wrap,
                      int *__restrict__ cell_cnt, CellAtom *__restrict__ cell_atoms, int *__restrict__ flags)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (types && types[i] != 0) atomicAdd(&flags[kFlagBadType], 1);   // one-type lists only
    if (!isfinite(x[3 * i]) || !isfinite(x[3 * i + 1]) || !isfinite(x[3 * i + 2])) atomicOr(&flags[kFlagBadCoord], 1);
    double L[3] = {Lx, Ly, Lz};
    int nc[3] = {ncx, ncy, ncz};
    int k[3], c[3];
    double w3[3];
    for (int a = 0; a < 3; a++) {
        double xa = x[3 * i + a];
        double fk = floor(xa / L[a]);
        double w = xa - fk * L[a];
        if (w >= L[a]) { w -= L[a]; fk += 1.0; }
        if (w < 0.0) { w += L[a]; fk -= 1.0; }
        // image index must fit the int8 shift encoding with room to spare
        if (fk > 60.0 || fk < -60.0) { atomicAdd(&flags[kFlagCapOverflow], 1); fk = 0.0; }
        k[a] = (int)fk;
        wpos[3 * i + a] = w;
        w3[a] = w;
        int ci = (int)(w * nc[a] / L[a]);
        c[a] = ci < 0 ? 0 : (ci >= nc[a] ? nc[a] - 1 : ci);
    }
    wrap[i] = pack_shift(k[0], k[1], k[2]);
    int cell = (c[0] * ncy + c[1]) * ncz + c[2];
    int slot = atomicAdd(&cell_cnt[cell], 1);
    if (slot < cellcap) {
        CellAtom e;
        e.x = w3[0];
        e.y = w3[1];
        e.z = w3[2];
        e.j = i;
        e.type = key_types ? key_types[i] : 0;
        cell_atoms[(long)cell * cellcap + slot] = e;
    } else {
        atomicAdd(&flags[kFlagCellOverflow], 1);
    }
}

// Sorts keys[0, 64 KPL) ascending with one wave: a bitonic network over
// the wave's registers, element e = lane KPL + r in register r of its lane.
// Exchanges between elements fewer than KPL apart stay in the lane; the
// others pair lane with lane ^ (distance / KPL) through a shuffle, each lane
// keeping the minimum or the maximum of the two.  keys is read once and
// written once (LDS); the caller synchronises around it.
template <int KPL>
__device__ void wave_sort(unsigned long long *keys)
{
    const int lane = threadIdx.x;
    unsigned long long v[KPL];
#pragma unroll
    for (int r = 0; r < KPL; r++) v[r] = keys[lane * KPL + r];
#pragma unroll
    for (int k = 2; k <= 64 * KPL; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= KPL) {
                const int m = j / KPL;
                const bool lower = (lane & m) == 0;
#pragma unroll
                for (int r = 0; r < KPL; r++) {
                    const bool up = ((lane * KPL + r) & k) == 0;   // ascending run
                    const unsigned long long o = __shfl_xor(v[r], m);
                    const bool keep_min = up == lower;
                    v[r] = (v[r] < o) == keep_min ? v[r] : o;
                }
            } else {
#pragma unroll
                for (int r = 0; r < KPL; r++) {
                    if (r & j) continue;
                    const bool up = ((lane * KPL + r) & k) == 0;
                    const unsigned long long a = v[r], b = v[r + j];
                    const bool sw = (a > b) == up;
                    v[r] = sw ? b : a;
                    v[r + j] = sw ? a : b;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < KPL; r++) keys[lane * KPL + r] = v[r];
}

// The same network on keys[0, P) in LDS, for P above 512 (rows of more than
// 512 candidates; sixteen keys per lane would triple the registers of the
// kernels that sort).
__device__ void lds_sort(unsigned long long *keys, int P)
{
    const int lane = threadIdx.x;
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < P / 2; t += 64) {
                const int i0 = ((t & ~(j - 1)) << 1) | (t & (j - 1));   // j is a power of two
                const int i1 = i0 + j;
                const bool up = (i0 & k) == 0;
                const unsigned long long a = keys[i0], b = keys[i1];
                if ((a > b) == up) {
                    keys[i0] = b;
                    keys[i1] = a;
                }
            }
            __syncthreads();
        }
    }
}

// keys[0, P) ascending, P = 64 .. 1024 a power of two.
__device__ void sort_keys(unsigned long long *keys, int P)
{
    switch (P) {
    case 64: wave_sort<1>(keys); break;
    case 128: wave_sort<2>(keys); break;
    case 256: wave_sort<4>(keys); break;
    case 512: wave_sort<8>(keys); break;
    default: lds_sort(keys, P); break;
    }
}

__device__ void finish_atom(int i, int cnt, int cap, unsigned long long *keys, const int *wrap,
                            int ki_packed, int *out_cnt, int *out_nei, int *out_shift, float *out_dist,
                            int *out_tcnt, int *flags, int joff)
{
    int lane = threadIdx.x;
    if (cnt > cap) {
        if (lane == 0) atomicAdd(&flags[kFlagCapOverflow], 1);
        cnt = cap;
    }
    int P = 64;   // <= the LDS array (the capacity rounded up to a power of two, >= 64)
    while (P < cnt) P <<= 1;
    for (int t = cnt + lane; t < P; t += 64) keys[t] = ~0ull;
    __syncthreads();
    sort_keys(keys, P);
    __syncthreads();
    int kix = (int)(signed char)(ki_packed & 0xFF), kiy = (int)(signed char)((ki_packed >> 8) & 0xFF),
        kiz = (int)(signed char)((ki_packed >> 16) & 0xFF);
    for (int t = lane; t < cnt; t += 64) {
        unsigned long long key = keys[t];
        int lo = (int)(key & 0x7FFFFFFFu);
        int j = lo >> 7;
        int code = lo & 127;
        int sx = code / 25 - 2, sy = (code / 5) % 5 - 2, sz = code % 5 - 2;
        int kj = wrap ? wrap[j] : 0;
        int kjx = (int)(signed char)(kj & 0xFF), kjy = (int)(signed char)((kj >> 8) & 0xFF),
            kjz = (int)(signed char)((kj >> 16) & 0xFF);
        out_nei[(long)i * cap + t] = j + joff;
        out_shift[(long)i * cap + t] = pack_shift(sx + kix - kjx, sy + kiy - kjy, sz + kiz - kjz);
        out_dist[(long)i * cap + t] = __uint_as_float((unsigned)((key >> 31) & 0x7FFFFFFFu));
    }
    // the rest of the row reads as beyond every candidate (the reverse
    // search loads a fixed window that may reach past the count)
    for (int t = cnt + lane; t < cap; t += 64) out_dist[(long)i * cap + t] = __builtin_huge_valf();
    if (out_tcnt) {
        int c[kMaxTypes] = {0, 0, 0, 0};
        for (int b = 0; b < cnt; b += 64) {
            int ty = b + lane < cnt ? key_type(keys[b + lane]) : -1;
            for (int q = 0; q < kMaxTypes; q++) c[q] += __popcll(__ballot(ty == q));
        }
        if (lane == 0)
            for (int q = 0; q < kMaxTypes; q++) out_tcnt[(long)i * kMaxTypes + q] = c[q];
    }
    if (lane == 0) out_cnt[i] = cnt;
}

// Candidates of one atom per 64-thread block: each lane takes cell offsets
// of the (2R+1)^3 window (two at most, R <= 2) and scans the atoms of that
// cell, whose positions sit in the cell's own slots (no gather through an
// index), four loads in flight at a time.
__global__ void __launch_bounds__(64) k_candidates_cells(
    int n, const double *__restrict__ wpos, const int *__restrict__ wrap, double Lx, double Ly,
    double Lz, int ncx, int ncy, int ncz, int Rx, int Ry, int Rz, int cellcap,
    const int *__restrict__ cell_cnt, const CellAtom *__restrict__ cell_atoms, double rcs2, int cap,
    int *__restrict__ out_cnt, int *__restrict__ out_nei, int *__restrict__ out_shift,
    float *__restrict__ out_dist, int *__restrict__ out_tcnt, int *__restrict__ flags, int joff)
{
    HIP_DYNAMIC_SHARED(unsigned long long, keys)
    __shared__ int count;
    int i = xcd_item(blockIdx.x, gridDim.x);
    if (i >= n) return;   // the whole (one-wave) block
    const int lane = threadIdx.x;
    if (lane == 0) count = 0;
    __syncthreads();
    const double wi0 = wpos[3 * i], wi1 = wpos[3 * i + 1], wi2 = wpos[3 * i + 2];
    const int ci0 = min((int)(wi0 * ncx / Lx), ncx - 1), ci1 = min((int)(wi1 * ncy / Ly), ncy - 1),
              ci2 = min((int)(wi2 * ncz / Lz), ncz - 1);
    const int wx = 2 * Rx + 1, wy = 2 * Ry + 1, wz = 2 * Rz + 1;
    const int noff = wx * wy * wz;
    for (int oc = lane; oc < noff; oc += 64) {
        int dx = oc / (wy * wz) - Rx, dy = (oc / wz) % wy - Ry, dz = oc % wz - Rz;
        int cx = ci0 + dx, cy = ci1 + dy, cz = ci2 + dz;
        // floor division / modulo for negative offsets
        int sx = (cx >= 0) ? cx / ncx : -((-cx + ncx - 1) / ncx);
        int sy = (cy >= 0) ? cy / ncy : -((-cy + ncy - 1) / ncy);
        int sz = (cz >= 0) ? cz / ncz : -((-cz + ncz - 1) / ncz);
        cx -= sx * ncx;
        cy -= sy * ncy;
        cz -= sz * ncz;
        const int cell = (cx * ncy + cy) * ncz + cz;
        const int m = min(cell_cnt[cell], cellcap);
        const double ox = sx * Lx - wi0, oy = sy * Ly - wi1, oz = sz * Lz - wi2;
        const int code = (sx + 2) * 25 + (sy + 2) * 5 + (sz + 2);
        const CellAtom *ca = cell_atoms + (long)cell * cellcap;
        for (int t = 0; t < m; t += 4) {
            CellAtom q[4];
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (t + u < m) q[u] = ca[t + u];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (t + u >= m) break;
                const double d0 = q[u].x + ox, d1 = q[u].y + oy, d2 = q[u].z + oz;
                const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                if (r2 < rcs2 && !(q[u].j == i && code == 62 /* image (0, 0, 0) */)) {
                    int slot = atomicAdd(&count, 1);
                    if (slot < cap) keys[slot] = make_key(q[u].type, (float)sqrt(r2), q[u].j, code);
                }
            }
        }
    }
    __syncthreads();
    finish_atom(i, count, cap, keys, wrap, wrap[i], out_cnt, out_nei, out_shift, out_dist, out_tcnt, flags,
                joff);
}

// Open boundary: brute force over all atoms (for clusters of modest size).
// check_types: one-type lists flag any type other than 0; key_types: the
// types that group a several-type list (NULL: one type).
__global__ void __launch_bounds__(64) k_candidates_open(int n, const double *__restrict__ x,
                                                        const int *__restrict__ check_types,
                                                        const int *__restrict__ key_types, double rcs2,
                                                        int cap, int *__restrict__ out_cnt,
                                                        int *__restrict__ out_nei,
                                                        int *__restrict__ out_shift,
                                                        float *__restrict__ out_dist,
                                                        int *__restrict__ out_tcnt,
                                                        int *__restrict__ flags, int joff)
{
    HIP_DYNAMIC_SHARED(unsigned long long, keys)
    __shared__ int count;
    int i = xcd_item(blockIdx.x, gridDim.x);
    if (i >= n) return;   // the whole (one-wave) block
    int lane = threadIdx.x;
    if (lane == 0) {
        count = 0;
        if (check_types && check_types[i] != 0) atomicAdd(&flags[kFlagBadType], 1);
        if (!isfinite(x[3 * i]) || !isfinite(x[3 * i + 1]) || !isfinite(x[3 * i + 2]))
            atomicOr(&flags[kFlagBadCoord], 1);
    }
    __syncthreads();
    double xi0 = x[3 * i], xi1 = x[3 * i + 1], xi2 = x[3 * i + 2];
    for (int j = lane; j < n; j += 64) {
        if (j == i) continue;
        double d0 = x[3 * j] - xi0, d1 = x[3 * j + 1] - xi1, d2 = x[3 * j + 2] - xi2;
        double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (r2 < rcs2) {
            int slot = atomicAdd(&count, 1);
            if (slot < cap)
                keys[slot] = make_key(key_types ? key_types[j] : 0, (float)sqrt(r2), j, 62 /* image (0,0,0) */);
        }
    }
    __syncthreads();
    finish_atom(i, count, cap, keys, nullptr, 0, out_cnt, out_nei, out_shift, out_dist, out_tcnt, flags, joff);
}

// Per atom (one wave) and type run: how many candidates have a build
// distance <= lim.  The runs are sorted by distance, so these are a prefix.
__global__ void __launch_bounds__(256) k_inner(int n, int cap, int ntypes, const int *__restrict__ cnt,
                                               const int *__restrict__ tcnt, const float *__restrict__ dist,
                                               float lim, int *__restrict__ inner)
{
    int lane = threadIdx.x & 63;
    int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;   // the whole wave
    const float *d = dist + (long)i * cap;
    int c0 = 0;
    for (int ty = 0; ty < ntypes; ty++) {
        int ct = tcnt ? tcnt[(long)i * kMaxTypes + ty] : cnt[i];
        int m = 0;
        for (int b = 0; b < ct; b += 64) m += __popcll(__ballot(b + lane < ct && d[c0 + b + lane] <= lim));
        if (lane == 0) inner[(long)i * kMaxTypes + ty] = m;
        c0 += ct;
    }
}

// Largest |x_i - x0_i|: per block a maximum, then one atomicMax on the bits
// (non-negative doubles order as their unsigned bit patterns).
// A block whose largest displacement d has 2 d >= lim (and d > 0) sets the
// skin flag: a pair now within the evaluating cut-off may have been beyond
// the list's reach at build.  A non-finite position counts as infinitely far
// and also sets the coordinate flag.
__global__ void __launch_bounds__(256) k_displacement(int n, const double *__restrict__ x,
                                                      const double *__restrict__ x0, double lim,
                                                      unsigned long long *__restrict__ disp,
                                                      int *__restrict__ flags)
{
    __shared__ double wmax[4];
    int i = blockIdx.x * 256 + threadIdx.x;
    double d = 0;
    bool bad = false;
    if (i < n) {
        double d0 = x[3 * i] - x0[3 * i], d1 = x[3 * i + 1] - x0[3 * i + 1], d2 = x[3 * i + 2] - x0[3 * i + 2];
        d = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        bad = !isfinite(d);
        if (bad) d = __builtin_huge_val();   // also turns the early end off
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&flags[kFlagBadCoord], 1);
    for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        if (m > 0) atomicMax(disp, (unsigned long long)__double_as_longlong(m));
        if (m > 0 && 2.0 * m >= lim) atomicOr(&flags[kFlagSkin], 1);
    }
}

}  // namespace

void launch_displacement(const dp_nlist *nl, int n, const double *x, double lim, hipStream_t st)
{
    if (!nl->x0 || n <= 0) return;
    launch_fill_zero_int(reinterpret_cast<int *>(nl->disp), 2, st);
    hipLaunchKernelGGL(k_displacement, dim3(div_up(n, 256)), dim3(256), 0, st, n, x, nl->x0, lim, nl->disp,
                       nl->flags);
}

void launch_fill_zero_int(int *p, long n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_zero_int, dim3(div_up(n, 256)), dim3(256), 0, st, p, n);
}

// The positions of the build and each atom's candidate prefixes within
// rcut + margin (lists that carry them).
static dp_status launch_prefix(const dp_model *m, dp_nlist *nl, const double *x, hipStream_t st)
{
    if (!nl->x0) return DP_OK;
    int n = nl->natoms;
    DP_HIP(hipMemcpyAsync(nl->x0, x, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToDevice, st));
    const bool typed = nl->ntypes > 1;
    hipLaunchKernelGGL(k_inner, dim3(div_up(n, 4)), dim3(256), 0, st, n, nl->cap, typed ? nl->ntypes : 1, nl->cnt,
                       typed ? nl->tcnt : nullptr, nl->dist, (float)(m->cfg.rcut + nl->margin), nl->inner);
    return DP_OK;
}

dp_status launch_build_nlist(const dp_model *m, dp_nlist *nl, const double *x, const int *types,
                             bool reset_flags, hipStream_t st)
{
    int n = nl->natoms;
    double rcs2 = nl->rc_build * nl->rc_build;
    // the sort pads the candidate count up to a power of two <= that of cap
    int cap2 = 1;
    while (cap2 < nl->cap) cap2 <<= 1;
    size_t lds = sizeof(unsigned long long) * cap2;
    // several types: the list's own copy (checked by build_type_layout) groups the candidates
    const bool typed = nl->ntypes > 1;
    const int *check = typed ? nullptr : types;
    const int *ktypes = typed ? nl->type : nullptr;
    int *tcnt = typed ? nl->tcnt : nullptr;
    if (reset_flags) launch_fill_zero_int(nl->flags, kNumFlags, st);
    if (!nl->periodic) {
        hipLaunchKernelGGL(k_candidates_open, dim3(xcd_grid(n)), dim3(64), lds, st, n, x, check, ktypes, rcs2,
                           nl->cap, nl->cnt, nl->nei, nl->shift, nl->dist, tcnt, nl->flags, 0);
        launch_reverse(nl, 0, n, st, true);   // open: every image shift is zero
        return launch_prefix(m, nl, x, st);
    }
    long ncell = (long)nl->nc[0] * nl->nc[1] * nl->nc[2];
    launch_fill_zero_int(nl->cell_cnt, ncell, st);
    hipLaunchKernelGGL(k_bin, dim3(div_up(n, 256)), dim3(256), 0, st, n, x, check, ktypes, nl->L[0], nl->L[1],
                       nl->L[2], nl->nc[0], nl->nc[1], nl->nc[2], nl->cellcap, nl->wpos, nl->wrap, nl->cell_cnt,
                       nl->cell_atoms, nl->flags);
    int R[3];
    for (int a = 0; a < 3; a++) {
        double c = nl->L[a] / nl->nc[a];
        R[a] = (int)ceil(nl->rc_build / c - 1e-12);
        if (R[a] > 2) return fail(DP_ERR_UNSUPPORTED, "box edge shorter than (rcut + skin) / 2");
    }
    hipLaunchKernelGGL(k_candidates_cells, dim3(xcd_grid(n)), dim3(64), lds, st, n,
                       nl->wpos, nl->wrap, nl->L[0], nl->L[1],
                       nl->L[2], nl->nc[0], nl->nc[1], nl->nc[2], R[0], R[1], R[2], nl->cellcap,
                       nl->cell_cnt, nl->cell_atoms, rcs2, nl->cap, nl->cnt, nl->nei, nl->shift, nl->dist, tcnt,
                       nl->flags, 0);
    // edges of at least 2 (rcut + skin): a list holds at most one image of
    // any atom, so j's slot for i is the one whose index is i
    const bool uniq = nl->L[0] >= 2 * nl->rc_build && nl->L[1] >= 2 * nl->rc_build && nl->L[2] >= 2 * nl->rc_build;
    launch_reverse(nl, 0, n, st, uniq);
    return launch_prefix(m, nl, x, st);
}

dp_status launch_build_nlist_range(dp_nlist *nl, const double *x, int off, int n, const double *L,
                                   hipStream_t st)
{
    double rcs = nl->rc_build, rcs2 = rcs * rcs;
    int cap2 = 1;
    while (cap2 < nl->cap) cap2 <<= 1;
    size_t lds = sizeof(unsigned long long) * cap2;
    long cap = nl->cap;
    const double *xr = x + 3L * off;
    int *cnt = nl->cnt + off, *nei = nl->nei + off * cap, *shift = nl->shift + off * cap;
    float *dist = nl->dist + off * cap;
    if (!L) {
        hipLaunchKernelGGL(k_candidates_open, dim3(xcd_grid(n)), dim3(64), lds, st, n, xr, (const int *)nullptr,
                           (const int *)nullptr, rcs2, nl->cap, cnt, nei, shift, dist, (int *)nullptr, nl->flags,
                           off);
        return DP_OK;
    }
    int nc[3], R[3];
    for (int a = 0; a < 3; a++) {
        nc[a] = (int)floor(L[a] / (0.5 * rcs));
        if (nc[a] < 1) nc[a] = 1;
        R[a] = (int)ceil(rcs / (L[a] / nc[a]) - 1e-12);
        if (R[a] > 2) return fail(DP_ERR_UNSUPPORTED, "box edge shorter than (rcut + skin) / 2");
    }
    long ncell = (long)nc[0] * nc[1] * nc[2];
    if ((size_t)(ncell * nl->cellcap) > nl->ncell_alloc) return fail(DP_ERR_STATE, "cell grid too small");
    launch_fill_zero_int(nl->cell_cnt, ncell, st);
    hipLaunchKernelGGL(k_bin, dim3(div_up(n, 256)), dim3(256), 0, st, n, xr, (const int *)nullptr,
                       (const int *)nullptr, L[0], L[1], L[2], nc[0], nc[1], nc[2], nl->cellcap, nl->wpos + 3L * off,
                       nl->wrap + off, nl->cell_cnt, nl->cell_atoms, nl->flags);
    hipLaunchKernelGGL(k_candidates_cells, dim3(xcd_grid(n)), dim3(64), lds, st, n, nl->wpos + 3L * off, nl->wrap + off, L[0],
                       L[1], L[2], nc[0], nc[1], nc[2], R[0], R[1], R[2], nl->cellcap, nl->cell_cnt, nl->cell_atoms,
                       rcs2, nl->cap, cnt, nei, shift, dist, (int *)nullptr, nl->flags, off);
    return DP_OK;
}

namespace {

// Expands per-request box edges to per-atom ones; one block per request.
__global__ void k_expand_boxes(const int *__restrict__ off, const double *__restrict__ Lreq,
                               double *__restrict__ atomL)
{
    int r = blockIdx.x;
    for (int i = off[r] + threadIdx.x; i < off[r + 1]; i += blockDim.x)
        for (int a = 0; a < 3; a++) atomL[3L * i + a] = Lreq[3 * r + a];
}

// Per request (block): E = sum of E_i and W = sum of W_i over its atoms, in
// an order fixed relative to the request's first atom (so the result does
// not depend on where the request sits in the batch).
__global__ void __launch_bounds__(256) k_segment_reduce(const int *__restrict__ off,
                                                        const double *__restrict__ e_atom,
                                                        const double *__restrict__ w_atom,
                                                        double *__restrict__ energy, double *__restrict__ virial,
                                                        int *__restrict__ flags)
{
    __shared__ double sh[256][10];
    int r = blockIdx.x, t = threadIdx.x;
    double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = off[r] + t; i < off[r + 1]; i += 256) {
        v[0] += e_atom[i];
        if (w_atom)
            for (int q = 0; q < 9; q++) v[1 + q] += w_atom[9L * i + q];
    }
    for (int q = 0; q < 10; q++) sh[t][q] = v[q];
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (t < s2)
            for (int q = 0; q < 10; q++) sh[t][q] += sh[t + s2][q];
        __syncthreads();
    }
    if (t == 0 && energy) energy[r] = sh[0][0];
    if (t < 9 && virial && w_atom) virial[9 * r + t] = sh[0][1 + t];
    if (t < 10 && !isfinite(sh[0][t])) atomicOr(&flags[kFlagNonFinite], 1);
}

}  // namespace

void launch_segment_reduce(int nreq, const int *offsets, const double *e_atom, const double *w_atom,
                           double *energy, double *virial, int *flags, hipStream_t st)
{
    hipLaunchKernelGGL(k_segment_reduce, dim3(nreq), dim3(256), 0, st, offsets, e_atom, w_atom, energy, virial,
                       flags);
}

void launch_expand_boxes(int nreq, const int *offsets, const double *Lreq, double *atomL, hipStream_t st)
{
    hipLaunchKernelGGL(k_expand_boxes, dim3(nreq), dim3(256), 0, st, offsets, Lreq, atomL);
}


namespace {

__global__ void k_fill_short(short *p, long n, short v)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ inline int neg_shift(int v)
{
    int a = (int)(signed char)(v & 0xFF), b = (int)(signed char)((v >> 8) & 0xFF),
        c = (int)(signed char)((v >> 16) & 0xFF);
    return pack_shift(-a, -b, -c);
}

// rev[i][c] = the slot of (i, -shift) in the list of j = nei[i][c], found
// by distance in j's sorted list (a few float ulps of slack: j computed the
// same distance from the other side), then a check of the entries in that
// distance window.  With several types the search stays inside the run of
// i's type in j's list (sorted by distance within the run).  Neighborhoods
// are alike, so the rank of r_ij in both lists is similar: each lane loads
// the kRevWindow entries of j's run around c's own rank at once, and when
// they bracket the distance window (the common case: in a thermalised FCC
// crystal the two ranks differ by at most 16 for all but about 1 pair in
// 2000) the slot is found in them; otherwise the search gallops outward from
// that rank and bisects.  Each pair is searched once, from its
// lower-indexed side (self-images: from the side with the larger shift
// code), and both slots are written.  -1 when j's list lacks i, which
// happens only at the edge of the skin, far outside rcut.  uniq (box edges
// of at least 2 (rcut + skin), or no box): a list holds at most one image of
// any atom, so an entry of the window is i's slot when its index is i (the
// image shift is not read).  One 64-thread block per atom.
constexpr int kRevWindow = 32;

__device__ inline int run_start(const int *tcnt, int a, int ty)
{
    int s = 0;
    for (int q = 0; q < ty; q++) s += tcnt[(long)a * kMaxTypes + q];
    return s;
}

template <bool TYPED>
__global__ void __launch_bounds__(64) k_reverse(int off, int n, int cap, const int *__restrict__ cnt,
                                                const int *__restrict__ nei, const int *__restrict__ shift,
                                                const float *__restrict__ dist, const int *__restrict__ type,
                                                const int *__restrict__ tcnt, short *__restrict__ rev, bool uniq)
{
    int ib = xcd_item(blockIdx.x, gridDim.x);
    if (ib >= n) return;
    int i = off + ib;
    int nc = cnt[i];
    int ti = TYPED ? type[i] : 0;
    for (int c = threadIdx.x; c < nc; c += 64) {
        long ic = (long)i * cap + c;
        int j = nei[ic];
        int sh = shift[ic];
        int want = neg_shift(sh);
        if (j < i || (j == i && sh < want)) continue;   // the other side searches
        float r = dist[ic];
        unsigned rb = __float_as_uint(r);
        float lo = __uint_as_float(rb > 8u ? rb - 8u : 0u), hi = __uint_as_float(rb + 8u);
        // j's run of type ti, and c's rank within i's run of j's type
        int j0 = 0, ncj = cnt[j], crel = c;
        if (TYPED) {
            j0 = run_start(tcnt, j, ti);
            ncj = tcnt[(long)j * kMaxTypes + ti];
            crel = c - run_start(tcnt, i, type[j]);
        }
        const float *dj = dist + (long)j * cap + j0;
        // the window [w0, w0 + kRevWindow) of the run around crel, inside the
        // row's allocation (cap - j0 >= kRevWindow entries from j0, else the
        // search below); entries at ncj and past it are loaded but not used
        const int lim = cap - j0;
        const int w0 = max(min(crel - kRevWindow / 2, lim - kRevWindow), 0);
        const int nw = min(kRevWindow, ncj - w0);   // entries of the run in the window
        // entries below lo and up to hi among the run's entries in the window
        // (prefixes, as the run is sorted), counted on the bits of the
        // non-negative distances (which order as integers)
        int na = 0, nb = 0;
        bool hit = false;
        if (lim >= kRevWindow && nw > 0) {
            unsigned wd[kRevWindow];
#pragma unroll
            for (int k = 0; k < kRevWindow; k++) wd[k] = __float_as_uint(dj[w0 + k]);
            const unsigned ulo = __float_as_uint(lo), uhi = __float_as_uint(hi);
#pragma unroll
            for (int k = 0; k < kRevWindow; k++) {
                // past the run: with one type the row's own +inf padding;
                // with several the next type's run, taken as above every
                // distance
                const unsigned d = TYPED && k >= nw ? 0x7FFFFFFFu : wd[k];
                na += d < ulo;
                nb += d <= uhi;
            }
            // the window holds every entry of the distance window
            hit = (w0 == 0 || na > 0) && (nb < nw || w0 + kRevWindow >= ncj);
        }
        if (hit) {
            int found = -1;
            for (int k = na; k < nb; k++) {
                const long jt = (long)j * cap + j0 + w0 + k;
                if (nei[jt] == i && (uniq || shift[jt] == want)) {
                    found = j0 + w0 + k;
                    break;
                }
            }
            rev[ic] = (short)found;
            if (found >= 0) rev[(long)j * cap + found] = (short)c;
            continue;
        }
        // first index a with dj[a] >= lo: gallop from min(crel, ncj - 1), then bisect
        int a, b;
        int p = crel < ncj ? crel : ncj - 1;
        if (ncj == 0) {
            a = b = 0;
        } else if (dj[p] < lo) {
            int step = 1;
            a = p + 1;
            b = p + 1;
            while (b < ncj && dj[b] < lo) {
                a = b + 1;
                b += step;
                step <<= 1;
            }
            if (b > ncj) b = ncj;
        } else {
            int step = 1;
            b = p;
            a = p - 1;
            while (a >= 0 && dj[a] >= lo) {
                b = a;
                a -= step;
                step <<= 1;
            }
            a = a < 0 ? 0 : a + 1;
        }
        while (a < b) {
            int mid = (a + b) >> 1;
            if (dj[mid] < lo) a = mid + 1;
            else b = mid;
        }
        int found = -1;
        for (int t = a; t < ncj && dj[t] <= hi; t++) {
            long jt = (long)j * cap + j0 + t;
            if (nei[jt] == i && (uniq || shift[jt] == want)) {
                found = j0 + t;
                break;
            }
        }
        rev[ic] = (short)found;
        if (found >= 0) rev[(long)j * cap + found] = (short)c;
    }
}

// Per atom i (one wave): F_i -= sum of dE_j/dr_ji over the atoms j that
// list i, read from j's pair-gradient slot for i (the reverse slot).  When i
// kept every neighbor within rcut, those j are exactly i's kept neighbors
// (membership within rcut is symmetric and their limits kept i, or they
// zeroed its slot), so only the forward's records are visited; otherwise
// every candidate within rcut, by the forward's own membership test.  Lanes
// take neighbors, four in flight (indices first, then pair gradients); the
// order of the sum is fixed.
template <typename real>
__device__ inline void add_pg(const real *p, double &f0, double &f1, double &f2)
{
    if (sizeof(real) == 4) {
        V4<float> g = *reinterpret_cast<const V4<float> *>(p);
        f0 += (double)g.x;
        f1 += (double)g.y;
        f2 += (double)g.z;
    } else {
        f0 += (double)p[0];
        f1 += (double)p[1];
        f2 += (double)p[2];
    }
}

template <typename real>
__global__ void __launch_bounds__(256) k_force_gather(int n, EnvArgs A, const short *__restrict__ rev,
                                                      double *__restrict__ force)
{
    constexpr int ST = sizeof(real) == 4 ? 4 : 3;   // reals per pair-gradient slot
    int lane = threadIdx.x & 63;
    int i = xcd_item(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const long cap = A.cap;
    const int *ni = A.nei + (long)i * cap;
    const short *ri = rev + (long)i * cap;
    const real *pg = reinterpret_cast<const real *>(A.pg);
    double f0 = 0, f1 = 0, f2 = 0;
    int code = A.rcnt[i];
    if (!(code & kTruncBit)) {
        int nn = code;
        const V4<real> *rec = reinterpret_cast<const V4<real> *>(A.rec) + (long)i * A.sel;
        for (int k0 = 0; k0 < nn; k0 += 256) {
            long off[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                int k = k0 + 64 * u + lane;
                off[u] = -1;
                if (k < nn) {
                    int c = record_slot(rec[k].w) & 0xFFFFFF;
                    int r = ri[c];
                    off[u] = r < 0 ? -1 : ((long)ni[c] * cap + r) * ST;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (off[u] >= 0) add_pg<real>(pg + off[u], f0, f1, f2);
        }
    } else {
        int nc = A.cnt[i];
        const int *si = A.shift + (long)i * cap;
        double xi0 = A.x[3 * i], xi1 = A.x[3 * i + 1], xi2 = A.x[3 * i + 2];
        double L0 = A.L0, L1 = A.L1, L2 = A.L2;
        if (A.atomL) {
            L0 = A.atomL[3 * i];
            L1 = A.atomL[3 * i + 1];
            L2 = A.atomL[3 * i + 2];
        }
        for (int c0 = 0; c0 < nc; c0 += 256) {
            long off[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                int c = c0 + 64 * u + lane;
                off[u] = -1;
                if (c < nc) {
                    int j = ni[c], r = ri[c];
                    double d0, d1, d2;
                    if (r >= 0 && within_cut(A.x, j, xi0, xi1, xi2, si[c], L0, L1, L2, A.rc2, d0, d1, d2))
                        off[u] = ((long)j * cap + r) * ST;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (off[u] >= 0) add_pg<real>(pg + off[u], f0, f1, f2);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        f0 += __shfl_xor(f0, o);
        f1 += __shfl_xor(f1, o);
        f2 += __shfl_xor(f2, o);
    }
    if (lane == 0) {
        force[3 * i] -= f0;
        force[3 * i + 1] -= f1;
        force[3 * i + 2] -= f2;
    }
}

}  // namespace

void launch_reverse(dp_nlist *nl, int off, int n, hipStream_t st, bool uniq)
{
    if (n <= 0) return;
    // every slot starts at -1: a pair is searched from one side only, so a
    // slot that no search writes (j's list lacks i) must already read -1
    long m = (long)n * nl->cap;
    hipLaunchKernelGGL(k_fill_short, dim3(div_up(m, 256)), dim3(256), 0, st, nl->rev + (long)off * nl->cap, m,
                       (short)-1);
    const bool typed = nl->ntypes > 1;
    if (typed)
        hipLaunchKernelGGL(k_reverse<true>, dim3(xcd_grid(n)), dim3(64), 0, st, off, n, nl->cap, nl->cnt, nl->nei,
                           nl->shift, nl->dist, nl->type, nl->tcnt, nl->rev, uniq);
    else
        hipLaunchKernelGGL(k_reverse<false>, dim3(xcd_grid(n)), dim3(64), 0, st, off, n, nl->cap, nl->cnt, nl->nei,
                           nl->shift, nl->dist, (const int *)nullptr, (const int *)nullptr, nl->rev, uniq);
}

void launch_force_gather(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision,
                         const void *rec, const int *rcnt, double *force, hipStream_t st)
{
    if (n <= 0) return;
    EnvArgs A = make_env_args(m, nl, x);
    A.rec = const_cast<void *>(rec);
    A.rcnt = const_cast<int *>(rcnt);
    A.pg = nl->pg;
    if (precision == DP_FP64)
        hipLaunchKernelGGL(k_force_gather<double>, dim3(xcd_grid(div_up(n, 4))), dim3(256), 0, st, n, A, nl->rev,
                           force);
    else
        hipLaunchKernelGGL(k_force_gather<float>, dim3(xcd_grid(div_up(n, 4))), dim3(256), 0, st, n, A, nl->rev,
                           force);
}

// ------------------------------------------------- rows grouped by type
namespace {

// Per block of 256 atoms: copy the types into the list (an out-of-range
// type is flagged and taken as 0) and count them per type.
__global__ void __launch_bounds__(256) k_type_count(int n, int ntypes, const int *__restrict__ types,
                                                    int *__restrict__ type_out, int *__restrict__ blk,
                                                    int *__restrict__ flags)
{
    __shared__ int c[kMaxTypes];
    if (threadIdx.x < kMaxTypes) c[threadIdx.x] = 0;
    __syncthreads();
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        int t = types ? types[i] : 0;
        if (t < 0 || t >= ntypes) {
            atomicAdd(&flags[kFlagBadType], 1);
            t = 0;
        }
        type_out[i] = t;
        atomicAdd(&c[t], 1);
    }
    __syncthreads();
    if (threadIdx.x < kMaxTypes) blk[(long)blockIdx.x * kMaxTypes + threadIdx.x] = c[threadIdx.x];
}

// Exclusive prefix of the block counts per type (one thread per type, in
// block order) and the totals.
__global__ void k_type_scan(int nblk, int *__restrict__ blk, int *__restrict__ tot)
{
    int t = threadIdx.x;
    if (t >= kMaxTypes) return;
    int s = 0;
    for (int b = 0; b < nblk; b++) {
        int v = blk[(long)b * kMaxTypes + t];
        blk[(long)b * kMaxTypes + t] = s;
        s += v;
    }
    tot[t] = s;
}

struct TypeRows {
    int v[kMaxTypes + 1];
};

// Row of atom i: its type group's first row, plus the atoms of its type
// before it (earlier blocks, then earlier threads of its block).
__global__ void __launch_bounds__(256) k_type_rows(int n, const int *__restrict__ type, const int *__restrict__ blk,
                                                   TypeRows trow, int *__restrict__ row, int *__restrict__ ratom)
{
    __shared__ int ts[256];
    int i = blockIdx.x * 256 + threadIdx.x;
    int t = i < n ? type[i] : -1;
    ts[threadIdx.x] = t;
    __syncthreads();
    if (i >= n) return;
    int r = 0;
    for (int k = 0; k < (int)threadIdx.x; k++) r += ts[k] == t ? 1 : 0;
    int rw = trow.v[t] + blk[(long)blockIdx.x * kMaxTypes + t] + r;
    row[i] = rw;
    ratom[rw] = i;
}

__global__ void k_fill_int(int *p, long n, int v)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

dp_status build_type_layout(dp_nlist *nl, const int *types, hipStream_t st)
{
    int n = nl->natoms, T = nl->ntypes;
    if (T <= 1) return DP_OK;
    int nblk = div_up(n, 256);
    int *tot = nl->tblk + (long)nblk * kMaxTypes;
    hipLaunchKernelGGL(k_type_count, dim3(nblk), dim3(256), 0, st, n, T, types, nl->type, nl->tblk, nl->flags);
    hipLaunchKernelGGL(k_type_scan, dim3(1), dim3(64), 0, st, nblk, nl->tblk, tot);
    int cnt[kMaxTypes];
    DP_HIP(hipGetLastError());
    DP_HIP(hipStreamSynchronize(st));
    DP_HIP(hipMemcpy(cnt, tot, sizeof(cnt), hipMemcpyDeviceToHost));
    TypeRows tr{};
    for (int t = 0; t < T; t++) tr.v[t + 1] = tr.v[t] + (int)round_up(cnt[t], kRowPad);
    for (int t = T + 1; t <= kMaxTypes; t++) tr.v[t] = tr.v[T];
    for (int t = 0; t <= kMaxTypes; t++) nl->trow[t] = tr.v[t];
    nl->rows = tr.v[T];
    if ((long)nl->rows > fit_rows(nl->alloc_atoms, T)) return fail(DP_ERR_STATE, "fitting rows exceed the workspace");
    hipLaunchKernelGGL(k_fill_int, dim3(div_up(nl->rows, 256)), dim3(256), 0, st, nl->ratom, (long)nl->rows, -1);
    hipLaunchKernelGGL(k_type_rows, dim3(nblk), dim3(256), 0, st, n, nl->type, nl->tblk, tr, nl->row, nl->ratom);
    return step_check("type_layout", st);
}

}  // namespace dp
