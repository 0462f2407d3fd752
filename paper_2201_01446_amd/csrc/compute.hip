// compute.hip -- one force step of the compressed model, and the
// velocity-Verlet kernels, as sequences of launches on one stream.
//
// Compressed step (per configuration, all on the caller's stream):
//   k_emb_fwd        env matrix + tabulated G fused with R^T G -> T, D
//   3 x GEMM         fitting net forward (tanh / shortcut epilogues)
//   k_energy         E_i, dz3
//   3 x GEMM         fitting-net input gradient -> dD
//   k_emb_bwd        dE/dT from dE/dD and T, then the adjoint of the fused
//                    step -> F_i's own part, dE_i/dr_ij per candidate, W_i
//   k_force_gather   F_j -= dE_i/dr_ij over the atoms i that list j
//   k_reduce_*       deterministic FP64 sums of E_i and W_i
// Buffers live in the neighbor list's workspace; rows are padded to 128 so
// the GEMM tiles never read past an allocation.

#include "dp_internal.h"

#include <mutex>
#include <type_traits>

namespace dp {

namespace {

struct WS {
    void *T, *D, *y1r, *y1o, *y2r, *y2o, *t2r, *t3r, *dz3o, *dy2r, *dz2o, *dz1o, *dDr, *dT;
    void *rec;   // the forward's compacted neighbors (r_ij, j) per atom, sel slots
    int *rcnt;   // their number per atom
    double *e_atom, *w_atom, *part;
};

size_t sizes(int precision, size_t &rs, size_t &os)
{
    rs = precision == DP_FP64 ? 8 : 4;
    os = precision == DP_FP64 ? 8 : (precision == DP_FP32 ? 4 : 2);
    return 0;
}

size_t ws_bytes_for(int np, int precision, int sel)
{
    size_t rs, os;
    sizes(precision, rs, os);
    os *= k_split(precision);
    auto al = [](size_t b) { return (size_t)round_up((long)b, 256); };
    size_t r = 0;
    r += al(np * 4 * kM * rs);          // T
    r += al(np * (size_t)kDdim * os);   // D
    r += 5 * al(np * (size_t)kFitPad * rs);   // y1r y2r t2r t3r dy2r
    r += 5 * al(np * (size_t)kFitPad * os);   // y1o y2o dz3o dz2o dz1o
    r += al(np * (size_t)kDdim * rs);   // dD
    r += al(np * 4 * kM * rs);          // dT
    r += al((size_t)np * sel * 4 * rs) + al(np * 4);   // neighbor records, counts
    r += al(np * 8) + al(np * 72) + al(256 * 10 * 8);
    return r;
}

WS carve(void *base, int np, int precision, int sel)
{
    size_t rs, os;
    sizes(precision, rs, os);
    os *= k_split(precision);
    char *p = (char *)base;
    auto take = [&](size_t b) {
        void *q = p;
        p += round_up((long)b, 256);
        return q;
    };
    WS w;
    w.T = take(np * 4 * kM * rs);
    w.D = take(np * (size_t)kDdim * os);
    w.y1r = take(np * (size_t)kFitPad * rs);
    w.y2r = take(np * (size_t)kFitPad * rs);
    w.t2r = take(np * (size_t)kFitPad * rs);
    w.t3r = take(np * (size_t)kFitPad * rs);
    w.dy2r = take(np * (size_t)kFitPad * rs);
    w.y1o = take(np * (size_t)kFitPad * os);
    w.y2o = take(np * (size_t)kFitPad * os);
    w.dz3o = take(np * (size_t)kFitPad * os);
    w.dz2o = take(np * (size_t)kFitPad * os);
    w.dz1o = take(np * (size_t)kFitPad * os);
    w.dDr = take(np * (size_t)kDdim * rs);
    w.dT = take(np * 4 * kM * rs);
    w.rec = take((size_t)np * sel * 4 * rs);
    w.rcnt = (int *)take(np * 4);
    w.e_atom = (double *)take(np * 8);
    w.w_atom = (double *)take(np * 72);
    w.part = (double *)take(256 * 10 * 8);
    return w;
}

template <typename TA, typename TR, bool PLAIN>
dp_status run_t(const ComputeArgs &a, const WS &w, int np, const FitWeights &fw, const TR *fb,
                hipStream_t st)
{
    const dp_model *m = a.m;
    int n = a.natoms;
    dp_status s = DP_OK;
    // vectors of type 0; a row group of type t reads them t * kFitB further
    const TR *c1 = fb, *c2 = fb + kFitPad, *c3 = fb + 2 * kFitPad, *w4 = fb + 3 * kFitPad;
    Epi e{};
    const int ks = k_split(a.precision);   // operand K multiplier (BF16 split)
    // GEMM rows: the live atoms rounded up to a whole 128-row tile (rows past
    // n hold stale finite values and their outputs are never read); with
    // several types, the type groups, each so rounded; the buffers
    // themselves are carved for the allocation's np rows.
    const dp_nlist *nl = a.nl;
    const bool typed = nl->ntypes > 1;
    const int mr = typed ? nl->rows : (int)round_up(n, kRowPad);
    (void)np;
    // the weights of a tile's type group: one type's Bt (N x K) further per type
    auto grouped = [&](Epi x, int N, int K) {
        if (typed) {
            x.ntr = nl->ntypes;
            for (int t = 0; t <= kMaxTypes; t++) x.trow[t] = nl->trow[t];
            x.bstride = (long)N * K;
            x.vstride = kFitB;
        }
        return x;
    };
    RowTypes rt;
    if (typed) {
        rt.ntr = nl->ntypes;
        for (int t = 0; t <= kMaxTypes; t++) rt.trow[t] = nl->trow[t];
        rt.ratom = nl->ratom;
    }
    for (int t = 0; t < kMaxTypes; t++) rt.b4[t] = m->b4[t];
    bool fwd = a.phase != 2, bwd = a.need_forces && a.phase != 1;
    // FP64 / FP32: every forward runs the fitting net's 256-wide layers, the
    // energy and their input gradients as one fused kernel (so a backward
    // that follows, in this call or a later one, starts at dz1); BF16 runs
    // them as separate GEMMs
    constexpr bool tail = std::is_same<TA, TR>::value;
    // FP32 / FP64 compressed forward: the first fitting layer forms D = T<^T T
    // from T as it stages its operand, and the embedding kernel writes no D
    // (unless the caller asks for D)
    const bool dfuse = tail && !PLAIN && a.mode == DP_COMPRESSED && !a.D_out;
    // decides the early end of the candidate scans, and flags moves beyond the list's reach
    launch_displacement(nl, n, a.x, nl->rc_build - m->cfg.rcut, st);
    if (fwd) {
        if (PLAIN) {
            bool tab = a.mode == DP_TAB_UNFUSED;
            if ((s = plain_forward<TR, TA>(m, a.nl, n, a.x, w.T, w.D, a.nnei_out, st, tab)) != DP_OK) return s;
        } else if (a.mode == DP_COMPRESSED) {
            DP_TIMED("emb_fwd", st, launch_emb_fwd(m, a.nl, n, a.x, a.precision, w.T, dfuse ? nullptr : w.D, w.rec, w.rcnt, a.nnei_out, a.nseg_out, st));
            if ((s = step_check("emb_fwd", st)) != DP_OK) return s;
        } else {
            bool pad = a.mode == DP_FUSED_PADDED;
            DP_TIMED("emb_fwd_pn", st, launch_emb_fwd_pn(m, a.nl, n, a.x, a.precision, w.T, w.D, w.rec, w.rcnt, pad, a.nnei_out, st));
            if ((s = step_check("emb_fwd", st)) != DP_OK) return s;
        }
        if (a.T_out) {
            // the compressed embedding kernel stores T by column
            if (!PLAIN && a.mode == DP_COMPRESSED) launch_tcol_to_double<TR>(n, (const TR *)w.T, a.T_out, st);
            else launch_to_double<TR>((long)n * 4 * kM, (const TR *)w.T, a.T_out, st);
        }
        if (a.D_out) launch_op_to_double<TA>(n, kDdim, (const TA *)w.D, typed ? nl->row : nullptr, a.D_out, st);
        // the fitting net's tanh: native, or the table (in the epilogue's precision) when enabled
        const float *ttab = m->tanh_on ? m->tanh_tab : nullptr;
        const double *ttab64 = m->tanh_on ? m->tanh_tab64 : nullptr;
        // when the operand type is the result type (FP32, FP64) the next
        // layer reads the result array itself; BF16 needs the split copy
        constexpr bool same = std::is_same<TA, TR>::value;
        void *y1op = same ? nullptr : w.y1o, *y2op = same ? nullptr : w.y2o;
        const TA *y1in = (const TA *)(same ? w.y1r : w.y1o), *y2in = (const TA *)(same ? w.y2r : w.y2o);
        e = Epi{c1, nullptr, nullptr, nullptr, w.y1r, y1op, nullptr};
        e.tanh_tab = ttab;
        e.tanh_tab64 = ttab64;
        e = grouped(e, kFitPad, ks * kDdim);
        if (dfuse) {
            e.dt_T = w.T;
            e.dt_ratom = typed ? nl->ratom : nullptr;
            e.dt_nlive = n;
            if constexpr (std::is_same<TA, TR>::value)
                DP_TIMED("fit_fwd1", st, launch_gemm_dt<TA, TR>(mr, kFitPad, (const TA *)fw.V1tp, e, st));
        } else {
            DP_TIMED("fit_fwd1", st, launch_gemm<TA, TR>(EPI_T1, mr, kFitPad, ks * kDdim, (const TA *)w.D, (const TA *)fw.V1t, e, st));
        }
        if (!tail) {
            e = Epi{c2, w.y1r, nullptr, nullptr, w.y2r, y2op, w.t2r};
            e.tanh_tab = ttab;
            e.tanh_tab64 = ttab64;
            e = grouped(e, kFitPad, ks * kFitPad);
            DP_TIMED("fit_fwd2", st, launch_gemm<TA, TR>(EPI_T2, mr, kFitPad, ks * kFitPad, y1in, (const TA *)fw.V2t, e, st));
            e = Epi{c3, nullptr, nullptr, nullptr, nullptr, nullptr, w.t3r};
            e.tanh_tab = ttab;
            e.tanh_tab64 = ttab64;
            e = grouped(e, kFitPad, ks * kFitPad);
            DP_TIMED("fit_fwd3", st, launch_gemm<TA, TR>(EPI_T3, mr, kFitPad, ks * kFitPad, y2in, (const TA *)fw.V3t, e, st));
        }
    }
    if (tail && fwd) {
        // y1 in; E_i and dz1 out
        TailLaunch tl;
        if (typed) {
            tl.ntr = nl->ntypes;
            for (int t = 0; t <= kMaxTypes; t++) tl.trow[t] = nl->trow[t];
            tl.ratom = nl->ratom;
        }
        tl.nlive = n;
        tl.width = m->f1;
        for (int t = 0; t < kMaxTypes; t++) tl.b4[t] = m->b4[t];
        if (m->tanh_on)
            tl.tanh_tab = std::is_same<TR, double>::value ? (const void *)m->tanh_tab64 : (const void *)m->tanh_tab;
        if constexpr (std::is_same<TA, TR>::value)
            DP_TIMED("fit_tail", st, launch_fit_tail<TA>(mr, (const TA *)w.y1r, fw, fb, tl, w.e_atom, (TA *)w.dz1o, (TA *)w.t2r, (TA *)w.dy2r, st));
        if ((s = step_check("fitting_tail", st)) != DP_OK) return s;
    } else if (!tail) {
        // E_i always (also from kept activations); dz3 = w4 (1 - t3^2) when the backward follows
        launch_energy<TA, TR>(typed ? mr : n, (const TR *)w.y2r, (const TR *)w.t3r, w4, rt, w.e_atom,
                              bwd ? (TA *)w.dz3o : nullptr, st);
        if ((s = step_check("fitting_forward", st)) != DP_OK) return s;
    }
    if (bwd) {
        if (!tail) {
            e = grouped(Epi{nullptr, nullptr, w4, w.t2r, w.dy2r, w.dz2o, nullptr}, kFitPad, ks * kFitPad);
            DP_TIMED("fit_bwd3", st, launch_gemm<TA, TR>(EPI_BWD, mr, kFitPad, ks * kFitPad, (const TA *)w.dz3o, (const TA *)fw.V3, e, st));
            e = grouped(Epi{nullptr, w.dy2r, nullptr, w.y1r, nullptr, w.dz1o, nullptr}, kFitPad, ks * kFitPad);
            DP_TIMED("fit_bwd2", st, launch_gemm<TA, TR>(EPI_BWD, mr, kFitPad, ks * kFitPad, (const TA *)w.dz2o, (const TA *)fw.V2, e, st));
        }
        e = grouped(Epi{nullptr, nullptr, nullptr, nullptr, w.dDr, nullptr, nullptr}, kDdim, ks * kFitPad);
        // K = the net's width in half K stages (dz1 and V1 are zero past it), rows kFitPad long
        int k1 = ks * kFitPad;
        if (ks == 1) {
            k1 = (int)std::min<long>(kFitPad, round_up(m->f1, 64 / (long)sizeof(TA)));
            e.kld = kFitPad;
        }
        DP_TIMED("fit_bwd1", st, launch_gemm<TA, TR>(EPI_LIN, mr, kDdim, k1, (const TA *)w.dz1o, (const TA *)fw.V1, e, st));
        if (PLAIN) {
            DP_TIMED("dT", st, launch_dT<TR>(n, (const TR *)w.dDr, (const TR *)w.T, (TR *)w.dT, st));
            if ((s = step_check("fitting_backward", st)) != DP_OK) return s;
            bool tab = a.mode == DP_TAB_UNFUSED;
            if ((s = plain_backward<TR>(m, a.nl, n, w.dT, a.force, w.w_atom, st, tab)) != DP_OK) return s;
        } else {
            if ((s = step_check("fitting_backward", st)) != DP_OK) return s;
            // dE/dT is formed inside the fused backward from dE/dD and T
            if (a.mode == DP_COMPRESSED) {
                DP_TIMED("emb_bwd", st, launch_emb_bwd(m, a.nl, n, a.x, a.precision, w.T, w.dDr, w.rec, w.rcnt, a.force, w.w_atom, st));
            } else {
                bool pad = a.mode == DP_FUSED_PADDED;
                DP_TIMED("emb_bwd_pn", st, launch_emb_bwd_pn(m, a.nl, n, a.x, a.precision, w.T, w.dDr, w.rec, w.rcnt, pad, a.force, w.w_atom, st));
            }
            DP_TIMED("force_gather", st, launch_force_gather(m, a.nl, n, a.x, a.precision, w.rec, w.rcnt, a.force, st));
            if ((s = step_check("emb_bwd", st)) != DP_OK) return s;
        }
    }
    double *energy = a.phase == 2 ? nullptr : a.energy;
    double *virial = bwd ? a.virial : nullptr;
    if (a.nseg > 0)
        launch_segment_reduce(a.nseg, a.seg_off, w.e_atom, bwd ? w.w_atom : nullptr, energy, virial, nl->flags, st);
    else
        launch_reduce(n, w.e_atom, bwd ? w.w_atom : nullptr, w.part, energy, virial, nl->flags, st);
    if (a.atom_energy && a.phase != 2)
        DP_HIP(hipMemcpyAsync(a.atom_energy, w.e_atom, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    return step_check("reduce", st);
}

}  // namespace

size_t ws_bytes_for_atoms(int natoms, int precision, int sel, int ntypes)
{
    return ws_bytes_for((int)fit_rows(natoms, ntypes), precision, sel);
}

dp_status ensure_ws(dp_nlist *nl, int precision, int sel)
{
    int np = (int)fit_rows(nl->alloc_atoms, nl->ntypes);
    size_t need = ws_bytes_for(np, DP_FP64, sel);
    size_t need_bf = ws_bytes_for(np, DP_MIXED_BF16, sel);
    if (need_bf > need) need = need_bf;   // the largest of the three layouts
    (void)precision;
    if (nl->ws_bytes >= need) return DP_OK;
    if (nl->ws) DP_HIP(hipFree(nl->ws));
    nl->ws = nullptr;
    nl->ws_bytes = 0;
    hipError_t e = hipMalloc(&nl->ws, need);
    if (e != hipSuccess) return fail(DP_ERR_OOM, "workspace allocation failed");
    nl->ws_bytes = need;
    // rows past natoms are read by GEMM tiles: keep them finite (zero)
    DP_HIP(hipMemset(nl->ws, 0, need));
    return DP_OK;
}

// Scratch of dp_compute_noalloc, for callers that cannot allocate device
// memory: one fixed array per device, shared by every such call on that
// device (calls that overlap on one device race).  Nothing in it needs
// clearing between calls: every element a call reads was written earlier in
// the same call, except the pad rows of the GEMM operands (rows past the
// last atom), whose outputs are never read and which cannot mix with other
// rows.  96 MiB holds the workspace of 512 atoms of any supported model
// (sel <= 512, up to 4 types) in any precision, or of up to 1,408 one-type
// atoms at sel = 192.
namespace {
constexpr size_t kNoAllocBytes = (size_t)96 << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (the host-side name of the array is not a device address).
dp_status scratch_on_device(void **out)
{
    int dev = 0;
    DP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DP_ERR_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(DP_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DP_OK;
}
}  // namespace

size_t noalloc_scratch_bytes() { return kNoAllocBytes; }

dp_status run_compressed(const ComputeArgs &a, hipStream_t st)
{
    int np;
    void *base;
    if (a.noalloc) {
        // carved for exactly the rows of this call
        np = (int)fit_rows(a.natoms, a.nl->ntypes);
        size_t need = ws_bytes_for(np, a.precision, a.m->cfg.sel);
        if (need > kNoAllocBytes)
            return fail(DP_ERR_CAPACITY, "the evaluation needs " + std::to_string(need) +
                                             " bytes of scratch, more than the static " +
                                             std::to_string(kNoAllocBytes) + " of dp_compute_noalloc");
        dp_status s = scratch_on_device(&base);
        if (s != DP_OK) return s;
    } else {
        np = (int)fit_rows(a.nl->alloc_atoms, a.nl->ntypes);
        base = a.nl->ws;
    }
    WS w = carve(base, np, a.precision, a.m->cfg.sel);
    if (a.precision == DP_FP64) return run_t<double, double, false>(a, w, np, a.m->w64, a.m->fitb_d, st);
    if (a.precision == DP_FP32) return run_t<float, float, false>(a, w, np, a.m->w32, a.m->fitb_f, st);
    return run_t<__bf16, float, false>(a, w, np, a.m->wbf, a.m->fitb_f, st);
}

dp_status run_plain(const ComputeArgs &a, hipStream_t st)
{
    int np = (int)fit_rows(a.nl->alloc_atoms, a.nl->ntypes);
    WS w = carve(a.nl->ws, np, a.precision, a.m->cfg.sel);
    if (a.precision == DP_FP64) return run_t<double, double, true>(a, w, np, a.m->w64, a.m->fitb_d, st);
    if (a.precision == DP_FP32) return run_t<float, float, true>(a, w, np, a.m->w32, a.m->fitb_f, st);
    return run_t<__bf16, float, true>(a, w, np, a.m->wbf, a.m->fitb_f, st);
}

// ---------------------------------------------------------------- Verlet
namespace {

// 1 eV/(A amu) in A/fs^2, and 1 amu A^2/fs^2 in eV.
constexpr double kAcc = 9.64853321e-3;
constexpr double kKe = 103.642691;

__global__ void k_kick_drift(double *__restrict__ x, double *__restrict__ v, const double *__restrict__ f,
                             long n3, const int *__restrict__ type, TypeScalars kick, double dt)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n3) return;
    double k = kick.v[type ? type[i / 3] : 0];
    double vi = v[i] + k * f[i];
    v[i] = vi;
    x[i] += dt * vi;
}

__global__ void k_kick(double *__restrict__ v, const double *__restrict__ f, long n3, const int *__restrict__ type,
                       TypeScalars kick)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n3) v[i] += kick.v[type ? type[i / 3] : 0] * f[i];
}

// Per block a fixed slice of sum_i ke[type_i] |v_i|^2.
__global__ void __launch_bounds__(256) k_vv_partial(long n3, const double *__restrict__ v,
                                                    const int *__restrict__ type, TypeScalars ke,
                                                    double *__restrict__ part)
{
    __shared__ double sh[256];
    long per = (n3 + gridDim.x - 1) / gridDim.x;
    long beg = blockIdx.x * per, end = min(n3, beg + per);
    double s = 0;
    for (long i = beg + threadIdx.x; i < end; i += 256) s += ke.v[type ? type[i / 3] : 0] * v[i] * v[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Kinetic energy from the 256 partials (a tree in LDS, fixed order) and the
// potential energy into one thermo row.
__global__ void __launch_bounds__(256) k_thermo_final(int nblk, const double *__restrict__ part,
                                                      const double *__restrict__ energy, double *row)
{
    __shared__ double sh[256];
    int t = threadIdx.x;
    sh[t] = t < nblk ? part[t] : 0.0;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    if (t == 0) {
        row[0] = *energy;
        row[1] = sh[0];
    }
}

}  // namespace

void launch_verlet_kick_drift(double *x, double *v, const double *f, int n, const int *type, TypeScalars kick,
                              double dt, hipStream_t st)
{
    long n3 = 3L * n;
    hipLaunchKernelGGL(k_kick_drift, dim3(div_up(n3, 256)), dim3(256), 0, st, x, v, f, n3, type, kick, dt);
}

void launch_verlet_kick(double *v, const double *f, int n, const int *type, TypeScalars kick, hipStream_t st)
{
    long n3 = 3L * n;
    hipLaunchKernelGGL(k_kick, dim3(div_up(n3, 256)), dim3(256), 0, st, v, f, n3, type, kick);
}

void launch_thermo(const double *v, const double *energy, int n, const int *type, TypeScalars ke, double *row,
                   double *part, hipStream_t st)
{
    hipLaunchKernelGGL(k_vv_partial, dim3(256), dim3(256), 0, st, 3L * n, v, type, ke, part);
    hipLaunchKernelGGL(k_thermo_final, dim3(1), dim3(256), 0, st, 256, part, energy, row);
}

double acc_unit() { return kAcc; }
double ke_unit() { return kKe; }

}  // namespace dp
