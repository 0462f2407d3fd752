// abi.hip -- the extern "C" entry points of libdp (declared in include/dp.h):
// argument checks, handle lifetimes, device allocations, and the order of
// kernel launches.  No arithmetic of the model lives here.

#include "dp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace dp {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

dp_status fail(dp_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

dp_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? DP_ERR_OOM : DP_ERR_HIP;
}

dp_status step_check(const char *name, hipStream_t st)
{
    static const bool sync = [] {
        const char *e = std::getenv("DP_SYNC_CHECK");
        return e && e[0] == '1';
    }();
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && sync) {
        e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e != hipSuccess) return hip_fail(e, name);
    return DP_OK;
}

namespace {

template <typename T>
dp_status upload(T **dst, const std::vector<T> &src)
{
    DP_HIP(hipMalloc((void **)dst, sizeof(T) * src.size()));
    DP_HIP(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return DP_OK;
}

// float -> bfloat16 bits, round to nearest even
uint16_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

dp_status upload_fit(FitWeights &w, const std::vector<double> *mats, int prec)
{
    // mats: V1 [2048][256], V1t [256][2048], V2, V2t, V3, V3t [256][256]
    void **dst[6] = {&w.V1, &w.V1t, &w.V2, &w.V2t, &w.V3, &w.V3t};
    // K (row length) of each matrix as a GEMM Bt operand
    const size_t kcols[6] = {(size_t)kFitPad, (size_t)kDdim, (size_t)kFitPad, (size_t)kFitPad, (size_t)kFitPad,
                             (size_t)kFitPad};
    for (int k = 0; k < 6; k++) {
        const std::vector<double> &m = mats[k];
        size_t n = m.size();
        if (prec == DP_FP64) {
            DP_HIP(hipMalloc(dst[k], n * 8));
            DP_HIP(hipMemcpy(*dst[k], m.data(), n * 8, hipMemcpyHostToDevice));
        } else if (prec == DP_FP32) {
            std::vector<float> f(n);
            for (size_t i = 0; i < n; i++) f[i] = (float)m[i];
            DP_HIP(hipMalloc(dst[k], n * 4));
            DP_HIP(hipMemcpy(*dst[k], f.data(), n * 4, hipMemcpyHostToDevice));
        } else {
            // rows of Bt as [hi | lo | hi] along K (see kSplitBf16)
            size_t K = kcols[k], rows = n / K;
            std::vector<uint16_t> b(3 * n);
            for (size_t r = 0; r < rows; r++)
                for (size_t c = 0; c < K; c++) {
                    float f = (float)m[r * K + c];
                    uint16_t hi = bf16_bits(f);
                    uint32_t hb = (uint32_t)hi << 16;
                    float hf;
                    std::memcpy(&hf, &hb, 4);
                    uint16_t lo = bf16_bits(f - hf);
                    b[r * 3 * K + c] = hi;
                    b[r * 3 * K + K + c] = lo;
                    b[r * 3 * K + 2 * K + c] = hi;
                }
            DP_HIP(hipMalloc(dst[k], 3 * n * 2));
            DP_HIP(hipMemcpy(*dst[k], b.data(), 3 * n * 2, hipMemcpyHostToDevice));
        }
    }
    if (prec == DP_FP64 || prec == DP_FP32) {
        // V1tp: the columns of V1t in the order k' = b M< + a of the operand
        // that the first layer forms from T
        const std::vector<double> &m = mats[1];
        size_t rows = m.size() / kDdim;
        std::vector<double> pm(m.size());
        for (size_t r = 0; r < rows; r++)
            for (int a = 0; a < kMlt; a++)
                for (int b = 0; b < kM; b++) pm[r * kDdim + (size_t)b * kMlt + a] = m[r * kDdim + (size_t)a * kM + b];
        if (prec == DP_FP64) {
            DP_HIP(hipMalloc(&w.V1tp, pm.size() * 8));
            DP_HIP(hipMemcpy(w.V1tp, pm.data(), pm.size() * 8, hipMemcpyHostToDevice));
        } else {
            std::vector<float> f(pm.begin(), pm.end());
            DP_HIP(hipMalloc(&w.V1tp, f.size() * 4));
            DP_HIP(hipMemcpy(w.V1tp, f.data(), f.size() * 4, hipMemcpyHostToDevice));
        }
    }
    return DP_OK;
}

void free_fit(FitWeights &w)
{
    void *p[7] = {w.V1, w.V1t, w.V2, w.V2t, w.V3, w.V3t, w.V1tp};
    for (void *q : p)
        if (q) (void)hipFree(q);
    w = FitWeights{};
}

size_t emb_params(const dp_model_config &c)
{
    size_t d1 = c.emb[0], d2 = c.emb[1], d3 = c.emb[2];
    return d1 + d1 + d1 * d2 + d2 + d2 * d3 + d3;
}

size_t fit_params(const dp_model_config &c)
{
    size_t f1 = c.fit[0], f2 = c.fit[1], f3 = c.fit[2];
    size_t nD = (size_t)c.m_lt * c.emb[2];
    return nD * f1 + f1 + f1 * f2 + f2 + f2 * f3 + f3 + f3 + 1;
}

// ntypes embedding nets, then ntypes fitting nets
size_t expected_params(const dp_model_config &c) { return (size_t)c.ntypes * (emb_params(c) + fit_params(c)); }

bool box_ok(const double *box, double L[3])
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            if (a != b && box[3 * a + b] != 0.0) return false;
    for (int a = 0; a < 3; a++) {
        L[a] = box[4 * a];
        if (!(L[a] > 0.0) || !std::isfinite(L[a])) return false;
    }
    return true;
}

void free_nlist_arrays(dp_nlist *nl)
{
    void *p[] = {nl->cell_cnt, nl->cell_atoms, nl->wpos, nl->wrap, nl->cnt, nl->nei, nl->shift,
                 nl->dist, nl->rev, nl->pg, nl->flags, nl->ws, nl->ws_plain, nl->force_tmp, nl->scal,
                 nl->type, nl->tcnt, nl->row, nl->ratom, nl->tblk, nl->x0, nl->inner, nl->disp, nl->nve_F};
    for (void *q : p)
        if (q) (void)hipFree(q);
}

// (Re)allocates the list for natoms atoms in box (NULL: open); no launch.
dp_status prepare_nlist(const dp_model *m, int natoms, const double *box, double skin, dp_nlist **inout)
{
    if (natoms <= 0) return fail(DP_ERR_ARG, "natoms must be positive");
    if (natoms >= (1 << 24)) return fail(DP_ERR_UNSUPPORTED, "at most 2^24 - 1 atoms");
    if (!(skin >= 0.0) || !std::isfinite(skin)) return fail(DP_ERR_ARG, "skin must be >= 0");
    dp_nlist *nl = *inout;
    bool fresh = nl == nullptr;
    if (fresh) nl = new dp_nlist();
    nl->nve_x = nullptr;   // a build or reallocation ends the trajectory dp_nve_continue would resume
    int dev = 0;
    DP_HIP(hipGetDevice(&dev));
    nl->device = dev;
    nl->rc_build = m->cfg.rcut + skin;
    nl->rcut_build = m->cfg.rcut;
    double rcs = nl->rc_build;
    int cap;
    if (box) {
        double L[3];
        if (!box_ok(box, L)) {
            if (fresh) delete nl;
            return fail(DP_ERR_UNSUPPORTED, "box must be orthorhombic with positive edges");
        }
        for (int a = 0; a < 3; a++)
            if (L[a] < 0.5 * rcs) {
                if (fresh) delete nl;
                return fail(DP_ERR_UNSUPPORTED, "box edge shorter than (rcut + skin) / 2");
            }
        nl->periodic = true;
        for (int a = 0; a < 3; a++) {
            nl->L[a] = L[a];
            nl->nc[a] = (int)std::floor(L[a] / (0.5 * rcs));
            if (nl->nc[a] < 1) nl->nc[a] = 1;
        }
        double vol = L[0] * L[1] * L[2];
        double expect = natoms / vol * 4.18879020478639 * rcs * rcs * rcs;   // 4/3 pi r^3
        cap = (int)round_up((long)std::ceil(1.3 * expect + 64.0), 64);
        long ncell = (long)nl->nc[0] * nl->nc[1] * nl->nc[2];
        int per = (int)std::ceil((double)natoms / ncell);
        int cellcap = (int)round_up(3 * per + 8, 8);
        if (cellcap < nl->cellcap) cellcap = nl->cellcap;   // keep a grown capacity
        if ((size_t)ncell * cellcap > nl->ncell_alloc) {
            if (nl->cell_atoms) DP_HIP(hipFree(nl->cell_atoms));
            if (nl->cell_cnt) DP_HIP(hipFree(nl->cell_cnt));
            nl->cell_atoms = nullptr;
            nl->cell_cnt = nullptr;
            DP_HIP(hipMalloc(&nl->cell_atoms, sizeof(CellAtom) * (size_t)ncell * cellcap));
            DP_HIP(hipMalloc(&nl->cell_cnt, sizeof(int) * (size_t)ncell));
            nl->ncell_alloc = (size_t)ncell * cellcap;
        }
        // cell_cnt must hold ncell entries even if ncell * cellcap fit before
        if ((size_t)ncell > nl->ncell_alloc) return fail(DP_ERR_STATE, "cell grid bookkeeping");
        nl->cellcap = cellcap;
    } else {
        nl->periodic = false;
        for (int a = 0; a < 3; a++) {
            nl->L[a] = 0.0;
            nl->nc[a] = 1;
        }
        cap = (int)round_up(natoms, 64);
    }
    if (cap < 128) cap = 128;
    if (cap < nl->cap_floor) cap = nl->cap_floor;
    if (cap > kCapMax) cap = kCapMax;
    bool grow_atoms = natoms > nl->alloc_atoms;
    bool grow = grow_atoms || cap > nl->cap;
    const int T = m->cfg.ntypes;
    // a list serves models of one type count; a change reallocates the type arrays
    bool retype = T != nl->ntypes;
    if (grow) {
        int alloc = natoms > nl->alloc_atoms ? natoms : nl->alloc_atoms;
        int capn = cap > nl->cap ? cap : nl->cap;
        void *p[] = {nl->wpos, nl->wrap, nl->cnt, nl->nei, nl->shift, nl->dist, nl->rev, nl->pg, nl->force_tmp,
                     nl->x0, nl->inner, nl->nve_F};
        for (void *q : p)
            if (q) DP_HIP(hipFree(q));
        DP_HIP(hipMalloc(&nl->wpos, sizeof(double) * 3 * (size_t)alloc));
        DP_HIP(hipMalloc(&nl->x0, sizeof(double) * 3 * (size_t)alloc));
        DP_HIP(hipMalloc(&nl->inner, sizeof(int) * kMaxTypes * (size_t)alloc));
        DP_HIP(hipMalloc(&nl->wrap, sizeof(int) * (size_t)alloc));
        DP_HIP(hipMalloc(&nl->cnt, sizeof(int) * (size_t)alloc));
        DP_HIP(hipMalloc(&nl->nei, sizeof(int) * (size_t)alloc * capn));
        DP_HIP(hipMalloc(&nl->shift, sizeof(int) * (size_t)alloc * capn));
        DP_HIP(hipMalloc(&nl->dist, sizeof(float) * (size_t)alloc * capn));
        DP_HIP(hipMalloc(&nl->rev, sizeof(short) * (size_t)alloc * capn));
        DP_HIP(hipMalloc(&nl->pg, sizeof(double) * 3 * (size_t)alloc * capn));
        DP_HIP(hipMalloc(&nl->force_tmp, sizeof(double) * 3 * (size_t)alloc));
        DP_HIP(hipMalloc(&nl->nve_F, sizeof(double) * 3 * (size_t)alloc));
        nl->alloc_atoms = alloc;
        nl->cap = capn;
    }
    // (the per-atom type arrays survive a capacity increase: a rebuild inside
    // an MD run reuses the list's copy of the types)
    if (grow_atoms || retype) {
        void *q[] = {nl->type, nl->tcnt, nl->row, nl->ratom, nl->tblk};
        for (void *v : q)
            if (v) DP_HIP(hipFree(v));
        nl->type = nl->tcnt = nl->row = nl->ratom = nl->tblk = nullptr;
        nl->ntypes = T;
        if (T > 1) {
            size_t A = (size_t)nl->alloc_atoms;
            DP_HIP(hipMalloc(&nl->type, sizeof(int) * A));
            DP_HIP(hipMalloc(&nl->tcnt, sizeof(int) * A * kMaxTypes));
            DP_HIP(hipMalloc(&nl->row, sizeof(int) * A));
            DP_HIP(hipMalloc(&nl->ratom, sizeof(int) * (size_t)fit_rows((long)A, T)));
            DP_HIP(hipMalloc(&nl->tblk, sizeof(int) * ((size_t)div_up((long)A, 256) + 1) * kMaxTypes));
        }
    }
    nl->cap = cap > nl->cap ? cap : nl->cap;
    if (!nl->flags) {
        DP_HIP(hipMalloc(&nl->flags, sizeof(int) * kNumFlags));
        DP_HIP(hipMemset(nl->flags, 0, sizeof(int) * kNumFlags));
    }
    if (!nl->scal) DP_HIP(hipMalloc(&nl->scal, sizeof(double) * 512));
    if (!nl->disp) DP_HIP(hipMalloc(&nl->disp, sizeof(unsigned long long)));
    nl->margin = 0.25 * skin;
    nl->natoms = natoms;
    dp_status s = ensure_ws(nl, DP_FP64, m->cfg.sel);
    if (s != DP_OK) return s;
    *inout = nl;
    return DP_OK;
}

dp_status read_flags(dp_nlist *nl, int *f, hipStream_t st)
{
    DP_HIP(hipStreamSynchronize(st));
    DP_HIP(hipMemcpy(f, nl->flags, sizeof(int) * kNumFlags, hipMemcpyDeviceToHost));
    return DP_OK;
}

dp_status check_build_flags(const int *f)
{
    if (f[kFlagBadCoord]) return fail(DP_ERR_ARG, "a coordinate is not finite");
    if (f[kFlagBadType]) return fail(DP_ERR_ARG, "an atom type lies outside [0, ntypes)");
    if (f[kFlagCapOverflow])
        return fail(DP_ERR_CAPACITY, "an atom has more skin candidates than the list capacity "
                                     "(or coordinates lie more than 60 boxes away)");
    if (f[kFlagCellOverflow]) return fail(DP_ERR_CAPACITY, "a cell holds more atoms than its capacity");
    return DP_OK;
}

// Conditions the evaluations since the last build have flagged.
dp_status check_eval_flags(const int *f)
{
    if (f[kFlagBadCoord]) return fail(DP_ERR_NONFINITE, "a coordinate became non-finite");
    if (f[kFlagNonFinite]) return fail(DP_ERR_NONFINITE, "an energy or virial was not finite");
    if (f[kFlagSkin])
        return fail(DP_ERR_SKIN, "an atom moved half the skin or more since the neighbor list was built, so "
                                 "pairs within rcut may be missing: rebuild more often or use a wider skin");
    return DP_OK;
}

// Capacity failures of a build that another attempt with larger capacities
// can cure: a crowded cell doubles the cell capacity, a truncated candidate
// list doubles the candidate capacity (up to kCapMax).  True when it grew one.
bool grow_after_overflow(dp_nlist *nl, const int *f)
{
    if (f[kFlagBadType] || f[kFlagBadCoord]) return false;
    bool grew = false;
    if (f[kFlagCellOverflow]) {
        nl->cellcap *= 2;
        grew = true;
    }
    if (f[kFlagCapOverflow] && nl->cap < kCapMax) {
        nl->cap_floor = (int)std::min<long>(kCapMax, round_up(2L * nl->cap, 64));
        grew = true;
    }
    return grew;
}

dp_status check_compute_args(const dp_model *m, const dp_nlist *nl, int natoms, const double *x, int mode,
                             int precision)
{
    if (!m || !nl || !x) return fail(DP_ERR_ARG, "NULL model, list or coordinates");
    if (natoms != nl->natoms) return fail(DP_ERR_ARG, "natoms differs from the list's");
    if (mode < DP_COMPRESSED || mode > DP_FUSED) return fail(DP_ERR_ARG, "unknown mode");
    if (precision < DP_FP64 || precision > DP_MIXED_BF16) return fail(DP_ERR_ARG, "unknown precision");
    if (mode != DP_PLAIN && !m->tab64) return fail(DP_ERR_STATE, "dp_tabulate has not run");
    if (nl->ntypes != m->cfg.ntypes) return fail(DP_ERR_ARG, "the list was built for a model of another type count");
    if (m->cfg.rcut >= nl->rc_build)
        return fail(DP_ERR_ARG, "the model's rcut reaches past the list's rcut + skin");
    if (m->cfg.ntypes > 1 && (mode == DP_PLAIN || mode == DP_TAB_UNFUSED))
        return fail(DP_ERR_UNSUPPORTED, "several atom types need a fused mode (0, 3 or 4)");
    return DP_OK;
}

// The list's build at coordinates x: types first (several types group the
// candidates by them), then the candidates and reverse slots.
dp_status build_all(const dp_model *m, dp_nlist *nl, const double *x, const int *types, hipStream_t st)
{
    launch_fill_zero_int(nl->flags, kNumFlags, st);
    dp_status s = build_type_layout(nl, types, st);
    if (s != DP_OK) return s;
    return launch_build_nlist(m, nl, x, types, false, st);
}

}  // namespace
}  // namespace dp

using namespace dp;

extern "C" {

dp_status dp_model_create(const dp_model_config *cfg, const double *params_h, size_t nparams, dp_model **out)
{
    if (!cfg || !params_h || !out) return fail(DP_ERR_ARG, "NULL argument");
    const dp_model_config &c = *cfg;
    if (c.ntypes < 1 || c.ntypes > kMaxTypes) return fail(DP_ERR_UNSUPPORTED, "ntypes must be in [1, 4]");
    if (c.ntypes > 1) {
        int sum = 0;
        for (int t = 0; t < c.ntypes; t++) {
            if (c.sel_t[t] < 1) return fail(DP_ERR_ARG, "each sel_t must be >= 1");
            sum += c.sel_t[t];
        }
        if (sum != c.sel) return fail(DP_ERR_ARG, "sel must equal the sum of sel_t");
    }
    if (!(c.rcut > 0) || !(c.rcut_smth >= 0) || !(c.rcut_smth < c.rcut))
        return fail(DP_ERR_ARG, "need 0 <= rcut_smth < rcut");
    // the kernels keep up to sel neighbors per atom in LDS (64 KB per block)
    if (c.sel < 1 || c.sel > 512) return fail(DP_ERR_UNSUPPORTED, "sel must be in [1, 512]");
    if (c.emb[2] != kM || c.emb[1] * 2 != c.emb[2] || c.emb[0] * 2 != c.emb[1])
        return fail(DP_ERR_UNSUPPORTED, "embedding widths must be 32, 64, 128");
    if (c.m_lt != kMlt) return fail(DP_ERR_UNSUPPORTED, "M< must be 16");
    if (c.fit[0] < 1 || c.fit[0] > kFitPad || c.fit[1] != c.fit[0] || c.fit[2] != c.fit[0])
        return fail(DP_ERR_UNSUPPORTED, "fitting widths must be equal and at most 256");
    if (!std::isfinite(c.desc_scale)) return fail(DP_ERR_ARG, "desc_scale must be finite");
    if (c.switch_kind != 0 && c.switch_kind != 1) return fail(DP_ERR_ARG, "switch_kind must be 0 or 1");
    if (nparams != expected_params(c)) return fail(DP_ERR_ARG, "parameter count does not match the config");
    for (size_t i = 0; i < nparams; i++)
        if (!std::isfinite(params_h[i])) return fail(DP_ERR_ARG, "non-finite parameter");

    dp_model *m = new dp_model();
    m->cfg = c;
    DP_HIP(hipGetDevice(&m->device));
    m->d1 = c.emb[0];
    m->d2 = c.emb[1];
    m->d3 = c.emb[2];
    m->f1 = c.fit[0];
    m->f2 = c.fit[1];
    m->f3 = c.fit[2];
    const int T = c.ntypes;
    m->ntypes = T;
    size_t nemb = emb_params(c), nfit = fit_params(c);
    int F = m->f1, P = kFitPad;
    // per center type: the GEMM operands (each matrix's copies back to back) and the vectors
    std::vector<double> mats[6];
    mats[0].assign((size_t)T * kDdim * P, 0.0);   // V1  [2048][256] per type
    mats[1].assign((size_t)T * P * kDdim, 0.0);   // V1t [256][2048] per type
    for (int k = 2; k < 6; k++) mats[k].assign((size_t)T * P * P, 0.0);
    std::vector<double> fb((size_t)T * kFitB, 0.0);
    for (int t = 0; t < T; t++) {
        const double *p = params_h + (size_t)T * nemb + (size_t)t * nfit;
        const double *V1 = p, *c1 = V1 + (size_t)kDdim * F, *V2 = c1 + F, *c2 = V2 + (size_t)F * F, *V3 = c2 + F,
                     *c3 = V3 + (size_t)F * F, *w4 = c3 + F, *b4 = w4 + F;
        double *M0 = mats[0].data() + (size_t)t * kDdim * P, *M1 = mats[1].data() + (size_t)t * P * kDdim;
        for (int a = 0; a < kDdim; a++)
            for (int o = 0; o < F; o++) {
                M0[(size_t)a * P + o] = V1[(size_t)a * F + o];
                M1[(size_t)o * kDdim + a] = V1[(size_t)a * F + o];
            }
        const double *Vs[2] = {V2, V3};
        for (int k = 0; k < 2; k++) {
            double *Ma = mats[2 + 2 * k].data() + (size_t)t * P * P, *Mb = mats[3 + 2 * k].data() + (size_t)t * P * P;
            for (int a = 0; a < F; a++)
                for (int o = 0; o < F; o++) {
                    Ma[(size_t)a * P + o] = Vs[k][(size_t)a * F + o];
                    Mb[(size_t)o * P + a] = Vs[k][(size_t)a * F + o];
                }
        }
        double *f = fb.data() + (size_t)t * kFitB;
        for (int o = 0; o < F; o++) {
            f[o] = c1[o];
            f[P + o] = c2[o];
            f[2 * P + o] = c3[o];
            f[3 * P + o] = w4[o];
        }
        f[4 * P] = b4[0];
        m->b4[t] = b4[0];
    }
    std::vector<float> fbf(fb.begin(), fb.end());
    std::vector<double> emb(params_h, params_h + (size_t)T * nemb);
    // embedding weights in the plain path's GEMM layouts (d1 = 32, d2 = 64, d3 = 128;
    // one type: the plain modes serve one-type models only)
    const double *W0 = params_h, *b0 = W0 + 32, *W1 = b0 + 32, *b1 = W1 + 32 * 64, *W2 = b1 + 64,
                 *b2 = W2 + 64 * 128;
    std::vector<double> eg(64 * 32 + 128 * 64 + 64 * 128 + 64 * 64 + 32 + 32 + 64 + 128, 0.0);
    double *W1t = eg.data(), *W2t = W1t + 64 * 32, *W2c = W2t + 128 * 64, *W1p = W2c + 64 * 128,
           *eW0 = W1p + 64 * 64, *eb0 = eW0 + 32, *eb1 = eb0 + 32, *eb2 = eb1 + 64;
    for (int a = 0; a < 32; a++)
        for (int o = 0; o < 64; o++) {
            W1t[o * 32 + a] = W1[a * 64 + o];
            W1p[a * 64 + o] = W1[a * 64 + o];
        }
    for (int a = 0; a < 64; a++)
        for (int o = 0; o < 128; o++) {
            W2t[o * 64 + a] = W2[a * 128 + o];
            W2c[a * 128 + o] = W2[a * 128 + o];
        }
    for (int a = 0; a < 32; a++) {
        eW0[a] = W0[a];
        eb0[a] = b0[a];
    }
    for (int a = 0; a < 64; a++) eb1[a] = b1[a];
    for (int a = 0; a < 128; a++) eb2[a] = b2[a];
    std::vector<float> egf(eg.begin(), eg.end());
    dp_status s;
    if ((s = upload(&m->emb_d, emb)) != DP_OK || (s = upload(&m->fitb_d, fb)) != DP_OK ||
        (s = upload(&m->fitb_f, fbf)) != DP_OK || (s = upload((double **)&m->embg64, eg)) != DP_OK ||
        (s = upload((float **)&m->embg32, egf)) != DP_OK || (s = upload_fit(m->w64, mats, DP_FP64)) != DP_OK ||
        (s = upload_fit(m->w32, mats, DP_FP32)) != DP_OK || (s = upload_fit(m->wbf, mats, DP_MIXED_BF16)) != DP_OK) {
        dp_model_destroy(m);
        return s;
    }
    *out = m;
    return DP_OK;
}

dp_status dp_model_destroy(dp_model *m)
{
    if (!m) return DP_OK;
    void *p[] = {m->emb_d, m->fitb_d, m->fitb_f, m->tab64, m->tab32, m->nodes, m->embg64, m->embg32, m->tanh_tab,
                 m->tanh_tab64};
    for (void *q : p)
        if (q) (void)hipFree(q);
    free_fit(m->w64);
    free_fit(m->w32);
    free_fit(m->wbf);
    delete m;
    return DP_OK;
}

dp_status dp_tabulate(dp_model *m, double s_max, double stride, double tail_max, double tail_stride, void *stream)
{
    if (!m) return fail(DP_ERR_ARG, "NULL model");
    if (!(s_max > 0) || !(stride > 0) || !(tail_max >= s_max) || !std::isfinite(tail_max))
        return fail(DP_ERR_ARG, "need s_max > 0, stride > 0, tail_max >= s_max");
    double nf = s_max / stride;
    if (nf > 1e6) return fail(DP_ERR_ARG, "too many intervals");
    int n_fine = (int)std::llround(nf);
    if (n_fine < 1 || std::fabs(n_fine * stride - s_max) > 1e-9 * s_max)
        return fail(DP_ERR_ARG, "s_max must be a multiple of stride");
    int n_tail = 0;
    if (tail_max > s_max) {
        if (!(tail_stride > 0)) return fail(DP_ERR_ARG, "tail_stride must be > 0");
        double nt = (tail_max - s_max) / tail_stride;
        if (nt > 1e6) return fail(DP_ERR_ARG, "too many tail intervals");
        n_tail = (int)std::llround(nt);
        if (n_tail < 1 || std::fabs(n_tail * tail_stride - (tail_max - s_max)) > 1e-9 * tail_max)
            return fail(DP_ERR_ARG, "tail_max - s_max must be a multiple of tail_stride");
    }
    void *p[] = {m->tab64, m->tab32, m->nodes};
    for (void *q : p)
        if (q) DP_HIP(hipFree(q));
    m->tab64 = nullptr;
    m->tab32 = nullptr;
    m->nodes = nullptr;
    m->tab.n_fine = n_fine;
    m->tab.n_tail = n_tail;
    m->tab.h = stride;
    m->tab.s_max = s_max;
    m->tab.h_tail = n_tail ? tail_stride : stride;
    m->tab.tail_max = n_tail ? tail_max : s_max;
    int n = n_fine + n_tail;
    size_t T = (size_t)m->ntypes;
    DP_HIP(hipMalloc(&m->tab64, sizeof(double) * T * n * kM * 6));
    DP_HIP(hipMalloc(&m->tab32, sizeof(float) * T * n * kM * 6));
    DP_HIP(hipMalloc(&m->nodes, sizeof(double) * T * (n + 1) * kM * 3));
    dp_status s = launch_tabulate(m, (hipStream_t)stream);
    if (s != DP_OK) return s;
    return step_check("tabulate", (hipStream_t)stream);
}

dp_status dp_fitting_tanh(dp_model *m, int tabulated, void *stream)
{
    if (!m || (tabulated != 0 && tabulated != 1)) return fail(DP_ERR_ARG, "bad argument");
    if (tabulated && !m->tanh_tab) {
        DP_HIP(hipMalloc(&m->tanh_tab, sizeof(float) * 4 * kTanhN));
        DP_HIP(hipMalloc(&m->tanh_tab64, sizeof(double) * 4 * kTanhN));
        launch_tanh_table(m->tanh_tab64, m->tanh_tab, (hipStream_t)stream);
        dp_status s = step_check("tanh_table", (hipStream_t)stream);
        if (s != DP_OK) return s;
    }
    m->tanh_on = tabulated;
    return DP_OK;
}

dp_status dp_tanh_table_download(dp_model *m, double *coef_h, int *n_int)
{
    if (!m) return fail(DP_ERR_ARG, "NULL model");
    if (n_int) *n_int = kTanhN;
    if (!coef_h) return DP_OK;
    if (!m->tanh_tab64) return fail(DP_ERR_STATE, "the tanh table has not been built (dp_fitting_tanh)");
    DP_HIP(hipDeviceSynchronize());
    DP_HIP(hipMemcpy(coef_h, m->tanh_tab64, sizeof(double) * 4 * kTanhN, hipMemcpyDeviceToHost));
    return DP_OK;
}

dp_status dp_table_download(dp_model *m, double *coef_h, int *n_int)
{
    if (!m) return fail(DP_ERR_ARG, "NULL model");
    if (!m->tab64) return fail(DP_ERR_STATE, "dp_tabulate has not run");
    int n = m->tab.n_int();
    if (n_int) *n_int = n;
    if (coef_h) {
        DP_HIP(hipDeviceSynchronize());
        DP_HIP(hipMemcpy(coef_h, m->tab64, sizeof(double) * (size_t)m->ntypes * n * kM * 6, hipMemcpyDeviceToHost));
    }
    return DP_OK;
}

dp_status dp_build_nlist(dp_model *m, int natoms, const double *coords_d, const int *types_d,
                         const double *box_h, double skin, dp_nlist **inout, void *stream)
{
    if (!m || !coords_d || !inout) return fail(DP_ERR_ARG, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    for (int attempt = 0; attempt < 4; attempt++) {
        dp_status s = prepare_nlist(m, natoms, box_h, skin, inout);
        if (s != DP_OK) return s;
        dp_nlist *nl = *inout;
        s = build_all(m, nl, coords_d, types_d, st);
        if (s != DP_OK) return s;
        if ((s = step_check("build_nlist", st)) != DP_OK) return s;
        int f[kNumFlags];
        if ((s = read_flags(nl, f, st)) != DP_OK) return s;
        if (attempt < 3 && grow_after_overflow(nl, f)) continue;   // retry with room to spare
        return check_build_flags(f);
    }
    return fail(DP_ERR_CAPACITY, "cell capacity");
}

dp_status dp_nlist_destroy(dp_nlist *nl)
{
    if (!nl) return DP_OK;
    free_nlist_arrays(nl);
    delete nl;
    return DP_OK;
}

static dp_status compute_common(dp_model *m, dp_nlist *nl, int natoms, const double *x, int mode, int precision,
                                double *energy, double *force, double *virial, double *atom_energy, int *nnei,
                                int *nseg, double *T, double *D, hipStream_t st, int phase = 0,
                                bool noalloc = false)
{
    dp_status s = check_compute_args(m, nl, natoms, x, mode, precision);
    if (s != DP_OK) return s;
    if (phase == 2 && nl->fwd_token != precision + 1 + 8 * mode)
        return fail(DP_ERR_STATE, "no kept forward of this precision and mode on this list");
    if (noalloc) {
        // the plain rungs keep their activations in a scratch of their own
        if (mode == DP_PLAIN || mode == DP_TAB_UNFUSED)
            return fail(DP_ERR_UNSUPPORTED, "dp_compute_noalloc runs the fused modes (0, 3, 4) only");
    } else if ((s = ensure_ws(nl, precision, m->cfg.sel)) != DP_OK) {
        return s;
    }
    ComputeArgs a;
    a.m = m;
    a.nl = nl;
    a.natoms = natoms;
    a.x = x;
    a.precision = precision;
    a.energy = energy;
    a.virial = virial;
    a.atom_energy = atom_energy;
    a.nnei_out = nnei;
    a.nseg_out = nseg;
    a.T_out = T;
    a.D_out = D;
    a.need_forces = force || virial;
    a.force = force ? force : nl->force_tmp;
    a.phase = phase;
    a.noalloc = noalloc;
    // any forward overwrites the kept activations
    nl->fwd_token = phase == 1 ? precision + 1 + 8 * mode : (phase == 2 ? nl->fwd_token : 0);
    a.mode = mode;
    return (mode == DP_PLAIN || mode == DP_TAB_UNFUSED) ? run_plain(a, st) : run_compressed(a, st);
}

// The box check shared by dp_compute and dp_compute_noalloc.
static dp_status check_box(const dp_nlist *nl, const double *box_h)
{
    if (nl && nl->periodic) {
        double L[3];
        if (!box_h || !box_ok(box_h, L) || L[0] != nl->L[0] || L[1] != nl->L[1] || L[2] != nl->L[2])
            return fail(DP_ERR_ARG, "box differs from the one the list was built for");
    } else if (nl && box_h) {
        return fail(DP_ERR_ARG, "the list was built for an open cluster");
    }
    return DP_OK;
}

dp_status dp_compute(dp_model *m, dp_nlist *nl, int natoms, const double *coords_d, const int *types_d,
                     const double *box_h, int mode, int precision, double *energy_d, double *force_d,
                     double *virial_d, double *atom_energy_d, void *stream)
{
    (void)types_d;
    dp_status s = check_box(nl, box_h);
    if (s != DP_OK) return s;
    return compute_common(m, nl, natoms, coords_d, mode, precision, energy_d, force_d, virial_d, atom_energy_d,
                          nullptr, nullptr, nullptr, nullptr, (hipStream_t)stream);
}

dp_status dp_compute_noalloc(dp_model *m, dp_nlist *nl, int natoms, const double *coords_d, const int *types_d,
                             const double *box_h, int mode, int precision, double *energy_d, double *force_d,
                             double *virial_d, double *atom_energy_d, void *stream)
{
    (void)types_d;
    dp_status s = check_box(nl, box_h);
    if (s != DP_OK) return s;
    timers_quiet(true);
    s = compute_common(m, nl, natoms, coords_d, mode, precision, energy_d, force_d, virial_d, atom_energy_d,
                       nullptr, nullptr, nullptr, nullptr, (hipStream_t)stream, 0, true);
    timers_quiet(false);
    return s;
}

dp_status dp_energy_forward(dp_model *m, dp_nlist *nl, int natoms, const double *coords_d, int mode,
                            int precision, double *energy_d, double *atom_energy_d, void *stream)
{
    return compute_common(m, nl, natoms, coords_d, mode, precision, energy_d, nullptr, nullptr, atom_energy_d,
                          nullptr, nullptr, nullptr, nullptr, (hipStream_t)stream, 1);
}

dp_status dp_energy_backward(dp_model *m, dp_nlist *nl, int natoms, const double *coords_d, int mode,
                             int precision, double *force_d, double *virial_d, void *stream)
{
    if (!force_d && !virial_d) return fail(DP_ERR_ARG, "nothing to compute");
    return compute_common(m, nl, natoms, coords_d, mode, precision, nullptr, force_d, virial_d, nullptr, nullptr,
                          nullptr, nullptr, nullptr, (hipStream_t)stream, 2);
}

dp_status dp_descriptor(dp_model *m, dp_nlist *nl, int natoms, const double *coords_d, const double *box_h,
                        int mode, int precision, int *nnei_d, int *nseg_d, double *T_d, double *D_d, void *stream)
{
    (void)box_h;
    return compute_common(m, nl, natoms, coords_d, mode, precision, nullptr, nullptr, nullptr, nullptr, nnei_d,
                          nseg_d, T_d, D_d, (hipStream_t)stream);
}

dp_status dp_nlist_stats(dp_nlist *nl, int *max_nei, int *n_sel_overflow, int *n_table_oob, int *n_cap_overflow)
{
    if (!nl) return fail(DP_ERR_ARG, "NULL list");
    int f[kNumFlags];
    DP_HIP(hipDeviceSynchronize());
    DP_HIP(hipMemcpy(f, nl->flags, sizeof(f), hipMemcpyDeviceToHost));
    if (max_nei) *max_nei = f[kFlagMaxNei];
    if (n_sel_overflow) *n_sel_overflow = f[kFlagSelOverflow];
    if (n_table_oob) *n_table_oob = f[kFlagTableOob];
    if (n_cap_overflow) *n_cap_overflow = f[kFlagCapOverflow];
    return DP_OK;
}

// nsteps of velocity Verlet from the list's trajectory state.  fresh: the
// list is (re)built at x and the forces evaluated first (dp_nve_run);
// otherwise the forces and energy the previous run left are used and the
// rebuild cadence continues from its last build (dp_nve_continue).
static dp_status nve_steps(dp_model *m, dp_nlist **nlp, int natoms, double *x, double *v, const int *types,
                           const double *box_h, const double *mass_h, double dt_fs, int nsteps, int rebuild_every,
                           double skin, int mode, int precision, double *thermo, hipStream_t st, bool fresh)
{
    const int T = m->cfg.ntypes;
    for (int t = 0; t < T; t++)
        if (!(mass_h[t] > 0) || !std::isfinite(mass_h[t])) return fail(DP_ERR_ARG, "need masses > 0");
    if (!(dt_fs > 0) || nsteps < 0 || rebuild_every < 1)
        return fail(DP_ERR_ARG, "need dt > 0, nsteps >= 0, rebuild_every >= 1");
    dp_status s;
    dp_nlist *nl = *nlp;
    if (fresh) {
        for (int attempt = 0;; attempt++) {   // the first build, checked as in dp_build_nlist
            if ((s = prepare_nlist(m, natoms, box_h, skin, nlp)) != DP_OK) return s;
            nl = *nlp;
            if ((s = check_compute_args(m, nl, natoms, x, mode, precision)) != DP_OK) return s;
            if ((s = build_all(m, nl, x, types, st)) != DP_OK) return s;
            if ((s = step_check("build_nlist", st)) != DP_OK) return s;
            int f[kNumFlags];
            if ((s = read_flags(nl, f, st)) != DP_OK) return s;
            if (attempt < 3 && grow_after_overflow(nl, f)) continue;
            if ((s = check_build_flags(f)) != DP_OK) return s;
            break;
        }
    } else {
        if (!nl || nl->nve_x != x || nl->nve_natoms != natoms || nl->nve_mode != mode || nl->nve_prec != precision)
            return fail(DP_ERR_STATE, "no trajectory to continue on this list: call dp_nve_run first (with the "
                                      "same positions array, atom count, mode and precision)");
        if ((s = check_compute_args(m, nl, natoms, x, mode, precision)) != DP_OK) return s;
    }
    // rebuilds inside the run reuse the list's copy of the types
    const int *tl = T > 1 ? nl->type : types;
    const int *tk = T > 1 ? nl->type : nullptr;   // per-atom type of the Verlet kernels
    double *F = nl->nve_F, *E = nl->scal, *part = nl->scal + 256;
    TypeScalars kick, kef;
    for (int t = 0; t < T; t++) {
        kick.v[t] = 0.5 * dt_fs * acc_unit() / mass_h[t];
        kef.v[t] = 0.5 * mass_h[t] * ke_unit();
    }
    // the box of the list, for a reallocation after a capacity overflow
    double box_l[9] = {nl->L[0], 0, 0, 0, nl->L[1], 0, 0, 0, nl->L[2]};
    const double *box = fresh ? box_h : (nl->periodic ? box_l : nullptr);
    const double skin_l = fresh ? skin : nl->rc_build - nl->rcut_build;
    int since = fresh ? 0 : nl->nve_since_build;
    nl->nve_x = nullptr;   // until this run ends normally
    if (fresh) {
        s = compute_common(m, nl, natoms, x, mode, precision, E, F, nullptr, nullptr, nullptr, nullptr, nullptr,
                           nullptr, st);
        if (s != DP_OK) return s;
    }
    if (thermo) launch_thermo(v, E, natoms, tk, kef, thermo, part, st);
    for (int step = 1; step <= nsteps; step++) {
        launch_verlet_kick_drift(x, v, F, natoms, tk, kick, dt_fs, st);
        if (++since % rebuild_every == 0) {
            // The counters of the run accumulate (no reset).  One
            // synchronisation per rebuild checks what the evaluations since the
            // last one flagged, and the build's capacities (grown and built
            // again on an overflow, as in dp_build_nlist).
            for (int attempt = 0;; attempt++) {
                DP_TIMED("nlist", st, s = launch_build_nlist(m, nl, x, tl, false, st));
                if (s != DP_OK) return s;
                if ((s = step_check("build_nlist", st)) != DP_OK) return s;
                int f[kNumFlags];
                if ((s = read_flags(nl, f, st)) != DP_OK) return s;
                if ((s = check_eval_flags(f)) != DP_OK) return s;
                if (attempt < 3 && grow_after_overflow(nl, f)) {
                    launch_fill_zero_int(nl->flags + kFlagCapOverflow, 1, st);
                    launch_fill_zero_int(nl->flags + kFlagCellOverflow, 1, st);
                    if ((s = prepare_nlist(m, natoms, box, skin_l, nlp)) != DP_OK) return s;
                    // a reallocation drops the forces of the step; they are
                    // evaluated again below at the same positions
                    F = nl->nve_F;
                    continue;
                }
                if ((s = check_build_flags(f)) != DP_OK) return s;
                break;
            }
            since = 0;
        }
        s = compute_common(m, nl, natoms, x, mode, precision, E, F, nullptr, nullptr, nullptr, nullptr, nullptr,
                           nullptr, st);
        if (s != DP_OK) return s;
        launch_verlet_kick(v, F, natoms, tk, kick, st);
        if (thermo) launch_thermo(v, E, natoms, tk, kef, thermo + 2 * step, part, st);
        if ((s = step_check("verlet", st)) != DP_OK) return s;
    }
    int f[kNumFlags];
    if ((s = read_flags(nl, f, st)) != DP_OK) return s;
    if ((s = check_eval_flags(f)) != DP_OK) return s;
    if ((s = check_build_flags(f)) != DP_OK) return s;
    nl->nve_x = x;
    nl->nve_natoms = natoms;
    nl->nve_mode = mode;
    nl->nve_prec = precision;
    nl->nve_since_build = since % rebuild_every;
    return DP_OK;
}

dp_status dp_nve_run(dp_model *m, dp_nlist **nlp, int natoms, double *x, double *v, const int *types,
                     const double *box_h, const double *mass_h, double dt_fs, int nsteps, int rebuild_every,
                     double skin, int mode, int precision, double *thermo, void *stream)
{
    if (!m || !nlp || !x || !v || !mass_h) return fail(DP_ERR_ARG, "NULL argument");
    return nve_steps(m, nlp, natoms, x, v, types, box_h, mass_h, dt_fs, nsteps, rebuild_every, skin, mode, precision,
                     thermo, (hipStream_t)stream, true);
}

dp_status dp_nve_continue(dp_model *m, dp_nlist *nl, int natoms, double *x, double *v, const double *mass_h,
                          double dt_fs, int nsteps, int rebuild_every, int mode, int precision, double *thermo,
                          void *stream)
{
    if (!m || !nl || !x || !v || !mass_h) return fail(DP_ERR_ARG, "NULL argument");
    dp_nlist *nlp = nl;
    return nve_steps(m, &nlp, natoms, x, v, nullptr, nullptr, mass_h, dt_fs, nsteps, rebuild_every, 0.0, mode,
                     precision, thermo, (hipStream_t)stream, false);
}

dp_status dp_nlist_check(dp_nlist *nl)
{
    if (!nl) return fail(DP_ERR_ARG, "NULL list");
    int f[kNumFlags];
    DP_HIP(hipDeviceSynchronize());
    DP_HIP(hipMemcpy(f, nl->flags, sizeof(f), hipMemcpyDeviceToHost));
    dp_status s = check_eval_flags(f);
    return s != DP_OK ? s : check_build_flags(f);
}

dp_status dp_nlist_export(dp_nlist *nl, int *natoms, int *cap, int *cnt_d, int *nei_d, int *shift_d,
                          float *dist_d, short *rev_d, void *stream)
{
    if (!nl || !natoms || !cap) return fail(DP_ERR_ARG, "NULL list or count pointer");
    *natoms = nl->natoms;
    *cap = nl->cap;
    hipStream_t st = (hipStream_t)stream;
    const size_t n = (size_t)nl->natoms, nc = n * (size_t)nl->cap;
    auto copy = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        return dst && bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) : hipSuccess;
    };
    DP_HIP(copy(cnt_d, nl->cnt, sizeof(int) * n));
    DP_HIP(copy(nei_d, nl->nei, sizeof(int) * nc));
    DP_HIP(copy(shift_d, nl->shift, sizeof(int) * nc));
    DP_HIP(copy(dist_d, nl->dist, sizeof(float) * nc));
    DP_HIP(copy(rev_d, nl->rev, sizeof(short) * nc));
    DP_HIP(hipStreamSynchronize(st));
    return DP_OK;
}

dp_status dp_footprint_bytes(const dp_model *m, int natoms, size_t *bytes)
{
    if (!m || natoms < 0 || !bytes) return fail(DP_ERR_ARG, "bad argument");
    // candidates (index, shift, distance, reverse slot, pair gradient), positions, boxes, counts
    size_t per = (size_t)kCapMax * (4 + 4 + 4 + 2 + 24) + 3 * 8 + 3 * 8 + 4 * 4 + 3 * 8 + 3 * 8 + 4 * kMaxTypes;
    size_t ws = std::max(ws_bytes_for_atoms(natoms, DP_FP64, m->cfg.sel, m->cfg.ntypes),
                         ws_bytes_for_atoms(natoms, DP_MIXED_BF16, m->cfg.sel, m->cfg.ntypes));
    if (m->cfg.ntypes > 1) per += 4 * (2 + kMaxTypes) + 4;   // type, row, per-type counts, row map
    *bytes = per * (size_t)natoms + ws;
    return DP_OK;
}

dp_status dp_batch_create(dp_model *m, int max_atoms, int max_requests, double skin, dp_batch **out)
{
    if (!m || !out || max_atoms < 1 || max_requests < 1 || !(skin >= 0)) return fail(DP_ERR_ARG, "bad argument");
    if (max_atoms >= (1 << 24)) return fail(DP_ERR_UNSUPPORTED, "at most 2^24 - 1 atoms");
    if (m->cfg.ntypes != 1) return fail(DP_ERR_UNSUPPORTED, "batches hold one-type models only");
    dp_batch *b = new dp_batch();
    b->max_atoms = max_atoms;
    b->max_req = max_requests;
    b->skin = skin;
    dp_nlist *nl = new dp_nlist();
    b->nl = nl;
    DP_HIP(hipGetDevice(&nl->device));
    nl->rc_build = m->cfg.rcut + skin;
    nl->rcut_build = m->cfg.rcut;
    nl->periodic = true;
    nl->cap = kCapMax;
    nl->alloc_atoms = max_atoms;
    size_t A = (size_t)max_atoms;
    DP_HIP(hipMalloc(&nl->wpos, sizeof(double) * 3 * A));
    DP_HIP(hipMalloc(&nl->wrap, sizeof(int) * A));
    DP_HIP(hipMalloc(&nl->cnt, sizeof(int) * A));
    DP_HIP(hipMalloc(&nl->nei, sizeof(int) * A * kCapMax));
    DP_HIP(hipMalloc(&nl->shift, sizeof(int) * A * kCapMax));
    DP_HIP(hipMalloc(&nl->dist, sizeof(float) * A * kCapMax));
    DP_HIP(hipMalloc(&nl->rev, sizeof(short) * A * kCapMax));
    DP_HIP(hipMalloc(&nl->pg, sizeof(double) * 3 * A * kCapMax));
    DP_HIP(hipMalloc(&nl->force_tmp, sizeof(double) * 3 * A));
    DP_HIP(hipMalloc(&nl->atomL, sizeof(double) * 3 * A));
    DP_HIP(hipMalloc(&nl->flags, sizeof(int) * kNumFlags));
    DP_HIP(hipMemset(nl->flags, 0, sizeof(int) * kNumFlags));
    DP_HIP(hipMalloc(&nl->scal, sizeof(double) * 512));
    DP_HIP(hipMalloc(&b->off_d, sizeof(int) * (max_requests + 1)));
    DP_HIP(hipMalloc(&b->Lreq_d, sizeof(double) * 3 * max_requests));
    DP_HIP(hipHostMalloc((void **)&b->off_h, sizeof(int) * (max_requests + 1), hipHostMallocDefault));
    DP_HIP(hipHostMalloc((void **)&b->Lreq_h, sizeof(double) * 3 * max_requests, hipHostMallocDefault));
    DP_HIP(hipEventCreateWithFlags(&b->staged, hipEventDisableTiming));
    dp_status s = ensure_ws(nl, DP_FP64, m->cfg.sel);
    if (s != DP_OK) return s;
    *out = b;
    return DP_OK;
}

dp_status dp_batch_destroy(dp_batch *b)
{
    if (!b) return DP_OK;
    if (b->nl) {
        (void)hipFree(b->nl->atomL);
        b->nl->atomL = nullptr;
        dp_nlist_destroy(b->nl);
    }
    (void)hipFree(b->off_d);
    (void)hipFree(b->Lreq_d);
    (void)hipHostFree(b->off_h);
    (void)hipHostFree(b->Lreq_h);
    if (b->staged) (void)hipEventDestroy(b->staged);
    delete b;
    return DP_OK;
}

dp_status dp_batch_compute(dp_model *m, dp_batch *b, int nreq, const dp_request *reqs, const double *coords_d,
                           int precision, double *energy_d, double *force_d, double *virial_d,
                           double *atom_energy_d, void *stream)
{
    if (!m || !b || !reqs || !coords_d || nreq < 1) return fail(DP_ERR_ARG, "bad argument");
    if (m->cfg.ntypes != 1) return fail(DP_ERR_UNSUPPORTED, "batches hold one-type models only");
    if (nreq > b->max_req) return fail(DP_ERR_CAPACITY, "more requests than the batch was created for");
    if (!m->tab64) return fail(DP_ERR_STATE, "dp_tabulate has not run");
    if (precision < DP_FP64 || precision > DP_MIXED_BF16) return fail(DP_ERR_ARG, "unknown precision");
    hipStream_t st = (hipStream_t)stream;
    dp_nlist *nl = b->nl;
    double rcs = nl->rc_build;
    long total = 0;
    size_t cells_needed = 0;
    int cellcap = 0;
    for (int r = 0; r < nreq; r++) {
        const dp_request &q = reqs[r];
        if (q.natoms < 1 || q.offset != total) return fail(DP_ERR_ARG, "requests must be contiguous and non-empty");
        total += q.natoms;
        if (q.periodic) {
            double L[3];
            if (!box_ok(q.box, L)) return fail(DP_ERR_UNSUPPORTED, "box must be orthorhombic");
            long ncell = 1;
            for (int a = 0; a < 3; a++) {
                if (L[a] < 0.5 * rcs) return fail(DP_ERR_UNSUPPORTED, "box edge shorter than (rcut + skin) / 2");
                int nc = (int)std::floor(L[a] / (0.5 * rcs));
                ncell *= nc < 1 ? 1 : nc;
            }
            int per = (int)std::ceil((double)q.natoms / ncell);
            int cc = (int)round_up(3 * per + 8, 8);
            cellcap = std::max(cellcap, cc);
            cells_needed = std::max(cells_needed, (size_t)ncell);
        } else if (q.natoms > kCapMax) {
            return fail(DP_ERR_UNSUPPORTED, "open clusters in a batch hold at most 1024 atoms");
        }
    }
    if (total > b->max_atoms) return fail(DP_ERR_CAPACITY, "batch exceeds max_atoms");
    cellcap = std::max(cellcap, nl->cellcap);
    if (cells_needed * cellcap > nl->ncell_alloc || (cells_needed && !nl->cell_cnt)) {
        // grow the shared cell grid (rare: only for a larger cell than seen before)
        DP_HIP(hipStreamSynchronize(st));
        if (nl->cell_atoms) DP_HIP(hipFree(nl->cell_atoms));
        if (nl->cell_cnt) DP_HIP(hipFree(nl->cell_cnt));
        size_t nc = std::max(cells_needed, (size_t)1);
        DP_HIP(hipMalloc(&nl->cell_atoms, sizeof(CellAtom) * nc * cellcap));
        DP_HIP(hipMalloc(&nl->cell_cnt, sizeof(int) * nc));
        nl->ncell_alloc = nc * cellcap;
    }
    nl->cellcap = cellcap ? cellcap : nl->cellcap;
    // request table: staging buffers are reused, so wait for the last upload
    DP_HIP(hipEventSynchronize(b->staged));
    for (int r = 0; r < nreq; r++) {
        b->off_h[r] = reqs[r].offset;
        for (int a = 0; a < 3; a++) b->Lreq_h[3 * r + a] = reqs[r].periodic ? reqs[r].box[4 * a] : 0.0;
    }
    b->off_h[nreq] = (int)total;
    DP_HIP(hipMemcpyAsync(b->off_d, b->off_h, sizeof(int) * (nreq + 1), hipMemcpyHostToDevice, st));
    DP_HIP(hipMemcpyAsync(b->Lreq_d, b->Lreq_h, sizeof(double) * 3 * nreq, hipMemcpyHostToDevice, st));
    DP_HIP(hipEventRecord(b->staged, st));
    launch_expand_boxes(nreq, b->off_d, b->Lreq_d, nl->atomL, st);
    launch_fill_zero_int(nl->flags, kNumFlags, st);
    for (int r = 0; r < nreq; r++) {
        double L[3];
        const double *Lp = nullptr;
        if (reqs[r].periodic) {
            box_ok(reqs[r].box, L);
            Lp = L;
        }
        dp_status s = launch_build_nlist_range(nl, coords_d, reqs[r].offset, reqs[r].natoms, Lp, st);
        if (s != DP_OK) return s;
    }
    launch_reverse(nl, 0, (int)total, st);
    dp_status s = step_check("batch_nlist", st);
    if (s != DP_OK) return s;
    nl->natoms = (int)total;
    nl->fwd_token = 0;
    ComputeArgs a{};
    a.m = m;
    a.nl = nl;
    a.natoms = (int)total;
    a.x = coords_d;
    a.precision = precision;
    a.energy = energy_d;
    a.virial = virial_d;
    a.atom_energy = atom_energy_d;
    a.need_forces = force_d || virial_d;
    a.force = force_d ? force_d : nl->force_tmp;
    a.phase = 0;
    a.nseg = nreq;
    a.seg_off = b->off_d;
    return run_compressed(a, st);
}

dp_status dp_batch_stats(dp_batch *b, int *max_nei, int *n_sel_overflow, int *n_table_oob, int *n_cap_overflow)
{
    if (!b) return fail(DP_ERR_ARG, "NULL batch");
    int f[kNumFlags];
    DP_HIP(hipDeviceSynchronize());
    DP_HIP(hipMemcpy(f, b->nl->flags, sizeof(f), hipMemcpyDeviceToHost));
    if (max_nei) *max_nei = f[kFlagMaxNei];
    if (n_sel_overflow) *n_sel_overflow = f[kFlagSelOverflow];
    if (n_table_oob) *n_table_oob = f[kFlagTableOob];
    if (n_cap_overflow) *n_cap_overflow = f[kFlagCapOverflow] + f[kFlagCellOverflow];
    return DP_OK;
}

const char *dp_last_error(void) { return g_err.c_str(); }

}  // extern "C"

