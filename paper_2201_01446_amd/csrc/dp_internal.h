// dp_internal.h -- handle layouts, launch helpers and device utilities shared
// by the HIP translation units of libdp (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/dp.h"

namespace dp {

// Fixed model shape of this build: M = 128 embedding columns, M< = 16.
constexpr int kM = 128;
constexpr int kMlt = 16;
constexpr int kDdim = kM * kMlt;     // 2048 descriptor entries per atom
constexpr int kFitPad = 256;         // fitting widths padded to 256 (zero columns)
constexpr int kCapMax = 1024;        // skin candidates per atom, upper bound
constexpr int kRowPad = 128;         // atom rows of every GEMM operand padded to 128
constexpr int kMaxTypes = DP_MAX_TYPES;
// Per-type block of the fitting net's vectors: c1, c2, c3, w4 (kFitPad each), b4
constexpr int kFitB = 4 * kFitPad + 64;

// Device-side sticky counters of a neighbor list, each on a 128-byte line of
// its own (atomics on one counter must not delay reads of another).
constexpr int kFlagStride = 32;
enum Flag {
    kFlagMaxNei = 0 * kFlagStride,        // atomicMax of neighbors within rcut
    kFlagSelOverflow = 1 * kFlagStride,   // atoms with more than sel neighbors within rcut
    kFlagTableOob = 2 * kFlagStride,      // table look-ups past the last node
    kFlagCapOverflow = 3 * kFlagStride,   // atoms whose candidate list hit cap
    kFlagCellOverflow = 4 * kFlagStride,  // atoms that did not fit their cell
    kFlagBadType = 5 * kFlagStride,       // atoms with a type outside [0, ntypes)
    kFlagSkin = 6 * kFlagStride,          // an evaluation found an atom moved too far since the build
    kFlagNonFinite = 7 * kFlagStride,     // an evaluation produced a non-finite energy or virial
    kFlagBadCoord = 8 * kFlagStride,      // a non-finite coordinate was seen
    kNumFlags = 12 * kFlagStride
};

struct TableInfo {
    int n_fine = 0, n_tail = 0;
    double h = 0, s_max = 0, h_tail = 0, tail_max = 0;
    int n_int() const { return n_fine + n_tail; }
};

// Fitting-net weights in one precision, widths padded to kFitPad, one copy
// per center type back to back (type t at t times one matrix's size).
//   Vk  : [in][kFitPad] forward operands, Vkt : [kFitPad][in] transposed
//   (backward operands), bias and output vector as float/double.
struct FitWeights {
    void *V1 = nullptr, *V2 = nullptr, *V3 = nullptr;
    void *V1t = nullptr, *V2t = nullptr, *V3t = nullptr;
    // V1t with its columns in the order k' = b M< + a of the D operand formed
    // from T (column a M + b of V1t at k'); FP32 and FP64
    void *V1tp = nullptr;
};

// An atom binned into a cell of the neighbor grid: its wrapped position,
// index and type, read together by the candidate search.
struct alignas(16) CellAtom {
    double x, y, z;
    int j, type;
};

}  // namespace dp

struct dp_model {
    dp_model_config cfg;
    int device = 0;
    int d1 = 0, d2 = 0, d3 = 0, f1 = 0, f2 = 0, f3 = 0;
    // parameters on the device
    int ntypes = 1;
    double *emb_d = nullptr;     // W0 b0 W1 b1 W2 b2 per neighbor type, FP64, file layout
    double *fitb_d = nullptr;    // per center type (kFitB apart): c1 c2 c3 w4 (each kFitPad, zero padded), b4
    float *fitb_f = nullptr;     // same in FP32
    double b4[dp::kMaxTypes] = {0, 0, 0, 0};   // output bias per center type
    dp::FitWeights w64, w32, wbf;   // double, float, bf16 GEMM operands
    void *embg64 = nullptr;      // embedding weights in GEMM layouts (plain path), FP64
    void *embg32 = nullptr;      // the same in FP32
    // table
    dp::TableInfo tab;
    double *tab64 = nullptr;     // [ntypes * n_int][M][6]: type t's table at interval t * n_int
    float *tab32 = nullptr;      // [ntypes * n_int][M][6]
    double *nodes = nullptr;     // scratch [ntypes][n_int+1][M][3] of node values g, g', g''
    // tanh of the fitting net: native, or the second-order table
    // [kTanhN][a0, a1, a2, 0] on [0, 8), in FP64 (FP64 epilogues) and FP32
    float *tanh_tab = nullptr;
    double *tanh_tab64 = nullptr;
    int tanh_on = 0;
};

struct dp_nlist {
    int device = 0;
    int natoms = 0;
    int alloc_atoms = 0;
    int cap = 0;
    bool periodic = false;
    double L[3] = {0, 0, 0};
    double rc_build = 0;
    // cell grid
    int nc[3] = {1, 1, 1};
    int cellcap = 0;
    size_t ncell_alloc = 0;
    int *cell_cnt = nullptr;
    dp::CellAtom *cell_atoms = nullptr;   // [ncell * cellcap]
    // wrapped positions and image index (int8 x3 packed) of every atom at build
    double *wpos = nullptr;
    int *wrap = nullptr;
    // candidates
    int *cnt = nullptr;      // [natoms]
    int *nei = nullptr;      // [natoms * cap]
    int *shift = nullptr;    // [natoms * cap], int8 x3 packed image shift
    float *dist = nullptr;   // [natoms * cap], distance at build (the sort key)
    short *rev = nullptr;    // [natoms * cap], slot of (i, -shift) in j's list, or -1
    void *pg = nullptr;      // [natoms * cap * 3] reals: dE_i/dr_ij per candidate slot
    int *flags = nullptr;    // [kNumFlags]
    // exact early end of the candidate scan: the positions at build, per atom
    // and type the candidates whose build distance is <= rcut + margin (a
    // prefix of the sorted run), and the largest displacement since the build
    // (FP64 bits, set before each evaluation); none of these in batch lists
    double *x0 = nullptr;                 // [natoms * 3]
    int *inner = nullptr;                 // [natoms * kMaxTypes]
    unsigned long long *disp = nullptr;   // [1]
    double margin = 0;                    // skin / 4
    // the model cut-off the list was built for (rc_build = rcut_build + skin),
    // and a lower bound on the candidate capacity (raised after an overflow)
    double rcut_build = 0;
    int cap_floor = 0;
    // several types: each atom's type, its candidates per type (the list is
    // grouped by type), and the fitting net's row of each atom: rows are
    // grouped by center type, group t at [trow[t], trow[t + 1]), each group
    // padded to a whole GEMM tile; ratom maps a row back to its atom (-1: pad)
    int ntypes = 1;
    int *type = nullptr;     // [natoms]
    int *tcnt = nullptr;     // [natoms * kMaxTypes]
    int *row = nullptr;      // [natoms]
    int *ratom = nullptr;    // [rows]
    int *tblk = nullptr;     // scratch of the row assignment
    int trow[dp::kMaxTypes + 1] = {0, 0, 0, 0, 0};
    int rows = 0;            // trow[ntypes] when ntypes > 1
    // per-configuration scratch of dp_compute
    void *ws = nullptr;
    size_t ws_bytes = 0;
    void *ws_plain = nullptr;
    size_t ws_plain_bytes = 0;
    double *atomL = nullptr;       // per-atom box edges when the list spans a batch of cells
    double *force_tmp = nullptr;   // forces when the caller wants only the virial
    int fwd_token = 0;             // precision+1 while a forward's activations are kept
    double *scal = nullptr;        // [16] device scalars (energy, partial sums)
    // the trajectory left by the last dp_nve_run / dp_nve_continue on this
    // list, from which dp_nve_continue resumes: forces (nve_F) and energy
    // (scal[0]) at the final positions nve_x, steps since the last build;
    // nve_x NULL when there is none (any (re)allocation or build clears it)
    double *nve_F = nullptr;
    const double *nve_x = nullptr;
    int nve_natoms = 0, nve_mode = -1, nve_prec = -1, nve_since_build = 0;
};

// A batch of independent cells (serving): one combined neighbor list and
// scratch sized for max_atoms, resident across calls.
struct dp_batch {
    dp_nlist *nl = nullptr;
    int max_atoms = 0, max_req = 0;
    double skin = 2.0;
    int *off_d = nullptr;        // [max_req + 1]
    double *Lreq_d = nullptr;    // [max_req][3]
    int *off_h = nullptr;        // pinned staging of the request table
    double *Lreq_h = nullptr;
    hipEvent_t staged = nullptr; // the last upload from the staging buffers has run
};

namespace dp {

// ----------------------------------------------------------------- errors
void set_error(const std::string &msg);
dp_status fail(dp_status st, const std::string &msg);
dp_status hip_fail(hipError_t e, const char *what);

#define DP_HIP(call)                                                   \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return dp::hip_fail(e_, #call);          \
    } while (0)

// Records HIP events around the enclosed launches on `st` when timing is
// enabled (dp_timers_enable); aggregated by name in dp_timers_read.
class TimerScope {
  public:
    TimerScope(const char *name, hipStream_t st);
    ~TimerScope();

  private:
    const char *name_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};
#define DP_TIMED(name, st, ...)              \
    do {                                     \
        dp::TimerScope ts_(name, st);        \
        __VA_ARGS__;                         \
    } while (0)

// After a group of launches: the launch error, if any; and, when the
// environment sets DP_SYNC_CHECK=1, a synchronisation that attributes an
// asynchronous kernel failure to the named step.
dp_status step_check(const char *name, hipStream_t st);

constexpr int div_up(long a, long b) { return (int)((a + b - 1) / b); }
constexpr long round_up(long a, long b) { return (a + b - 1) / b * b; }

// XCD-aware work order.  The dispatcher deals the blocks of a grid round-robin
// over the 8 XCDs (each with its own L2), so block b runs on XCD b % 8.  A
// kernel whose neighboring items share data (atoms and their neighbors) gives
// XCD x the contiguous item range [x G/8, (x+1) G/8) instead; the grid is
// padded to a multiple of 8 (xcd_grid) and items past the real count exit.
// Only locality depends on the dealing order, never correctness.
constexpr int kXcd = 8;

// Waves (atoms) per block for a kernel that needs per_wave bytes of LDS per
// wave: 4 when they fit 64 KB, else 2, else 1 (0: too large).
inline int lds_wpb(size_t per_wave)
{
    for (int w = 4; w >= 1; w >>= 1)
        if ((size_t)w * per_wave <= 65536) return w;
    return 0;
}
inline int xcd_grid(long nblocks) { return (int)round_up(nblocks, kXcd); }
__device__ inline int xcd_item(int b, int grid) { return (b % kXcd) * (grid / kXcd) + b / kXcd; }

// ------------------------------------------------------------- launchers
// (defined in the kernel translation units; all enqueue on `st`)
void launch_fill_zero(double *p, long n, hipStream_t st);
void launch_fill_zero_bytes(void *p, size_t nbytes, hipStream_t st);
void launch_fill_zero_int(int *p, long n, hipStream_t st);
// The largest |x_i - x0_i| into nl->disp (no-op for lists without x0); sets
// kFlagSkin when twice it reaches `lim` (the list's reach beyond the
// evaluating model's cut-off: a pair within that cut-off may then lack its
// candidate) and kFlagBadCoord on a non-finite position.
void launch_displacement(const dp_nlist *nl, int n, const double *x, double lim, hipStream_t st);
dp_status launch_tabulate(dp_model *m, hipStream_t st);
constexpr int kTanhN = 1024;   // tanh table intervals of width 1/128 on [0, 8)
void launch_tanh_table(double *tab64, float *tab32, hipStream_t st);
dp_status launch_build_nlist(const dp_model *m, dp_nlist *nl, const double *x, const int *types,
                             bool reset_flags, hipStream_t st);
// Candidates of the atoms [off, off + n) of a batch, all inside one cell with
// box edges L (NULL: open); neighbor indices are global (j + off).
dp_status launch_build_nlist_range(dp_nlist *nl, const double *x, int off, int n, const double *L,
                                   hipStream_t st);
void launch_segment_reduce(int nreq, const int *offsets, const double *e_atom, const double *w_atom,
                           double *energy, double *virial, int *flags, hipStream_t st);
void launch_expand_boxes(int nreq, const int *offsets, const double *Lreq, double *atomL, hipStream_t st);

// BF16 operands of the fitting net are kept as an exact-ish split
// x = hi + lo (hi = bf16(x), lo = bf16(x - hi)) laid out along K as
// [hi | hi | lo] for A and [hi | lo | hi] for Bt, so one BF16 GEMM over 3K
// accumulates hi*hi + hi*lo + lo*hi (the lo*lo term, ~2^-18 relative, is
// dropped).  kSplit is the K multiplier of a precision's operands.
constexpr int kSplitBf16 = 3;
__host__ __device__ inline int k_split(int precision) { return precision == DP_MIXED_BF16 ? kSplitBf16 : 1; }

// Epilogues of the fitting-net GEMM C = A Bt^T (see fit.hip).
//   EPI_LIN  out_r = acc
//   EPI_T1   out_r = out_o = tanh(acc + bias)
//   EPI_T2   t = tanh(acc + bias); out_t = t; out_r = out_o = res + t
//   EPI_T3   out_t = tanh(acc + bias)
//   EPI_BWD  dy = (resv or res) + acc; out_r = dy; out_o = dy (1 - tt^2)
//   EPI_EMB  t = tanh(acc + bias); out_t = t; out_r = res[m][n mod resw] + t
//            (the (x, x) shortcut of an embedding layer)
//   EPI_FOLD columns n < half only: dy = res[m][n] + res[m][n + half] + acc;
//            out_o[m][n] = dy (1 - tt[m][n]^2), with row pitch `half` for tt
//            and out_o, 2 half for res (adjoint of the (x, x) shortcut)
enum EpiKind { EPI_LIN = 0, EPI_T1 = 1, EPI_T2 = 2, EPI_T3 = 3, EPI_BWD = 4, EPI_EMB = 5, EPI_FOLD = 6 };
struct Epi {
    const void *bias;  // TR[N]
    const void *res;   // TR[M][N]
    const void *resv;  // TR[N], broadcast over rows
    const void *tt;    // TR[M][N] tanh outputs
    void *out_r;       // TR[M][N]
    void *out_o;       // TA[M][N]
    void *out_t;       // TR[M][N]
    int resw = 0;      // EPI_EMB: width of the residual input
    int half = 0;      // EPI_FOLD
    const float *tanh_tab = nullptr;     // FP32 epilogues: tanh from this table (kTanhN x 4), or native
    const double *tanh_tab64 = nullptr;  // FP64 epilogues: the same table in FP64, or native
    // rows grouped by type (several types): a tile whose first row lies in
    // [trow[t], trow[t + 1]) takes Bt + t bstride and bias / resv + t vstride
    int ntr = 0;
    int trow[dp::kMaxTypes + 1] = {0, 0, 0, 0, 0};
    long bstride = 0;
    int vstride = 0;
    // launch_gemm_dt: T (TA[atoms][kM][4], by column) whose D = T<^T T is the A operand,
    // the atom of each row (several types; -1: padding) or, with one type,
    // the rows below dt_nlive are the atoms
    const void *dt_T = nullptr;
    const int *dt_ratom = nullptr;
    int dt_nlive = 0;
    // row length of A and Bt (elements) when it exceeds K: the last kld - K
    // elements of every row are zero padding that the product skips; 0: K.
    // K is a whole number of half stages (64 bytes of K); a K that ends in
    // half a stage needs rows that reach the whole stage (kld)
    int kld = 0;
};
template <typename TA, typename TR>
void launch_gemm(int epi, int M, int N, int K, const TA *A, const TA *Bt, const Epi &e, hipStream_t st);
// y1 = tanh(D V1 + c1) (the EPI_T1 epilogue) with D formed from e.dt_T as the
// operand is staged; Bt is V1tp, K = kDdim (FP32, FP64)
template <typename TA, typename TR>
void launch_gemm_dt(int M, int N, const TA *Bt, const Epi &e, hipStream_t st);
// E_i and dz3 for rows [0, rows); several types: w4 and b4 of the row's
// type group (Epi trow / vstride), E written to e_atom[ratom[row]] (pad rows
// skipped); one type: e_atom[row].
struct RowTypes {
    int ntr = 0;
    int trow[dp::kMaxTypes + 1] = {0, 0, 0, 0, 0};
    double b4[kMaxTypes] = {0, 0, 0, 0};
    const int *ratom = nullptr;
};
template <typename TA, typename TR>
void launch_energy(int rows, const TR *y2, const TR *t3, const TR *w4, const RowTypes &rt, double *e_atom,
                   TA *dz3, hipStream_t st);
// The fused tail of the fitting net (FP64 and FP32): the two 256-wide
// forward products, E_i, and the two 256-wide input-gradient products, per
// tile of 64 rows (rows: a multiple of 64).  Reads y1, writes E_i (at the
// row's atom) and dz1 = dE/d(first layer's pre-activation); t2s and dy2s
// ([rows][256]) are its scratch.
struct TailLaunch {
    int ntr = 0;                            // several types: rows grouped by type (trow), ratom row -> atom
    int trow[kMaxTypes + 1] = {0, 0, 0, 0, 0};
    const int *ratom = nullptr;
    int nlive = 0;                          // one type: rows below nlive are atoms
    double b4[kMaxTypes] = {0, 0, 0, 0};
    const void *tanh_tab = nullptr;         // tanh table of the precision, or NULL
    int width = kFitPad;                    // the net's width: the products run over K = width
};
template <typename T>
void launch_fit_tail(int rows, const T *y1, const FitWeights &fw, const T *fb, const TailLaunch &tl, double *e_atom,
                     T *dz1, T *t2s, T *dy2s, hipStream_t st);
template <typename TR>
void launch_dT(int n, const TR *dD, const TR *T, TR *dT, hipStream_t st);
// E = sum E_i and W = sum W_i in a fixed order; kFlagNonFinite when either
// is not finite.
void launch_reduce(int n, const double *e_atom, const double *w_atom, double *part, double *energy,
                   double *virial, int *flags, hipStream_t st);
template <typename T>
void launch_to_double(long n, const T *a, double *b, hipStream_t st);
// T stored by column (n atoms x kM columns of (T_0c, .., T_3c)) to FP64 [n][4][kM]
template <typename T>
void launch_tcol_to_double(int n, const T *a, double *b, hipStream_t st);
// GEMM operand matrix (n atoms, ncols logical columns) to FP64 (hi + lo for
// BF16); atom i's row is row[i] (NULL: i)
template <typename T>
void launch_op_to_double(int n, int ncols, const T *a, const int *row, double *b, hipStream_t st);
// The per-neighbor rungs of the ablation (padded: rows up to sel included).
void launch_emb_fwd_pn(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision, void *T,
                       void *D, void *rec, int *rcnt, bool padded, int *nnei, hipStream_t st);
void launch_emb_bwd_pn(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision, const void *T,
                       const void *dD, const void *rec, const int *rcnt, bool padded, double *force, double *w_atom,
                       hipStream_t st);
// rec/rcnt: the forward's compacted neighbor records (sel slots per atom) and
// their counts, written by launch_emb_fwd and read by launch_emb_bwd
void launch_emb_fwd(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision, void *T,
                    void *D, void *rec, int *rcnt, int *nnei, int *nseg, hipStream_t st);
void launch_emb_bwd(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision,
                    const void *T, const void *dD, const void *rec, const int *rcnt, double *force,
                    double *w_atom, hipStream_t st);

struct ComputeArgs {
    const dp_model *m;
    dp_nlist *nl;
    int natoms;
    const double *x;
    int precision;
    double *energy, *force, *virial, *atom_energy;   // force: never NULL when need_forces
    int *nnei_out;
    int *nseg_out = nullptr;
    double *T_out, *D_out;
    bool need_forces;
    int phase;   // 0: whole step; 1: forward only, activations kept; 2: backward from kept activations
    int mode = 0;                  // dp_mode
    int nseg = 0;                  // >0: E and W per segment (request) of a batch instead of totals
    const int *seg_off = nullptr;  // device [nseg + 1] atom offsets of the segments
    bool noalloc = false;          // scratch from the library's static device array, not the list's
};
// tabulated: the tabulated-but-unfused rung (G materialised from the table)
template <typename real, typename TD>
dp_status plain_forward(const dp_model *m, dp_nlist *nl, int n, const double *x, void *T, void *D, int *nnei,
                        hipStream_t st, bool tabulated);
template <typename real>
dp_status plain_backward(const dp_model *m, dp_nlist *nl, int n, const void *dT, double *force, double *w_atom,
                         hipStream_t st, bool tabulated);
dp_status ensure_ws(dp_nlist *nl, int precision, int sel);
// GEMM rows a list of alloc_atoms atoms of ntypes types may need
inline long fit_rows(long atoms, int ntypes) { return round_up(atoms, kRowPad) + (long)kRowPad * (ntypes - 1); }
// Copies the types into the list, checks them, counts them per type and
// assigns every atom its fitting-net row (synchronises once).
dp_status build_type_layout(dp_nlist *nl, const int *types, hipStream_t st);
// Reverse slots of the candidate lists of atoms [off, off + n) (after a build).
// uniq: no list holds two images of one atom (the slot match needs only the index)
void launch_reverse(dp_nlist *nl, int off, int n, hipStream_t st, bool uniq = false);
// F_i = (F_i as written by the backward: sum_j dE_i/dr_ij) - sum over the
// atoms j that list i of dE_j/dr_ji, read from the pair gradients at the
// reverse slot (rec / rcnt: the forward's neighbor records); deterministic
// (fixed order), no atomics.
void launch_force_gather(const dp_model *m, const dp_nlist *nl, int n, const double *x, int precision,
                         const void *rec, const int *rcnt, double *force, hipStream_t st);
size_t ws_bytes_for_atoms(int natoms, int precision, int sel, int ntypes);
// The static scratch of dp_compute_noalloc: its size in bytes (fixed at
// build time) and the calling thread's switch that keeps the kernel timers
// from creating events during such a call.
size_t noalloc_scratch_bytes();
void timers_quiet(bool on);
dp_status run_compressed(const ComputeArgs &a, hipStream_t st);
dp_status run_plain(const ComputeArgs &a, hipStream_t st);
// Per-type kick factors 0.5 dt / m (A/fs per eV/A) and kinetic-energy
// factors 0.5 m; type[i] of each atom (NULL: type 0).
struct TypeScalars {
    double v[kMaxTypes] = {0, 0, 0, 0};
};
void launch_verlet_kick_drift(double *x, double *v, const double *f, int n, const int *type, TypeScalars kick,
                              double dt, hipStream_t st);
void launch_verlet_kick(double *v, const double *f, int n, const int *type, TypeScalars kick, hipStream_t st);
void launch_thermo(const double *v, const double *energy, int n, const int *type, TypeScalars ke, double *row,
                   double *part, hipStream_t st);
double acc_unit();
double ke_unit();

}  // namespace dp
