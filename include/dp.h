/*
 * dp.h -- C-ABI of the MI355X (gfx950) compressed Deep Potential force step.
 *
 * The library computes, for one configuration of atoms, the Deep Potential
 * energy E = sum_i E_i, the forces F_i = -grad_i E and the virial, as the
 * paper defines them in Sec. 2.1 (Eqs. 1-5), with the embedding net replaced
 * by its fifth-order-polynomial tabulation (Sec. 3.2) and evaluated fused
 * with the R^T G contraction, padded neighbors skipped (Sec. 3.3, 3.4).
 *
 * Conventions for every entry point:
 *   - Arrays named *_d are DEVICE pointers owned by the caller (for example
 *     the storage of torch tensors on the current HIP device).  They are
 *     borrowed until the work enqueued on `stream` has completed.  Arrays
 *     named *_h are HOST pointers, read before the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; entry points do not synchronise unless their
 *     comment says so.
 *   - Coordinates are Angstrom, energies eV, forces eV/A; all results are
 *     FP64 whatever the precision mode.
 *   - Boxes are 9 doubles on the HOST, row vectors a, b, c; only
 *     orthorhombic boxes (off-diagonals zero) are accepted.  box_h == NULL
 *     means an open (non-periodic) cluster.
 *   - Return value: DP_OK or a negative dp_status.  On error nothing has been
 *     enqueued, and dp_last_error() describes the cause.
 *   - Handles (dp_model, dp_nlist) are owned by the library and released by
 *     their *_destroy call.  A model may serve several streams at once once
 *     its table is built; each configuration needs its own dp_nlist (the
 *     nlist also owns that configuration's scratch buffers).
 */
#ifndef DP_H
#define DP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DP_OK = 0,
    DP_ERR_ARG = -1,         /* a bad argument (NULL, size, shape)              */
    DP_ERR_HIP = -2,         /* a HIP runtime call failed                       */
    DP_ERR_OOM = -3,         /* device allocation failed                        */
    DP_ERR_CAPACITY = -4,    /* a neighbor-list or cell capacity was exceeded   */
    DP_ERR_UNSUPPORTED = -5, /* a valid request the library does not implement  */
    DP_ERR_STATE = -6,       /* call order violated (e.g. no table yet)         */
    DP_ERR_NONFINITE = -7,   /* a non-finite energy, virial or coordinate       */
    DP_ERR_SKIN = -8         /* an atom moved skin/2 or more since the list's build */
} dp_status;

typedef enum {
    DP_FP64 = 0,        /* everything in double precision                            */
    DP_FP32 = 1,        /* table, contraction, fitting net in FP32 (FP32 MFMA)       */
    DP_MIXED_BF16 = 2   /* as FP32, fitting-net GEMMs on BF16 MFMA, FP32 accumulate */
} dp_precision;

/* How the embedding stage is evaluated.  All modes compute the same model;
 * modes 1-4 are the rungs of the paper's step-by-step evaluation of its
 * optimizations (Sec. 3, and the ablation in its evaluation section). */
typedef enum {
    DP_COMPRESSED = 0,    /* tabulated, fused, per table-interval run of neighbors (default) */
    DP_PLAIN = 1,         /* embedding net evaluated layer by layer, padded to sel            */
    DP_TAB_UNFUSED = 2,   /* G and G' of every padded row from the table, materialised         */
    DP_FUSED_PADDED = 3,  /* tabulated and fused per neighbor, padded rows included (Sec. 3.4.1) */
    DP_FUSED = 4          /* as 3 without the padded rows (redundancy removal, Sec. 3.4.2)    */
} dp_mode;

/* Model hyper-parameters (Sec. 2.1 and the physical-systems section).
 *   ntypes      atom types (chemical species), 1..DP_MAX_TYPES: copper has
 *               one, water two (O, H).  With several types the embedding net
 *               is chosen by the neighbor's type and the fitting net by the
 *               center's type;
 *   rcut        cut-off R_c (A); rcut_smth: start of the gate w(r) (A);
 *   sel         N_m: neighbors kept per atom (the nearest sel within rcut), 1..512;
 *               with several types the sum of sel_t;
 *   sel_t       (ntypes > 1) neighbors kept per neighbor type: of each type t
 *               the nearest sel_t within rcut; each >= 1;
 *   emb         embedding widths d1, 2 d1, 4 d1 (M = emb[2]); emb[2] must be 128;
 *   m_lt        M<, columns of G kept in G< (Eq. 2); must be 16;
 *   fit         fitting-net hidden widths (each at most 256);
 *   desc_scale  factor multiplying R^T G (1/sel by default);
 *   switch_kind 0: gate 1-10u^3+15u^4-6u^5, 1: (cos(pi u)+1)/2, u=(r-rs)/(rc-rs). */
#define DP_MAX_TYPES 4
typedef struct {
    int ntypes;
    double rcut;
    double rcut_smth;
    int sel;
    int emb[3];
    int m_lt;
    int fit[3];
    double desc_scale;
    int switch_kind;
    int sel_t[DP_MAX_TYPES];
} dp_model_config;

typedef struct dp_model dp_model;
typedef struct dp_nlist dp_nlist;

/* Creates a model from the flat FP64 parameter vector params_h (HOST,
 * nparams doubles, copied).  Layout, row-major [fan_in][fan_out]: ntypes
 * embedding nets (for neighbors of type 0, 1, ...), then ntypes fitting nets
 * (for centers of type 0, 1, ...), each
 *   embedding  W0[1][d1] b0[d1] W1[d1][2d1] b1[2d1] W2[2d1][4d1] b2[4d1]
 *   fitting    V1[M< * M][f1] c1[f1] V2[f1][f2] c2[f2] V3[f2][f3] c3[f3]
 *              w4[f3] b4[1]
 * Embedding layers follow Eqs. 4-5 (tanh; the shortcut (x,x) is the
 * concatenation [x, x]); fitting layers are tanh with a shortcut where the
 * input and output widths match, and a linear output (Sec. 2.1).
 * Allocates device memory on the current device.  Errors: DP_ERR_ARG on a
 * bad config or count, DP_ERR_UNSUPPORTED for other widths or ntypes. */
dp_status dp_model_create(const dp_model_config *cfg, const double *params_h, size_t nparams,
                          dp_model **out);
dp_status dp_model_destroy(dp_model *model);

/* Builds the coefficient table of the embedding net (Sec. 3.2), one per
 * neighbor type on the same intervals: on each interval the M quintics whose value, first and second derivative match the
 * net at both nodes.  Intervals of width `stride` cover [0, s_max), then
 * intervals of width `tail_stride` cover [s_max, tail_max) (tail_max ==
 * s_max: no tail).  A polynomial is written in the offset t = s - x_lo from
 * its interval's left node; s past tail_max is clamped to tail_max and
 * counted (dp_nlist_stats).  Runs on `stream`, in FP64 on the device; the
 * FP32 copy is derived from it.  Must precede every compressed dp_compute. */
dp_status dp_tabulate(dp_model *model, double s_max, double stride, double tail_max,
                      double tail_stride, void *stream);

/* Selects the tanh of the fitting net, in every precision: 0 the native
 * tanh (default), 1 a second-order polynomial per interval of width 1/128 on
 * [0, 8) with the value and slope of tanh at the left node and its value at
 * the right node, odd extension, 1 beyond 8 (the tabulated tanh of Sec. 3.5;
 * its largest error, 2.3e-7, is the saturation at 8, and 2.4e-8 inside the
 * range).  The table is built on `stream` at the first call with
 * tabulated = 1, in FP64 (read by the FP64 mode) and rounded to FP32 (read by
 * the FP32 and mixed modes).  DP_ERR_ARG on other values. */
dp_status dp_fitting_tanh(dp_model *model, int tabulated, void *stream);

/* Copies the FP64 tanh table to the host: coef_h[4 k + q] (k < *n_int) is
 * the coefficient of t^q (q < 3; q = 3 is 0) on [k/128, (k+1)/128), with t
 * the offset from the interval's left node.  *n_int receives the interval
 * count (1024); coef_h may be NULL to query it.  DP_ERR_STATE when the table
 * has not been built.  Synchronises. */
dp_status dp_tanh_table_download(dp_model *model, double *coef_h, int *n_int);

/* Copies the FP64 tables to the host: coef_h[((type * n + theta) * M + eta)
 * * 6 + xi] is the coefficient of t^xi of column eta on interval theta of the
 * table of neighbor type `type` (ntypes tables of n intervals).  *n_int
 * receives n (coef_h may be NULL to query it).  Synchronises. */
dp_status dp_table_download(dp_model *model, double *coef_h, int *n_int);

/* Neighbor list with a skin (paper Sec. 2.1 L_Rc(i); the MD protocol keeps a
 * 2 A buffer): for every atom i all (j, periodic image) with
 * |x_j + n L - x_i| < rcut + skin, sorted by that distance, stored on the
 * device.  Images are handled for any box edge >= (rcut + skin) / 2, so cells
 * smaller than the cut-off sphere see several images of each atom (and of
 * the atom itself).  *inout: NULL creates a list, else it is rebuilt in place
 * (reallocated if natoms grew).  types_d (natoms int32, device) holds each
 * atom's type in [0, ntypes) (NULL: all 0); with several types every list is
 * grouped by neighbor type, nearest first within a type, and the list keeps
 * its own copy of the types (they are fixed for the life of the list).
 * The list also keeps the positions it was built at and, per atom and type,
 * how many candidates lay within rcut + skin/4: an evaluation whose atoms
 * have all moved at most skin/8 - 5e-4 A since then scans only those (the
 * others are provably beyond rcut); any other evaluation scans every
 * candidate.  Results do not depend on which scan runs.
 * Synchronises to check the capacity flags: a crowded cell or an atom with
 * more candidates than the list holds grows that capacity and builds again
 * (up to three times); DP_ERR_CAPACITY when an atom has more than 1024
 * candidates, DP_ERR_ARG for a type out of range or a non-finite
 * coordinate. */
dp_status dp_build_nlist(dp_model *model, int natoms, const double *coords_d, const int *types_d,
                         const double *box_h, double skin, dp_nlist **inout, void *stream);
dp_status dp_nlist_destroy(dp_nlist *nlist);

/* Energy, forces and virial of the configuration the list was built for, at
 * coordinates coords_d (natoms x 3), which may have moved by less than
 * skin / 2 since the build (more than that may lose pairs within rcut: the
 * evaluation sets a sticky flag that dp_nlist_check reports as DP_ERR_SKIN;
 * a non-finite energy, virial or coordinate is reported as
 * DP_ERR_NONFINITE).  The model's rcut must lie below the list's
 * rcut + skin (DP_ERR_ARG).  Neighbors beyond rcut are skipped; when more
 * than sel remain, the sel nearest are kept (counted in dp_nlist_stats).
 * Outputs (device, FP64; NULL skips):
 *   energy_d[1]        E = sum_i E_i
 *   force_d[natoms*3]  F_i = -dE/dx_i (overwritten)
 *   virial_d[9]        W = -sum_i sum_j r_ij (x) dE_i/dr_ij, r_ij = x_j - x_i
 *   atom_energy_d[natoms]  E_i
 * Passing force_d == NULL and virial_d == NULL runs the forward pass only.
 * mode DP_PLAIN evaluates the embedding net layer by layer over sel padded
 * rows (the untabulated baseline); every other mode needs dp_tabulate first.
 * The types are those the list was built with (types_d is not read).  With
 * several types, modes DP_PLAIN and DP_TAB_UNFUSED return DP_ERR_UNSUPPORTED. */
dp_status dp_compute(dp_model *model, dp_nlist *nlist, int natoms, const double *coords_d,
                     const int *types_d, const double *box_h, int mode, int precision,
                     double *energy_d, double *force_d, double *virial_d,
                     double *atom_energy_d, void *stream);

/* dp_compute for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, hosts that forbid allocation.  Same
 * arguments, same results (bit for bit) as dp_compute in the fused modes 0, 3
 * and 4; the plain modes 1 and 2 return DP_ERR_UNSUPPORTED.  The list must
 * have been built beforehand (dp_build_nlist allocates; this call does not).
 * Its scratch (embedding outputs, descriptor, fitting-net activations and
 * gradients, neighbor records) is not the list's but one static device
 * array of 96 MiB per GPU, held from the library's first use on that GPU
 * until the process ends; the call makes no hipMalloc, hipFree or other
 * allocating call (kernel timers stay off during it).  The scratch must
 * hold the evaluation: any natoms <= 512 of any supported model in any
 * precision fits, one-type models at sel = 192 up to 1,408 atoms; a larger
 * evaluation returns DP_ERR_CAPACITY before anything is enqueued.  Every
 * call on one GPU shares that GPU's array: two calls whose work overlaps
 * on the device (different streams, or different host threads) race and
 * give wrong results; calls in one stream are ordered and safe.  The
 * array needs no clearing: results depend only on what the call itself wrote. */
dp_status dp_compute_noalloc(dp_model *model, dp_nlist *nlist, int natoms, const double *coords_d,
                             const int *types_d, const double *box_h, int mode, int precision,
                             double *energy_d, double *force_d, double *virial_d,
                             double *atom_energy_d, void *stream);

/* The two halves of dp_compute, for an autograd function.  dp_energy_forward
 * computes E (and E_i) and keeps in the list's scratch what the adjoint
 * needs: T, the neighbor records, and the fitting net's activations (mixed
 * precision) or, in FP64 and FP32, where the 256-wide layers and their input
 * gradients run as one fused kernel with the forward, the gradient at the
 * first layer.  dp_energy_backward then runs only the rest of the adjoint:
 * the fitting-net input gradient, dE/dT, and the backward of the fused step,
 * which recomputes G and G' from the table (G is never stored).  The two
 * halves give E, F and W bit-identical to one dp_compute call.
 * It writes F = -dE/dx and/or W.  coords_d must be the forward's coordinates.
 * DP_ERR_STATE if no forward of the same mode and precision is kept (any other
 * compute on the list discards it). */
dp_status dp_energy_forward(dp_model *model, dp_nlist *nlist, int natoms, const double *coords_d,
                            int mode, int precision, double *energy_d, double *atom_energy_d,
                            void *stream);
dp_status dp_energy_backward(dp_model *model, dp_nlist *nlist, int natoms, const double *coords_d,
                             int mode, int precision, double *force_d, double *virial_d,
                             void *stream);

/* Intermediate results for testing: per atom the number of neighbors used
 * (nnei_d, int32: those within rcut, after the neighbor limits), the number
 * of runs of equal table interval in its neighbor list, grouped by type and
 * distance-sorted within a type (nseg_d, int32; compressed mode only, the
 * work unit of the kernels' interval-moment contraction; left untouched in
 * the other modes), T = desc_scale * R^T G (T_d, natoms x 4 x M, row k of the
 * 4 environment columns) and D = (T<)^T T (D_d, natoms x M< x M, in atom
 * order), all FP64 copies; any may be NULL. */
dp_status dp_descriptor(dp_model *model, dp_nlist *nlist, int natoms, const double *coords_d,
                        const double *box_h, int mode, int precision, int *nnei_d, int *nseg_d,
                        double *T_d, double *D_d, void *stream);

/* Sticky counters of the list since its last build (synchronises):
 * max_nei: most neighbors within rcut seen for one atom; n_sel_overflow:
 * atoms that had more than sel (several types: more than sel_t of some
 * type), counted once per evaluation; n_table_oob: look-ups past the table
 * end; n_cap_overflow: atoms whose candidate list was truncated at build. */
dp_status dp_nlist_stats(dp_nlist *nlist, int *max_nei, int *n_sel_overflow, int *n_table_oob,
                         int *n_cap_overflow);

/* The list's candidate arrays, for tests and inspection (paper Sec. 2.1,
 * L_Rc(i) with the skin).  *natoms_h and *cap_h (host, required) receive the
 * atom count N and the per-atom capacity C; call once with every array NULL
 * to size them.  Each device array that is not NULL receives a copy (enqueued
 * on `stream`, which is then synchronised):
 *   cnt_d[N]       candidates of atom i (all (j, n) within rcut + skin)
 *   nei_d[N * C]   row i, entries 0 .. cnt_i - 1: neighbor index j
 *   shift_d[N * C] its image shift n, r_ij = x_j - x_i + n L, as three int8
 *                  in bits 0-7 (x), 8-15 (y), 16-23 (z)
 *   dist_d[N * C]  |r_ij| at build in FP32 (the sort key: ascending within
 *                  a row, or within each type's run with several types)
 *   rev_d[N * C]   (int16) the position of (i, -n) in j's row, -1 if absent
 * Entries past cnt_i are undefined.  DP_ERR_ARG for a NULL list or count
 * pointer. */
dp_status dp_nlist_export(dp_nlist *nlist, int *natoms_h, int *cap_h, int *cnt_d, int *nei_d, int *shift_d,
                          float *dist_d, short *rev_d, void *stream);

/* Synchronises and returns what the evaluations on the list since its last
 * build have flagged: DP_ERR_NONFINITE (a non-finite energy, virial or
 * coordinate), DP_ERR_SKIN (an atom had moved skin/2 or more since the build,
 * so pairs within rcut may have been missed), else DP_ERR_CAPACITY or
 * DP_ERR_ARG for a failed build, else DP_OK.  The flags stay set until the
 * next dp_build_nlist. */
dp_status dp_nlist_check(dp_nlist *nlist);

/* Velocity-Verlet NVE (the MD protocol of the physical-systems section):
 * nsteps of half kick, drift, [neighbor rebuild every rebuild_every steps],
 * force, half kick, all on `stream` in FP64 (positions x_d and velocities
 * v_d, natoms x 3, updated in place; A and A/fs).  mass_h (HOST, ntypes
 * values) is the mass of each type in amu, dt_fs in fs; types_d as for
 * dp_build_nlist.  thermo_d (device, nsteps+1 rows of 2 doubles: potential
 * and kinetic energy, row 0 = start) may be NULL.  The nlist is built at
 * the start and rebuilt every rebuild_every steps; each build synchronises
 * once to check the capacities (grown and built again on an overflow, as in
 * dp_build_nlist) and what the evaluations since the previous build flagged.
 * The run stops at the first such check that fails, returning
 * DP_ERR_NONFINITE, DP_ERR_SKIN (an atom moved skin/2 or more between
 * builds) or DP_ERR_CAPACITY; x_d and v_d then hold the state of that step.
 * The same checks run at the end.  The list's counters (dp_nlist_stats)
 * accumulate over the run. */
dp_status dp_nve_run(dp_model *model, dp_nlist **nlist, int natoms, double *x_d, double *v_d,
                     const int *types_d, const double *box_h, const double *mass_h, double dt_fs,
                     int nsteps, int rebuild_every, double skin, int mode, int precision,
                     double *thermo_d, void *stream);

/* Continues the trajectory that the last dp_nve_run or dp_nve_continue on
 * `nlist` left (the same MD protocol): no build at the start and no first
 * evaluation; the forces and energy of the final positions, which the list
 * keeps, start the first half kick, and the rebuild cadence counts on from
 * the list's last build (rebuild_every as before).  So n steps of dp_nve_run
 * followed by m steps of dp_nve_continue give exactly the state of n + m
 * steps of dp_nve_run.  The positions array must be the one the previous run
 * updated (x_d, natoms, mode and precision as then; x_d and v_d not changed
 * in between); otherwise, or after a dp_build_nlist on the list or a failed
 * run, DP_ERR_STATE.  thermo_d: nsteps+1 rows, row 0 the state continued
 * from.  Checks, errors and counters as in dp_nve_run.  (An MD loop timed
 * this way excludes the set-up of the first build and evaluation, as a
 * steady-state step count does.) */
dp_status dp_nve_continue(dp_model *model, dp_nlist *nlist, int natoms, double *x_d, double *v_d,
                          const double *mass_h, double dt_fs, int nsteps, int rebuild_every, int mode,
                          int precision, double *thermo_d, void *stream);

/* ---------------------------------------------------------------- serving
 * A batch evaluates several independent configurations ("requests") in one
 * chain of launches: their atoms are concatenated (request r owns atoms
 * [offset, offset + natoms) of coords_d), each request's neighbor list is
 * built for its own box into one combined list, every per-atom kernel and
 * fitting-net GEMM runs once over all atoms of the batch, and E and W are
 * reduced per request in an order fixed relative to the request's first atom,
 * so a request's energy and virial do not depend on its batch-mates, nor do
 * its forces (gathered per atom in a fixed order).  The batch's neighbor
 * list and scratch are allocated once (for max_atoms) and stay resident.
 * Batches hold one-type models only (DP_ERR_UNSUPPORTED otherwise). */
typedef struct {
    int natoms;      /* atoms of this request                                */
    int offset;      /* first atom in the batch (requests are contiguous)    */
    int periodic;    /* 1: orthorhombic box below; 0: open cluster (<= 1024) */
    double box[9];   /* host, row vectors                                    */
} dp_request;
typedef struct dp_batch dp_batch;

dp_status dp_batch_create(dp_model *model, int max_atoms, int max_requests, double skin,
                          dp_batch **out);
dp_status dp_batch_destroy(dp_batch *batch);
/* energy_d[nreq], force_d[total*3], virial_d[nreq*9], atom_energy_d[total]
 * (device, FP64, NULL skips).  Enqueued on `stream`; one batch object must
 * not be used by two streams at once.  Returns DP_ERR_CAPACITY when the
 * requests exceed max_atoms or max_requests. */
dp_status dp_batch_compute(dp_model *model, dp_batch *batch, int nreq, const dp_request *reqs_h,
                           const double *coords_d, int precision, double *energy_d,
                           double *force_d, double *virial_d, double *atom_energy_d, void *stream);
/* Counters of the last batch (synchronises), as dp_nlist_stats. */
dp_status dp_batch_stats(dp_batch *batch, int *max_nei, int *n_sel_overflow, int *n_table_oob,
                         int *n_cap_overflow);
/* Device bytes one evaluation of natoms atoms needs (neighbor list and
 * scratch): the unit of the serving loop's HBM admission. */
dp_status dp_footprint_bytes(const dp_model *model, int natoms, size_t *bytes);

/* Kernel timing for measurement: while enabled, every kernel launch of the
 * library is bracketed by HIP events recorded on the stream it is launched
 * on.  dp_timers_read synchronises on those events, returns per kernel name
 * (names: max_names slots of 32 chars) the summed duration in ms and the
 * launch count, and clears the records. */
dp_status dp_timers_enable(int on);
dp_status dp_timers_read(int max_names, char *names, double *total_ms, int *counts, int *n_names);

/* Message of the last failed call on this thread ("" if none); valid until
 * the next call on the thread. */
const char *dp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DP_H */
