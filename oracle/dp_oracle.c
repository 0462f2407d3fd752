/*
 * dp_oracle.c -- plain FP64 CPU oracle for the Deep Potential force step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library never links, includes or calls it, and it shares no code with it.
 *
 * What it computes (paper: "Extending the limit of molecular dynamics with
 * ab initio accuracy to 10 billion atoms", PPoPP'22):
 *   - neighbor sets L_Rc(i) within the cut-off R_c               (Sec. 2.1)
 *   - the smooth environment matrix rows s(r)(1, x/r, y/r, z/r)   (Sec. 2.1, Eq. 1)
 *   - the embedding net G = L2 o L1 o L0 (s), tanh layers, the
 *     width-doubling shortcut (x,x)+tanh(xW+b)                    (Sec. 2.1, Eqs. 3-5)
 *   - the descriptor D = (G<)^T R R^T G                           (Sec. 2.1, Eq. 2)
 *   - the fitting net with shortcuts between equal-width layers,
 *     per-atom energy E_i and E = sum_i E_i                       (Sec. 2.1)
 *   - forces F_i = -grad_i E by hand-written reverse mode and
 *     the virial                                                  (Sec. 2.1, Sec. 3.4.3)
 *   - the tabulation of the embedding net by fifth-order
 *     polynomials matching value, first and second derivative at
 *     both interval nodes                                         (Sec. 3.2)
 *   - optionally, tanh of the fitting net by a second-order
 *     polynomial per interval on [0, 8], odd extension, 1 beyond 8 (Sec. 3.5)
 *
 * Readings where the paper is silent (stated once, used everywhere here):
 *   - gate w(r): 1 below r_s, the quintic smoothstep 1-10u^3+15u^4-6u^5 with
 *     u=(r-r_s)/(r_c-r_s) on [r_s, r_c), 0 from r_c on (switch_kind 0); or the
 *     cosine gate (cos(pi u)+1)/2 (switch_kind 1);
 *   - no normalisation of the environment matrix;
 *   - the contraction R^T G is multiplied by desc_scale (default 1/sel);
 *   - the embedding input is the raw s;
 *   - "(x,x)" is concatenation [x, x];
 *   - fitting shortcuts only where input and output widths match, linear
 *     output layer;
 *   - the tabulated polynomial is written in the local variable t = s - x_lo
 *     of its interval; interval index min(floor(s/h), n-1) (left-closed);
 *     beyond the last node s is clamped to the table end;
 *   - more than sel neighbors: keep the sel nearest by (r, j, image);
 *   - several atom types (the paper's water has two; its text does not
 *     spell out how types enter): the embedding net is chosen by the
 *     NEIGHBOR's type, the fitting net by the CENTER's type, and of each
 *     neighbor type t only the sel_t nearest are kept; the sum over j in
 *     R^T G runs over all kept neighbors of all types, scaled by
 *     desc_scale (default 1 / sum_t sel_t);
 *   - virial W = - sum_i sum_j r_ij (x) dE_i/dr_ij;
 *   - tabulated tanh (tanh_table = 1): intervals of width 1/128 on [0, 8);
 *     on [x0, x0 + h] the quadratic with the value and slope of tanh at x0
 *     and its value at x0 + h; its derivative in the backward is taken as
 *     1 - y^2 of the tabulated y, as for tanh itself.
 *
 * Boxes are orthorhombic (diagonal 3x3, row vectors) or NULL for an open
 * cluster.  Everything is double precision.  Threads: OpenMP over atoms.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_TYPES 4

typedef struct {
    double rcut, rcut_smth;
    int sel;
    int d1, d2, d3;      /* embedding widths; d2 = 2 d1, d3 = 2 d2 = M   */
    int m_lt;            /* M< : columns of G kept in G<                  */
    int f1, f2, f3;      /* fitting-net hidden widths                     */
    double desc_scale;   /* factor on R^T G                               */
    int switch_kind;     /* 0 quintic smoothstep, 1 cosine                */
    int tanh_table;      /* 1: tabulated tanh in the fitting net          */
    int ntypes;          /* atom types (chemical species); <= 1 means one */
    int sel_t[ORC_MAX_TYPES];  /* neighbors kept per neighbor type (ntypes > 1) */
} orc_config;

static int n_types(const orc_config *c) { return c->ntypes > 1 ? c->ntypes : 1; }

/* A tabulated embedding net: n_int intervals, each with M quintics in the
 * local variable t = s - lo[theta].  coef[(theta*M + eta)*6 + xi]. */
typedef struct {
    int n_fine, n_tail;
    double h, s_max, h_tail, tail_max;
    int M;
    const double *coef;
} orc_table;

/* ------------------------------------------------------- tabulated tanh */

/* tanh of the fitting net by a second-order polynomial per interval of
 * width 1/128 on [0, 8): value and slope of tanh at the left node, value at
 * the right node; odd extension; 1 from 8 on (Sec. 3.5 states the order,
 * the range, the symmetry and the saturation). */
double orc_tanh_table(double x)
{
    const double h = 1.0 / 128.0;
    double ax = fabs(x);
    if (ax >= 8.0) return x < 0 ? -1.0 : 1.0;
    int k = (int)floor(ax / h);
    double x0 = k * h, t = ax - x0;
    double a0 = tanh(x0), a1 = 1.0 - a0 * a0;
    double a2 = (tanh(x0 + h) - a0 - a1 * h) / (h * h);
    double y = a0 + t * (a1 + t * a2);
    return x < 0 ? -y : y;
}

static double act(const orc_config *c, double z) { return c->tanh_table ? orc_tanh_table(z) : tanh(z); }

/* ---------------------------------------------------------------- params */

typedef struct {
    const double *W0, *b0, *W1, *b1, *W2, *b2;          /* embedding */
} orc_emb_params;
typedef struct {
    const double *V1, *c1, *V2, *c2, *V3, *c3, *w4, *b4; /* fitting   */
} orc_fit_params;

static long emb_count(const orc_config *c)
{
    return (long)1 * c->d1 + c->d1 + (long)c->d1 * c->d2 + c->d2 + (long)c->d2 * c->d3 + c->d3;
}

static long fit_count(const orc_config *c)
{
    long dD = (long)c->m_lt * c->d3;
    return dD * c->f1 + c->f1 + (long)c->f1 * c->f2 + c->f2 + (long)c->f2 * c->f3 + c->f3 + c->f3 + 1;
}

/* The parameter vector holds one embedding net per neighbor type, then one
 * fitting net per center type (types in increasing order). */
long orc_param_count(const orc_config *c)
{
    return n_types(c) * (emb_count(c) + fit_count(c));
}

/* Embedding net applied to neighbors of type t. */
static orc_emb_params emb_params(const orc_config *c, const double *p, int t)
{
    orc_emb_params q;
    p += t * emb_count(c);
    q.W0 = p; p += c->d1;
    q.b0 = p; p += c->d1;
    q.W1 = p; p += (long)c->d1 * c->d2;
    q.b1 = p; p += c->d2;
    q.W2 = p; p += (long)c->d2 * c->d3;
    q.b2 = p;
    return q;
}

/* Fitting net of centers of type t. */
static orc_fit_params fit_params(const orc_config *c, const double *p, int t)
{
    orc_fit_params q;
    p += n_types(c) * emb_count(c) + t * fit_count(c);
    q.V1 = p; p += (long)c->m_lt * c->d3 * c->f1;
    q.c1 = p; p += c->f1;
    q.V2 = p; p += (long)c->f1 * c->f2;
    q.c2 = p; p += c->f2;
    q.V3 = p; p += (long)c->f2 * c->f3;
    q.c3 = p; p += c->f3;
    q.w4 = p; p += c->f3;
    q.b4 = p;
    return q;
}

/* ---------------------------------------------------------- gate, Eq. 1 */

void orc_switch(const orc_config *c, double r, double *w, double *dw)
{
    double rs = c->rcut_smth, rc = c->rcut;
    if (r < rs) { *w = 1.0; *dw = 0.0; return; }
    if (r >= rc) { *w = 0.0; *dw = 0.0; return; }
    double L = rc - rs;
    double u = (r - rs) / L;
    if (c->switch_kind == 1) {
        *w = 0.5 * cos(M_PI * u) + 0.5;
        *dw = -0.5 * M_PI * sin(M_PI * u) / L;
    } else {
        *w = 1.0 - 10.0 * u * u * u + 15.0 * u * u * u * u - 6.0 * u * u * u * u * u;
        *dw = (-30.0 * u * u + 60.0 * u * u * u - 30.0 * u * u * u * u) / L;
    }
}

/* ------------------------------------------- embedding net, Eqs. 3-5 */

/* G(s) of the embedding net of neighbor type `type` and its first two
 * derivatives by forward-mode differentiation.  Any of G, dG, ddG may be NULL.  Layer 0: tanh(s W0 + b0); layers 1, 2:
 * [x, x] + tanh(x W + b). */
void orc_embed(const orc_config *c, const double *params, int type, double s,
               double *G, double *dG, double *ddG)
{
    orc_emb_params q = emb_params(c, params, type);
    int d1 = c->d1, d2 = c->d2, d3 = c->d3;
    double *h = malloc(sizeof(double) * 3 * d3);
    double *hn = malloc(sizeof(double) * 3 * d3);
    double *h1 = h + d3, *h2 = h + 2 * d3;        /* first, second derivative */
    double *hn1 = hn + d3, *hn2 = hn + 2 * d3;

    for (int a = 0; a < d1; a++) {
        double z = s * q.W0[a] + q.b0[a];
        double t = tanh(z);
        double dt = 1.0 - t * t;
        h[a] = t;
        h1[a] = dt * q.W0[a];
        h2[a] = -2.0 * t * dt * q.W0[a] * q.W0[a];
    }
    int win = d1;
    const double *Ws[2] = {q.W1, q.W2}, *bs[2] = {q.b1, q.b2};
    int wout_arr[2] = {d2, d3};
    for (int l = 0; l < 2; l++) {
        int wout = wout_arr[l];
        const double *W = Ws[l], *b = bs[l];
        for (int o = 0; o < wout; o++) {
            double z = b[o], z1 = 0.0, z2 = 0.0;
            for (int a = 0; a < win; a++) {
                z += h[a] * W[(long)a * wout + o];
                z1 += h1[a] * W[(long)a * wout + o];
                z2 += h2[a] * W[(long)a * wout + o];
            }
            double t = tanh(z);
            double dt = 1.0 - t * t;
            double t1 = dt * z1;
            double t2 = -2.0 * t * dt * z1 * z1 + dt * z2;
            /* shortcut [x, x]: output o takes input o mod win */
            int src = o % win;
            hn[o] = h[src] + t;
            hn1[o] = h1[src] + t1;
            hn2[o] = h2[src] + t2;
        }
        memcpy(h, hn, sizeof(double) * wout);
        memcpy(h1, hn1, sizeof(double) * wout);
        memcpy(h2, hn2, sizeof(double) * wout);
        win = wout;
    }
    for (int o = 0; o < d3; o++) {
        if (G) G[o] = h[o];
        if (dG) dG[o] = h1[o];
        if (ddG) ddG[o] = h2[o];
    }
    free(h);
    free(hn);
}

/* -------------------------------------------------- tabulation, Sec. 3.2 */

/* Coefficients a[0..5] of the quintic p(t), t in [0, h], whose value, first
 * and second derivative equal (y0, d0, dd0) at t = 0 and (y1, d1, dd1) at
 * t = h.  The lower three follow from t = 0; the upper three solve the 3x3
 * system left at t = h, written in the residuals of the quadratic part. */
void orc_hermite(double y0, double d0, double dd0, double y1, double d1, double dd1,
                 double h, double *a)
{
    a[0] = y0;
    a[1] = d0;
    a[2] = 0.5 * dd0;
    double r0 = y1 - (a[0] + a[1] * h + a[2] * h * h);
    double r1 = d1 - (a[1] + 2.0 * a[2] * h);
    double r2 = dd1 - 2.0 * a[2];
    double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
    a[3] = (20.0 * r0 - 8.0 * h * r1 + h2 * r2) / (2.0 * h3);
    a[4] = (-30.0 * r0 + 14.0 * h * r1 - 2.0 * h2 * r2) / (2.0 * h4);
    a[5] = (12.0 * r0 - 6.0 * h * r1 + h2 * r2) / (2.0 * h5);
}

int orc_table_intervals(double s_max, double h, double tail_max, double h_tail)
{
    int n_fine = (int)llround(s_max / h);
    int n_tail = (tail_max > s_max) ? (int)llround((tail_max - s_max) / h_tail) : 0;
    return n_fine + n_tail;
}

/* Left node of interval theta. */
static double table_node(const orc_table *t, int theta)
{
    if (theta < t->n_fine) return theta * t->h;
    return t->s_max + (theta - t->n_fine) * t->h_tail;
}

/* Table of the embedding net of neighbor type `type`: fills
 * coef[(theta*M + eta)*6 + xi]; returns the interval count. */
int orc_tabulate(const orc_config *c, const double *params, int type, double s_max, double h,
                 double tail_max, double h_tail, double *coef)
{
    orc_table t;
    t.n_fine = (int)llround(s_max / h);
    t.n_tail = (tail_max > s_max) ? (int)llround((tail_max - s_max) / h_tail) : 0;
    t.h = h; t.s_max = s_max; t.h_tail = h_tail; t.tail_max = tail_max; t.M = c->d3;
    int n = t.n_fine + t.n_tail, M = c->d3;
    #pragma omp parallel for schedule(dynamic)
    for (int th = 0; th < n; th++) {
        double lo = table_node(&t, th), hi, w;
        if (th < t.n_fine) {
            hi = (th + 1) * h;
            w = h;
        } else {
            hi = s_max + (th + 1 - t.n_fine) * h_tail;
            w = h_tail;
        }
        double *g0 = malloc(sizeof(double) * 6 * M);
        double *g1 = g0 + M, *g2 = g0 + 2 * M, *G0 = g0 + 3 * M, *G1 = g0 + 4 * M, *G2 = g0 + 5 * M;
        orc_embed(c, params, type, lo, g0, g1, g2);
        orc_embed(c, params, type, hi, G0, G1, G2);
        for (int e = 0; e < M; e++)
            orc_hermite(g0[e], g1[e], g2[e], G0[e], G1[e], G2[e], w,
                        coef + ((long)th * M + e) * 6);
        free(g0);
    }
    return n;
}

/* Interval and local offset of s; *oob set when s is past the table end. */
static void table_locate(const orc_table *t, double s, int *theta, double *loc, int *oob)
{
    *oob = 0;
    if (s < t->s_max) {
        int k = (int)floor(s / t->h);
        if (k > t->n_fine - 1) k = t->n_fine - 1;
        if (k < 0) k = 0;
        *theta = k;
        *loc = s - k * t->h;
        return;
    }
    if (t->n_tail > 0 && s < t->tail_max) {
        int k = (int)floor((s - t->s_max) / t->h_tail);
        if (k > t->n_tail - 1) k = t->n_tail - 1;
        *theta = t->n_fine + k;
        *loc = s - (t->s_max + k * t->h_tail);
        return;
    }
    /* past the end: clamp to the last node */
    *oob = 1;
    if (t->n_tail > 0) {
        *theta = t->n_fine + t->n_tail - 1;
        *loc = t->h_tail;
    } else {
        *theta = t->n_fine - 1;
        *loc = t->h;
    }
}

/* G and dG/ds from the table: p(t) and p'(t) of each column. */
static void table_eval(const orc_table *t, double s, double *G, double *dG, int *oob)
{
    int th;
    double x;
    table_locate(t, s, &th, &x, oob);
    for (int e = 0; e < t->M; e++) {
        const double *a = t->coef + ((long)th * t->M + e) * 6;
        double v = 0.0, d = 0.0, xp = 1.0;
        for (int k = 0; k < 6; k++) {        /* sum of a_k t^k, written out */
            v += a[k] * xp;
            xp *= x;
        }
        xp = 1.0;
        for (int k = 1; k < 6; k++) {
            d += k * a[k] * xp;
            xp *= x;
        }
        G[e] = v;
        dG[e] = *oob ? 0.0 : d;
    }
}

void orc_table_eval(const orc_config *c, int n_fine, int n_tail, double h, double s_max,
                    double h_tail, double tail_max, const double *coef, double s,
                    double *G, double *dG)
{
    orc_table t = {n_fine, n_tail, h, s_max, h_tail, tail_max, c->d3, coef};
    int oob;
    table_eval(&t, s, G, dG, &oob);
}

/* --------------------------------------------------------- neighbors */

typedef struct { double r; int j; int n[3]; double d[3]; } orc_nbr;

static int nbr_less(const orc_nbr *a, const orc_nbr *b)
{
    if (a->r != b->r) return a->r < b->r;
    if (a->j != b->j) return a->j < b->j;
    for (int k = 0; k < 3; k++)
        if (a->n[k] != b->n[k]) return a->n[k] < b->n[k];
    return 0;
}

static int nbr_cmp(const void *x, const void *y)
{
    const orc_nbr *a = x, *b = y;
    if (nbr_less(a, b)) return -1;
    if (nbr_less(b, a)) return 1;
    return 0;
}

/* Every (j, image n) with r_ij = x_j + n L - x_i, 0 < |r_ij| < rc, by brute
 * force over all atoms and images.  An image shift is only tried in a
 * direction where its component alone is already within rc.  Result sorted
 * by (r, j, n).  Returns the number found (all of them, even past cap). */
static int find_neighbors(const orc_config *c, int natoms, const double *x, const double *box,
                          int i, orc_nbr *out, int cap)
{
    double rc = c->rcut;
    int K[3] = {0, 0, 0};
    double L[3] = {0, 0, 0};
    if (box) {
        for (int a = 0; a < 3; a++) {
            L[a] = box[a * 3 + a];
            K[a] = (int)ceil(rc / L[a]) + 1;
        }
    }
    int cnt = 0;
    for (int j = 0; j < natoms; j++) {
        double d0[3];
        for (int a = 0; a < 3; a++) d0[a] = x[3 * j + a] - x[3 * i + a];
        for (int n0 = -K[0]; n0 <= K[0]; n0++) {
            double dx = d0[0] + n0 * L[0];
            if (fabs(dx) >= rc) continue;
            for (int n1 = -K[1]; n1 <= K[1]; n1++) {
                double dy = d0[1] + n1 * L[1];
                if (fabs(dy) >= rc) continue;
                for (int n2 = -K[2]; n2 <= K[2]; n2++) {
                    double dz = d0[2] + n2 * L[2];
                    if (fabs(dz) >= rc) continue;
                    if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
                    double r = sqrt(dx * dx + dy * dy + dz * dz);
                    if (r >= rc) continue;
                    if (cnt < cap) {
                        orc_nbr *o = out + cnt;
                        o->r = r; o->j = j;
                        o->n[0] = n0; o->n[1] = n1; o->n[2] = n2;
                        o->d[0] = dx; o->d[1] = dy; o->d[2] = dz;
                    }
                    cnt++;
                }
            }
        }
    }
    int m = cnt < cap ? cnt : cap;
    qsort(out, m, sizeof(orc_nbr), nbr_cmp);
    return cnt;
}

/* Neighbor set of atom i for tests: up to cap entries (j, image, r). */
int orc_neighbors(const orc_config *c, int natoms, const double *x, const double *box, int i,
                  int cap, int *j_out, int *img_out, double *r_out)
{
    orc_nbr *buf = malloc(sizeof(orc_nbr) * (size_t)cap);
    int cnt = find_neighbors(c, natoms, x, box, i, buf, cap);
    int m = cnt < cap ? cnt : cap;
    for (int k = 0; k < m; k++) {
        j_out[k] = buf[k].j;
        for (int a = 0; a < 3; a++) img_out[3 * k + a] = buf[k].n[a];
        r_out[k] = buf[k].r;
    }
    free(buf);
    return cnt;
}

/* ------------------------------------------------- one atom, Eqs. 1-5 */

/* Energy E_i of one atom of type ctype from its neighbor displacements
 * d[nn][3] and the neighbors' types ntype[nn], and g[nn][3] = dE_i / d r_ij.
 * T (4 x M) and D (M< x M) are written when not NULL.  tabs == NULL: the
 * embedding nets are evaluated directly; else by tabs[type] (one table per
 * neighbor type).  Returns the number of table look-ups past the table end. */
static int atom_eval(const orc_config *c, const double *params, const orc_table *tabs,
                     int nn, const double (*d)[3], const int *ntype, int ctype,
                     double *E, double (*g)[3], double *T_out, double *D_out)
{
    orc_fit_params fq = fit_params(c, params, ctype);
    const orc_fit_params *q = &fq;
    int M = c->d3, Ml = c->m_lt, f1 = c->f1, f2 = c->f2, f3 = c->f3;
    double sig = c->desc_scale;
    int nD = Ml * M;
    int oob_total = 0;

    double *s = malloc(sizeof(double) * nn);
    double *dsdr = malloc(sizeof(double) * nn);
    double *rr = malloc(sizeof(double) * nn);
    double *u = malloc(sizeof(double) * nn * 4);
    double *R = malloc(sizeof(double) * nn * 4);
    double *G = malloc(sizeof(double) * (size_t)nn * M);
    double *dG = malloc(sizeof(double) * (size_t)nn * M);
    double *T = calloc(4 * M, sizeof(double));
    double *D = calloc(nD, sizeof(double));

    /* Eq. 1: rows s(r) (1, x/r, y/r, z/r) */
    for (int j = 0; j < nn; j++) {
        double r = sqrt(d[j][0] * d[j][0] + d[j][1] * d[j][1] + d[j][2] * d[j][2]);
        double w, dw;
        orc_switch(c, r, &w, &dw);
        rr[j] = r;
        s[j] = w / r;
        dsdr[j] = dw / r - w / (r * r);
        u[4 * j + 0] = 1.0;
        for (int a = 0; a < 3; a++) u[4 * j + 1 + a] = d[j][a] / r;
        for (int k = 0; k < 4; k++) R[4 * j + k] = s[j] * u[4 * j + k];
        /* Eqs. 3-5 (or the table of Sec. 3.2) */
        if (tabs) {
            int oob;
            table_eval(&tabs[ntype[j]], s[j], G + (size_t)j * M, dG + (size_t)j * M, &oob);
            oob_total += oob;
        } else {
            orc_embed(c, params, ntype[j], s[j], G + (size_t)j * M, dG + (size_t)j * M, NULL);
        }
    }
    /* T = sig * R^T G  (4 x M) */
    for (int k = 0; k < 4; k++)
        for (int e = 0; e < M; e++) {
            double acc = 0.0;
            for (int j = 0; j < nn; j++) acc += R[4 * j + k] * G[(size_t)j * M + e];
            T[k * M + e] = sig * acc;
        }
    /* Eq. 2: D = (T<)^T T, D[a][b] = sum_k T[k][a] T[k][b], a < M< */
    for (int a = 0; a < Ml; a++)
        for (int b = 0; b < M; b++) {
            double acc = 0.0;
            for (int k = 0; k < 4; k++) acc += T[k * M + a] * T[k * M + b];
            D[a * M + b] = acc;
        }

    /* fitting net */
    double *z1 = malloc(sizeof(double) * f1), *y1 = malloc(sizeof(double) * f1);
    double *z2 = malloc(sizeof(double) * f2), *y2 = malloc(sizeof(double) * f2);
    double *z3 = malloc(sizeof(double) * f3), *y3 = malloc(sizeof(double) * f3);
    for (int o = 0; o < f1; o++) {
        double acc = q->c1[o];
        for (int a = 0; a < nD; a++) acc += D[a] * q->V1[(long)a * f1 + o];
        z1[o] = acc;
        y1[o] = act(c, acc) + (nD == f1 ? D[o] : 0.0);
    }
    for (int o = 0; o < f2; o++) {
        double acc = q->c2[o];
        for (int a = 0; a < f1; a++) acc += y1[a] * q->V2[(long)a * f2 + o];
        z2[o] = acc;
        y2[o] = act(c, acc) + (f1 == f2 ? y1[o] : 0.0);
    }
    for (int o = 0; o < f3; o++) {
        double acc = q->c3[o];
        for (int a = 0; a < f2; a++) acc += y2[a] * q->V3[(long)a * f3 + o];
        z3[o] = acc;
        y3[o] = act(c, acc) + (f2 == f3 ? y2[o] : 0.0);
    }
    double Ei = q->b4[0];
    for (int a = 0; a < f3; a++) Ei += y3[a] * q->w4[a];
    *E = Ei;

    if (g) {
        /* reverse mode through the fitting net */
        double *dy3 = malloc(sizeof(double) * f3), *dy2 = malloc(sizeof(double) * f2);
        double *dy1 = malloc(sizeof(double) * f1), *dD = malloc(sizeof(double) * nD);
        double *dz = malloc(sizeof(double) * (f1 > f2 ? (f1 > f3 ? f1 : f3) : (f2 > f3 ? f2 : f3)));
        for (int a = 0; a < f3; a++) dy3[a] = q->w4[a];
        for (int o = 0; o < f3; o++) { double t = act(c, z3[o]); dz[o] = dy3[o] * (1.0 - t * t); }
        for (int a = 0; a < f2; a++) {
            double acc = (f2 == f3) ? dy3[a] : 0.0;
            for (int o = 0; o < f3; o++) acc += q->V3[(long)a * f3 + o] * dz[o];
            dy2[a] = acc;
        }
        for (int o = 0; o < f2; o++) { double t = act(c, z2[o]); dz[o] = dy2[o] * (1.0 - t * t); }
        for (int a = 0; a < f1; a++) {
            double acc = (f1 == f2) ? dy2[a] : 0.0;
            for (int o = 0; o < f2; o++) acc += q->V2[(long)a * f2 + o] * dz[o];
            dy1[a] = acc;
        }
        for (int o = 0; o < f1; o++) { double t = act(c, z1[o]); dz[o] = dy1[o] * (1.0 - t * t); }
        for (int a = 0; a < nD; a++) {
            double acc = (nD == f1) ? dy1[a] : 0.0;
            for (int o = 0; o < f1; o++) acc += q->V1[(long)a * f1 + o] * dz[o];
            dD[a] = acc;
        }
        /* D[a][b] = sum_k T[k][a] T[k][b]: dT[k][c] gets dD[c][b] T[k][b]
         * (c < M<) and dD[a][c] T[k][a] */
        double *dT = calloc(4 * M, sizeof(double));
        for (int k = 0; k < 4; k++)
            for (int a = 0; a < Ml; a++)
                for (int b = 0; b < M; b++) {
                    double v = dD[a * M + b];
                    dT[k * M + a] += v * T[k * M + b];
                    dT[k * M + b] += v * T[k * M + a];
                }
        /* T = sig R^T G: per neighbor dR[k] and dG[e] */
        for (int j = 0; j < nn; j++) {
            double dR[4], dsG = 0.0;
            for (int k = 0; k < 4; k++) {
                double acc = 0.0;
                for (int e = 0; e < M; e++) acc += dT[k * M + e] * G[(size_t)j * M + e];
                dR[k] = sig * acc;
            }
            for (int e = 0; e < M; e++) {
                double dGe = 0.0;
                for (int k = 0; k < 4; k++) dGe += dT[k * M + e] * R[4 * j + k];
                dsG += sig * dGe * dG[(size_t)j * M + e];
            }
            /* R[k] = s u[k]:  dE/ds = dsG + sum_k dR[k] u[k];  dE/du[k] = s dR[k] */
            double dEds = dsG;
            for (int k = 0; k < 4; k++) dEds += dR[k] * u[4 * j + k];
            double r = rr[j], rhat[3], du[3], dudotr = 0.0;
            for (int a = 0; a < 3; a++) {
                rhat[a] = d[j][a] / r;
                du[a] = s[j] * dR[1 + a];
                dudotr += du[a] * rhat[a];
            }
            /* d(x_a/r)/d x_b = (delta_ab - rhat_a rhat_b)/r */
            for (int b = 0; b < 3; b++)
                g[j][b] = dEds * dsdr[j] * rhat[b] + (du[b] - dudotr * rhat[b]) / r;
        }
        free(dT); free(dy3); free(dy2); free(dy1); free(dD); free(dz);
    }
    if (T_out) memcpy(T_out, T, sizeof(double) * 4 * M);
    if (D_out) memcpy(D_out, D, sizeof(double) * nD);
    free(z1); free(y1); free(z2); free(y2); free(z3); free(y3);
    free(s); free(dsdr); free(rr); free(u); free(R); free(G); free(dG); free(T); free(D);
    return oob_total;
}

/* ------------------------------------------------ whole configurations */

/* Keeps, of the sorted neighbor list nb[0..n), the nearest sel of each
 * neighbor type (one type: the nearest sel), in place and in order; fills
 * their types and returns how many were kept. */
static int select_neighbors(const orc_config *c, const int *types, orc_nbr *nb, int n, int *ntype)
{
    int T = n_types(c), taken[ORC_MAX_TYPES] = {0}, nn = 0;
    for (int k = 0; k < n; k++) {
        int t = types ? types[nb[k].j] : 0;
        int lim = T > 1 ? c->sel_t[t] : c->sel;
        if (taken[t] >= lim) continue;
        taken[t]++;
        nb[nn] = nb[k];
        ntype[nn] = t;
        nn++;
    }
    return nn;
}

/* Evaluates the atoms listed in `centers` (all atoms when centers == NULL,
 * ncent ignored).  types[natoms] gives each atom's type (NULL: all type 0).
 * Outputs (NULL to skip):
 *   e_atom[ncent]        E_i of each center
 *   force[natoms*3]      contributions -grad E_i of the centers only
 *                        (the full force when every atom is a center)
 *   virial[9]            - sum over centers of sum_j r_ij (x) dE_i/dr_ij
 *   nnei[ncent]          neighbor count within rc (before truncation to sel)
 *   T_out[ncent*4*M], D_out[ncent*M<*M]
 * tab_* describe the tables (tab_coef == NULL: untabulated); tab_coef holds
 * one table per neighbor type, back to back.
 * Returns the total number of neighbors dropped by the sel truncation, or -1
 * on an allocation failure. */
long orc_evaluate(const orc_config *c, const double *params, int natoms, const double *x,
                  const double *box, const int *types, int ncent, const int *centers,
                  int tab_n_fine, int tab_n_tail, double tab_h, double tab_s_max,
                  double tab_h_tail, double tab_tail_max, const double *tab_coef,
                  double *e_atom, double *force, double *virial, int *nnei,
                  double *T_out, double *D_out, long *table_oob)
{
    int T = n_types(c), M = c->d3;
    orc_table tabs[ORC_MAX_TYPES];
    long per_type = (long)(tab_n_fine + tab_n_tail) * M * 6;
    for (int t = 0; t < T; t++) {
        orc_table tb = {tab_n_fine, tab_n_tail, tab_h, tab_s_max, tab_h_tail, tab_tail_max,
                        M, tab_coef ? tab_coef + t * per_type : NULL};
        tabs[t] = tb;
    }
    const orc_table *tp = tab_coef ? tabs : NULL;
    int nc = centers ? ncent : natoms;
    int sel = 0;
    if (T > 1)
        for (int t = 0; t < T; t++) sel += c->sel_t[t];
    else
        sel = c->sel;
    int cap = 4096;  /* neighbors scanned per atom; far above any sel here */
    long dropped = 0, oob = 0;
    if (force) memset(force, 0, sizeof(double) * 3 * (size_t)natoms);
    double W[9] = {0};

    const int CHUNK = 2048;
    int *cnt = malloc(sizeof(int) * CHUNK);
    orc_nbr *nb = malloc(sizeof(orc_nbr) * (size_t)CHUNK * cap);
    double (*g)[3] = malloc(sizeof(double) * 3 * (size_t)CHUNK * sel);
    double *Wc = malloc(sizeof(double) * 9 * (size_t)CHUNK);
    int fail = (!cnt || !nb || !g || !Wc);
    for (int c0 = 0; c0 < nc && !fail; c0 += CHUNK) {
        int m = nc - c0 < CHUNK ? nc - c0 : CHUNK;
        long drop_c = 0, oob_c = 0;
        #pragma omp parallel for schedule(dynamic, 4) reduction(+:drop_c, oob_c)
        for (int k = 0; k < m; k++) {
            int i = centers ? centers[c0 + k] : c0 + k;
            orc_nbr *mine = nb + (size_t)k * cap;
            int n = find_neighbors(c, natoms, x, box, i, mine, cap);
            if (n > cap) n = cap;   /* cap far exceeds any neighbor count here */
            if (nnei) nnei[c0 + k] = n;
            int *ntype = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
            int nn = select_neighbors(c, types, mine, n, ntype);
            drop_c += n - nn;
            cnt[k] = nn;
            double (*d)[3] = malloc(sizeof(double) * 3 * (size_t)(nn > 0 ? nn : 1));
            for (int j = 0; j < nn; j++)
                for (int a = 0; a < 3; a++) d[j][a] = mine[j].d[a];
            double Ei;
            oob_c += atom_eval(c, params, tp, nn, (const double (*)[3])d, ntype,
                               types ? types[i] : 0, &Ei,
                               (force || virial) ? g + (size_t)k * sel : NULL,
                               T_out ? T_out + (size_t)(c0 + k) * 4 * M : NULL,
                               D_out ? D_out + (size_t)(c0 + k) * c->m_lt * M : NULL);
            if (e_atom) e_atom[c0 + k] = Ei;
            double *w = Wc + 9 * (size_t)k;
            for (int t = 0; t < 9; t++) w[t] = 0.0;
            if (force || virial)
                for (int j = 0; j < nn; j++)
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            w[3 * a + b] -= d[j][a] * g[(size_t)k * sel + j][b];
            free(d);
            free(ntype);
        }
        dropped += drop_c;
        oob += oob_c;
        /* scatter serially: F_i += g_ij, F_j -= g_ij */
        for (int k = 0; k < m; k++) {
            int i = centers ? centers[c0 + k] : c0 + k;
            if (force)
                for (int j = 0; j < cnt[k]; j++) {
                    int jj = nb[(size_t)k * cap + j].j;
                    for (int a = 0; a < 3; a++) {
                        double v = g[(size_t)k * sel + j][a];
                        force[3 * i + a] += v;
                        force[3 * jj + a] -= v;
                    }
                }
            for (int t = 0; t < 9; t++) W[t] += Wc[9 * (size_t)k + t];
        }
    }
    if (virial) memcpy(virial, W, sizeof(W));
    if (table_oob) *table_oob = oob;
    free(cnt); free(nb); free(g); free(Wc);
    return fail ? -1 : dropped;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
