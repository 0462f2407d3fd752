// tabulate.hip -- the embedding net as a table of fifth-order polynomials
// (paper Sec. 3.2), built on the device in FP64.
//
// The domain of s is cut into equal intervals (stride h on [0, s_max), then
// stride h_tail on [s_max, tail_max)).  On each interval every one of the M
// columns of the net is replaced by the quintic that matches the net's
// value, first and second derivative at both nodes.  Here the quintic is
// assembled from the six quintic Hermite basis functions on [0, 1] (value,
// slope and curvature at either end) and expanded into monomials of the
// offset t from the left node, a_k = c_k / w^k.
//
// Layouts written: tab64[theta][eta][6] (FP64) and tab32[theta][eta][6]
// (FP32; a column is 24 bytes, three 8-byte loads).  With several atom types the tables of the neighbor types follow
// each other: type t's interval theta is row t n_int + theta.

#include "dp_internal.h"

namespace dp {

namespace {

// Net value, slope and curvature at every node: one block of 128 threads
// per (node, type), thread o owns output column o of each layer.  emb holds
// the nets of the types back to back, emb_stride doubles apart.
__global__ void __launch_bounds__(128) k_nodes(int n_fine, int n_tail, double h, double s_max,
                                               double h_tail, const double *__restrict__ emb_all,
                                               long emb_stride, int d1, int d2, int d3,
                                               double *__restrict__ out_all)
{
    __shared__ double v[3][256], vn[3][256];
    int node = blockIdx.x, o = threadIdx.x;
    const double *emb = emb_all + blockIdx.y * emb_stride;
    double *out = out_all + (long)blockIdx.y * (n_fine + n_tail + 1) * d3 * 3;
    double x = node <= n_fine ? node * h : s_max + (node - n_fine) * h_tail;
    const double *W0 = emb, *b0 = W0 + d1, *W1 = b0 + d1, *b1 = W1 + d1 * d2, *W2 = b1 + d2,
                 *b2 = W2 + d2 * d3;
    if (o < d1) {
        double w = W0[o];
        double t = tanh(x * w + b0[o]);
        double g1 = 1.0 - t * t;
        v[0][o] = t;
        v[1][o] = g1 * w;
        v[2][o] = -2.0 * t * g1 * w * w;
    }
    __syncthreads();
    int win = d1;
    for (int layer = 0; layer < 2; layer++) {
        const double *W = layer == 0 ? W1 : W2;
        const double *b = layer == 0 ? b1 : b2;
        int wout = layer == 0 ? d2 : d3;
        if (o < wout) {
            double z0 = b[o], z1 = 0.0, z2 = 0.0;
            for (int a = 0; a < win; a++) {
                double w = W[a * wout + o];
                z0 = fma(v[0][a], w, z0);
                z1 = fma(v[1][a], w, z1);
                z2 = fma(v[2][a], w, z2);
            }
            double t = tanh(z0);
            double q = 1.0 - t * t;                   // tanh'
            int src = o - (o >= win ? win : 0);      // [x, x]: column o repeats input o mod win
            vn[0][o] = v[0][src] + t;
            vn[1][o] = v[1][src] + q * z1;
            vn[2][o] = v[2][src] + q * z2 - 2.0 * t * q * z1 * z1;
        }
        __syncthreads();
        if (o < wout)
            for (int c = 0; c < 3; c++) v[c][o] = vn[c][o];
        __syncthreads();
        win = wout;
    }
    if (o < d3)
        for (int c = 0; c < 3; c++) out[((long)node * d3 + o) * 3 + c] = v[c][o];
}

// One thread per (type, interval, column).
__global__ void k_hermite(int ntypes, int n_int, int n_fine, double h, double h_tail, int M,
                          const double *__restrict__ nodes, double *__restrict__ tab64,
                          float *__restrict__ tab32)
{
    long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (id >= (long)ntypes * n_int * M) return;
    int ty = (int)(id / ((long)n_int * M));
    int th = (int)(id / M % n_int), e = (int)(id % M);
    double w = th < n_fine ? h : h_tail;
    const double *nt = nodes + (long)ty * (n_int + 1) * M * 3;
    const double *L = nt + ((long)th * M + e) * 3, *R = nt + ((long)(th + 1) * M + e) * 3;
    // end values in the unit variable tau = t / w
    double y0 = L[0], p0 = w * L[1], q0 = w * w * L[2];
    double y1 = R[0], p1 = w * R[1], q1 = w * w * R[2];
    // monomial coefficients in tau of
    //   y0 H0 + p0 H1 + q0 H2 + y1 H3 + p1 H4 + q1 H5,  with
    //   H0 = 1 - 10 tau^3 + 15 tau^4 - 6 tau^5,   H3 = 1 - H0,
    //   H1 = tau - 6 tau^3 + 8 tau^4 - 3 tau^5,   H4 = -4 tau^3 + 7 tau^4 - 3 tau^5,
    //   H2 = (tau^2 - 3 tau^3 + 3 tau^4 - tau^5)/2, H5 = (tau^3 - 2 tau^4 + tau^5)/2
    double c[6];
    c[0] = y0;
    c[1] = p0;
    c[2] = 0.5 * q0;
    c[3] = -10.0 * y0 - 6.0 * p0 - 1.5 * q0 + 10.0 * y1 - 4.0 * p1 + 0.5 * q1;
    c[4] = 15.0 * y0 + 8.0 * p0 + 1.5 * q0 - 15.0 * y1 + 7.0 * p1 - q1;
    c[5] = -6.0 * y0 - 3.0 * p0 - 0.5 * q0 + 6.0 * y1 - 3.0 * p1 + 0.5 * q1;
    double inv = 1.0 / w, sc = 1.0;
    double *o64 = tab64 + id * 6;
    float *o32 = tab32 + id * 6;
    for (int k = 0; k < 6; k++) {
        o64[k] = c[k] * sc;
        o32[k] = (float)(c[k] * sc);
        sc *= inv;
    }
}

}  // namespace

dp_status launch_tabulate(dp_model *m, hipStream_t st)
{
    const TableInfo &t = m->tab;
    int n_int = t.n_int();
    long emb_stride = (long)m->d1 * 2 + (long)m->d1 * m->d2 + m->d2 + (long)m->d2 * m->d3 + m->d3;
    hipLaunchKernelGGL(k_nodes, dim3(n_int + 1, m->ntypes), dim3(128), 0, st, t.n_fine, t.n_tail, t.h, t.s_max,
                       t.h_tail, m->emb_d, emb_stride, m->d1, m->d2, m->d3, m->nodes);
    long nthr = (long)m->ntypes * n_int * kM;
    hipLaunchKernelGGL(k_hermite, dim3(div_up(nthr, 256)), dim3(256), 0, st, m->ntypes, n_int, t.n_fine, t.h,
                       t.h_tail, kM, m->nodes, m->tab64, m->tab32);
    return DP_OK;
}

namespace {

// tanh on [0, 8) by a quadratic per interval of width 1/128: the value and
// slope of tanh at the left node x0 and its value at x0 + h (paper Sec. 3.5
// fixes the order, the range, the odd extension and the saturation at 8).
__global__ void k_tanh_table(double *tab64, float *tab32)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kTanhN) return;
    const double h = 8.0 / kTanhN;
    double x0 = k * h;
    double a0 = tanh(x0), a1 = 1.0 - a0 * a0;
    double a2 = (tanh(x0 + h) - a0 - a1 * h) / (h * h);
    double a[4] = {a0, a1, a2, 0.0};
    for (int q = 0; q < 4; q++) {
        tab64[4 * k + q] = a[q];
        tab32[4 * k + q] = (float)a[q];
    }
}

}  // namespace

void launch_tanh_table(double *tab64, float *tab32, hipStream_t st)
{
    hipLaunchKernelGGL(k_tanh_table, dim3(div_up(kTanhN, 256)), dim3(256), 0, st, tab64, tab32);
}

}  // namespace dp
