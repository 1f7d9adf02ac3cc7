/*
 * hrkan_oracle.c -- plain FP64 CPU oracle for one HRKAN physics-informed
 * training step. TEST INFRASTRUCTURE ONLY (see hrkan_oracle.h).
 *
 * Everything here is the definition written out, point by point, in double
 * precision:
 *   basis  (Sec. 3, Eq. 2):   v(z) = c_m * ReLU(e - z)^m * ReLU(z - s)^m,
 *                              c_m = (2 / (e - s))^(2m)
 *   derivatives:              Leibniz rule on the product of the two powers
 *   supports (Sec. 2.1-2.2):  those of the n = G + k order-k B-splines on a
 *                              uniform grid of G intervals over [lo, hi]
 *   layer (Sec. 3):           u_j = sum_i sum_b W[i*n_b + b][j] * v_b(z_i)
 *   jets:                     Faa di Bruno's formula with partial Bell
 *                              polynomials, derivatives of order 1..n (n <= 5)
 *                              along each input coordinate (Sec. 3 remarks that
 *                              a PDE with a fifth derivative takes m = 6)
 *   residual, loss (Sec. 4.1, 4.2): L = alpha * mean(r^2) + mean((u - g)^2);
 *                              also a linear PDE of any order up to n whose
 *                              source makes sin(pi x) sin(pi y) its solution
 *   gradient:                 reverse mode through the same expressions
 *
 * Terms whose basis factor is exactly zero (z outside the open support) are
 * skipped; that changes no value.
 *
 * Parallelism: OpenMP over points. Weight gradients are summed into one
 * buffer per thread (static schedule), then added in thread order.
 */
#include "hrkan_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* optional rounding model (off unless hro_set_rounding is called)      */
/* ------------------------------------------------------------------ */

static int g_mode = 0, g_split = 1;

void hro_set_rounding(int mode, int split)
{
    g_mode = mode;
    g_split = split < 1 ? 1 : (split > 2 ? 2 : split);
}

static double to_f32(double v) { return (double)(float)v; }

/* Nearest-even rounding of a float to the 8-bit-mantissa bfloat16 grid. */
static double to_bf16(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;   /* Inf, NaN */
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double round_feature(double a)
{
    if (g_mode == 0) return a;
    a = to_f32(a);
    if (g_mode == 2) {
        const double hi = to_bf16(a);
        a = g_split >= 2 ? hi + to_bf16(a - hi) : hi;
    }
    return a;
}

static double round_store(double v) { return g_mode == 0 ? v : to_f32(v); }

/* BF16 mode only: an output bar entering the input-bar contraction (with
 * W) is the split operand, like a feature; entering the weight-gradient
 * product (with a feature) it is the second operand, of which only the
 * high BF16 piece is used for split <= 2. Other modes leave bars as
 * stored. */
static double round_bar_split(double v) { return g_mode == 2 ? round_feature(v) : v; }
static double round_bar_hi(double v) { return g_mode == 2 ? to_bf16(to_f32(v)) : v; }

/* one step of a contraction's running sum, acc + w * a; in the rounding
 * model it is an FP32 fused multiply-add of the operands held in FP32: the
 * exact value of acc + w * a rounded once to FP32 (C99 fmaf). */
static double acc_step(double acc, double w, double a)
{
    return g_mode == 0 ? acc + w * a : (double)fmaf((float)w, (float)a, (float)acc);
}

double hro_model_round(int what, double v)
{
    switch (what) {
    case 0: return round_feature(v);
    case 1: return round_store(v);
    case 2: return round_bar_split(v);
    case 3: return round_bar_hi(v);
    default: return v;
    }
}

double hro_model_acc(double acc, double w, double a) { return acc_step(acc, w, a); }

/* ------------------------------------------------------------------ */
/* grid and basis                                                      */
/* ------------------------------------------------------------------ */

static int net_ok(const hro_net *net)
{
    if (!net || net->n_layers < 1 || net->n_layers > HRO_MAX_LAYERS) return 0;
    if (net->widths[0] != 2 || net->widths[net->n_layers] != 1) return 0;
    for (int l = 0; l <= net->n_layers; ++l)
        if (net->widths[l] < 1) return 0;
    if (net->G < 1 || net->k < 0 || net->m < 1) return 0;
    if (net->order < 0 || net->order > HRO_MAX_ORDER) return 0;
    if (!(net->hi > net->lo)) return 0;
    return 1;
}

int hro_n_basis(const hro_net *net) { return net->G + net->k; }

void hro_supports(const hro_net *net, double *s, double *e)
{
    /* Knots of the order-k B-spline basis on G uniform intervals, extended
     * by k intervals on each side; basis b lives on knots b .. b+k+1. */
    const int nb = hro_n_basis(net);
    const double h = (net->hi - net->lo) / net->G;
    for (int b = 0; b < nb; ++b) {
        s[b] = net->lo + (double)(b - net->k) * h;
        e[b] = net->lo + (double)(b + 1) * h;
    }
}

static double falling(int m, int j)  /* m! / (m - j)! */
{
    double f = 1.0;
    for (int t = 0; t < j; ++t) f *= (double)(m - t);
    return f;
}

static double binom(int n, int j)
{
    double c = 1.0;
    for (int t = 1; t <= j; ++t) c = c * (double)(n - j + t) / (double)t;
    return c;
}

void hro_basis(int m, double s, double e, double z, int nmax, double *out)
{
    for (int n = 0; n <= nmax; ++n) out[n] = 0.0;
    if (!(z > s && z < e)) return;               /* a ReLU factor is zero */
    const double c = pow(2.0 / (e - s), 2.0 * m);
    const double a = z - s;                       /* ReLU(z - s)  */
    const double be = e - z;                      /* ReLU(e - z)  */
    for (int n = 0; n <= nmax; ++n) {
        double sum = 0.0;
        for (int j = 0; j <= n; ++j) {
            const int i = n - j;                  /* derivatives on (e - z)^m */
            if (j > m || i > m) continue;
            const double da = falling(m, j) * pow(a, m - j);
            const double db = falling(m, i) * pow(be, m - i) * ((i & 1) ? -1.0 : 1.0);
            sum += binom(n, j) * da * db;
        }
        out[n] = c * sum;
    }
}

/* ------------------------------------------------------------------ */
/* jets of order n: slots and Faa di Bruno                             */
/* ------------------------------------------------------------------ */

/* Jet order per coordinate of a network (0 in the struct means 2). */
static int net_order(const hro_net *net) { return net->order == 0 ? 2 : net->order; }

int hro_slots(int order) { return 1 + 2 * order; }

/* Partial Bell polynomials B[k][j] = B_{k,j}(d_1, ..., d_{k-j+1}) for
 * 0 <= j <= k <= n, by the recurrence
 *   B_{0,0} = 1,  B_{k,0} = 0 (k >= 1),  B_{0,j} = 0 (j >= 1),
 *   B_{k,j} = sum_{i=1}^{k-j+1} C(k-1, i-1) d_i B_{k-i,j-1}.
 * d[i] is the i-th derivative of the inner function (d[0] unused). */
static void bell_table(int n, const double *d, double B[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1])
{
    for (int k = 0; k <= n; ++k)
        for (int j = 0; j <= n; ++j) B[k][j] = 0.0;
    B[0][0] = 1.0;
    for (int k = 1; k <= n; ++k)
        for (int j = 1; j <= k; ++j) {
            double sum = 0.0;
            for (int i = 1; i <= k - j + 1; ++i) sum += binom(k - 1, i - 1) * d[i] * B[k - i][j - 1];
            B[k][j] = sum;
        }
}

/* The derivatives along one coordinate of the feature f(z) of one basis
 * function, by Faa di Bruno's formula:
 *   d^k/dx^k f(z(x)) = sum_{j=1}^{k} f^(j)(z) B_{k,j}(z', ..., z^(k-j+1)),
 * k = 1..n; ph[j] = f^(j)(z). */
static void faa_di_bruno(int n, const double *ph, double B[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1], double *A)
{
    for (int k = 1; k <= n; ++k) {
        double sum = 0.0;
        for (int j = 1; j <= k; ++j) sum += ph[j] * B[k][j];
        A[k - 1] = sum;
    }
}

/* One input's jets for one point, zin [S][win] with S = 1 + 2n slots: the
 * value, then d^k/dx0^k (k = 1..n), then d^k/dx1^k. */
static void input_bells(int n, const double *zin, int win, int i,
                        double Bx[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1],
                        double By[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1],
                        double *dx, double *dy)
{
    dx[0] = dy[0] = 0.0;
    for (int k = 1; k <= n; ++k) {
        dx[k] = zin[k * win + i];
        dy[k] = zin[(n + k) * win + i];
    }
    bell_table(n, dx, Bx);
    bell_table(n, dy, By);
}

/* The features of basis function b of one input: slot 0 the value, slots
 * 1..n the x0-derivatives, n+1..2n the x1-derivatives. */
static void features_point(int n, const double *ph,
                           double Bx[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1],
                           double By[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1], double *A)
{
    A[0] = ph[0];
    faa_di_bruno(n, ph, Bx, A + 1);
    faa_di_bruno(n, ph, By, A + 1 + n);
    for (int q = 0; q < 1 + 2 * n; ++q) A[q] = round_feature(A[q]);
}

/* ------------------------------------------------------------------ */
/* one point through one layer                                         */
/* ------------------------------------------------------------------ */

/* zin: [S][win] for one point, zout: [S][wout], S = 1 + 2n. */
static void fwd_point(int m, int nb, const double *s, const double *e, int n,
                      int win, int wout, const double *W,
                      const double *zin, double *zout)
{
    const int S = hro_slots(n);
    for (int q = 0; q < S * wout; ++q) zout[q] = 0.0;
    for (int i = 0; i < win; ++i) {
        const double z = zin[0 * win + i];
        double Bx[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1], By[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1];
        double dx[HRO_MAX_ORDER + 1], dy[HRO_MAX_ORDER + 1];
        input_bells(n, zin, win, i, Bx, By, dx, dy);
        for (int b = 0; b < nb; ++b) {
            if (!(z > s[b] && z < e[b])) continue;
            double ph[HRO_MAX_ORDER + 2];
            hro_basis(m, s[b], e[b], z, n, ph);
            double A[HRO_MAX_SLOTS];
            features_point(n, ph, Bx, By, A);
            const double *wrow = W + (size_t)(i * nb + b) * wout;
            for (int j = 0; j < wout; ++j)
                for (int q = 0; q < S; ++q)
                    zout[q * wout + j] = acc_step(zout[q * wout + j], wrow[j], A[q]);
        }
    }
    if (g_mode)
        for (int q = 0; q < S * wout; ++q) zout[q] = round_store(zout[q]);
}

/* Bars of one input's jets from the bars Ab of one basis function's
 * features (one coordinate, slots 1..n of that coordinate): with
 * A_k = sum_j f^(j)(z) B_{k,j}(d) and dB_{k,j}/dd_i = C(k, i) B_{k-i,j-1},
 *   dA_k/dz   = sum_j f^(j+1)(z) B_{k,j},
 *   dA_k/dd_i = sum_j f^(j)(z) C(k, i) B_{k-i,j-1}. */
static void faa_di_bruno_adjoint(int n, const double *ph,
                                 double B[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1],
                                 const double *Ab, double *z0bar, double *dbar)
{
    for (int k = 1; k <= n; ++k) {
        const double a = Ab[k - 1];
        double dz = 0.0;
        for (int j = 1; j <= k; ++j) dz += ph[j + 1] * B[k][j];
        *z0bar += a * dz;
        for (int i = 1; i <= k; ++i) {
            double di = 0.0;
            for (int j = 1; j <= k - i + 1; ++j) di += ph[j] * B[k - i][j - 1];
            dbar[i] += a * binom(k, i) * di;
        }
    }
}

/* Reverse of fwd_point. ybar: [S][wout]; zbar: [S][win] (overwritten, may
 * be NULL); gW accumulated. */
static void bwd_point(int m, int nb, const double *s, const double *e, int n,
                      int win, int wout, const double *W,
                      const double *zin, const double *ybar,
                      double *zbar, double *gW)
{
    const int S = hro_slots(n);
    if (zbar)
        for (int q = 0; q < S * win; ++q) zbar[q] = 0.0;
    for (int i = 0; i < win; ++i) {
        const double z = zin[0 * win + i];
        double Bx[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1], By[HRO_MAX_ORDER + 1][HRO_MAX_ORDER + 1];
        double dx[HRO_MAX_ORDER + 1], dy[HRO_MAX_ORDER + 1];
        input_bells(n, zin, win, i, Bx, By, dx, dy);
        for (int b = 0; b < nb; ++b) {
            if (!(z > s[b] && z < e[b])) continue;
            double ph[HRO_MAX_ORDER + 2];
            hro_basis(m, s[b], e[b], z, n + 1, ph);
            double A[HRO_MAX_SLOTS];
            features_point(n, ph, Bx, By, A);
            const size_t row = (size_t)(i * nb + b);
            const double *wrow = W + row * wout;
            double *grow = gW + row * wout;
            double Ab[HRO_MAX_SLOTS];
            for (int q = 0; q < S; ++q) Ab[q] = 0.0;
            for (int j = 0; j < wout; ++j) {
                double g = 0.0;
                for (int q = 0; q < S; ++q) {
                    const double yb = ybar[q * wout + j];
                    Ab[q] = acc_step(Ab[q], wrow[j], round_bar_split(yb));   /* dL/dA = W * dL/dY */
                    g += A[q] * round_bar_hi(yb);                            /* dL/dW = A * dL/dY */
                }
                grow[j] += g;
            }
            if (!zbar) continue;
            /* every feature depends on the input's jets through the basis
             * derivatives at z and the Bell polynomials of its derivatives */
            double z0 = Ab[0] * ph[1];
            double dxb[HRO_MAX_ORDER + 1] = {0}, dyb[HRO_MAX_ORDER + 1] = {0};
            faa_di_bruno_adjoint(n, ph, Bx, Ab + 1, &z0, dxb);
            faa_di_bruno_adjoint(n, ph, By, Ab + 1 + n, &z0, dyb);
            zbar[0 * win + i] += z0;
            for (int k = 1; k <= n; ++k) {
                zbar[k * win + i] += dxb[k];
                zbar[(n + k) * win + i] += dyb[k];
            }
        }
    }
    if (zbar && g_mode)
        for (int q = 0; q < S * win; ++q) zbar[q] = round_store(zbar[q]);
}

static void gather(int S, const double *src, int w, int64_t n, int64_t p, double *dst)
{
    for (int q = 0; q < S; ++q)
        for (int i = 0; i < w; ++i)
            dst[q * w + i] = src[((int64_t)q * w + i) * n + p];
}

static void scatter(int S, const double *src, int w, int64_t n, int64_t p, double *dst)
{
    for (int q = 0; q < S; ++q)
        for (int i = 0; i < w; ++i)
            dst[((int64_t)q * w + i) * n + p] = src[q * w + i];
}

static void point_input(int order, const double *x, int64_t p, double *z /* [S][2] */)
{
    /* z_0 = x, z_1 = y (or t); d/dx0 z_0 = 1, d/dx1 z_1 = 1, every other
     * derivative zero */
    for (int q = 0; q < 2 * hro_slots(order); ++q) z[q] = 0.0;
    z[0] = x[2 * p];
    z[1] = x[2 * p + 1];
    z[2 * 1 + 0] = 1.0;                 /* slot 1 (d/dx0), input 0 */
    z[2 * (order + 1) + 1] = 1.0;       /* slot n+1 (d/dx1), input 1 */
}

int hro_input_jets(const double *x, int64_t n, int order, double *zin)
{
    if (order < 1 || order > HRO_MAX_ORDER) return -1;
    for (int64_t p = 0; p < n; ++p) {
        double z[2 * HRO_MAX_SLOTS];
        point_input(order, x, p, z);
        scatter(hro_slots(order), z, 2, n, p, zin);
    }
    return 0;
}

static int max_width(const hro_net *net)
{
    int w = 0;
    for (int l = 0; l <= net->n_layers; ++l)
        if (net->widths[l] > w) w = net->widths[l];
    return w;
}

/* ------------------------------------------------------------------ */
/* teacher-forced single layers                                        */
/* ------------------------------------------------------------------ */

int hro_layer_forward(const hro_net *net, int layer, const double *W,
                      const double *zin, int64_t n, double *zout)
{
    if (!net_ok(net) || layer < 0 || layer >= net->n_layers) return -1;
    const int nb = hro_n_basis(net), win = net->widths[layer],
              wout = net->widths[layer + 1];
    const int no = net_order(net), S = hro_slots(no);
    double *s = malloc(sizeof(double) * nb), *e = malloc(sizeof(double) * nb);
    hro_supports(net, s, e);
#pragma omp parallel
    {
        double *a = malloc(sizeof(double) * S * win);
        double *y = malloc(sizeof(double) * S * wout);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            gather(S, zin, win, n, p, a);
            fwd_point(net->m, nb, s, e, no, win, wout, W, a, y);
            scatter(S, y, wout, n, p, zout);
        }
        free(a); free(y);
    }
    free(s); free(e);
    return 0;
}

int hro_layer_backward(const hro_net *net, int layer, const double *W,
                       const double *zin, const double *ybar, int64_t n,
                       double *zbar, double *gW)
{
    if (!net_ok(net) || layer < 0 || layer >= net->n_layers) return -1;
    const int nb = hro_n_basis(net), win = net->widths[layer],
              wout = net->widths[layer + 1];
    const size_t np = (size_t)win * nb * wout;
    const int no = net_order(net), S = hro_slots(no);
    double *s = malloc(sizeof(double) * nb), *e = malloc(sizeof(double) * nb);
    hro_supports(net, s, e);
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *part = calloc((size_t)nt * np, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *a = malloc(sizeof(double) * S * win);
        double *yb = malloc(sizeof(double) * S * wout);
        double *zb = malloc(sizeof(double) * S * win);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            gather(S, zin, win, n, p, a);
            gather(S, ybar, wout, n, p, yb);
            bwd_point(net->m, nb, s, e, no, win, wout, W, a, yb, zb, part + (size_t)tid * np);
            if (zbar) scatter(S, zb, win, n, p, zbar);
        }
        free(a); free(yb); free(zb);
    }
    for (int t = 0; t < nt; ++t)
        for (size_t q = 0; q < np; ++q) gW[q] += part[(size_t)t * np + q];
    free(part); free(s); free(e);
    return 0;
}

/* ------------------------------------------------------------------ */
/* whole network                                                       */
/* ------------------------------------------------------------------ */

typedef struct {
    double *jets;      /* per layer l: [S][w_l], concatenated */
    double *bar_a, *bar_b;
    size_t off[HRO_MAX_LAYERS + 1];
} point_ws;

static void ws_init(const hro_net *net, point_ws *w)
{
    size_t tot = 0;
    for (int l = 0; l <= net->n_layers; ++l) {
        w->off[l] = tot;
        tot += (size_t)hro_slots(net_order(net)) * net->widths[l];
    }
    w->jets = malloc(sizeof(double) * tot);
    w->bar_a = malloc(sizeof(double) * hro_slots(net_order(net)) * max_width(net));
    w->bar_b = malloc(sizeof(double) * hro_slots(net_order(net)) * max_width(net));
}

static void ws_free(point_ws *w)
{
    free(w->jets); free(w->bar_a); free(w->bar_b);
}

static void net_fwd_point(const hro_net *net, const double *const *W,
                          const double *s, const double *e,
                          const double *x, int64_t p, point_ws *w)
{
    const int nb = hro_n_basis(net);
    point_input(net_order(net), x, p, w->jets + w->off[0]);
    for (int l = 0; l < net->n_layers; ++l)
        fwd_point(net->m, nb, s, e, net_order(net), net->widths[l], net->widths[l + 1], W[l],
                  w->jets + w->off[l], w->jets + w->off[l + 1]);
}

/* seed: [S] bars of the output jets. gW accumulated. */
static void net_bwd_point(const hro_net *net, const double *const *W,
                          const double *s, const double *e,
                          const double *seed, point_ws *w, double *const *gW)
{
    const int nb = hro_n_basis(net);
    double *cur = w->bar_a, *nxt = w->bar_b;
    for (int q = 0; q < hro_slots(net_order(net)); ++q) cur[q] = seed[q];
    for (int l = net->n_layers - 1; l >= 0; --l) {
        bwd_point(net->m, nb, s, e, net_order(net), net->widths[l], net->widths[l + 1], W[l],
                  w->jets + w->off[l], cur, l > 0 ? nxt : NULL, gW[l]);
        double *t = cur; cur = nxt; nxt = t;
    }
}

int hro_forward(const hro_net *net, const double *const *W, const double *x,
                int64_t n, double *u_jets, double *all_jets)
{
    if (!net_ok(net) || n < 0) return -1;
    const int nb = hro_n_basis(net), L = net->n_layers, S = hro_slots(net_order(net));
    double *s = malloc(sizeof(double) * nb), *e = malloc(sizeof(double) * nb);
    hro_supports(net, s, e);
    size_t blk[HRO_MAX_LAYERS + 1], acc = 0;
    for (int l = 0; l <= L; ++l) { blk[l] = acc; acc += (size_t)S * net->widths[l] * n; }
#pragma omp parallel
    {
        point_ws w;
        ws_init(net, &w);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            net_fwd_point(net, W, s, e, x, p, &w);
            if (u_jets)
                for (int q = 0; q < S; ++q)
                    u_jets[(int64_t)q * n + p] = w.jets[w.off[L] + q];
            if (all_jets)
                for (int l = 0; l <= L; ++l)
                    scatter(S, w.jets + w.off[l], net->widths[l], n, p, all_jets + blk[l]);
        }
        ws_free(&w);
    }
    free(s); free(e);
    return 0;
}

static double poisson_source(double x, double y)
{
    /* nabla^2 u = -2 pi^2 sin(pi x) sin(pi y)  (Sec. 4.1, Eq. 3) */
    return 2.0 * PI * PI * sin(PI * x) * sin(PI * y);
}

/* d^k/dx^k sin(pi x) = pi^k sin(pi x + k pi / 2): the derivatives of sin
 * cycle through sin, cos, -sin, -cos. */
static double dsin(int k, double x)
{
    const double v = (k & 1) ? cos(PI * x) : sin(PI * x);
    return pow(PI, k) * ((k & 2) ? -v : v);
}

/* Highest derivative order of a linear PDE along each coordinate (0 when
 * it has no such term). */
static void linear_orders(const hro_pde *pde, int *ox, int *oy)
{
    *ox = *oy = 0;
    for (int k = 1; k <= HRO_MAX_ORDER; ++k) {
        if (pde->cx[k - 1] != 0.0) *ox = k;
        if (pde->cy[k - 1] != 0.0) *oy = k;
    }
}

/* The linear PDE's operator applied to u* = sin(pi x) sin(pi y), the source
 * that makes u* its solution. */
static double linear_source(const hro_pde *pde, double x, double y)
{
    double f = pde->c0 * sin(PI * x) * sin(PI * y);
    for (int k = 1; k <= HRO_MAX_ORDER; ++k) {
        f += pde->cx[k - 1] * dsin(k, x) * sin(PI * y);
        f += pde->cy[k - 1] * sin(PI * x) * dsin(k, y);
    }
    return f;
}

/* Residual of one interior point from its output jets j[S] (slot order:
 * value, d^k/dx0^k for k = 1..n, d^k/dx1^k for k = 1..n). */
static double residual_point(const hro_pde *pde, int n, const double *xp,
                             const double *j)
{
    if (pde->kind == HRO_POISSON2D)
        return j[2] + j[n + 2] + poisson_source(xp[0], xp[1]);
    if (pde->kind == HRO_LINEAR2D) {
        /* c0 u + sum_k cx_k d^k u/dx^k + sum_k cy_k d^k u/dy^k - f */
        double r = pde->c0 * j[0];
        for (int k = 1; k <= n; ++k) r += pde->cx[k - 1] * j[k] + pde->cy[k - 1] * j[n + k];
        return r - linear_source(pde, xp[0], xp[1]);
    }
    /* u_t + adv * u * u_x - nu * u_xx  (Sec. 4.2, Eq. 5 and Eq. 6) */
    return j[n + 1] + pde->adv * j[0] * j[1] - pde->nu * j[2];
}

/* dL/d(jets) of one interior point, given rho = dL/dr. */
static void seed_point(const hro_pde *pde, int n, const double *j, double rho,
                       double *sd)
{
    for (int q = 0; q < hro_slots(n); ++q) sd[q] = 0.0;
    if (pde->kind == HRO_POISSON2D) {
        sd[2] = rho;                       /* dr/du_xx = 1 */
        sd[n + 2] = rho;                   /* dr/du_yy = 1 */
    } else if (pde->kind == HRO_LINEAR2D) {
        sd[0] = rho * pde->c0;
        for (int k = 1; k <= n; ++k) {
            sd[k] = rho * pde->cx[k - 1];
            sd[n + k] = rho * pde->cy[k - 1];
        }
    } else {
        sd[0] = rho * pde->adv * j[1];     /* dr/du    = adv * u_x */
        sd[1] = rho * pde->adv * j[0];     /* dr/du_x  = adv * u   */
        sd[2] = -rho * pde->nu;            /* dr/du_xx = -nu       */
        sd[n + 1] = rho;                   /* dr/du_t  = 1         */
    }
}

/* The PDE's kind is known and its derivatives fit jets of order n. */
static int pde_ok(const hro_pde *pde, int n)
{
    if (!pde || n < 1 || n > HRO_MAX_ORDER) return 0;
    if (pde->kind == HRO_POISSON2D || pde->kind == HRO_BURGERS1D) return n >= 2;
    if (pde->kind != HRO_LINEAR2D) return 0;
    int ox, oy;
    linear_orders(pde, &ox, &oy);
    return ox <= n && oy <= n;
}

int hro_residual(const hro_pde *pde, int order, const double *x_int,
                 const double *jets_int, int64_t n_int,
                 const double *u_bc, const double *g_bc, int64_t n_bc,
                 double *r, double *loss, double *seed_int, double *seed_bc)
{
    if (!pde_ok(pde, order)) return -1;
    const int S = hro_slots(order);
    double spde = 0.0, sbc = 0.0;
    for (int64_t p = 0; p < n_int; ++p) {
        double j[HRO_MAX_SLOTS];
        for (int q = 0; q < S; ++q) j[q] = jets_int[(int64_t)q * n_int + p];
        const double rp = residual_point(pde, order, x_int + 2 * p, j);
        if (r) r[p] = rp;
        spde += rp * rp;
        if (seed_int) {
            double sd[HRO_MAX_SLOTS];
            seed_point(pde, order, j, 2.0 * pde->alpha * rp / (double)n_int, sd);
            for (int q = 0; q < S; ++q) seed_int[(int64_t)q * n_int + p] = sd[q];
        }
    }
    for (int64_t p = 0; p < n_bc; ++p) {
        const double d = u_bc[p] - g_bc[p];
        sbc += d * d;
        if (seed_bc) seed_bc[p] = 2.0 * d / (double)n_bc;
    }
    const double lpde = n_int > 0 ? spde / (double)n_int : 0.0;
    const double lbc = n_bc > 0 ? sbc / (double)n_bc : 0.0;
    loss[0] = pde->alpha * lpde + lbc;
    loss[1] = lpde;
    loss[2] = lbc;
    return 0;
}

int hro_backward(const hro_net *net, const double *const *W, const double *x,
                 int64_t n, const double *seed, double *const *gW)
{
    if (!net_ok(net) || n < 0) return -1;
    const int nb = hro_n_basis(net), L = net->n_layers, S = hro_slots(net_order(net));
    double *s = malloc(sizeof(double) * nb), *e = malloc(sizeof(double) * nb);
    hro_supports(net, s, e);
    size_t np[HRO_MAX_LAYERS], tot = 0;
    for (int l = 0; l < L; ++l) { np[l] = (size_t)net->widths[l] * nb * net->widths[l + 1]; tot += np[l]; }
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *part = calloc((size_t)nt * tot, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine[HRO_MAX_LAYERS];
        size_t o = (size_t)tid * tot;
        for (int l = 0; l < L; ++l) { mine[l] = part + o; o += np[l]; }
        point_ws w;
        ws_init(net, &w);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            double sd[HRO_MAX_SLOTS];
            for (int q = 0; q < S; ++q) sd[q] = seed[(int64_t)q * n + p];
            net_fwd_point(net, W, s, e, x, p, &w);
            net_bwd_point(net, W, s, e, sd, &w, mine);
        }
        ws_free(&w);
    }
    for (int t = 0; t < nt; ++t) {
        size_t o = (size_t)t * tot;
        for (int l = 0; l < L; ++l) {
            for (size_t q = 0; q < np[l]; ++q) gW[l][q] += part[o + q];
            o += np[l];
        }
    }
    free(part); free(s); free(e);
    return 0;
}

int hro_step(const hro_net *net, const hro_pde *pde, const double *const *W,
             const double *x_int, int64_t n_int,
             const double *x_bc, int64_t n_bc, const double *g_bc,
             double *loss, double *const *gW,
             double *r_out, double *jets_out, double *ubc_out)
{
    if (!net_ok(net) || n_int < 0 || n_bc < 0) return -1;
    const int no = net_order(net), S = hro_slots(no);
    if (!pde_ok(pde, no)) return -1;
    const int nb = hro_n_basis(net), L = net->n_layers;
    for (int l = 0; l < L; ++l)
        memset(gW[l], 0, sizeof(double) * (size_t)net->widths[l] * nb * net->widths[l + 1]);

    /* forward jets at every point */
    double *ji = malloc(sizeof(double) * S * (size_t)(n_int > 0 ? n_int : 1));
    double *jb = malloc(sizeof(double) * S * (size_t)(n_bc > 0 ? n_bc : 1));
    if (hro_forward(net, W, x_int, n_int, ji, NULL)) return -1;
    if (hro_forward(net, W, x_bc, n_bc, jb, NULL)) return -1;

    /* residual, loss and seeds */
    double *si = malloc(sizeof(double) * S * (size_t)(n_int > 0 ? n_int : 1));
    double *sbc = malloc(sizeof(double) * (size_t)(n_bc > 0 ? n_bc : 1));
    double *sb = calloc(S * (size_t)(n_bc > 0 ? n_bc : 1), sizeof(double));
    hro_residual(pde, no, x_int, ji, n_int, jb /* slot 0 = u */, g_bc, n_bc,
                 r_out, loss, si, sbc);
    for (int64_t p = 0; p < n_bc; ++p) sb[p] = sbc[p];   /* only du is seeded */

    /* reverse: gW = dL/dW summed over both point sets */
    hro_backward(net, W, x_int, n_int, si, gW);
    hro_backward(net, W, x_bc, n_bc, sb, gW);

    if (jets_out) memcpy(jets_out, ji, sizeof(double) * S * (size_t)n_int);
    if (ubc_out) memcpy(ubc_out, jb, sizeof(double) * (size_t)n_bc);
    free(ji); free(jb); free(si); free(sbc); free(sb);
    return 0;
}

int hro_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
