/*
 * hrkan_oracle.h -- plain FP64 CPU oracle for one physics-informed training
 * step of a Higher-order-ReLU KAN (HRKAN).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no source,
 * header, table or helper with the GPU library and must never be used as a
 * fallback for it.
 *
 * What it computes (all in double precision, scalar loops, no tiling):
 *   - the HR basis of order m and its derivatives (Sec. 3, Eq. 2),
 *   - the KAN layer as "basis tensor times weight matrix" (Sec. 3, the
 *     matrix-operation remark; Sec. 2.1-2.2 for the supports),
 *   - forward-mode jets (value and the derivatives of order 1..n along each
 *     input direction, n = 2 by default, up to 5) through every layer, as
 *     needed by the PDE residuals (Sec. 4.1 loss, Sec. 4.2 loss; Sec. 3
 *     on higher derivatives with a larger m),
 *   - the residuals and the loss L = alpha*L_pde + L_bc (Sec. 4.1 and 4.2),
 *     and a linear PDE of any order up to n,
 *   - the exact reverse-mode gradient of L with respect to every weight.
 *
 * Jet layout used throughout, for jet order n (hro_net.order): S = 1 + 2n
 * slots per feature,
 *   slot 0 = value, slot k = d^k/dx0^k (k = 1..n), slot n + k = d^k/dx1^k,
 * where x0 is the first input coordinate (x) and x1 the second (y, or t for
 * Burgers). For n = 2 that is value, d/dx0, d2/dx0^2, d/dx1, d2/dx1^2.
 * Arrays of jets are [S][width][n] (slot, feature, point), doubles. Slots
 * that a caller does not need are still computed; they cost time only.
 *
 * Weights of layer l: [w_l * n_b][w_{l+1}] row-major, row index i*n_b + b
 * (input feature i, basis function b), n_b = G + k.
 */
#ifndef HRKAN_ORACLE_H
#define HRKAN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HRO_MAX_LAYERS 8
#define HRO_MAX_ORDER 5
#define HRO_MAX_SLOTS (1 + 2 * HRO_MAX_ORDER)

typedef struct {
    int32_t n_layers;                     /* number of KAN layers L          */
    int32_t widths[HRO_MAX_LAYERS + 1];   /* widths[0] = 2, widths[L] = 1    */
    int32_t G;                            /* grid intervals on [lo, hi]      */
    int32_t k;                            /* B-spline order of the supports  */
    int32_t m;                            /* HR order                        */
    double lo, hi;                        /* grid range                      */
    int32_t order;                        /* jet order n, 1..5 (0 means 2)   */
} hro_net;

enum { HRO_POISSON2D = 0, HRO_BURGERS1D = 1, HRO_LINEAR2D = 2 };

typedef struct {
    int32_t kind;    /* HRO_POISSON2D, HRO_BURGERS1D or HRO_LINEAR2D          */
    double nu;       /* Burgers viscosity                                    */
    double alpha;    /* weight of the PDE term in the loss                   */
    double adv;      /* Burgers advection coefficient (1 for u_t+u u_x-nu u_xx) */
    /* HRO_LINEAR2D: r = c0 u + sum_k cx[k-1] d^k u/dx^k + sum_k cy[k-1]
     * d^k u/dy^k - f, f the same operator applied to sin(pi x) sin(pi y)
     * (so that function solves it); every order with a non-zero
     * coefficient must be at most the jet order. */
    double c0;
    double cx[HRO_MAX_ORDER];
    double cy[HRO_MAX_ORDER];
} hro_pde;

/* Slots per feature for jet order n: 1 + 2n. */
int hro_slots(int order);

/* n_b = G + k basis functions per input. */
int hro_n_basis(const hro_net *net);

/* Support [s_b, e_b] of every basis function b = 0..n_b-1. */
void hro_supports(const hro_net *net, double *s, double *e);

/* d^n/dz^n of the order-m HR bump on [s,e] at z, n = 0..nmax (nmax <= 8),
 * written to out[0..nmax]. Zero outside the open interval (s, e). */
void hro_basis(int m, double s, double e, double z, int nmax, double *out);

/* Teacher-forced layer forward: zin [S][w_l][n] -> zout [S][w_{l+1}][n]. */
int hro_layer_forward(const hro_net *net, int layer, const double *W,
                      const double *zin, int64_t n, double *zout);

/* Teacher-forced layer reverse: given the input jets zin [S][w_l][n] and the
 * bars of the output jets ybar [S][w_{l+1}][n], write the bars of the input
 * jets to zbar [S][w_l][n] (may be NULL) and ADD the weight gradient to gW. */
int hro_layer_backward(const hro_net *net, int layer, const double *W,
                       const double *zin, const double *ybar, int64_t n,
                       double *zbar, double *gW);

/* Layer-0 input jets of points x [n][2] for jet order `order`: value x,
 * unit first derivative along its own direction, every other derivative
 * zero. zin is [S][2][n]. Returns -1 for an order outside 1..5. */
int hro_input_jets(const double *x, int64_t n, int order, double *zin);

/* Whole network forward: x [n][2] -> jets of the output u, [S][n].
 * If all_jets is not NULL it receives the jets entering every layer l = 0..L,
 * concatenated: block l is [S][w_l][n]. */
int hro_forward(const hro_net *net, const double *const *W, const double *x,
                int64_t n, double *u_jets, double *all_jets);

/* Residual, loss and seeds. jets_int [S][n_int] (jet order `order`) are the
 * output jets at the interior points x_int [n_int][2]; u_bc [n_bc] are the
 * values at the boundary/initial points with targets g_bc [n_bc].
 * loss[0] = L, loss[1] = L_pde, loss[2] = L_bc.
 * r [n_int], seed_int [S][n_int] (dL/d jets) and seed_bc [n_bc] (dL/du) may
 * be NULL. Returns -1 if the PDE needs derivatives above `order`. */
int hro_residual(const hro_pde *pde, int order, const double *x_int,
                 const double *jets_int, int64_t n_int,
                 const double *u_bc, const double *g_bc, int64_t n_bc,
                 double *r, double *loss, double *seed_int, double *seed_bc);

/* Whole network reverse: given seeds [S][n] on the output jets of points
 * x [n][2], ADD dL/dW of every layer to gW[l]. */
int hro_backward(const hro_net *net, const double *const *W, const double *x,
                 int64_t n, const double *seed, double *const *gW);

/* One full step: forward jets at interior and boundary points, residual,
 * loss, and the gradient of L with respect to every weight. gW[l] is
 * OVERWRITTEN. r_out [n_int], jets_out [S][n_int] and ubc_out [n_bc] may be
 * NULL. */
int hro_step(const hro_net *net, const hro_pde *pde, const double *const *W,
             const double *x_int, int64_t n_int,
             const double *x_bc, int64_t n_bc, const double *g_bc,
             double *loss, double *const *gW,
             double *r_out, double *jets_out, double *ubc_out);

/* Rounding model, OFF by default (mode 0: every value exact in double).
 * It only serves to estimate how much error storage in a narrower type alone
 * causes through the network's conditioning, for tolerance gates:
 *   mode 1: every basis feature, every partial sum of a contraction over
 *           the basis (as an FP32 fused multiply-add chain, in the oracle's
 *           summation order) and every stored layer output (and input bar
 *           in the reverse pass) is rounded to FP32;
 *   mode 2: as mode 1, and every basis feature is further replaced by the sum
 *           of its first `split` BF16 pieces (hi, then lo = the BF16 rounding
 *           of the remainder), each rounded to nearest even; in the reverse
 *           pass an output bar is split the same way where it multiplies W
 *           (input bars) and rounded to its high BF16 piece where it
 *           multiplies a feature (weight gradient).
 * Weights are never rounded here: callers pass already rounded weights. */
void hro_set_rounding(int mode, int split);

/* The rounding model's primitives under the current mode, exposed so that
 * tests can pin them against independent FP32/BF16 conversions:
 *   what 0: a basis feature; 1: a stored layer output or input bar;
 *   2: an output bar where it multiplies W; 3: an output bar where it
 *   multiplies a feature.  Mode 0 returns v unchanged. */
double hro_model_round(int what, double v);
/* One step acc + w * a of a contraction's running sum (mode >= 1: one FP32
 * fused multiply-add of the FP32-held operands). */
double hro_model_acc(double acc, double w, double a);

/* Number of OpenMP threads the oracle runs with. */
int hro_num_threads(void);

#ifdef __cplusplus
}
#endif

#endif
