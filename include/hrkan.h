/*
 * hrkan.h -- C ABI of the MI355X (gfx950) library for one physics-informed
 * training step of a Higher-order-ReLU KAN (HRKAN, So & Yung).
 *
 * The step (Sec. 3 and Sec. 4 of the paper):
 *   1. every KAN layer evaluates, for each input feature z_i, the HR basis
 *        v_b(z) = c_m * ReLU(e_b - z)^m * ReLU(z - s_b)^m,  c_m = (2/(e_b-s_b))^(2m)
 *      (Sec. 3, Eq. 2) on the supports of the order-k B-splines of a uniform
 *      grid of G intervals on [lo, hi] (Sec. 2.1-2.2; n_b = G + k functions),
 *      and contracts the basis tensor [points x (w_in * n_b)] with the layer's
 *      weight matrix [w_in * n_b, w_out] (the matrix operation of Sec. 3);
 *   2. the value is carried together with its first and second derivatives
 *      along each input coordinate (forward jets) through every layer;
 *   3. the PDE residual and the loss L = alpha * L_pde + L_bc are formed
 *      (Poisson: Sec. 4.1, Eq. 3 and its loss; viscous Burgers: Sec. 4.2,
 *      Eq. 5/6 and Eq. 7);
 *   4. L is differentiated back to every weight (reverse mode through the
 *      jets, with the basis recomputed rather than stored).
 *
 * Conventions shared by every call
 *   - Every array argument is DEVICE memory owned by the caller, unless the
 *     argument says "host". The library never allocates device memory in these
 *     calls; scratch lives in the caller's workspace `ws`.
 *   - Calls are asynchronous on `stream` (0 = the null stream). They validate
 *     every argument on the host before anything is enqueued and return a
 *     status code; no C++ exception crosses this interface. A non-zero code
 *     means nothing was enqueued, except HRKAN_ERR_DEVICE (a HIP launch error;
 *     the stream may hold part of the work).
 *   - Results are deterministic run to run on one device: every reduction has
 *     a fixed order and no floating-point atomics are used.
 *   - Calls are re-entrant for distinct workspaces. Two calls in flight on the
 *     same workspace race. The first 256 bytes of a workspace hold the device
 *     status word (hrkan_read_status): zero them once before first use.
 *   - Floating-point arrays use the "array type" of the network's dtype:
 *       HRKAN_F64  -> double;
 *       HRKAN_F32  -> float;
 *       HRKAN_BF16 -> float (FP32 master weights and FP32 jets; the basis x W
 *                     contractions run on BF16 matrix cores, see bf16_split).
 *   - Points x are [n][2] row-major: (x, y) for Poisson, (x, t) for Burgers.
 *   - Jets are channel-major [C][n]; the channels present are the set bits of
 *     a channel mask, in the order U, then the x0-derivatives X, XX, X3, X4,
 *     X5, then the x1-derivatives Y, YY, Y3, Y4, Y5 (X = d/dx0, Xk =
 *     d^k/dx0^k, likewise Y; x1 is y for Poisson and t for Burgers). For the
 *     masks of order at most two that is U, X, XX, Y, YY.
 *   - Weights of layer l are [w_l * n_b][w_{l+1}] row-major, row i*n_b + b for
 *     input feature i and basis function b, 16-byte aligned. Weight gradients
 *     use the same layout, alignment and array type.
 */
#ifndef HRKAN_H
#define HRKAN_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HRKAN_MAX_LAYERS 8
#define HRKAN_MAX_WIDTH 1024

/* status codes */
#define HRKAN_OK 0
#define HRKAN_ERR_INVALID_ARG (-1)   /* null/misaligned pointer, bad size, bad field */
#define HRKAN_ERR_UNSUPPORTED (-2)   /* valid but not implemented: dtype, m, mask, width */
#define HRKAN_ERR_WORKSPACE (-3)     /* ws_bytes smaller than required */
#define HRKAN_ERR_DEVICE (-4)        /* a HIP call failed; see hrkan_last_error() */
#define HRKAN_ERR_PLAN_MISMATCH (-5) /* plan used with another shape or freed */
#define HRKAN_ERR_HOST_MEMORY (-6)   /* a host allocation failed (plan tables) */

/* bits of the device status word (hrkan_read_status) */
#define HRKAN_STATUS_NONFINITE 1u    /* a loss partial was NaN or Inf */

/* contraction precision (hrkan_net_desc.dtype) */
#define HRKAN_F64 0
#define HRKAN_F32 1
#define HRKAN_BF16 2

/* PDE kinds (hrkan_pde_desc.kind) */
#define HRKAN_POISSON2D 0   /* u_xx + u_yy = -2 pi^2 sin(pi x) sin(pi y), Sec. 4.1 Eq. 3 */
#define HRKAN_BURGERS1D 1   /* u_t + adv * u * u_x - nu * u_xx = 0, Sec. 4.2 Eq. 5 / Eq. 6 */
#define HRKAN_LINEAR2D 2    /* linear, derivatives up to fifth order (Sec. 3's remark on
                               higher derivatives); see hrkan_pde_desc */

/* jet channels: the value and the derivatives of order 1..5 along each
 * coordinate (orders above two need HR order m >= 3, and the reverse pass
 * of order n uses the basis derivative n + 1) */
#define HRKAN_MAX_ORDER 5
#define HRKAN_CH_U 1u
#define HRKAN_CH_X 2u
#define HRKAN_CH_XX 4u
#define HRKAN_CH_Y 8u
#define HRKAN_CH_YY 16u
#define HRKAN_CH_X3 32u
#define HRKAN_CH_X4 64u
#define HRKAN_CH_X5 128u
#define HRKAN_CH_Y3 256u
#define HRKAN_CH_Y4 512u
#define HRKAN_CH_Y5 1024u
#define HRKAN_MASK_POISSON (HRKAN_CH_U | HRKAN_CH_X | HRKAN_CH_XX | HRKAN_CH_Y | HRKAN_CH_YY)
#define HRKAN_MASK_BURGERS (HRKAN_CH_U | HRKAN_CH_X | HRKAN_CH_XX | HRKAN_CH_Y)
#define HRKAN_MASK_VALUE HRKAN_CH_U

/* Network description (host struct).
 *   n_layers   1..HRKAN_MAX_LAYERS; widths[0] = 2, widths[n_layers] = 1,
 *              every width in 1..HRKAN_MAX_WIDTH.
 *   G, k, m    grid intervals (>= 1), B-spline order of the supports (0..8),
 *              HR order (2..8; the paper uses m = 4). Every layer uses the
 *              same grid [lo, hi] (lo < hi).
 *   dtype      HRKAN_F64, HRKAN_F32 or HRKAN_BF16.
 *   bf16_split number of BF16 product terms S for HRKAN_BF16 (1, 2 or 3):
 *              1: a_hi*b_hi; 2: adds a_lo*b_hi (the weight is used in BF16,
 *              the basis/bar operand in two BF16 pieces); 3: also adds
 *              a_hi*b_lo (both operands split). Ignored for F32/F64.          */
typedef struct {
    int32_t n_layers;
    int32_t widths[HRKAN_MAX_LAYERS + 1];
    int32_t G, k, m;
    double lo, hi;
    int32_t dtype;
    int32_t bf16_split;
} hrkan_net_desc;

/* PDE description (host struct). alpha weighs L_pde in L = alpha L_pde + L_bc
 * (the paper uses 0.05). For Burgers, nu is the viscosity and adv the
 * coefficient of u*u_x (1 for Eq. 5; 1/4 with nu/16 for the rescaled Eq. 6).
 * For HRKAN_LINEAR2D the residual is
 *   r = c0 u + sum_{k=1..5} cx[k-1] d^k u/dx^k + sum_{k=1..5} cy[k-1] d^k u/dy^k - f,
 * f being the same operator applied to sin(pi x) sin(pi y), which therefore
 * solves it (and vanishes on the edges of [-1,1]^2); the interior jets carry
 * the derivatives up to the highest order with a non-zero coefficient along
 * each coordinate. */
typedef struct {
    int32_t kind;
    double nu;
    double alpha;
    double adv;
    double c0;
    double cx[HRKAN_MAX_ORDER];
    double cy[HRKAN_MAX_ORDER];
} hrkan_pde_desc;

/* Collocation sets (host struct holding device pointers).
 *   x_int [n_int][2]   interior points (residual)
 *   x_bc  [n_bc][2]    boundary / initial points (value misfit)
 *   g_bc  [n_bc]       target values at x_bc (0 on walls, the initial
 *                      condition on t = 0)
 * Either count may be 0 (the pointer may then be NULL); the matching loss
 * term is then 0. */
typedef struct {
    const void *x_int;
    int64_t n_int;
    const void *x_bc;
    int64_t n_bc;
    const void *g_bc;
} hrkan_points;

/* Fill *net / *pde with the paper's defaults (G=5, k=3, m=4, [-1,1], F32,
 * S=2; alpha=0.05, adv=1, nu=0.01/pi for Burgers). Returns HRKAN_OK. */
int hrkan_net_init(hrkan_net_desc *net);
int hrkan_pde_init(hrkan_pde_desc *pde, int32_t kind);

/* Number of channels of a mask, or a negative status if it is not a
 * supported set: it must hold U, and along each coordinate the derivatives
 * of order 1..o for some o in 0..5 (HRKAN_ERR_INVALID_ARG otherwise). Masks
 * with an order above two (or the sets U,X; U,Y; U,X,Y,YY; ...) run on the
 * vector-ALU kernels in FP64 and FP32 only (HRKAN_BF16 is refused with
 * HRKAN_ERR_UNSUPPORTED); U alone, U,X,Y, U,X,XX, U,X,XX,Y and
 * U,X,XX,Y,YY also run on the matrix cores. */
int hrkan_mask_channels(uint32_t channel_mask);

/* The mask of the value and the derivatives of order 1..ox along x0 and
 * 1..oy along x1 (0 <= ox, oy <= 5), or 0 if an order is out of range. */
uint32_t hrkan_mask_of_orders(int32_t ox, int32_t oy);

/* Bytes of the `saved` buffer that hrkan_forward_jets fills and
 * hrkan_backward reads for n points: the jets entering layers 1..L-1, in the
 * array type, [C][w_l][n] per layer. */
int hrkan_saved_bytes(const hrkan_net_desc *net, int64_t n, uint32_t channel_mask,
                      size_t *bytes /* host */);

/* Bytes of workspace that every call below needs for at most n_int interior
 * and n_bc boundary points (hrkan_forward_jets / hrkan_backward with
 * n <= max(n_int, n_bc) included). ws must be 256-byte aligned. */
int hrkan_workspace_bytes(const hrkan_net_desc *net, const hrkan_pde_desc *pde,
                          int64_t n_int, int64_t n_bc, size_t *bytes /* host */);

/* Forward jets: the network's output u and the derivatives selected by
 * channel_mask at n points x [n][2].
 *   W        host array of n_layers device pointers, W[l] as documented above
 *   jets_out [C][n] (array type)
 *   saved    NULL, or hrkan_saved_bytes(...) bytes that receive the inner
 *            jets needed by hrkan_backward for the same x, W and mask */
int hrkan_forward_jets(const hrkan_net_desc *net, const void *const *W, const void *x,
                       int64_t n, uint32_t channel_mask, void *jets_out, void *saved,
                       void *ws, size_t ws_bytes, hipStream_t stream);

/* Residual, loss and seeds (Sec. 4.1 / 4.2 losses).
 *   jets_int [C][n_int]  output jets at pts->x_int with the PDE's mask
 *                        (HRKAN_MASK_POISSON, HRKAN_MASK_BURGERS, or for
 *                        HRKAN_LINEAR2D the mask of its highest orders)
 *   u_bc     [n_bc]      network values at pts->x_bc
 *   r_out    [n_int]     residual (may be NULL)
 *   loss_out device double[3] = {L, L_pde, L_bc}
 *   seed_int [C][n_int]  dL/d(jets_int) (may be NULL)
 *   seed_bc  [n_bc]      dL/d(u_bc) (may be NULL)
 * dtype is the array type of jets/seeds (HRKAN_F64 or HRKAN_F32; BF16 runs
 * pass HRKAN_F32). Partial sums are reduced in double precision. */
int hrkan_residual(const hrkan_pde_desc *pde, int32_t dtype, const void *jets_int,
                   const void *u_bc, const hrkan_points *pts, void *r_out, double *loss_out,
                   void *seed_int, void *seed_bc, void *ws, size_t ws_bytes,
                   hipStream_t stream);

/* Reverse pass: given seed [C][n] = dL/d(output jets) at points x, write
 * dL/dW to gW_out[l] (host array of device pointers), overwriting it, or
 * adding to it when accumulate != 0. `saved` is what hrkan_forward_jets
 * wrote for the same x, W, n and mask. The basis is recomputed from the
 * saved jets. */
int hrkan_backward(const hrkan_net_desc *net, const void *const *W, const void *x, int64_t n,
                   uint32_t channel_mask, const void *seed, const void *saved,
                   void *const *gW_out, int32_t accumulate, void *ws, size_t ws_bytes,
                   hipStream_t stream);

/* One full training step: forward jets at both point sets, residual, loss
 * (loss_out device double[3] = {L, L_pde, L_bc}) and gW_out[l] = dL/dW[l]
 * (overwritten). The interior mask is the PDE's (Poisson: 5 channels,
 * Burgers: 4, linear: up to 11); only the value enters the boundary loss. Execution depends on
 * the set sizes (the results do not, up to rounding): small sets run as one
 * set, medium ones put the boundary set on a second stream that the library
 * creates for `stream` on first use (default priority; every fork is joined
 * back into `stream` within the call's work, and under graph capture the
 * fork and join become graph edges), large ones run on `stream` alone.
 * hrkan_workspace_bytes gives the size for the same counts. */
int hrkan_step(const hrkan_net_desc *net, const hrkan_pde_desc *pde, const void *const *W,
               const hrkan_points *pts, double *loss_out, void *const *gW_out, void *ws,
               size_t ws_bytes, hipStream_t stream);

/* hrkan_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same step, with the workspace taken from a static device array of the
 * library, HRKAN_STATIC_SCRATCH_BYTES (64 MiB) per GPU, which each GPU the
 * library runs on holds until the process ends. The caller still passes
 * weights, points, loss_out and gW_out (same meaning and layouts as
 * hrkan_step). The call allocates nothing: no hipMalloc, no stream or event
 * (both point sets run on `stream`). Its first call on a device looks up that
 * device's array and clears its status word on `stream`.
 * Errors: HRKAN_ERR_WORKSPACE (nothing enqueued) when the step needs more
 * workspace than the array holds (hrkan_workspace_bytes for the same
 * counts; e.g. the [2,32,32,1] Burgers network fits up to about 14,000
 * interior points); HRKAN_ERR_UNSUPPORTED while per-launch profiling is on;
 * otherwise those of hrkan_step. All calls on one GPU share its array, which
 * keeps the last call's contents: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller. */
#define HRKAN_STATIC_SCRATCH_BYTES (64u << 20)
int hrkan_step_static(const hrkan_net_desc *net, const hrkan_pde_desc *pde, const void *const *W,
                      const hrkan_points *pts, double *loss_out, void *const *gW_out,
                      hipStream_t stream);

/* Adam update of every layer's weights in place, for training with the
 * optimiser the paper uses (Sec. 4.1, 4.2: Adam, 3000 epochs), with the
 * published update of Kingma and Ba: with t = *step_dev + 1,
 *   m = beta1 m + (1 - beta1) g,   v = beta2 v + (1 - beta2) g^2,
 *   W -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
 * elementwise over W[l], gW[l], m[l], v[l] (host arrays of n_layers device
 * pointers, each [w_l * n_b, w_{l+1}], array type of the net: FP64 for
 * HRKAN_F64, else FP32; m and v zero before the first update). step_dev is
 * a device int64 (zero before the first update) that the call advances by
 * one after the update, so a step and its update captured together in a
 * HIP graph replay with the right bias corrections. Requires lr >= 0,
 * 0 <= beta1, beta2 < 1, eps > 0; asynchronous on `stream`. */
int hrkan_adam(const hrkan_net_desc *net, void *const *W, const void *const *gW, void *const *m,
               void *const *v, int64_t *step_dev, double lr, double beta1, double beta2, double eps,
               hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Batched step: many independent instances of one network shape, each with */
/* its own weights, PDE coefficients and point counts, run by one           */
/* persistent kernel whose launches are captured in a HIP graph.            */
/* ---------------------------------------------------------------------- */
typedef struct hrkan_plan hrkan_plan;

/* Create a plan (host call; may allocate host memory and run the tile
 * autotuner, which times candidate tile shapes on `stream` with the caller's
 * buffers; it never allocates device memory). The autotuner's choice is
 * kept in a cache file keyed by the device architecture, the network shape,
 * dtype, PDE kind and the instance and interior point counts rounded up to
 * powers of two; a later plan with the same key reads it instead of timing
 * the candidates. The file is $HRKAN_AUTOTUNE_CACHE (an empty value turns
 * the cache off), else $XDG_CACHE_HOME/hrkan/autotune.json, else
 * $HOME/.cache/hrkan/autotune.json; it is written atomically (temporary
 * file and rename), and a missing, unreadable or unwritable file only costs
 * the timing.
 *   n_inst     number of instances (>= 1)
 *   pdes       host array [n_inst] (kind must be HRKAN_BURGERS1D or
 *              HRKAN_POISSON2D, one kind for all instances)
 *   W_packed   [n_inst][n_params] weights, instance-major, each instance's
 *              layers concatenated in order (array type)
 *   pts        host array [n_inst] of collocation sets (device pointers)
 *   loss_out   device double [n_inst][3]
 *   gW_packed  [n_inst][n_params] gradients (overwritten at each execute)
 *   ws         workspace of hrkan_plan_workspace_bytes(...) bytes
 * The plan keeps every pointer until hrkan_plan_destroy. HRKAN_F32 and
 * HRKAN_BF16 (the block-sparse matrix-core kernels with bf16_split product
 * terms; FP32 master weights) are supported, HRKAN_F64 is refused. */
int hrkan_plan_workspace_bytes(const hrkan_net_desc *net, int32_t n_inst,
                               const hrkan_points *pts /* host [n_inst] */,
                               size_t *bytes /* host */);
int hrkan_plan_create(hrkan_plan **out, const hrkan_net_desc *net, int32_t n_inst,
                      const hrkan_pde_desc *pdes, const void *W_packed, const hrkan_points *pts,
                      double *loss_out, void *gW_packed, void *ws, size_t ws_bytes,
                      hipStream_t stream);
/* Enqueue one batched step (one graph launch) on stream. */
int hrkan_plan_execute(hrkan_plan *plan, hipStream_t stream);
/* Tile configuration the autotuner chose (host ints: points per tile, work
 * items per persistent block); either pointer may be NULL. */
int hrkan_plan_config(const hrkan_plan *plan, int32_t *tile_points, int32_t *blocks);
/* Whether the plan's configuration came from the autotune cache (host int,
 * 1 or 0) and the step time (ms, host double) measured for it when it was
 * tuned; either pointer may be NULL. */
int hrkan_plan_autotune_info(const hrkan_plan *plan, int32_t *from_cache, double *step_ms);
void hrkan_plan_destroy(hrkan_plan *plan);

/* Read and clear the device status word kept in ws (synchronises stream).
 * *flags (host) receives a set of HRKAN_STATUS_* bits. */
int hrkan_read_status(void *ws, size_t ws_bytes, hipStream_t stream, uint32_t *flags);

/* Static description of a status code, and the detailed message of the last
 * failing call on this host thread (empty if none). */
const char *hrkan_status_string(int code);
const char *hrkan_last_error(void);

/* Kernel timing, for benchmarks. While enabled (on != 0), every kernel the
 * library launches is bracketed by two HIP events recorded on the stream it
 * runs on. hrkan_profile_read waits for those events, writes one line
 * "<kernel> <launches> <total_ms>\n" per kernel name into buf (host,
 * NUL-terminated, truncated to buflen) and forgets the recorded events. The
 * names are "<stage>_l<layer>" for per-layer kernels (stage fwd, dx, dw,
 * reduce) and plain names otherwise. Not thread-safe; off by default. */
int hrkan_profile_enable(int32_t on);
int hrkan_profile_read(char *buf, size_t buflen);

/* ABI version (major * 100 + minor). */
int hrkan_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HRKAN_H */
