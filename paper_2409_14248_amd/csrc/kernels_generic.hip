// kernels_generic.hip -- the FP32 instances of the vector-ALU layer kernels
// (generic_layers.h), and the reduction, Adam, residual and loss kernels of
// the HRKAN step for both array types.
#include "generic_layers.h"

namespace hrk {

int dw_generic_splits(int64_t n, LayerShape ls)
{
    const int64_t tiles = (int64_t)((ls.win + DW_IB - 1) / DW_IB) * ((ls.wout + DW_JB - 1) / DW_JB);
    int64_t s = (2048 + tiles - 1) / tiles;
    const int64_t maxs = (n + 4 * DW_TP - 1) / (4 * DW_TP);   // >= 128 points per slice
    if (s > maxs) s = maxs;
    if (s < 1) s = 1;
    if (s > 1024) s = 1024;
    return (int)s;
}

size_t dw_generic_lds_bytes(int elem, int C, int nb)
{
    (void)nb;
    const int tp = C > 5 ? 8 : DW_TP;
    return (size_t)elem * (DW_IB * NBMAX * DW_JB + DW_IB * KBMAX * C * tp + C * DW_JB * (tp + 1)) +
           sizeof(int) * DW_IB * tp;
}


// ---------------------------------------------------------------------------
// out[e] (+)= sum over slices. A block takes 32 elements; its 8 slice lanes
// each sum a fixed residue class of slices in double, then one thread adds
// the 8 lane sums in order: a fixed summation order for every element.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over the block (256 threads = 4 waves), fixed order; valid in
// thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// Loss from the per-block partials (interior squared residuals, boundary
// squared misfits), one block of NT threads: L = alpha L_pde + L_bc.
__device__ __forceinline__ void loss_block(const double *__restrict__ partials, int nblk, double inv_int,
                                           double inv_bc, double alpha, double *__restrict__ loss_out,
                                           uint32_t *__restrict__ status, double *sh)
{
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += NT) {
        a += partials[2 * i];
        b += partials[2 * i + 1];
    }
    const double sa = block_sum(a, sh);
    const double sb = block_sum(b, sh);
    if (threadIdx.x == 0) {
        const double lpde = sa * inv_int, lbc = sb * inv_bc;
        const double L = alpha * lpde + lbc;
        loss_out[0] = L;
        loss_out[1] = lpde;
        loss_out[2] = lbc;
        if (!isfinite(L)) status[0] |= HRKAN_STATUS_NONFINITE;
    }
}

constexpr int RD_EB = 32, RD_SL = NT / RD_EB;

// Every layer's reduction in one launch: blocks [blk0[l], blk0[l+1]) take
// layer l. A block takes RD_EB elements: its RD_SL slice lanes add slices
// sl, sl + RD_SL, ... in increasing order (8 loads in flight) in FP64, and
// the lanes' sums are added in lane order, so each element has one fixed
// summation order.
template <typename T>
__global__ __launch_bounds__(NT) void k_reduce_layers(ReduceTable<T> tab, int accumulate)
{
    __shared__ double sh[RD_SL][RD_EB];
    if (tab.loss_part && (int64_t)blockIdx.x == tab.blk0[tab.L]) {
        loss_block(tab.loss_part, tab.loss_nblk, tab.inv_int, tab.inv_bc, tab.alpha, tab.loss_out,
                   tab.status, &sh[0][0]);
        return;
    }
    int l = 0;
    while (l + 1 < tab.L && (int64_t)blockIdx.x >= tab.blk0[l + 1]) ++l;
    const T *part = tab.part[l];
    const int nsplit = tab.nsplit[l];
    const int64_t count = tab.count[l];
    T *out = tab.out[l];
    const int el = threadIdx.x % RD_EB, sl = threadIdx.x / RD_EB;
    const int64_t e = ((int64_t)blockIdx.x - tab.blk0[l]) * RD_EB + el;
    double s = 0.0;
    if (e < count) {
        int k = sl;
        for (; k + 7 * RD_SL < nsplit; k += 8 * RD_SL) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(k + u * RD_SL) * count + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += (double)v[u];
        }
        for (; k < nsplit; k += RD_SL) s += (double)part[(int64_t)k * count + e];
    }
    sh[sl][el] = s;
    __syncthreads();
    if (sl == 0 && e < count) {
        double t = accumulate ? (double)out[e] : 0.0;
        for (int k = 0; k < RD_SL; ++k) t += sh[k][el];
        out[e] = (T)t;
    }
}

// Adam update of every layer's weights (one launch): with t = *tdev + 1,
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
//   W -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
// blocks [blk0[l], blk0[l+1]) take layer l. The step count lives in device
// memory (k_adam_count advances it), so a captured step replays correctly.
template <typename T>
__global__ __launch_bounds__(NT) void k_adam(AdamTable<T> tab, const int64_t *__restrict__ tdev, double lr,
                                             double b1, double b2, double eps)
{
    int l = 0;
    while (l + 1 < tab.L && (int64_t)blockIdx.x >= tab.blk0[l + 1]) ++l;
    const int64_t e = ((int64_t)blockIdx.x - tab.blk0[l]) * NT + threadIdx.x;
    if (e >= tab.count[l]) return;
    const double t = (double)(*tdev + 1);
    const double c1 = 1.0 / (1.0 - pow(b1, t)), c2 = 1.0 / (1.0 - pow(b2, t));
    const T g = tab.g[l][e];
    const T m = (T)b1 * tab.m[l][e] + (T)(1.0 - b1) * g;
    const T v = (T)b2 * tab.v[l][e] + (T)(1.0 - b2) * g * g;
    tab.m[l][e] = m;
    tab.v[l][e] = v;
    tab.W[l][e] -= (T)lr * (m * (T)c1) / (sqrt(v * (T)c2) + (T)eps);
}

__global__ void k_adam_count(int64_t *tdev) { tdev[0] += 1; }

template <typename T>
hipError_t launch_adam(AdamTable<T> tab, int64_t *tdev, double lr, double b1, double b2, double eps,
                       hipStream_t st)
{
    int64_t b = 0;
    for (int l = 0; l < tab.L; ++l) {
        tab.blk0[l] = b;
        b += (tab.count[l] + NT - 1) / NT;
    }
    tab.blk0[tab.L] = b;
    if (b > 0) k_adam<T><<<(unsigned)b, NT, 0, st>>>(tab, tdev, lr, b1, b2, eps);
    k_adam_count<<<1, 1, 0, st>>>(tdev);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce_layers(ReduceTable<T> tab, int accumulate, hipStream_t st)
{
    int64_t b = 0;
    for (int l = 0; l < tab.L; ++l) {
        tab.blk0[l] = b;
        b += (tab.count[l] + RD_EB - 1) / RD_EB;
    }
    tab.blk0[tab.L] = b;
    if (tab.loss_part) ++b;
    if (b == 0) return hipSuccess;
    k_reduce_layers<T><<<(unsigned)b, NT, 0, st>>>(tab, accumulate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// residual, seeds and per-block loss partials
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T sin_pi(T v);
template <> __device__ __forceinline__ double sin_pi<double>(double v) { return sinpi(v); }
template <> __device__ __forceinline__ float sin_pi<float>(float v) { return sinpif(v); }
template <typename T> __device__ __forceinline__ T cos_pi(T v);
template <> __device__ __forceinline__ double cos_pi<double>(double v) { return cospi(v); }
template <> __device__ __forceinline__ float cos_pi<float>(float v) { return cospif(v); }

// Coefficients of the PDE in the array type.
template <typename T>
struct PdeK {
    T nu, adv;
    T c0, cx[HRKAN_MAX_ORDER], cy[HRKAN_MAX_ORDER];   // linear kind
    int ox, oy;                                        // its jet orders
};

template <typename T>
PdeK<T> pde_k(const PdeParams &p)
{
    PdeK<T> k{};
    k.nu = (T)p.nu;
    k.adv = (T)p.adv;
    k.c0 = (T)p.c0;
    for (int i = 0; i < HRKAN_MAX_ORDER; ++i) {
        k.cx[i] = (T)p.cx[i];
        k.cy[i] = (T)p.cy[i];
    }
    k.ox = p.ox;
    k.oy = p.oy;
    return k;
}

// d^k/dt^k sin(pi t) = pi^k times sin, cos, -sin, -cos (pi t) for k mod 4 =
// 0, 1, 2, 3, from s = sin(pi t), c = cos(pi t).
template <typename T>
__device__ __forceinline__ T dsin_pi(int k, T s, T c)
{
    T pk = T(1);
    for (int i = 0; i < k; ++i) pk *= T(3.14159265358979323846);
    const T v = (k & 1) ? c : s;
    return (k & 2) ? -pk * v : pk * v;
}

// Residual of the linear kind at one point and its seeds: r is the operator
// applied to u minus the operator applied to u* = sin(pi x) sin(pi y),
// channel by channel; the seed of a channel is rho times its coefficient.
// jets/seed are [C][stride] with C = 1 + ox + oy.
template <typename T>
__device__ __forceinline__ T linear_residual(const PdeK<T> &k, const T *__restrict__ jets, int64_t stride, int64_t p,
                                             T x, T y)
{
    const T sx = sin_pi(x), sy = sin_pi(y), cx = cos_pi(x), cy = cos_pi(y);
    T r = k.c0 * (jets[p] - sx * sy);
    for (int q = 1; q <= k.ox; ++q) r += k.cx[q - 1] * (jets[q * stride + p] - dsin_pi(q, sx, cx) * sy);
    for (int q = 1; q <= k.oy; ++q) r += k.cy[q - 1] * (jets[(k.ox + q) * stride + p] - sx * dsin_pi(q, sy, cy));
    return r;
}

template <typename T>
__device__ __forceinline__ void linear_seed(const PdeK<T> &k, T rho, T *__restrict__ seed, int64_t stride, int64_t p)
{
    seed[p] = rho * k.c0;
    for (int q = 1; q <= k.ox; ++q) seed[q * stride + p] = rho * k.cx[q - 1];
    for (int q = 1; q <= k.oy; ++q) seed[(k.ox + q) * stride + p] = rho * k.cy[q - 1];
}

// Points 0..n_int-1 are interior (residual), n_int..n_int+n_bc-1 boundary.
template <typename T, int KIND>
__global__ __launch_bounds__(NT) void k_residual(const T *__restrict__ jets,
                                                 const T *__restrict__ x_int, int64_t n_int,
                                                 const T *__restrict__ u_bc,
                                                 const T *__restrict__ g_bc, int64_t n_bc,
                                                 T *__restrict__ r_out, T *__restrict__ seed_int,
                                                 T *__restrict__ seed_bc,
                                                 double *__restrict__ partials, PdeK<T> pk,
                                                 T sc_int, T sc_bc)
{
    const T nu = pk.nu, adv = pk.adv;
    __shared__ double sh[4];
    const int64_t p = (int64_t)blockIdx.x * NT + threadIdx.x;
    double e_pde = 0.0, e_bc = 0.0;
    if (p < n_int) {
        T r;
        if constexpr (KIND == 0) {
            // Poisson: jets (u, ux, uxx, uy, uyy); r = uxx + uyy + 2 pi^2 sin(pi x) sin(pi y)
            const T uxx = jets[2 * n_int + p], uyy = jets[4 * n_int + p];
            const T x = x_int[2 * p], y = x_int[2 * p + 1];
            const T f = T(2.0 * 9.869604401089358) * sin_pi(x) * sin_pi(y);
            r = uxx + uyy + f;
            if (seed_int) {
                const T rho = sc_int * r;            // dL/dr = 2 alpha r / n_int
                seed_int[0 * n_int + p] = T(0);
                seed_int[1 * n_int + p] = T(0);
                seed_int[2 * n_int + p] = rho;
                seed_int[3 * n_int + p] = T(0);
                seed_int[4 * n_int + p] = rho;
            }
        } else if constexpr (KIND == 1) {
            // Burgers: jets (u, ux, uxx, ut); r = ut + adv u ux - nu uxx
            const T u = jets[p], ux = jets[n_int + p], uxx = jets[2 * n_int + p],
                    ut = jets[3 * n_int + p];
            r = ut + adv * u * ux - nu * uxx;
            if (seed_int) {
                const T rho = sc_int * r;
                seed_int[0 * n_int + p] = rho * adv * ux;
                seed_int[1 * n_int + p] = rho * adv * u;
                seed_int[2 * n_int + p] = -rho * nu;
                seed_int[3 * n_int + p] = rho;
            }
        } else {
            // linear, jets (u, x-derivatives 1..ox, y-derivatives 1..oy)
            r = linear_residual(pk, jets, n_int, p, x_int[2 * p], x_int[2 * p + 1]);
            if (seed_int) linear_seed(pk, sc_int * r, seed_int, n_int, p);
        }
        if (r_out) r_out[p] = r;
        e_pde = (double)r * (double)r;
    } else if (p < n_int + n_bc) {
        const int64_t q = p - n_int;
        const T d = u_bc[q] - g_bc[q];
        if (seed_bc) seed_bc[q] = sc_bc * d;     // dL/du = 2 (u - g) / n_bc
        e_bc = (double)d * (double)d;
    }
    const double s0 = block_sum(e_pde, sh);
    const double s1 = block_sum(e_bc, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s0;
        partials[2 * blockIdx.x + 1] = s1;
    }
}

int residual_blocks(int64_t n_int, int64_t n_bc)
{
    // room for the two sets in launches of their own
    const int64_t b = (n_int + NT - 1) / NT + (n_bc + NT - 1) / NT;
    return (int)(b < 1 ? 1 : b);
}
int residual_blocks_of(int64_t n) { return (int)((n + NT - 1) / NT); }

template <typename T>
hipError_t launch_residual(const PdeParams &pde, int C, const T *jets, const T *x_int,
                           int64_t n_int, const T *u_bc, const T *g_bc, int64_t n_bc, T *r_out,
                           T *seed_int, T *seed_bc, double *partials, int nblk, hipStream_t st)
{
    (void)C;
    const T sc_int = n_int > 0 ? (T)(2.0 * pde.alpha / (double)n_int) : T(0);
    const T sc_bc = n_bc > 0 ? (T)(2.0 / (double)n_bc) : T(0);
    const PdeK<T> pk = pde_k<T>(pde);
    if (pde.kind == HRKAN_POISSON2D)
        k_residual<T, 0><<<nblk, NT, 0, st>>>(jets, x_int, n_int, u_bc, g_bc, n_bc, r_out, seed_int,
                                              seed_bc, partials, pk, sc_int, sc_bc);
    else if (pde.kind == HRKAN_BURGERS1D)
        k_residual<T, 1><<<nblk, NT, 0, st>>>(jets, x_int, n_int, u_bc, g_bc, n_bc, r_out, seed_int,
                                              seed_bc, partials, pk, sc_int, sc_bc);
    else
        k_residual<T, 2><<<nblk, NT, 0, st>>>(jets, x_int, n_int, u_bc, g_bc, n_bc, r_out, seed_int,
                                              seed_bc, partials, pk, sc_int, sc_bc);
    return hipGetLastError();
}

// One block: each thread sums a fixed strided subset of the block partials,
// then a fixed tree combines the threads.
__global__ __launch_bounds__(NT) void k_loss_final(const double *__restrict__ partials, int nblk,
                                                   double inv_int, double inv_bc, double alpha,
                                                   double *__restrict__ loss_out,
                                                   uint32_t *__restrict__ status)
{
    __shared__ double sh[4];
    loss_block(partials, nblk, inv_int, inv_bc, alpha, loss_out, status, sh);
}

// One point set of both: the interior points, then the boundary points
// (interleaved coordinate pairs).
template <typename T>
__global__ __launch_bounds__(NT) void k_concat_points(const T *__restrict__ x_int, int64_t n_int,
                                                      const T *__restrict__ x_bc, int64_t n_bc,
                                                      T *__restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e < 2 * n_int)
        out[e] = x_int[e];
    else if (e < 2 * (n_int + n_bc))
        out[e] = x_bc[e - 2 * n_int];
}

template <typename T>
hipError_t launch_concat_points(const T *x_int, int64_t n_int, const T *x_bc, int64_t n_bc, T *out,
                                hipStream_t st)
{
    const int64_t m = 2 * (n_int + n_bc);
    if (m == 0) return hipSuccess;
    k_concat_points<T><<<(unsigned)((m + NT - 1) / NT), NT, 0, st>>>(x_int, n_int, x_bc, n_bc, out);
    return hipGetLastError();
}

// Residual, misfit and seeds of the merged set: jets and seeds are
// [C][n_int + n_bc]; points p < n_int are interior (as k_residual), the rest
// boundary points, whose seed is the misfit's on the value channel and zero
// on the others (their derivative channels carry no loss term).
template <typename T, int KIND>
__global__ __launch_bounds__(NT) void k_residual_merged(const T *__restrict__ jets,
                                                        const T *__restrict__ x_int, int64_t n_int,
                                                        const T *__restrict__ g_bc, int64_t n_bc, int C,
                                                        T *__restrict__ seed,
                                                        double *__restrict__ partials, PdeK<T> pk,
                                                        T sc_int, T sc_bc)
{
    const T nu = pk.nu, adv = pk.adv;
    __shared__ double sh[4];
    const int64_t ns = n_int + n_bc;
    const int64_t p = (int64_t)blockIdx.x * NT + threadIdx.x;
    double e_pde = 0.0, e_bc = 0.0;
    if (p < n_int) {
        T r;
        if constexpr (KIND == 0) {
            const T uxx = jets[2 * ns + p], uyy = jets[4 * ns + p];
            const T x = x_int[2 * p], y = x_int[2 * p + 1];
            const T f = T(2.0 * 9.869604401089358) * sin_pi(x) * sin_pi(y);
            r = uxx + uyy + f;
            const T rho = sc_int * r;
            seed[0 * ns + p] = T(0);
            seed[1 * ns + p] = T(0);
            seed[2 * ns + p] = rho;
            seed[3 * ns + p] = T(0);
            seed[4 * ns + p] = rho;
        } else if constexpr (KIND == 1) {
            const T u = jets[p], ux = jets[ns + p], uxx = jets[2 * ns + p], ut = jets[3 * ns + p];
            r = ut + adv * u * ux - nu * uxx;
            const T rho = sc_int * r;
            seed[0 * ns + p] = rho * adv * ux;
            seed[1 * ns + p] = rho * adv * u;
            seed[2 * ns + p] = -rho * nu;
            seed[3 * ns + p] = rho;
        } else {
            r = linear_residual(pk, jets, ns, p, x_int[2 * p], x_int[2 * p + 1]);
            linear_seed(pk, sc_int * r, seed, ns, p);
        }
        e_pde = (double)r * (double)r;
    } else if (p < ns) {
        const T d = jets[p] - g_bc[p - n_int];
        seed[p] = sc_bc * d;
        for (int c = 1; c < C; ++c) seed[c * ns + p] = T(0);
        e_bc = (double)d * (double)d;
    }
    const double s0 = block_sum(e_pde, sh);
    const double s1 = block_sum(e_bc, sh);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s0;
        partials[2 * blockIdx.x + 1] = s1;
    }
}

template <typename T>
hipError_t launch_residual_merged(const PdeParams &pde, int C, const T *jets, const T *x_int, int64_t n_int,
                                  const T *g_bc, int64_t n_bc, T *seed, double *partials, int nblk,
                                  hipStream_t st)
{
    const T sc_int = n_int > 0 ? (T)(2.0 * pde.alpha / (double)n_int) : T(0);
    const T sc_bc = n_bc > 0 ? (T)(2.0 / (double)n_bc) : T(0);
    const PdeK<T> pk = pde_k<T>(pde);
    if (pde.kind == HRKAN_POISSON2D)
        k_residual_merged<T, 0><<<nblk, NT, 0, st>>>(jets, x_int, n_int, g_bc, n_bc, C, seed, partials, pk,
                                                     sc_int, sc_bc);
    else if (pde.kind == HRKAN_BURGERS1D)
        k_residual_merged<T, 1><<<nblk, NT, 0, st>>>(jets, x_int, n_int, g_bc, n_bc, C, seed, partials, pk,
                                                     sc_int, sc_bc);
    else
        k_residual_merged<T, 2><<<nblk, NT, 0, st>>>(jets, x_int, n_int, g_bc, n_bc, C, seed, partials, pk,
                                                     sc_int, sc_bc);
    return hipGetLastError();
}

hipError_t launch_loss_final(const double *partials, int nblk, int64_t n_int, int64_t n_bc,
                             double alpha, double *loss_out, uint32_t *status, hipStream_t st)
{
    k_loss_final<<<1, NT, 0, st>>>(partials, nblk, n_int > 0 ? 1.0 / (double)n_int : 0.0,
                                   n_bc > 0 ? 1.0 / (double)n_bc : 0.0, alpha, loss_out, status);
    return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_fwd_generic<float>(ChanCfg, bool, const float *, const float *, float *, int64_t,
                                              LayerShape, const GridP<float> &, hipStream_t);
template hipError_t launch_dx_generic<float>(ChanCfg, const float *, const float *, const float *, float *,
                                             int64_t, LayerShape, const GridP<float> &, hipStream_t);
template hipError_t launch_dw_generic<float>(ChanCfg, bool, const float *, const float *, float *, int,
                                             int64_t, LayerShape, const GridP<float> &, hipStream_t);

#define HRK_INST(T)                                                                              \
    template hipError_t launch_reduce_layers<T>(ReduceTable<T>, int, hipStream_t);                 \
    template hipError_t launch_adam<T>(AdamTable<T>, int64_t *, double, double, double, double, hipStream_t); \
    template hipError_t launch_residual<T>(const PdeParams &, int, const T *, const T *, int64_t, \
                                           const T *, const T *, int64_t, T *, T *, T *,         \
                                           double *, int, hipStream_t);                          \
    template hipError_t launch_concat_points<T>(const T *, int64_t, const T *, int64_t, T *, hipStream_t); \
    template hipError_t launch_residual_merged<T>(const PdeParams &, int, const T *, const T *, int64_t, \
                                                  const T *, int64_t, T *, double *, int, hipStream_t);
HRK_INST(float)
HRK_INST(double)

}  // namespace hrk
