// kernels_generic.hip -- vector-ALU kernels of the HRKAN step for any array
// type T (double or float): one KAN layer forward with jets, its reverse to
// the input jets, its weight gradient, and the residual / loss kernels.
//
// Only the k+1 basis functions whose support contains z are evaluated (the
// others are zero by the ReLU factors of Eq. 2); their values are staged in
// LDS once per (point, input) and reused by every output column.
//
// Jet arrays are [C][w][n] (channel, feature, point): consecutive threads
// touch consecutive points.
#include "internal.h"

namespace hrk {

constexpr int NT = 256;      // threads per block
constexpr int TP = 64;       // points per block (forward, input bars)
constexpr int KBMAX = 4;     // at most k+1 = 4 live basis functions per input
constexpr int NBMAX = 32;    // n_b limit of the weight-gradient kernel
constexpr int NOQ = -(1 << 20);

#define HRK_CH_SWITCH(ch, ...)                                   \
    switch ((ch).o0 * 3 + (ch).o1) {                              \
    case 0: { constexpr int O0 = 0, O1 = 0; __VA_ARGS__; } break;        \
    case 4: { constexpr int O0 = 1, O1 = 1; __VA_ARGS__; } break;        \
    case 6: { constexpr int O0 = 2, O1 = 0; __VA_ARGS__; } break;        \
    case 7: { constexpr int O0 = 2, O1 = 1; __VA_ARGS__; } break;        \
    case 8: { constexpr int O0 = 2, O1 = 2; __VA_ARGS__; } break;        \
    default: return hipErrorInvalidValue;                         \
    }

// Load the jets of input feature i at point p (layer 0 reads x directly).
template <typename T, int O0, int O1, bool FIRST>
__device__ __forceinline__ void load_jets(const T *__restrict__ zin, int64_t n, int win, int i,
                                          int64_t p, T *zj)
{
    constexpr int C = Ch<O0, O1>::C;
    if constexpr (FIRST) {
        input_jets<T, O0, O1>(zin, p, i, zj);
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) zj[c] = zin[((int64_t)c * win + i) * n + p];
    }
}

// ---------------------------------------------------------------------------
// forward: zout[c][j][p] = sum_i sum_b W[i*nb+b][j] * A_c(p, i, b)
// grid (ceil(n/64), ceil(N/32)); each thread owns one point and 8 outputs.
// ---------------------------------------------------------------------------
template <typename T, int O0, int O1, bool FIRST>
__global__ __launch_bounds__(NT) void k_fwd_generic(const T *__restrict__ zin,
                                                    const T *__restrict__ W,
                                                    T *__restrict__ zout, int64_t n, int win,
                                                    int N, GridP<T> g)
{
    constexpr int C = Ch<O0, O1>::C;
    constexpr int KI = 8;                 // inputs staged per pass
    constexpr int JS = NT / TP;           // output sub-columns per point
    constexpr int NJ = 8;                 // outputs per thread
    __shared__ int sq[KI][TP];
    __shared__ T sA[KI][KBMAX][C][TP];

    const int tid = threadIdx.x, tp = tid % TP, js = tid / TP;
    const int64_t p0 = (int64_t)blockIdx.x * TP;
    const int j0 = blockIdx.y * (NJ * JS);
    const int kb = g.k + 1;
    T acc[NJ][C];
#pragma unroll
    for (int r = 0; r < NJ; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[r][c] = T(0);

    for (int i0 = 0; i0 < win; i0 += KI) {
        for (int it = tid; it < KI * TP; it += NT) {
            const int il = it / TP, pp = it % TP, i = i0 + il;
            const int64_t p = p0 + pp;
            T zj[C];
            T zt = T(0);
            int q = NOQ;
            if (i < win && p < n) {
                load_jets<T, O0, O1, FIRST>(zin, n, win, i, p, zj);
                zt = zeta_of(g, zj[0]);
                q = interval_of(g, zt);
            }
            sq[il][pp] = q;
#pragma unroll
            for (int t = 0; t < KBMAX; ++t) {
                T A[C];
                if (t < kb && q != NOQ) {
                    T v[3];
                    hr_bump<T, 2>(g, zt, q + t, v);
                    features<T, O0, O1>(v, zj, A);
                } else {
#pragma unroll
                    for (int c = 0; c < C; ++c) A[c] = T(0);
                }
#pragma unroll
                for (int c = 0; c < C; ++c) sA[il][t][c][pp] = A[c];
            }
        }
        __syncthreads();
        const int ilmax = min(KI, win - i0);
        for (int il = 0; il < ilmax; ++il) {
            const int q = sq[il][tp];
#pragma unroll
            for (int t = 0; t < KBMAX; ++t) {
                const int b = q + t;
                if (t >= kb || b < 0 || b >= g.nb) continue;
                const T *wr = W + (size_t)((i0 + il) * g.nb + b) * N;
                T a[C];
#pragma unroll
                for (int c = 0; c < C; ++c) a[c] = sA[il][t][c][tp];
#pragma unroll
                for (int r = 0; r < NJ; ++r) {
                    const int j = j0 + js + JS * r;
                    if (j < N) {
                        const T w = wr[j];
#pragma unroll
                        for (int c = 0; c < C; ++c) acc[r][c] += a[c] * w;
                    }
                }
            }
        }
        __syncthreads();
    }
    const int64_t p = p0 + tp;
    if (p < n) {
#pragma unroll
        for (int r = 0; r < NJ; ++r) {
            const int j = j0 + js + JS * r;
            if (j < N)
#pragma unroll
                for (int c = 0; c < C; ++c) zout[((int64_t)c * N + j) * n + p] = acc[r][c];
        }
    }
}

template <typename T>
hipError_t launch_fwd_generic(ChanCfg ch, bool first, const T *zin, const T *W, T *zout,
                              int64_t n, LayerShape ls, const GridP<T> &g, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + TP - 1) / TP), (unsigned)((ls.wout + 31) / 32));
    HRK_CH_SWITCH(ch, {
        if (first)
            k_fwd_generic<T, O0, O1, true><<<grid, NT, 0, st>>>(zin, W, zout, n, ls.win, ls.wout, g);
        else
            k_fwd_generic<T, O0, O1, false><<<grid, NT, 0, st>>>(zin, W, zout, n, ls.win, ls.wout, g);
    });
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reverse to the input jets:
//   Ab_c(p,i,b) = sum_j W[i*nb+b][j] * ybar[c][j][p]   (live b only)
//   zbar[.][i][p] = adjoint of the features through v, v', v'', v'''
// grid (ceil(n/64), ceil(win/8)); each thread owns one point and 2 inputs.
// ---------------------------------------------------------------------------
template <typename T, int O0, int O1>
__global__ __launch_bounds__(NT) void k_dx_generic(const T *__restrict__ zin,
                                                   const T *__restrict__ ybar,
                                                   const T *__restrict__ W,
                                                   T *__restrict__ zbar, int64_t n, int win,
                                                   int N, GridP<T> g)
{
    constexpr int C = Ch<O0, O1>::C;
    constexpr int RI = 2;
    constexpr int IS = NT / TP;
    constexpr int JC = 32;
    __shared__ T sY[C][JC][TP];

    const int tid = threadIdx.x, tp = tid % TP, ig = tid / TP;
    const int64_t p0 = (int64_t)blockIdx.x * TP, p = p0 + tp;
    const int ib = blockIdx.y * (RI * IS);
    const int kb = g.k + 1;
    T zj[RI][C];
    T zt[RI];
    int q[RI];
    T Ab[RI][KBMAX][C];
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int i = ib + ig + IS * r;
        q[r] = NOQ;
        zt[r] = T(0);
#pragma unroll
        for (int c = 0; c < C; ++c) zj[r][c] = T(0);
        if (i < win && p < n) {
            load_jets<T, O0, O1, false>(zin, n, win, i, p, zj[r]);
            zt[r] = zeta_of(g, zj[r][0]);
            q[r] = interval_of(g, zt[r]);
        }
#pragma unroll
        for (int t = 0; t < KBMAX; ++t)
#pragma unroll
            for (int c = 0; c < C; ++c) Ab[r][t][c] = T(0);
    }
    for (int j0 = 0; j0 < N; j0 += JC) {
        for (int it = tid; it < C * JC * TP; it += NT) {
            const int c = it / (JC * TP), rem = it % (JC * TP), jj = rem / TP, pp = rem % TP;
            const int j = j0 + jj;
            const int64_t pq = p0 + pp;
            sY[c][jj][pp] = (j < N && pq < n) ? ybar[((int64_t)c * N + j) * n + pq] : T(0);
        }
        __syncthreads();
        const int jmax = min(JC, N - j0);
        for (int jj = 0; jj < jmax; ++jj) {
            T y[C];
#pragma unroll
            for (int c = 0; c < C; ++c) y[c] = sY[c][jj][tp];
#pragma unroll
            for (int r = 0; r < RI; ++r) {
                const int i = ib + ig + IS * r;
#pragma unroll
                for (int t = 0; t < KBMAX; ++t) {
                    const int b = q[r] + t;
                    if (t >= kb || b < 0 || b >= g.nb) continue;
                    const T w = W[(size_t)(i * g.nb + b) * N + j0 + jj];
#pragma unroll
                    for (int c = 0; c < C; ++c) Ab[r][t][c] += w * y[c];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RI; ++r) {
        const int i = ib + ig + IS * r;
        if (i >= win || p >= n) continue;
        T zb[C];
#pragma unroll
        for (int c = 0; c < C; ++c) zb[c] = T(0);
#pragma unroll
        for (int t = 0; t < KBMAX; ++t) {
            if (t >= kb) continue;
            T v[4];
            hr_bump<T, 3>(g, zt[r], q[r] + t, v);
            features_adjoint<T, O0, O1>(v, zj[r], Ab[r][t], zb);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) zbar[((int64_t)c * win + i) * n + p] = zb[c];
    }
}

template <typename T>
hipError_t launch_dx_generic(ChanCfg ch, const T *zin, const T *ybar, const T *W, T *zbar,
                             int64_t n, LayerShape ls, const GridP<T> &g, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + TP - 1) / TP), (unsigned)((ls.win + 7) / 8));
    HRK_CH_SWITCH(ch, {
        k_dx_generic<T, O0, O1><<<grid, NT, 0, st>>>(zin, ybar, W, zbar, n, ls.win, ls.wout, g);
    });
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// weight gradient of one point slice:
//   part[s][(i*nb+b)*N + j] = sum_{p in slice s} sum_c A_c(p,i,b) * ybar[c][j][p]
// grid (ceil(win/8), ceil(N/32), nsplit); the block accumulates its
// 8 x nb x 32 tile in LDS, each (i, j) column owned by one thread, so the
// sum over points has a fixed order.
// ---------------------------------------------------------------------------
constexpr int DW_IB = 8, DW_JB = 32, DW_TP = 32;

template <typename T, int O0, int O1, bool FIRST>
__global__ __launch_bounds__(NT) void k_dw_generic(const T *__restrict__ zin,
                                                   const T *__restrict__ ybar,
                                                   T *__restrict__ part, int64_t n, int win,
                                                   int N, int nsplit, GridP<T> g)
{
    constexpr int C = Ch<O0, O1>::C;
    __shared__ T gacc[DW_IB * NBMAX * DW_JB];
    __shared__ int sq[DW_IB][DW_TP];
    __shared__ T sA[DW_IB][KBMAX][C][DW_TP];
    __shared__ T sY[C][DW_JB][DW_TP + 1];

    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * DW_IB, j0 = blockIdx.y * DW_JB, split = blockIdx.z;
    const int nb = g.nb, kb = g.k + 1;
    const int64_t per = ((n + nsplit - 1) / nsplit + DW_TP - 1) / DW_TP * DW_TP;
    const int64_t ps = (int64_t)split * per;
    const int64_t pe = min(n, ps + per);
    for (int it = tid; it < DW_IB * nb * DW_JB; it += NT) gacc[it] = T(0);
    const int il = tid / DW_JB, jj = tid % DW_JB;

    for (int64_t pc = ps; pc < pe; pc += DW_TP) {
        for (int it = tid; it < DW_IB * DW_TP; it += NT) {
            const int il2 = it / DW_TP, pp = it % DW_TP, i = i0 + il2;
            const int64_t p = pc + pp;
            T zj[C];
            T zt = T(0);
            int q = NOQ;
            if (i < win && p < pe) {
                load_jets<T, O0, O1, FIRST>(zin, n, win, i, p, zj);
                zt = zeta_of(g, zj[0]);
                q = interval_of(g, zt);
            }
            sq[il2][pp] = q;
#pragma unroll
            for (int t = 0; t < KBMAX; ++t) {
                T A[C];
                if (t < kb && q != NOQ) {
                    T v[3];
                    hr_bump<T, 2>(g, zt, q + t, v);
                    features<T, O0, O1>(v, zj, A);
                } else {
#pragma unroll
                    for (int c = 0; c < C; ++c) A[c] = T(0);
                }
#pragma unroll
                for (int c = 0; c < C; ++c) sA[il2][t][c][pp] = A[c];
            }
        }
        for (int it = tid; it < C * DW_JB * DW_TP; it += NT) {
            const int c = it / (DW_JB * DW_TP), rem = it % (DW_JB * DW_TP);
            const int j2 = rem / DW_TP, pp = rem % DW_TP;
            const int j = j0 + j2;
            const int64_t p = pc + pp;
            sY[c][j2][pp] = (j < N && p < pe) ? ybar[((int64_t)c * N + j) * n + p] : T(0);
        }
        __syncthreads();
        for (int pp = 0; pp < DW_TP; ++pp) {
            const int q = sq[il][pp];
            if (q == NOQ) continue;
            T y[C];
#pragma unroll
            for (int c = 0; c < C; ++c) y[c] = sY[c][jj][pp];
#pragma unroll
            for (int t = 0; t < KBMAX; ++t) {
                const int b = q + t;
                if (t >= kb || b < 0 || b >= nb) continue;
                T s = T(0);
#pragma unroll
                for (int c = 0; c < C; ++c) s += sA[il][t][c][pp] * y[c];
                gacc[(il * nb + b) * DW_JB + jj] += s;
            }
        }
        __syncthreads();
    }
    const int64_t KN = (int64_t)win * nb * N;
    for (int it = tid; it < DW_IB * nb * DW_JB; it += NT) {
        const int il2 = it / (nb * DW_JB), rem = it % (nb * DW_JB), b = rem / DW_JB,
                  j2 = rem % DW_JB;
        const int i = i0 + il2, j = j0 + j2;
        if (i < win && j < N) part[split * KN + (int64_t)(i * nb + b) * N + j] = gacc[it];
    }
}

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
    return (size_t)elem * (DW_IB * NBMAX * DW_JB + DW_IB * KBMAX * C * DW_TP + C * DW_JB * (DW_TP + 1)) +
           sizeof(int) * DW_IB * DW_TP;
}

template <typename T>
hipError_t launch_dw_generic(ChanCfg ch, bool first, const T *zin, const T *ybar, T *part,
                             int nsplit, int64_t n, LayerShape ls, const GridP<T> &g,
                             hipStream_t st)
{
    if (ls.nb > NBMAX || g.k + 1 > KBMAX) return hipErrorInvalidValue;
    dim3 grid((unsigned)((ls.win + DW_IB - 1) / DW_IB), (unsigned)((ls.wout + DW_JB - 1) / DW_JB),
              (unsigned)nsplit);
    HRK_CH_SWITCH(ch, {
        if (first)
            k_dw_generic<T, O0, O1, true><<<grid, NT, 0, st>>>(zin, ybar, part, n, ls.win, ls.wout, nsplit, g);
        else
            k_dw_generic<T, O0, O1, false><<<grid, NT, 0, st>>>(zin, ybar, part, n, ls.win, ls.wout, nsplit, g);
    });
    return hipGetLastError();
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

// Points 0..n_int-1 are interior (residual), n_int..n_int+n_bc-1 boundary.
template <typename T, int KIND>
__global__ __launch_bounds__(NT) void k_residual(const T *__restrict__ jets,
                                                 const T *__restrict__ x_int, int64_t n_int,
                                                 const T *__restrict__ u_bc,
                                                 const T *__restrict__ g_bc, int64_t n_bc,
                                                 T *__restrict__ r_out, T *__restrict__ seed_int,
                                                 T *__restrict__ seed_bc,
                                                 double *__restrict__ partials, T alpha, T nu,
                                                 T adv, T sc_int, T sc_bc)
{
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
        } else {
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
    (void)alpha;
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
    if (pde.kind == 0)
        k_residual<T, 0><<<nblk, NT, 0, st>>>(jets, x_int, n_int, u_bc, g_bc, n_bc, r_out, seed_int,
                                              seed_bc, partials, (T)pde.alpha, (T)pde.nu,
                                              (T)pde.adv, sc_int, sc_bc);
    else
        k_residual<T, 1><<<nblk, NT, 0, st>>>(jets, x_int, n_int, u_bc, g_bc, n_bc, r_out, seed_int,
                                              seed_bc, partials, (T)pde.alpha, (T)pde.nu,
                                              (T)pde.adv, sc_int, sc_bc);
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
                                                        double *__restrict__ partials, T nu, T adv,
                                                        T sc_int, T sc_bc)
{
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
        } else {
            const T u = jets[p], ux = jets[ns + p], uxx = jets[2 * ns + p], ut = jets[3 * ns + p];
            r = ut + adv * u * ux - nu * uxx;
            const T rho = sc_int * r;
            seed[0 * ns + p] = rho * adv * ux;
            seed[1 * ns + p] = rho * adv * u;
            seed[2 * ns + p] = -rho * nu;
            seed[3 * ns + p] = rho;
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
    if (pde.kind == 0)
        k_residual_merged<T, 0><<<nblk, NT, 0, st>>>(jets, x_int, n_int, g_bc, n_bc, C, seed, partials,
                                                     (T)pde.nu, (T)pde.adv, sc_int, sc_bc);
    else
        k_residual_merged<T, 1><<<nblk, NT, 0, st>>>(jets, x_int, n_int, g_bc, n_bc, C, seed, partials,
                                                     (T)pde.nu, (T)pde.adv, sc_int, sc_bc);
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
#define HRK_INST(T)                                                                              \
    template hipError_t launch_fwd_generic<T>(ChanCfg, bool, const T *, const T *, T *, int64_t, \
                                              LayerShape, const GridP<T> &, hipStream_t);        \
    template hipError_t launch_dx_generic<T>(ChanCfg, const T *, const T *, const T *, T *,      \
                                             int64_t, LayerShape, const GridP<T> &, hipStream_t); \
    template hipError_t launch_dw_generic<T>(ChanCfg, bool, const T *, const T *, T *, int,      \
                                             int64_t, LayerShape, const GridP<T> &, hipStream_t); \
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
