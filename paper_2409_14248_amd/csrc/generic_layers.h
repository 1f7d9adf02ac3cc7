// generic_layers.h -- the vector-ALU layer kernels of the HRKAN step for any
// array type T (double or float) and any pair of jet orders: one KAN layer
// forward with jets, its reverse to the input jets and its weight gradient.
// Included by kernels_generic.hip (FP32 instances) and kernels_generic_f64.hip
// (FP64 instances), so that the two sets compile in parallel.
//
// Only the k+1 basis functions whose support contains z are evaluated (the
// others are zero by the ReLU factors of Eq. 2); their values are staged in
// LDS once per (point, input) and reused by every output column.
//
// Jet arrays are [C][w][n] (channel, feature, point): consecutive threads
// touch consecutive points.
#pragma once

#include "internal.h"

namespace hrk {

constexpr int NT = 256;      // threads per block
constexpr int TP = 64;       // points per block (forward, input bars)
constexpr int KBMAX = 4;     // at most k+1 = 4 live basis functions per input
constexpr int NBMAX = 32;    // n_b limit of the weight-gradient kernel
constexpr int NOQ = -(1 << 20);

// Every pair of jet orders (O0, O1) in 0..5 x 0..5.
#define HRK_GEN_CASE(a, b, ...) \
    case (a) * 8 + (b): { constexpr int O0 = a, O1 = b; __VA_ARGS__; } break;
#define HRK_GEN_ROW(a, ...)                                                                     \
    HRK_GEN_CASE(a, 0, __VA_ARGS__) HRK_GEN_CASE(a, 1, __VA_ARGS__) HRK_GEN_CASE(a, 2, __VA_ARGS__) \
    HRK_GEN_CASE(a, 3, __VA_ARGS__) HRK_GEN_CASE(a, 4, __VA_ARGS__) HRK_GEN_CASE(a, 5, __VA_ARGS__)
#define HRK_CH_SWITCH(ch, ...)                                                                  \
    switch ((ch).o0 * 8 + (ch).o1) {                                                            \
    HRK_GEN_ROW(0, __VA_ARGS__) HRK_GEN_ROW(1, __VA_ARGS__) HRK_GEN_ROW(2, __VA_ARGS__)           \
    HRK_GEN_ROW(3, __VA_ARGS__) HRK_GEN_ROW(4, __VA_ARGS__) HRK_GEN_ROW(5, __VA_ARGS__)           \
    default: return hipErrorInvalidValue;                                                       \
    }

// The bump's value and z-derivatives up to ND at zeta: the specialised
// forms for the jets of order at most two (ND <= 3), the general one above.
template <typename T, int O0, int O1, int EXTRA>
__device__ __forceinline__ void bump_for(const GridP<T> &g, T zeta, int b, T *v)
{
    using CH = Ch<O0, O1>;
    if constexpr (CH::LOW)
        hr_bump<T, 2 + EXTRA>(g, zeta, b, v);
    else
        hr_bump_n<T, CH::OM + EXTRA>(g, zeta, b, v);
}
template <int O0, int O1, int EXTRA>
constexpr int bump_len() { return Ch<O0, O1>::LOW ? 3 + EXTRA : Ch<O0, O1>::OM + 1 + EXTRA; }

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
    constexpr int KI = C > 5 ? 4 : 8;     // inputs staged per pass (LDS)
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
                    T v[bump_len<O0, O1, 0>()];
                    bump_for<T, O0, O1, 0>(g, zt, q + t, v);
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

// inputs per thread of the input-bar kernel (registers: C bars per live
// basis function and input)
template <int O0, int O1>
constexpr int dx_generic_ri() { return Ch<O0, O1>::C > 5 ? 1 : 2; }

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
    constexpr int RI = dx_generic_ri<O0, O1>();   // inputs per thread
    constexpr int IS = NT / TP;
    constexpr int JC = C > 5 ? 16 : 32;           // outputs staged per pass (LDS)
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
            T v[bump_len<O0, O1, 1>()];
            bump_for<T, O0, O1, 1>(g, zt[r], q[r] + t, v);
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
    HRK_CH_SWITCH(ch, {
        constexpr int per_block = dx_generic_ri<O0, O1>() * (NT / TP);
        dim3 grid((unsigned)((n + TP - 1) / TP), (unsigned)((ls.win + per_block - 1) / per_block));
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

// points per staged chunk of the weight-gradient kernel (LDS)
template <int O0, int O1>
constexpr int dw_generic_tp() { return Ch<O0, O1>::C > 5 ? 8 : DW_TP; }

template <typename T, int O0, int O1, bool FIRST>
__global__ __launch_bounds__(NT) void k_dw_generic(const T *__restrict__ zin,
                                                   const T *__restrict__ ybar,
                                                   T *__restrict__ part, int64_t n, int win,
                                                   int N, int nsplit, GridP<T> g)
{
    constexpr int C = Ch<O0, O1>::C;
    constexpr int DW_TP = dw_generic_tp<O0, O1>();
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
                    T v[bump_len<O0, O1, 0>()];
                    bump_for<T, O0, O1, 0>(g, zt, q + t, v);
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


}  // namespace hrk
