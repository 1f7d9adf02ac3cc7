// kernels_bs32.hip -- FP32 matrix-core kernels of one KAN layer.
//
// Forward and input-bar contractions use the 16-block 4x4x1 FP32 MFMA with
// ONE COLLOCATION POINT PER BLOCK: the block's 4 rows are the point's jet
// channels, its K = 1 is one live basis function (the HR basis of Eq. 2 has
// k+1 = 4 non-zero functions per input, the rest are zero by the ReLU
// factors), and its 4 columns are 4 outputs. Each block gathers the weight
// rows of its own point's live functions from LDS, so no zero of the basis
// tensor is ever multiplied.
//
// Lane roles inside a wave (64 lanes, 16 blocks): block b = lane >> 2 holds
// point p0 + b; s = lane & 3 is the block row (channel) for the A operand and
// the block column for the B operand and the result.
//
// The weight gradient is a dense 32x32x2 FP32 MFMA GEMM over points:
// gW[K x N] = A^T [K x (points*C)] * Ybar [(points*C) x N], with the A
// operand assembled from LDS-staged live features (zeros elsewhere).
#include <algorithm>

#include "internal.h"
#include "kernels_bs.h"

namespace hrk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int NT = 256;                 // threads per block (4 waves)
constexpr int PW = 16;                  // points per wave
constexpr int PB = 4 * PW;              // points per block
constexpr int LDS_W_BYTES = 112 * 1024; // weight staging budget

// Broadcast lane T of each quad (DPP quad_perm [T,T,T,T]).
template <int T>
__device__ __forceinline__ float qbcast(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), T * 0x55, 0xF, 0xF, false));
}

// Sum over the 4 lanes of each quad (result in every lane of the quad).
__device__ __forceinline__ float quad_sum(float v)
{
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
    return v;
}

// Coefficients (of v, v', v'') of the feature of channel c:
//   U: v   X: v' zx   XX: v'' zx^2 + v' zxx   Y: v' zy   YY: v'' zy^2 + v' zyy
template <int O0, int O1>
__device__ __forceinline__ void channel_coeffs(int c, const float *zj, float &a0, float &a1, float &a2)
{
    using CH = Ch<O0, O1>;
    a0 = 0.f; a1 = 0.f; a2 = 0.f;
    if (c == CH::U) a0 = 1.f;
    if constexpr (CH::X >= 0) if (c == CH::X) a1 = zj[CH::X];
    if constexpr (CH::XX >= 0) if (c == CH::XX) { a1 = zj[CH::XX]; a2 = zj[CH::X] * zj[CH::X]; }
    if constexpr (CH::Y >= 0) if (c == CH::Y) a1 = zj[CH::Y];
    if constexpr (CH::YY >= 0) if (c == CH::YY) { a1 = zj[CH::YY]; a2 = zj[CH::Y] * zj[CH::Y]; }
}

template <typename T, int O0, int O1, bool FIRST>
__device__ __forceinline__ void load_jets_guarded(const T *__restrict__ zin, int64_t n, int win,
                                                  int i, int64_t p, bool ok, T *zj)
{
    constexpr int C = Ch<O0, O1>::C;
    if (!ok) {
#pragma unroll
        for (int c = 0; c < C; ++c) zj[c] = T(0);
        return;
    }
    if constexpr (FIRST) {
        input_jets<T, O0, O1>(zin, p, i, zj);
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) zj[c] = zin[((int64_t)c * win + i) * n + p];
    }
}

// Stage weight rows [r0, r0 + nrows) x N into LDS with row stride NS.
__device__ __forceinline__ void stage_rows(float *sW, const float *__restrict__ W, int r0, int nrows,
                                           int N, int NS)
{
    const int n4 = N / 4;
    for (int e = threadIdx.x; e < nrows * n4; e += NT) {
        const int r = e / n4, c4 = e % n4;
        const f4 v = *reinterpret_cast<const f4 *>(W + (size_t)(r0 + r) * N + 4 * c4);
        *reinterpret_cast<f4 *>(sW + r * NS + 4 * c4) = v;
    }
}

// ---------------------------------------------------------------------------
// Staging of input jets. A tile is PB = 64 points; its inputs are taken in
// chunks of KJ. A chunk's jets are loaded from HBM into registers one chunk
// ahead (all loads of a chunk in flight together) and written to LDS as
// [input][channel][point] while the previous chunk is being computed.
// ---------------------------------------------------------------------------
constexpr int KJ = 8;

template <int O0, int O1, bool FIRST>
struct JetChunk {
    static constexpr int C = Ch<O0, O1>::C;
    static constexpr int E = KJ * C * PB;            // elements per chunk
    static constexpr int R = (E + NT - 1) / NT;      // registers per thread
    float r[R];

    __device__ __forceinline__ void load(const float *__restrict__ zin, int64_t n, int win,
                                         int64_t tile, int jc)
    {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int e = threadIdx.x + k * NT;
            const int pp = e % PB, rest = e / PB, c = rest % C, il = rest / C;
            const int i = jc * KJ + il;
            const int64_t p = tile * PB + pp;
            float v = 0.f;
            if (e < E && i < win && p < n) {
                if constexpr (FIRST) {
                    float zj[C];
                    input_jets<float, O0, O1>(zin, p, i, zj);
                    v = zj[c];
                } else {
                    v = zin[((int64_t)c * win + i) * n + p];
                }
            }
            r[k] = v;
        }
    }
    __device__ __forceinline__ void store(float *sZ) const
    {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < E) sZ[e] = r[k];
        }
    }
};

// ---------------------------------------------------------------------------
// forward: zout[c][j][p] = sum_i sum_t W[i*nb + q + t][j] * A_c(p, i, t)
// Persistent blocks walk tiles of 64 points (16 per wave). NQ = N/4 output
// chunks; block column s owns outputs j = s*NQ + k, k < NQ.
// ---------------------------------------------------------------------------
template <int O0, int O1, bool FIRST, int NQ>
__global__ __launch_bounds__(NT) void k_fwd_bs(const float *__restrict__ zin,
                                               const float *__restrict__ W,
                                               float *__restrict__ zout, int64_t n, int win,
                                               int KI, GridP<float> g)
{
    constexpr int C = Ch<O0, O1>::C;
    constexpr int RG = (C + 3) / 4;
    constexpr int N = 4 * NQ;
    constexpr int NS = N + 4;
    using JCk = JetChunk<O0, O1, FIRST>;
    extern __shared__ float smem[];
    const int nb = g.nb;
    float *sW = smem;
    float *sZ = smem + KI * nb * NS;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int bl = lane >> 2, s = lane & 3;
    const int64_t ntiles = (n + PB - 1) / PB;
    const int njc = (win + KJ - 1) / KJ;
    const bool single = KI >= win;
    if (single) stage_rows(sW, W, 0, win * nb, N, NS);

    JCk pre;
    int64_t tile = blockIdx.x;
    int jc = 0;
    if (tile < ntiles) pre.load(zin, n, win, tile, 0);
    f4 acc[RG][NQ];
    while (tile < ntiles) {
        if (jc == 0) {
#pragma unroll
            for (int r = 0; r < RG; ++r)
#pragma unroll
                for (int k = 0; k < NQ; ++k) acc[r][k] = (f4){0.f, 0.f, 0.f, 0.f};
        }
        const int ib = jc * KJ;                         // first input of this chunk
        const int iW = single ? 0 : (ib / KI) * KI;     // first input of the staged W rows
        __syncthreads();
        pre.store(sZ);
        if (!single && ib % KI == 0) stage_rows(sW, W, iW * nb, (min(win, iW + KI) - iW) * nb, N, NS);
        __syncthreads();
        // prefetch the next chunk (next inputs of this tile, or the next tile)
        const int64_t cur_tile = tile;
        if (++jc == njc) {
            jc = 0;
            tile += gridDim.x;
        }
        if (tile < ntiles) pre.load(zin, n, win, tile, jc);

        const int64_t p = cur_tile * PB + wv * PW + bl;
        const int ie = min(win, ib + KJ);
        for (int i = ib; i < ie; ++i) {
            const float *zp = sZ + ((i - ib) * C) * PB + wv * PW + bl;
            float zj[C];
#pragma unroll
            for (int c = 0; c < C; ++c) zj[c] = zp[c * PB];
            const float zt = zeta_of(g, zj[0]);
            const int q = interval_of(g, zt);
            // this lane evaluates live function t = s; the quad shares it
            float v[3];
            hr_bump<float, 2, 4>(g, zt, q + s, v);
            float a0[RG], a1[RG], a2[RG];
#pragma unroll
            for (int r = 0; r < RG; ++r) channel_coeffs<O0, O1>(4 * r + s, zj, a0[r], a1[r], a2[r]);
            float vt[4][3];
            vt[0][0] = qbcast<0>(v[0]); vt[0][1] = qbcast<0>(v[1]); vt[0][2] = qbcast<0>(v[2]);
            vt[1][0] = qbcast<1>(v[0]); vt[1][1] = qbcast<1>(v[1]); vt[1][2] = qbcast<1>(v[2]);
            vt[2][0] = qbcast<2>(v[0]); vt[2][1] = qbcast<2>(v[1]); vt[2][2] = qbcast<2>(v[2]);
            vt[3][0] = qbcast<3>(v[0]); vt[3][1] = qbcast<3>(v[1]); vt[3][2] = qbcast<3>(v[2]);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int b = q + t;
                const bool live = b >= 0 && b < nb;
                const int row = (i - iW) * nb + (live ? b : 0);
                const float *wr = sW + row * NS + s * NQ;
                float bw[NQ];
#pragma unroll
                for (int k4 = 0; k4 < NQ / 4; ++k4) {
                    const f4 w4 = *reinterpret_cast<const f4 *>(wr + 4 * k4);
                    bw[4 * k4 + 0] = live ? w4[0] : 0.f;
                    bw[4 * k4 + 1] = live ? w4[1] : 0.f;
                    bw[4 * k4 + 2] = live ? w4[2] : 0.f;
                    bw[4 * k4 + 3] = live ? w4[3] : 0.f;
                }
#pragma unroll
                for (int r = 0; r < RG; ++r) {
                    const float A = a0[r] * vt[t][0] + a1[r] * vt[t][1] + a2[r] * vt[t][2];
#pragma unroll
                    for (int k = 0; k < NQ; ++k)
                        acc[r][k] = __builtin_amdgcn_mfma_f32_4x4x1f32(A, bw[k], acc[r][k], 0, 0, 0);
                }
            }
        }
        if (jc == 0 && p < n) {                 // the tile is complete
#pragma unroll
            for (int r = 0; r < RG; ++r)
#pragma unroll
                for (int k = 0; k < NQ; ++k)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = 4 * r + e;
                        if (c < C) zout[((int64_t)c * N + s * NQ + k) * n + p] = acc[r][k][e];
                    }
        }
    }
}

// ---------------------------------------------------------------------------
// input bars: Ab_c(p,i,t) = sum_j W[i*nb + q + t][j] * ybar[c][j][p]; then the
// adjoint of the features through v..v''' gives zbar[.][i][p].
// Block row = channel, block column = live function t. Two inputs are in
// flight at a time so consecutive MFMAs accumulate into different results.
// ---------------------------------------------------------------------------
template <int O0, int O1, int NQ>
__global__ __launch_bounds__(NT) void k_dx_bs(const float *__restrict__ zin,
                                              const float *__restrict__ ybar,
                                              const float *__restrict__ W,
                                              float *__restrict__ zbar, int64_t n, int win, int KI,
                                              GridP<float> g)
{
    constexpr int C = Ch<O0, O1>::C;
    constexpr int RG = (C + 3) / 4;
    constexpr int N = 4 * NQ;
    constexpr int NS = N + 4;
    using JCk = JetChunk<O0, O1, false>;
    extern __shared__ float smem[];
    const int nb = g.nb;
    float *sW = smem;
    float *sZ = smem + KI * nb * NS;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int bl = lane >> 2, s = lane & 3;
    const int64_t ntiles = (n + PB - 1) / PB;
    const int njc = (win + KJ - 1) / KJ;
    const bool single = KI >= win;
    if (single) stage_rows(sW, W, 0, win * nb, N, NS);

    JCk pre;
    int64_t tile = blockIdx.x;
    int jc = 0;
    if (tile < ntiles) pre.load(zin, n, win, tile, 0);
    float yb[RG][N];
    while (tile < ntiles) {
        const int64_t p = tile * PB + wv * PW + bl;
        const bool ok = p < n;
        if (jc == 0) {
            // the output bars of this lane's channel rows, all N outputs
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                const int c = 4 * r + s;
#pragma unroll
                for (int j = 0; j < N; ++j)
                    yb[r][j] = (ok && c < C) ? ybar[((int64_t)c * N + j) * n + p] : 0.f;
            }
        }
        const int ib = jc * KJ;
        const int iW = single ? 0 : (ib / KI) * KI;
        __syncthreads();
        pre.store(sZ);
        if (!single && ib % KI == 0) stage_rows(sW, W, iW * nb, (min(win, iW + KI) - iW) * nb, N, NS);
        __syncthreads();
        if (++jc == njc) {
            jc = 0;
            tile += gridDim.x;
        }
        if (tile < ntiles) pre.load(zin, n, win, tile, jc);

        const int ie = min(win, ib + KJ);
        for (int i = ib; i < ie; i += 2) {
            const int npair = (i + 1 < ie) ? 2 : 1;
            float zj[2][C], zt[2];
            int q[2];
            f4 ab[2][RG];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float *zp = sZ + ((i + (u < npair ? u : 0) - ib) * C) * PB + wv * PW + bl;
#pragma unroll
                for (int c = 0; c < C; ++c) zj[u][c] = (u < npair) ? zp[c * PB] : 0.f;
                zt[u] = zeta_of(g, zj[u][0]);
                q[u] = interval_of(g, zt[u]);
#pragma unroll
                for (int r = 0; r < RG; ++r) ab[u][r] = (f4){0.f, 0.f, 0.f, 0.f};
            }
            // this lane (column t = s) reads the weight row of function q + s
            const float *wr[2];
            bool live[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int b = q[u] + s;
                live[u] = u < npair && b >= 0 && b < nb;
                wr[u] = sW + ((i + (u < npair ? u : 0) - iW) * nb + (live[u] ? b : 0)) * NS;
            }
#pragma unroll
            for (int j4 = 0; j4 < NQ; ++j4) {
                f4 w4[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    w4[u] = *reinterpret_cast<const f4 *>(wr[u] + 4 * j4);
                    if (!live[u]) w4[u] = (f4){0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int r = 0; r < RG; ++r)
                            ab[u][r] = __builtin_amdgcn_mfma_f32_4x4x1f32(yb[r][4 * j4 + e], w4[u][e],
                                                                          ab[u][r], 0, 0, 0);
            }
            // lane (b, t): ab[u][r][e] = Abar of channel 4r+e for function t = s
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                float v[4];
                hr_bump<float, 3, 4>(g, zt[u], q[u] + s, v);
                float Ab[C];
#pragma unroll
                for (int c = 0; c < C; ++c) Ab[c] = ab[u][c / 4][c % 4];
                float zb[C];
#pragma unroll
                for (int c = 0; c < C; ++c) zb[c] = 0.f;
                features_adjoint<float, O0, O1>(v, zj[u], Ab, zb);
#pragma unroll
                for (int c = 0; c < C; ++c) zb[c] = quad_sum(zb[c]);
                if (ok && u < npair) {
#pragma unroll
                    for (int r = 0; r < RG; ++r) {
                        const int c = 4 * r + s;
                        float val = zb[0];
#pragma unroll
                        for (int cc = 1; cc < C; ++cc) val = (c == cc) ? zb[cc] : val;
                        if (c < C) zbar[((int64_t)c * win + i + u) * n + p] = val;
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient, block-sparse:
//   gW[i*nb + q + t][j] += sum_c A_c(p, i, t) * ybar[c][j][p]
// One 4x4x1 MFMA block is (input feature, chunk of 4 outputs) of ONE point:
// rows = live function t, columns = 4 outputs, K = one jet channel (C MFMAs
// accumulate the channels). Each lane then adds its 4 results to rows
// q..q+3 of its input in the block's LDS copy of the gradient. A wave owns II
// inputs (disjoint gradient rows) and walks every point of the slice in a
// fixed order, so each LDS word has a single writer and the sums are
// deterministic. A block owns 4*II inputs and all N outputs of one slice; the
// next chunk of points is loaded while the current one is computed.
// ---------------------------------------------------------------------------
template <int NQ> constexpr int dw_pc() { return NQ >= 32 ? 8 : 16; }

template <int O0, int O1, bool FIRST, int NQ>
__global__ __launch_bounds__(NT) void k_dw_bs(const float *__restrict__ zin,
                                              const float *__restrict__ ybar,
                                              float *__restrict__ part, int64_t n, int win,
                                              int nsplit, GridP<float> g)
{
    constexpr int C = Ch<O0, O1>::C;
    constexpr int CP = C <= 4 ? 4 : 8;       // padded channel stride in LDS
    constexpr int N = 4 * NQ;
    constexpr int GS = N + 1;                // gradient row stride (spreads banks)
    constexpr int II = 64 / NQ;              // inputs per wave (II * N = 256)
    constexpr int IB = 4 * II;               // inputs per block
    constexpr int JC = 16 / II;              // 4-output chunks per MFMA
    constexpr int PASSES = NQ / JC;
    constexpr int PC = dw_pc<NQ>();
    constexpr int JS = IB * CP + 1;          // staged jets: stride per point
    constexpr int YS = N * CP + 1;           // staged bars: stride per point
    constexpr int EJ = C * IB * PC, EY = C * N * PC;
    constexpr int RJ = (EJ + NT - 1) / NT, RY = (EY + NT - 1) / NT;
    extern __shared__ float smem[];
    const int nb = g.nb;
    float *sG = smem;                                  // [IB * nb][GS], then 256 scratch words
    float *sJ = sG + IB * nb * GS + NT;                // [PC][JS]
    float *sY = sJ + PC * JS;                          // [PC][YS]

    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int blk = lane >> 2, s = lane & 3;
    const int ii = wv * II + blk / JC, jc = blk % JC;  // block-local input of this lane
    const int i0 = blockIdx.x * IB;
    const bool iok = i0 + ii < win;
    const int trash = IB * nb * GS + threadIdx.x;      // this lane's scratch word
    const int lane_row = ii * nb * GS;                 // first gradient row of this lane's input
    const int colbase = 4 * jc + s;
    const int split = blockIdx.y;
    const int64_t per = ((n + nsplit - 1) / nsplit + PC - 1) / PC * PC;
    const int64_t ps = (int64_t)split * per, pe = min(n, ps + per);
    for (int e = threadIdx.x; e < IB * nb * GS + NT; e += NT) sG[e] = 0.f;

    float rj[RJ], ry[RY];
    auto load = [&](int64_t pc) {
#pragma unroll
        for (int k = 0; k < RJ; ++k) {
            const int e = threadIdx.x + k * NT;
            const int pp = e % PC, rest = e / PC, il = rest % IB, c = rest / IB;
            const int64_t p = pc + pp;
            float v = 0.f;
            if (e < EJ && p < pe && i0 + il < win) {
                if constexpr (FIRST) {
                    float zj[C];
                    input_jets<float, O0, O1>(zin, p, i0 + il, zj);
                    v = zj[c];
                } else {
                    v = zin[((int64_t)c * win + i0 + il) * n + p];
                }
            }
            rj[k] = v;
        }
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int e = threadIdx.x + k * NT;
            const int pp = e % PC, rest = e / PC, j = rest % N, c = rest / N;
            const int64_t p = pc + pp;
            ry[k] = (e < EY && p < pe) ? ybar[((int64_t)c * N + j) * n + p] : 0.f;
        }
    };
    if (ps < pe) load(ps);
    for (int64_t pc = ps; pc < pe; pc += PC) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RJ; ++k) {
            const int e = threadIdx.x + k * NT;
            const int pp = e % PC, rest = e / PC, il = rest % IB, c = rest / IB;
            if (e < EJ) sJ[pp * JS + il * CP + c] = rj[k];
        }
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int e = threadIdx.x + k * NT;
            const int pp = e % PC, rest = e / PC, j = rest % N, c = rest / N;
            if (e < EY) sY[pp * YS + j * CP + c] = ry[k];
        }
        __syncthreads();
        if (pc + PC < pe) load(pc + PC);         // next chunk in flight during this one
        const int npts = (int)min<int64_t>(PC, pe - pc);
        for (int pp = 0; pp < npts; ++pp) {
            float zj[C];
#pragma unroll
            for (int c = 0; c < C; ++c) zj[c] = sJ[pp * JS + ii * CP + c];
            const float zt = zeta_of(g, zj[0]);
            const int q = interval_of(g, zt);
            float v[3], A[C];
            hr_bump<float, 2, 4>(g, zt, q + s, v);     // this lane's row: live function t = s
            features<float, O0, O1>(v, zj, A);
            f4 d[PASSES];
#pragma unroll
            for (int ps_ = 0; ps_ < PASSES; ++ps_) {
                const int jb = 4 * (ps_ * JC + jc);
                const float *yp = sY + pp * YS + (jb + s) * CP;
                d[ps_] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int c = 0; c < C; ++c)
                    d[ps_] = __builtin_amdgcn_mfma_f32_4x4x1f32(A[c], yp[c], d[ps_], 0, 0, 0);
            }
            // each (input, column) word belongs to one lane of one wave:
            // plain read-add-write, no atomics. All reads are issued before
            // any write; a row outside the basis goes to this lane's own
            // scratch word, so the live addresses are all distinct.
            int addr[PASSES][4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = q + r;
                // all-ones when row b of this input is a live gradient row
                const int keep = -(int)(iok & ((unsigned)b < (unsigned)nb));
#pragma unroll
                for (int ps_ = 0; ps_ < PASSES; ++ps_) {
                    const int a = lane_row + b * GS + 4 * (ps_ * JC) + colbase;
                    addr[ps_][r] = trash + ((a - trash) & keep);
                }
            }
            float old[PASSES][4];
#pragma unroll
            for (int ps_ = 0; ps_ < PASSES; ++ps_)
#pragma unroll
                for (int r = 0; r < 4; ++r) old[ps_][r] = sG[addr[ps_][r]];
#pragma unroll
            for (int ps_ = 0; ps_ < PASSES; ++ps_)
#pragma unroll
                for (int r = 0; r < 4; ++r) sG[addr[ps_][r]] = old[ps_][r] + d[ps_][r];
        }
    }
    __syncthreads();
    const int64_t KN = (int64_t)win * nb * N;
    for (int e = threadIdx.x; e < IB * nb * N; e += NT) {
        const int row = e / N, col = e % N;
        if (i0 + row / nb >= win) continue;
        part[split * KN + (int64_t)(i0 * nb + row) * N + col] = sG[row * GS + col];
    }
}

static size_t dw_bs_lds(int C, int nb, int N)
{
    const int CP = C <= 4 ? 4 : 8, IB = 4 * (256 / N), PC = N >= 128 ? 8 : 16;
    return sizeof(float) * ((size_t)IB * nb * (N + 1) + NT + (size_t)PC * (IB * CP + 1) +
                            (size_t)PC * (N * CP + 1));
}

// ---------------------------------------------------------------------------
// last layer (one output): plain vector-ALU kernels
// ---------------------------------------------------------------------------
// u_c[p] = sum_i sum_t W[i*nb + q + t] * A_c(p, i, t); one thread per point
template <int O0, int O1>
__global__ __launch_bounds__(NT) void k_fwd_last(const float *__restrict__ zin,
                                                 const float *__restrict__ W,
                                                 float *__restrict__ out, int64_t n, int win,
                                                 GridP<float> g)
{
    constexpr int C = Ch<O0, O1>::C;
    extern __shared__ float sW[];
    const int nb = g.nb;
    for (int e = threadIdx.x; e < win * nb; e += NT) sW[e] = W[e];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (p >= n) return;
    float acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.f;
    constexpr int U = 8;                        // inputs whose loads are in flight together
    for (int i0 = 0; i0 < win; i0 += U) {
        float zj[U][C];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < C; ++c)
                zj[u][c] = (i0 + u < win) ? zin[((int64_t)c * win + i0 + u) * n + p] : 0.f;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            if (i >= win) break;
            const float zt = zeta_of(g, zj[u][0]);
            const int q = interval_of(g, zt);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int b = q + t;
                if (b < 0 || b >= nb) continue;
                float v[3], A[C];
                hr_bump<float, 2, 4>(g, zt, b, v);
                features<float, O0, O1>(v, zj[u], A);
                const float w = sW[i * nb + b];
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] += w * A[c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) out[(int64_t)c * n + p] = acc[c];
}

// zbar[c][i][p] from ubar[c][p]; one thread per (point, input)
template <int O0, int O1>
__global__ __launch_bounds__(NT) void k_dx_last(const float *__restrict__ zin,
                                                const float *__restrict__ ybar,
                                                const float *__restrict__ W,
                                                float *__restrict__ zbar, int64_t n, int win,
                                                GridP<float> g)
{
    constexpr int C = Ch<O0, O1>::C;
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= n * win) return;
    const int i = (int)(e / n);
    const int64_t p = e % n;
    const int nb = g.nb;
    float zj[C], yb[C], zb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        zj[c] = zin[((int64_t)c * win + i) * n + p];
        yb[c] = ybar[(int64_t)c * n + p];
        zb[c] = 0.f;
    }
    const float zt = zeta_of(g, zj[0]);
    const int q = interval_of(g, zt);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int b = q + t;
        if (b < 0 || b >= nb) continue;
        float v[4], Ab[C];
        hr_bump<float, 3, 4>(g, zt, b, v);
        const float w = W[i * nb + b];
#pragma unroll
        for (int c = 0; c < C; ++c) Ab[c] = w * yb[c];
        features_adjoint<float, O0, O1>(v, zj, Ab, zb);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) zbar[((int64_t)c * win + i) * n + p] = zb[c];
}

// gW[i*nb + b] for one point slice; thread (i, lane-slot) owns a private
// accumulator row in LDS, so every sum has a fixed order.
constexpr int DL_SL = 8;   // point lanes per input
template <int O0, int O1>
__global__ __launch_bounds__(NT) void k_dw_last(const float *__restrict__ zin,
                                                const float *__restrict__ ybar,
                                                float *__restrict__ part, int64_t n, int win,
                                                int nsplit, GridP<float> g)
{
    constexpr int C = Ch<O0, O1>::C;
    constexpr int IB = NT / DL_SL;        // inputs per block
    __shared__ float sacc[NT][33];
    const int nb = g.nb;
    const int li = threadIdx.x / DL_SL, sl = threadIdx.x % DL_SL;
    const int i = blockIdx.x * IB + li;
    const int split = blockIdx.y;
    const int64_t per = (n + nsplit - 1) / nsplit;
    const int64_t ps = (int64_t)split * per, pe = min(n, ps + per);
    for (int b = 0; b < nb; ++b) sacc[threadIdx.x][b] = 0.f;
    if (i < win) {
        constexpr int U = 4;                    // points whose loads are in flight together
        for (int64_t p0 = ps + sl; p0 < pe; p0 += U * DL_SL) {
            float zj[U][C], yb[U][C];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t p = p0 + (int64_t)u * DL_SL;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    zj[u][c] = p < pe ? zin[((int64_t)c * win + i) * n + p] : 0.f;
                    yb[u][c] = p < pe ? ybar[(int64_t)c * n + p] : 0.f;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (p0 + (int64_t)u * DL_SL >= pe) break;
                const float zt = zeta_of(g, zj[u][0]);
                const int q = interval_of(g, zt);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int b = q + t;
                    if (b < 0 || b >= nb) continue;
                    float v[3], A[C];
                    hr_bump<float, 2, 4>(g, zt, b, v);
                    features<float, O0, O1>(v, zj[u], A);
                    float sum = 0.f;
#pragma unroll
                    for (int c = 0; c < C; ++c) sum += A[c] * yb[u][c];
                    sacc[threadIdx.x][b] += sum;
                }
            }
        }
    }
    __syncthreads();
    // fixed-order sum over the point lanes of each input
    for (int e = threadIdx.x; e < IB * nb; e += NT) {
        const int l2 = e / nb, b = e % nb;
        const int i2 = blockIdx.x * IB + l2;
        if (i2 >= win) continue;
        float sum = 0.f;
        for (int k = 0; k < DL_SL; ++k) sum += sacc[l2 * DL_SL + k][b];
        part[(int64_t)split * win * nb + i2 * nb + b] = sum;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define HRK_CH_SWITCH32(ch, ...)                                  \
    switch ((ch).o0 * 3 + (ch).o1) {                              \
    case 0: { constexpr int O0 = 0, O1 = 0; __VA_ARGS__; } break; \
    case 4: { constexpr int O0 = 1, O1 = 1; __VA_ARGS__; } break; \
    case 6: { constexpr int O0 = 2, O1 = 0; __VA_ARGS__; } break; \
    case 7: { constexpr int O0 = 2, O1 = 1; __VA_ARGS__; } break; \
    case 8: { constexpr int O0 = 2, O1 = 2; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                         \
    }

#define HRK_NQ_SWITCH(N, ...)                                     \
    switch (N) {                                                  \
    case 32: { constexpr int NQ = 8; __VA_ARGS__; } break;        \
    case 64: { constexpr int NQ = 16; __VA_ARGS__; } break;       \
    case 128: { constexpr int NQ = 32; __VA_ARGS__; } break;      \
    default: return hipErrorInvalidValue;                         \
    }

bool bs32_supported(LayerShape ls)
{
    if (ls.nb < 2 || ls.nb > 32) return false;
    if (ls.wout == 1) return true;
    if (ls.wout != 32 && ls.wout != 64 && ls.wout != 128) return false;
    return dw_bs_lds(5, ls.nb, ls.wout) <= 160 * 1024;
}

// Raise a kernel's dynamic-LDS limit once (outside any graph capture: the
// first launch of each kernel happens eagerly).
static void set_lds_limit(const void *kf, size_t bytes)
{
    static const void *done[256];
    static int ndone = 0;
    for (int k = 0; k < ndone; ++k)
        if (done[k] == kf) return;
    (void)hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (ndone < 256) done[ndone++] = kf;
    (void)bytes;
}

static int grid_blocks(int64_t tiles, int cap) { return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, cap)); }

// inputs whose weight rows are staged at once (a multiple of KJ, or all of
// them), and the LDS bytes of those rows plus one chunk of jets
static void w_stage(LayerShape ls, int C, int &KI, size_t &bytes)
{
    const size_t per_in = (size_t)ls.nb * (ls.wout + 4) * sizeof(float);
    const size_t jets = (size_t)KJ * C * PB * sizeof(float);
    size_t ki = (LDS_W_BYTES - jets) / per_in;
    if (ki >= (size_t)ls.win)
        ki = ls.win;
    else
        ki = std::max<size_t>(KJ, ki / KJ * KJ);
    KI = (int)ki;
    bytes = per_in * ki + jets;
}

hipError_t launch_fwd_bs32(ChanCfg ch, bool first, const float *zin, const float *W, float *zout,
                           int64_t n, LayerShape ls, const GridP<float> &g, int cu_blocks, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (ls.wout == 1) {
        const size_t sh = sizeof(float) * ls.win * ls.nb;
        HRK_CH_SWITCH32(ch, {
            k_fwd_last<O0, O1><<<(unsigned)((n + NT - 1) / NT), NT, sh, st>>>(zin, W, zout, n, ls.win, g);
        });
        return hipGetLastError();
    }
    int KI;
    size_t sh;
    w_stage(ls, ch.C(), KI, sh);
    const int grid = grid_blocks((n + PB - 1) / PB, cu_blocks);
    HRK_CH_SWITCH32(ch, {
        HRK_NQ_SWITCH(ls.wout, {
            if (first) {
                auto kf = k_fwd_bs<O0, O1, true, NQ>;
                set_lds_limit((const void *)kf, sh);
                kf<<<grid, NT, sh, st>>>(zin, W, zout, n, ls.win, KI, g);
            } else {
                auto kf = k_fwd_bs<O0, O1, false, NQ>;
                set_lds_limit((const void *)kf, sh);
                kf<<<grid, NT, sh, st>>>(zin, W, zout, n, ls.win, KI, g);
            }
        });
    });
    return hipGetLastError();
}

hipError_t launch_dx_bs32(ChanCfg ch, const float *zin, const float *ybar, const float *W, float *zbar,
                          int64_t n, LayerShape ls, const GridP<float> &g, int cu_blocks, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (ls.wout == 1) {
        HRK_CH_SWITCH32(ch, {
            k_dx_last<O0, O1><<<(unsigned)((n * ls.win + NT - 1) / NT), NT, 0, st>>>(zin, ybar, W, zbar, n,
                                                                                   ls.win, g);
        });
        return hipGetLastError();
    }
    int KI;
    size_t sh;
    w_stage(ls, ch.C(), KI, sh);
    const int grid = grid_blocks((n + PB - 1) / PB, cu_blocks);
    HRK_CH_SWITCH32(ch, {
        HRK_NQ_SWITCH(ls.wout, {
            auto kf = k_dx_bs<O0, O1, NQ>;
            set_lds_limit((const void *)kf, sh);
            kf<<<grid, NT, sh, st>>>(zin, ybar, W, zbar, n, ls.win, KI, g);
        });
    });
    return hipGetLastError();
}

int dw_bs32_splits(int64_t n, LayerShape ls)
{
    if (n <= 0) return 0;
    // enough blocks to fill the chip, but at least 256 points per slice
    const int64_t maxs = std::max<int64_t>(1, n / 128);
    int64_t tiles;
    if (ls.wout == 1)
        tiles = (ls.win + NT / DL_SL - 1) / (NT / DL_SL);
    else
        tiles = (ls.win + 4 * (256 / ls.wout) - 1) / (4 * (256 / ls.wout));
    const int64_t s = (512 + tiles - 1) / tiles;
    return (int)std::max<int64_t>(1, std::min<int64_t>(std::min(s, maxs), 1024));
}

hipError_t launch_dw_bs32(ChanCfg ch, bool first, const float *zin, const float *ybar, float *part,
                          int nsplit, int64_t n, LayerShape ls, const GridP<float> &g, hipStream_t st)
{
    if (ls.wout == 1) {
        dim3 grid((unsigned)((ls.win + NT / DL_SL - 1) / (NT / DL_SL)), (unsigned)nsplit);
        HRK_CH_SWITCH32(ch, {
            k_dw_last<O0, O1><<<grid, NT, 0, st>>>(zin, ybar, part, n, ls.win, nsplit, g);
        });
        return hipGetLastError();
    }
    HRK_CH_SWITCH32(ch, {
        HRK_NQ_SWITCH(ls.wout, {
            constexpr int IB = 4 * (64 / NQ);
            dim3 grid((unsigned)((ls.win + IB - 1) / IB), (unsigned)nsplit);
            const size_t sh = dw_bs_lds(ch.C(), ls.nb, ls.wout);
            if (first) {
                auto kf = k_dw_bs<O0, O1, true, NQ>;
                set_lds_limit((const void *)kf, sh);
                kf<<<grid, NT, sh, st>>>(zin, ybar, part, n, ls.win, nsplit, g);
            } else {
                auto kf = k_dw_bs<O0, O1, false, NQ>;
                set_lds_limit((const void *)kf, sh);
                kf<<<grid, NT, sh, st>>>(zin, ybar, part, n, ls.win, nsplit, g);
            }
        });
    });
    return hipGetLastError();
}

}  // namespace hrk
