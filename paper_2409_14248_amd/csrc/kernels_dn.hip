// kernels_dn.hip -- BF16 matrix-core kernels of a hidden KAN layer (k = 3,
// m = 4) in the dense form of the contraction: a tile of the basis tensor,
// zeros included, is generated in registers and multiplied on the 16x16x32
// BF16 MFMA (the basis-times-weights product of Sec. 3 with the HR basis of
// Eq. 2; forward jets, input bars and weight gradient).
//
// Rows: each input's n_b basis functions are padded to NBP = 8, 16 or 24
// rows (kk = i * NBP + b), so that the 8 consecutive K values one lane holds
// of an operand belong to one input. The weights enter as BF16 copies in that
// padded order with zero padding rows, written once per call by k_w_prep:
//   Wt[j][kk]   kk contiguous: the forward's B operand
//   Wr[kk][j]   row-major:     the input-bar's A operand
// plus, for S = 3, the low pieces of both.
//
// Products follow the BF16 splitting of the block-sparse kernels: a = a_hi +
// a_lo, b = b_hi + b_lo; S = 1: a_hi b_hi, S = 2: + a_lo b_hi, S = 3: +
// a_hi b_lo, where b is the weight (forward, input bars) or the output bar
// (weight gradient).
//
// Bumps: with u = clamp(zt - b/2 + 1/2, -1, 1) the offset from the support
// midpoint, t = 1 - u^2 (= a (2 - a) for a = u + 1 the distance to the
// support start) is exactly zero off the support, d = 2 - 2a = -2u, and
// 3 d^2 - 2 t = 14 u^2 - 2; every power stays bounded, so padding rows and
// far-away coordinates give finite zeros; a NaN coordinate is carried by
// adding a NaN to t. Near the support ends 1 - u^2 is the difference of
// nearly equal values: its error there is a few FP32 units of 1, where the
// bump value t^4 is below 1e-10.
//
// MFMA lane layout (16x16x32 BF16, wave of 64): lane l, r16 = l % 16,
// g = l / 16:  A[r16][8g .. 8g+7],  B[8g .. 8g+7][r16],  D[4g + r][r16].
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "kernels_dn.h"

namespace hrk {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));
typedef unsigned short hw;   // the bits of one BF16 value

constexpr int DN_T = 512;    // forward / input-bar block: 8 waves of 16 points
constexpr int DN_P = 128;    // points per forward / input-bar block
constexpr int DW_T = 512;    // weight-gradient block: 8 waves of 2 inputs each
constexpr int DN_LDS_MAX = 160 * 1024;

__device__ __forceinline__ unsigned int pk2(float a, float b)
{
    return __builtin_bit_cast(unsigned int, __builtin_convertvector((f2v){a, b}, bf2v));
}
__device__ __forceinline__ float lo_f(unsigned int w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_f(unsigned int w) { return __uint_as_float(w & 0xffff0000u); }

// 8 FP32 values as one BF16 operand (round to nearest even) ...
__device__ __forceinline__ bf8 pack8(const float *v)
{
    const u4 w = {pk2(v[0], v[1]), pk2(v[2], v[3]), pk2(v[4], v[5]), pk2(v[6], v[7])};
    return __builtin_bit_cast(bf8, w);
}
// ... and with the low pieces v - bf16(v)
__device__ __forceinline__ void split8(const float *v, bf8 &hi, bf8 &lo)
{
    u4 h, l;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = pk2(v[2 * q], v[2 * q + 1]);
        l[q] = pk2(v[2 * q] - lo_f(h[q]), v[2 * q + 1] - hi_f(h[q]));
    }
    hi = __builtin_bit_cast(bf8, h);
    lo = __builtin_bit_cast(bf8, l);
}

__device__ __forceinline__ f4 mfma(bf8 a, bf8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Scaled jets of one (point, input): the scaled coordinate zt, 1 plus the
// NaN carrier, and the chain-rule factors of the features
//   A_U = t^4,  A_X = kX tu,  A_XX = kXX2 v2 + kXX1 tu  (A_Y, A_YY alike),
// tu = t^3 u, v2 = t^2 (u^2 - 1/7); kX = -8w zx, kXX1 = -8w zxx,
// kXX2 = 56 w^2 zx^2 (w = inv_w), so that v' = 4w t^3 d = -8w tu and
// v'' = 4w^2 t^2 (3 d^2 - 2 t) = 56 w^2 v2.
enum { SZ = 0, SN = 1, SX = 2, SXX1 = 3, SXX2 = 4, SY = 5, SYY1 = 6, SYY2 = 7 };

template <int O0, int O1>
__device__ __forceinline__ void scale_jets(const float *zj, float inv_w, float zoff, float *s)
{
    using CH = Ch<O0, O1>;
    const float w1 = -8.f * inv_w, w2 = 56.f * inv_w * inv_w;
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = 0.f;
    s[SZ] = zj[CH::U] * inv_w + zoff;
    s[SN] = 1.f + (__builtin_isnan(s[SZ]) ? s[SZ] : 0.f);
    if constexpr (CH::X >= 0) s[SX] = w1 * zj[CH::X];
    if constexpr (CH::XX >= 0) {
        s[SXX1] = w1 * zj[CH::XX];
        s[SXX2] = w2 * (zj[CH::X] * zj[CH::X]);
    }
    if constexpr (CH::Y >= 0) s[SY] = w1 * zj[CH::Y];
    if constexpr (CH::YY >= 0) {
        s[SYY1] = w1 * zj[CH::YY];
        s[SYY2] = w2 * (zj[CH::Y] * zj[CH::Y]);
    }
}

// Features of every channel for the basis row with offset cb = 1/2 - b/2.
template <int O0, int O1>
__device__ __forceinline__ void dn_features(const float *s, float cb, float *A)
{
    using CH = Ch<O0, O1>;
    const float u = fminf(fmaxf(s[SZ] + cb, -1.f), 1.f);
    const float u2 = u * u;
    const float t = s[SN] - u2;
    const float t2 = t * t;
    A[CH::U] = t2 * t2;
    if constexpr (CH::X >= 0 || CH::Y >= 0) {
        const float tu = t2 * t * u;
        if constexpr (CH::X >= 0) A[CH::X] = s[SX] * tu;
        if constexpr (CH::Y >= 0) A[CH::Y] = s[SY] * tu;
        if constexpr (CH::XX >= 0 || CH::YY >= 0) {
            const float v2 = t2 * (u2 - (1.f / 7.f));
            if constexpr (CH::XX >= 0) A[CH::XX] = fmaf(s[SXX2], v2, s[SXX1] * tu);
            if constexpr (CH::YY >= 0) A[CH::YY] = fmaf(s[SYY2], v2, s[SYY1] * tu);
        }
    }
}

// ---------------------------------------------------------------------------
// weight copies: W [win * nb][N] FP32 -> Wr [kpad][N], Wt [N][kpad] BF16
// (padded rows zero), low pieces into Wrl / Wtl where those are given
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_w_prep(const float *__restrict__ W, hw *__restrict__ Wr,
                                                hw *__restrict__ Wt, hw *__restrict__ Wrl,
                                                hw *__restrict__ Wtl, int win, int nb, int nbp, int N,
                                                int kpad)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)kpad * N) return;
    const int kk = (int)(e / N), j = (int)(e % N);
    const int i = kk / nbp, b = kk % nbp;
    const float v = (i < win && b < nb) ? W[(int64_t)(i * nb + b) * N + j] : 0.f;
    const unsigned int h = pk2(v, 0.f);
    Wr[(int64_t)kk * N + j] = (hw)h;
    Wt[(int64_t)j * kpad + kk] = (hw)h;
    const hw l = (hw)pk2(v - lo_f(h), 0.f);
    if (Wrl) Wrl[(int64_t)kk * N + j] = l;
    if (Wtl) Wtl[(int64_t)j * kpad + kk] = l;
}

// ---------------------------------------------------------------------------
// forward: zout[c][j][p] = sum_kk A_c[p][kk] W[kk][j]
// A block of 8 waves takes 128 points (16 per wave: the MFMA rows) and walks
// the inputs in chunks of 4 (4 NBP rows of K); every chunk's weight columns
// Wt[.][chunk] and the scaled jets of its (point, input) pairs are staged in
// LDS by the whole block, the next chunk's loads in flight meanwhile. A lane
// evaluates the 8 rows of its K group for its point, all channels at once,
// and each channel's operand meets every 16-output tile (C x N/16
// accumulators).
// ---------------------------------------------------------------------------
template <int O0, int O1, int S, int NQ, int NBP>
struct FwdDn {
    static constexpr int C = Ch<O0, O1>::C;
    static constexpr int N = 16 * NQ;
    static constexpr int KC = 4 * NBP;         // padded rows per chunk
    static constexpr int KS = KC / 32;         // K steps per chunk
    static constexpr int RS = KC + 8;          // halfwords per staged weight column
    static constexpr int NWP = S == 3 ? 2 : 1; // weight pieces
    static constexpr int WEL = N * RS;         // halfwords of one staged piece
    static constexpr int JEL = 4 * DN_P * 8;   // floats of one staged jet chunk
    static constexpr size_t lds() { return 2 * (size_t)NWP * WEL * sizeof(hw) + 2 * (size_t)JEL * sizeof(float); }
};

template <int O0, int O1, int S, int NQ, int NBP>
__global__ __launch_bounds__(DN_T) void k_fwd_dn(const float *__restrict__ zin, const hw *__restrict__ Wt,
                                                 const hw *__restrict__ Wtl, float *__restrict__ zout,
                                                 int64_t n, int win, int kpad, float inv_w, float zoff)
{
    using F = FwdDn<O0, O1, S, NQ, NBP>;
    constexpr int C = F::C, N = F::N, KC = F::KC, KS = F::KS, RS = F::RS, NWP = F::NWP, WEL = F::WEL;
    constexpr int GPI = NBP / 8;               // 8-row groups per input
    constexpr int WV = N * KC / 8;             // 16-byte weight vectors per piece and chunk
    constexpr int RW = (WV + DN_T - 1) / DN_T;
    static_assert(4 * DN_P == DN_T, "one staged (point, input) pair per thread");
    extern __shared__ __align__(16) float smem[];
    hw *sW = reinterpret_cast<hw *>(smem);                         // [2][NWP][N][RS]
    float *sJ = smem + (2 * NWP * WEL) / 2;                        // [2][2 planes][4][DN_P][4]

    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int64_t pb = (int64_t)blockIdx.x * DN_P;
    const int nch = (win + 3) / 4;

    u4 rw[NWP][RW];
    float rj[C];
    const int sj_il = threadIdx.x / DN_P, sj_pp = threadIdx.x % DN_P;
    auto load = [&](int ci) {
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int e = threadIdx.x + k * DN_T;
            if (e < WV) {
                const int j = e / (KC / 8), v = e % (KC / 8);
                const size_t o = (size_t)j * kpad + (size_t)ci * KC + 8 * v;
                rw[0][k] = *reinterpret_cast<const u4 *>(Wt + o);
                if constexpr (NWP == 2) rw[1][k] = *reinterpret_cast<const u4 *>(Wtl + o);
            }
        }
        const int i = 4 * ci + sj_il;
        const int64_t p = pb + sj_pp;
        const bool ok = i < win && p < n;
#pragma unroll
        for (int c = 0; c < C; ++c) rj[c] = ok ? zin[((int64_t)c * win + i) * n + p] : 0.f;
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int e = threadIdx.x + k * DN_T;
            if (e < WV) {
                const int j = e / (KC / 8), v = e % (KC / 8);
#pragma unroll
                for (int w = 0; w < NWP; ++w)
                    *reinterpret_cast<u4 *>(sW + (size_t)(buf * NWP + w) * WEL + j * RS + 8 * v) = rw[w][k];
            }
        }
        float s[8];
        scale_jets<O0, O1>(rj, inv_w, zoff, s);
        // slots 0..3 and 4..7 in separate planes: consecutive lanes read
        // consecutive 16-byte words
        float *d = sJ + (size_t)buf * F::JEL + (sj_il * DN_P + sj_pp) * 4;
        *reinterpret_cast<f4 *>(d) = (f4){s[0], s[1], s[2], s[3]};
        *reinterpret_cast<f4 *>(d + F::JEL / 2) = (f4){s[4], s[5], s[6], s[7]};
    };

    f4 acc[C][NQ];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[c][q] = (f4){0.f, 0.f, 0.f, 0.f};

    load(0);
    store(0);
    __syncthreads();
    for (int ci = 0; ci < nch; ++ci) {
        const int buf = ci & 1;
        if (ci + 1 < nch) load(ci + 1);
        const hw *W0 = sW + (size_t)buf * NWP * WEL;
        const float *J0 = sJ + (size_t)buf * F::JEL;
#pragma unroll 1
        for (int ks = 0; ks < KS; ++ks) {
            const int G = 4 * ks + g;              // this lane's 8-row group in the chunk
            const int il = G / GPI, b0 = 8 * (G % GPI);
            const float *sp = J0 + (il * DN_P + wv * 16 + r16) * 4;
            const f4 s0 = *reinterpret_cast<const f4 *>(sp), s1 = *reinterpret_cast<const f4 *>(sp + F::JEL / 2);
            const float s[8] = {s0[0], s0[1], s0[2], s0[3], s1[0], s1[1], s1[2], s1[3]};
            const float cb0 = 0.5f - 0.5f * (float)b0;
            float A[C][8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float f[C];
                dn_features<O0, O1>(s, cb0 - 0.5f * (float)e, f);
#pragma unroll
                for (int c = 0; c < C; ++c) A[c][e] = f[c];
            }
            bf8 ah[C], al[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if constexpr (S >= 2)
                    split8(A[c], ah[c], al[c]);
                else
                    ah[c] = pack8(A[c]);
            }
            // weight operands one output tile ahead: a tile's read is in
            // flight during the previous tile's products
            auto ldw = [&](int q, bf8 &bh, bf8 &bl) {
                const int o = (16 * q + r16) * RS + 32 * ks + 8 * g;
                bh = *reinterpret_cast<const bf8 *>(W0 + o);
                if constexpr (S == 3) bl = *reinterpret_cast<const bf8 *>(W0 + WEL + o);
            };
            bf8 nh, nl;
            ldw(0, nh, nl);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const bf8 bh = nh, bl = nl;
                if (q + 1 < NQ) ldw(q + 1, nh, nl);
                // consecutive products go to different accumulators
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c][q] = mfma(ah[c], bh, acc[c][q]);
                if constexpr (S >= 2)
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[c][q] = mfma(al[c], bh, acc[c][q]);
                if constexpr (S == 3)
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[c][q] = mfma(ah[c], bl, acc[c][q]);
            }
        }
        if (ci + 1 < nch) store(buf ^ 1);
        __syncthreads();
    }

    // lane holds points p0 + 4g + r of output 16q + r16
    const int64_t p0 = pb + wv * 16 + 4 * g;
    const bool vec = (n % 4 == 0) && p0 + 3 < n && (reinterpret_cast<uintptr_t>(zout) & 15) == 0;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            float *o = zout + ((int64_t)c * N + 16 * q + r16) * n + p0;
            if (vec) {
                *reinterpret_cast<f4 *>(o) = acc[c][q];
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (p0 + r < n) o[r] = acc[c][q][r];
            }
        }
}

// ---------------------------------------------------------------------------
// input bars: Abar_c[p][kk] = sum_j ybar_c[j][p] W[kk][j] on the MFMA (rows
// kk, columns p, K = outputs), then the reverse of the features for the 4
// rows (consecutive b of one input) each lane holds, summed over b: the
// lane's own 4 rows, its row tiles, then the 4 lane groups of the wave.
// A block of 8 waves takes 128 points; each wave keeps its 16 points' output
// bars as B operands in registers and walks the inputs in chunks of 2, whose
// weight rows Wr[chunk][.] the block stages in LDS.
// ---------------------------------------------------------------------------
template <int O0, int O1, int S, int NQ, int NBP>
struct DxDn {
    static constexpr int C = Ch<O0, O1>::C;
    static constexpr int N = 16 * NQ;
    static constexpr int KC = 2 * NBP;         // padded rows per chunk: 2 inputs
    static constexpr int MT = KC / 16;         // row tiles per chunk
    static constexpr int RS = N + 8;           // halfwords per staged weight row
    static constexpr int NWP = S == 3 ? 2 : 1;
    static constexpr int WEL = KC * RS;
    static constexpr size_t lds() { return 2 * (size_t)NWP * WEL * sizeof(hw); }
};

template <int O0, int O1, int S, int NQ, int NBP>
__global__ __launch_bounds__(DN_T) void k_dx_dn(const float *__restrict__ zin, const float *__restrict__ ybar,
                                                const hw *__restrict__ Wr, const hw *__restrict__ Wrl,
                                                float *__restrict__ zbar, int64_t n, int win, float inv_w,
                                                float zoff)
{
    using F = DxDn<O0, O1, S, NQ, NBP>;
    using CH = Ch<O0, O1>;
    constexpr int C = F::C, N = F::N, KC = F::KC, MT = F::MT, RS = F::RS, NWP = F::NWP, WEL = F::WEL;
    constexpr int KJ = N / 32;                 // K steps over the outputs
    constexpr int WV = KC * N / 8;
    constexpr int RW = (WV + DN_T - 1) / DN_T;
    static_assert(N % 32 == 0, "outputs in whole K steps");
    extern __shared__ __align__(16) float smem[];
    hw *sW = reinterpret_cast<hw *>(smem);     // [2][NWP][KC][RS]

    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int64_t p = (int64_t)blockIdx.x * DN_P + wv * 16 + r16;   // this lane's point (D column)
    const bool pin = p < n;
    const int nch = (win + 1) / 2;
    const float w1 = -8.f * inv_w, w2 = 56.f * inv_w * inv_w, w3 = -336.f * inv_w * inv_w * inv_w;

    // output bars of this lane's point, outputs 32 ks + 8 g + e, as B operands
    bf8 yh[C][KJ], yl[C][KJ];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int ks = 0; ks < KJ; ++ks) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                v[e] = pin ? ybar[((int64_t)c * N + 32 * ks + 8 * g + e) * n + p] : 0.f;
            if constexpr (S >= 2)
                split8(v, yh[c][ks], yl[c][ks]);
            else
                yh[c][ks] = pack8(v);
        }

    u4 rw[NWP][RW];
    float zn[2][C];                            // next chunk's jets of this lane's point
    auto load = [&](int ci) {
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int e = threadIdx.x + k * DN_T;
            if (e < WV) {
                const int row = e / (N / 8), v = e % (N / 8);
                const size_t o = (size_t)(ci * KC + row) * N + 8 * v;
                rw[0][k] = *reinterpret_cast<const u4 *>(Wr + o);
                if constexpr (NWP == 2) rw[1][k] = *reinterpret_cast<const u4 *>(Wrl + o);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = 2 * ci + h;
            const bool ok = pin && i < win;
#pragma unroll
            for (int c = 0; c < C; ++c) zn[h][c] = ok ? zin[((int64_t)c * win + i) * n + p] : 0.f;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int k = 0; k < RW; ++k) {
            const int e = threadIdx.x + k * DN_T;
            if (e < WV) {
                const int row = e / (N / 8), v = e % (N / 8);
#pragma unroll
                for (int w = 0; w < NWP; ++w)
                    *reinterpret_cast<u4 *>(sW + (size_t)(buf * NWP + w) * WEL + row * RS + 8 * v) = rw[w][k];
            }
        }
    };

    load(0);
    store(0);
    float zj[2][C];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < C; ++c) zj[h][c] = zn[h][c];
    __syncthreads();
    for (int ci = 0; ci < nch; ++ci) {
        const int buf = ci & 1;
        if (ci + 1 < nch) load(ci + 1);
        const hw *W0 = sW + (size_t)buf * NWP * WEL;
        float zb[2][C];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < C; ++c) zb[h][c] = 0.f;
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            f4 acc[C];
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KJ; ++ks) {
                const int o = (16 * t + r16) * RS + 32 * ks + 8 * g;
                const bf8 ah = *reinterpret_cast<const bf8 *>(W0 + o);
                bf8 al;
                if constexpr (S == 3) al = *reinterpret_cast<const bf8 *>(W0 + WEL + o);
#pragma unroll
                for (int c = 0; c < C; ++c) acc[c] = mfma(ah, yh[c][ks], acc[c]);
                if constexpr (S >= 2)
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[c] = mfma(ah, yl[c][ks], acc[c]);
                if constexpr (S == 3)
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[c] = mfma(al, yh[c][ks], acc[c]);
            }
            // rows 16 t + 4 g + r of the chunk: input h, basis rows b0 + r
            const int row0 = 16 * t + 4 * g;
            const int h = row0 >= NBP ? 1 : 0;
            const int b0 = row0 - h * NBP;
            float z[C];
#pragma unroll
            for (int c = 0; c < C; ++c) z[c] = h ? zj[1][c] : zj[0][c];
            const float zt = z[CH::U] * inv_w + zoff;
            const float one = 1.f + (__builtin_isnan(zt) ? zt : 0.f);   // 1 plus the NaN carrier
            // P = sum of first-order bars times z', Q = second-order bars
            // times z'^2
            float zbt[C];
#pragma unroll
            for (int c = 0; c < C; ++c) zbt[c] = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // u = offset from the support midpoint, t = 1 - u^2, d = -2u:
                // v' = -8w t^3 u, v'' = 56 w^2 t^2 (u^2 - 1/7),
                // v''' = -336 w^3 t u (u^2 - 3/7)
                const float u = fminf(fmaxf(zt + (0.5f - 0.5f * (float)(b0 + r)), -1.f), 1.f);
                const float u2 = u * u;
                const float tt = one - u2;
                const float t2 = tt * tt;
                float Ab[C];
#pragma unroll
                for (int c = 0; c < C; ++c) Ab[c] = acc[c][r];
                if constexpr (C == 1) {
                    zbt[0] = fmaf(w1 * (t2 * tt * u), Ab[0], zbt[0]);
                } else {
                    const float v1 = w1 * (t2 * tt * u);
                    const float v2 = w2 * (t2 * (u2 - (1.f / 7.f)));
                    const float v3 = w3 * (tt * u * (u2 - (3.f / 7.f)));
                    float P = 0.f, Q = 0.f;
                    if constexpr (CH::X >= 0) {
                        P = fmaf(Ab[CH::X], z[CH::X], P);
                        zbt[CH::X] = fmaf(v1, Ab[CH::X], zbt[CH::X]);
                    }
                    if constexpr (CH::XX >= 0) {
                        P = fmaf(Ab[CH::XX], z[CH::XX], P);
                        Q = fmaf(Ab[CH::XX], z[CH::X] * z[CH::X], Q);
                        zbt[CH::X] = fmaf(v2, 2.f * z[CH::X] * Ab[CH::XX], zbt[CH::X]);
                        zbt[CH::XX] = fmaf(v1, Ab[CH::XX], zbt[CH::XX]);
                    }
                    if constexpr (CH::Y >= 0) {
                        P = fmaf(Ab[CH::Y], z[CH::Y], P);
                        zbt[CH::Y] = fmaf(v1, Ab[CH::Y], zbt[CH::Y]);
                    }
                    if constexpr (CH::YY >= 0) {
                        P = fmaf(Ab[CH::YY], z[CH::YY], P);
                        Q = fmaf(Ab[CH::YY], z[CH::Y] * z[CH::Y], Q);
                        zbt[CH::Y] = fmaf(v2, 2.f * z[CH::Y] * Ab[CH::YY], zbt[CH::Y]);
                        zbt[CH::YY] = fmaf(v1, Ab[CH::YY], zbt[CH::YY]);
                    }
                    zbt[CH::U] = fmaf(v1, Ab[CH::U], fmaf(v2, P, fmaf(v3, Q, zbt[CH::U])));
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                zb[0][c] += h ? 0.f : zbt[c];
                zb[1][c] += h ? zbt[c] : 0.f;
            }
        }
        // sum over the 4 lane groups (rows of other b); group h writes input h
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float v = zb[hh][c];
                v += __shfl_xor(v, 16, 64);
                v += __shfl_xor(v, 32, 64);
                zb[hh][c] = v;
            }
        if (g < 2 && pin) {
            const int i = 2 * ci + g;
            if (i < win) {
#pragma unroll
                for (int c = 0; c < C; ++c) zbar[((int64_t)c * win + i) * n + p] = g ? zb[1][c] : zb[0][c];
            }
        }
        if (ci + 1 < nch) {
            store(buf ^ 1);
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int c = 0; c < C; ++c) zj[h][c] = zn[h][c];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// weight gradient: part[split][i nb + b][j] = sum over the slice's points
// and channels of A_c[p][i, b] ybar_c[j][p]; MFMA rows = gradient rows,
// columns = outputs, K = (point, channel) pairs. A block of 8 waves owns 16
// inputs (2 per wave) and all outputs of one point slice; the slice's bars
// (BF16, [j][point][channel]) and scaled jets are staged in chunks,
// the next chunk's loads in flight meanwhile. Row tile t of a wave holds
// basis rows 8t .. 8t+7 of its two inputs (MFMA row m: input m / 8,
// b = 8t + m % 8), so a lane's rows in every tile belong to one input: each
// K step it reads that input's scaled jets once per point and evaluates its
// NBP / 8 basis rows.
// ---------------------------------------------------------------------------
template <int O0, int O1, int S, int NQ, int NBP>
struct DwDn {
    static constexpr int C = Ch<O0, O1>::C;
    static constexpr int CP = C == 1 ? 1 : C <= 4 ? 4 : 8;   // channels per point in a K group
    static constexpr int PG = 8 / CP;                      // points per 8-value K group
    static constexpr int KP = 4 * PG;                      // points per K step
    static constexpr int PC = KP > 16 ? KP : 16;           // points per staged chunk
    static constexpr int KSC = PC / KP;                    // K steps per chunk
    static constexpr int N = 16 * NQ;
    static constexpr int MT = NBP / 8;                     // row tiles per wave
    static constexpr int IB = 2 * (DW_T / 64);             // inputs per block
    static constexpr int YR = PC * CP + 8;                 // halfwords per staged bar row
    static constexpr int NYP = S == 3 ? 2 : 1;             // bar pieces
    static constexpr int YEL = N * YR;
    static constexpr int SJN = C == 1 ? 2 : 8;             // scaled-jet slots kept
    static constexpr int JPS = IB * SJN + 4;               // floats per staged point (padded: the lane
                                                           // groups' points fall on distinct banks)
    static constexpr int JEL = PC * JPS;
    static constexpr size_t lds() { return 2 * (size_t)NYP * YEL * sizeof(hw) + 2 * (size_t)JEL * sizeof(float); }
};

template <int O0, int O1, int S, int NQ, int NBP>
__global__ __launch_bounds__(DW_T) void k_dw_dn(const float *__restrict__ zin, const float *__restrict__ ybar,
                                                float *__restrict__ part, int64_t n, int win, int nb,
                                                int nsplit, int nkb, float inv_w, float zoff)
{
    using F = DwDn<O0, O1, S, NQ, NBP>;
    constexpr int C = F::C, CP = F::CP, PG = F::PG, KP = F::KP, PC = F::PC, KSC = F::KSC, N = F::N;
    constexpr int MT = F::MT, IB = F::IB, YR = F::YR, NYP = F::NYP, YEL = F::YEL, SJN = F::SJN;
    constexpr int EY = N * PC;                 // (output, point) pairs per chunk
    constexpr int RY = (EY + DW_T - 1) / DW_T;
    constexpr int EJ = PC * IB;                // (point, input) pairs per chunk
    constexpr int RJ = (EJ + DW_T - 1) / DW_T;
    extern __shared__ __align__(16) float smem[];
    hw *sY = reinterpret_cast<hw *>(smem);                         // [2][NYP][N][YR]
    float *sJ = smem + (2 * NYP * YEL) / 2;                        // [2][PC][JPS]

    // XCD-aware order: the input blocks of one slice run on one XCD (blocks
    // are dealt to the 8 XCDs round robin), so its bars come from one L2
    int kb, split;
    if (nsplit % 8 == 0) {
        const int x = blockIdx.x % 8, slot = blockIdx.x / 8;
        kb = slot % nkb;
        split = (slot / nkb) * 8 + x;
    } else {
        kb = blockIdx.x % nkb;
        split = blockIdx.x / nkb;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int i0 = kb * IB;                    // first input of the block
    const int64_t per = ((n + nsplit - 1) / nsplit + PC - 1) / PC * PC;
    const int64_t ps = (int64_t)split * per, pe = min(n, ps + per);

    // this lane's input (block-local) and the offsets cb = 1/2 - b/2 of its rows
    const int jl = 2 * wv + (r16 >> 3);
    float cb[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) cb[t] = 0.5f - 0.5f * (float)(8 * t + (r16 & 7));

    float ry[RY][C];
    float rj[RJ][C];
    auto load = [&](int64_t pc) {
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int e = threadIdx.x + k * DW_T;
            const int pp = e % PC, j = e / PC;
            const bool ok = e < EY && pc + pp < pe;
#pragma unroll
            for (int c = 0; c < C; ++c) ry[k][c] = ok ? ybar[((int64_t)c * N + j) * n + pc + pp] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < RJ; ++k) {
            const int e = threadIdx.x + k * DW_T;
            const int pp = e % PC, il = e / PC;
            const bool ok = e < EJ && i0 + il < win && pc + pp < pe;
#pragma unroll
            for (int c = 0; c < C; ++c) rj[k][c] = ok ? zin[((int64_t)c * win + i0 + il) * n + pc + pp] : 0.f;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int e = threadIdx.x + k * DW_T;
            if (e < EY) {
                const int pp = e % PC, j = e / PC;
                hw *d = sY + (size_t)buf * NYP * YEL + j * YR + pp * CP;
                float v[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) v[c] = c < C ? ry[k][c < C ? c : 0] : 0.f;
                if constexpr (CP == 1) {
                    const unsigned int h = pk2(v[0], 0.f);
                    d[0] = (hw)h;
                    if constexpr (NYP == 2) d[YEL] = (hw)pk2(v[0] - lo_f(h), 0.f);
                } else if constexpr (CP == 4) {
                    const u2 h = {pk2(v[0], v[1]), pk2(v[2], v[3])};
                    *reinterpret_cast<u2 *>(d) = h;
                    if constexpr (NYP == 2) {
                        const u2 l = {pk2(v[0] - lo_f(h[0]), v[1] - hi_f(h[0])),
                                      pk2(v[2] - lo_f(h[1]), v[3] - hi_f(h[1]))};
                        *reinterpret_cast<u2 *>(d + YEL) = l;
                    }
                } else {
                    bf8 h, l;
                    if constexpr (NYP == 2) {
                        split8(v, h, l);
                        *reinterpret_cast<bf8 *>(d + YEL) = l;
                    } else {
                        h = pack8(v);
                    }
                    *reinterpret_cast<bf8 *>(d) = h;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < RJ; ++k) {
            const int e = threadIdx.x + k * DW_T;
            if (e >= EJ) break;
            const int pp = e % PC, il = e / PC;
            float s[8];
            scale_jets<O0, O1>(rj[k], inv_w, zoff, s);
            float *d = sJ + (size_t)buf * F::JEL + pp * F::JPS + il * SJN;
            if constexpr (SJN == 2) {
                *reinterpret_cast<f2v *>(d) = (f2v){s[0], s[1]};
            } else {
                *reinterpret_cast<f4 *>(d) = (f4){s[0], s[1], s[2], s[3]};
                *reinterpret_cast<f4 *>(d + 4) = (f4){s[4], s[5], s[6], s[7]};
            }
        }
    };

    f4 acc[MT][NQ];
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[t][q] = (f4){0.f, 0.f, 0.f, 0.f};

    if (ps < pe) {
        load(ps);
        store(0);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t pc = ps; pc < pe; pc += PC) {
        if (pc + PC < pe) load(pc + PC);
        const hw *Y0 = sY + (size_t)buf * NYP * YEL;
        const float *J0 = sJ + (size_t)buf * F::JEL;
#pragma unroll 1
        for (int ks = 0; ks < KSC; ++ks) {
            const int pp0 = ks * KP + g * PG;      // first point of this lane's K group
            float v[MT][8];
#pragma unroll
            for (int e = 0; e < PG; ++e) {
                const float *sp = J0 + (pp0 + e) * F::JPS + jl * SJN;
                float s[8];
                if constexpr (SJN == 2) {
                    const f2v s0 = *reinterpret_cast<const f2v *>(sp);
                    s[0] = s0[0];
                    s[1] = s0[1];
                } else {
                    const f4 s0 = *reinterpret_cast<const f4 *>(sp), s1 = *reinterpret_cast<const f4 *>(sp + 4);
                    s[0] = s0[0]; s[1] = s0[1]; s[2] = s0[2]; s[3] = s0[3];
                    s[4] = s1[0]; s[5] = s1[1]; s[6] = s1[2]; s[7] = s1[3];
                }
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    float f[C];
                    dn_features<O0, O1>(s, cb[t], f);
#pragma unroll
                    for (int c = 0; c < CP; ++c) v[t][e * CP + c] = c < C ? f[c < C ? c : 0] : 0.f;
                }
            }
            bf8 ah[MT], al[MT];
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                if constexpr (S >= 2)
                    split8(v[t], ah[t], al[t]);
                else
                    ah[t] = pack8(v[t]);
            }
            // bar operands one output tile ahead: a tile's read is in flight
            // during the previous tile's products
            auto ldy = [&](int q, bf8 &bh, bf8 &bl) {
                const int o = (16 * q + r16) * YR + pp0 * CP;
                bh = *reinterpret_cast<const bf8 *>(Y0 + o);
                if constexpr (S == 3) bl = *reinterpret_cast<const bf8 *>(Y0 + YEL + o);
            };
            bf8 nh, nl;
            ldy(0, nh, nl);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const bf8 bh = nh, bl = nl;
                if (q + 1 < NQ) ldy(q + 1, nh, nl);
                // consecutive products go to different accumulators
#pragma unroll
                for (int t = 0; t < MT; ++t) acc[t][q] = mfma(ah[t], bh, acc[t][q]);
                if constexpr (S >= 2)
#pragma unroll
                    for (int t = 0; t < MT; ++t) acc[t][q] = mfma(al[t], bh, acc[t][q]);
                if constexpr (S == 3)
#pragma unroll
                    for (int t = 0; t < MT; ++t) acc[t][q] = mfma(ah[t], bl, acc[t][q]);
            }
        }
        if (pc + PC < pe) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    // D row 4 g + r of tile t: input g / 2 of the wave, basis row 8 t + 4 (g % 2) + r
    const int64_t KN = (int64_t)win * nb * N;
    const int i = i0 + 2 * wv + (g >> 1);
    if (i < win) {
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = 8 * t + 4 * (g & 1) + r;
                if (b < nb) {
                    float *o = part + split * KN + (int64_t)(i * nb + b) * N + r16;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) o[16 * q] = acc[t][q][r];
                }
            }
    }
}

int nbp_of(int nb) { return nb <= 8 ? 8 : nb <= 16 ? 16 : nb <= 24 ? 24 : 0; }
int kpad_of(LayerShape ls) { return (ls.win + 3) / 4 * 4 * nbp_of(ls.nb); }

static void set_lds_limit(const void *kf)
{
    static const void *done[256];
    static int ndone = 0;
    for (int k = 0; k < ndone; ++k)
        if (done[k] == kf) return;
    (void)hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, DN_LDS_MAX);
    if (ndone < 256) done[ndone++] = kf;
}

#define DN_CH_SWITCH(ch, ...)                                     \
    switch ((ch).o0 * 3 + (ch).o1) {                              \
    case 0: { constexpr int O0 = 0, O1 = 0; __VA_ARGS__; } break; \
    case 7: { constexpr int O0 = 2, O1 = 1; __VA_ARGS__; } break; \
    case 8: { constexpr int O0 = 2, O1 = 2; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                         \
    }
#define DN_S_SWITCH(S_, ...)                                      \
    switch (S_) {                                                 \
    case 1: { constexpr int S = 1; __VA_ARGS__; } break;          \
    case 2: { constexpr int S = 2; __VA_ARGS__; } break;          \
    case 3: { constexpr int S = 3; __VA_ARGS__; } break;          \
    default: return hipErrorInvalidValue;                         \
    }
#define DN_NQ_SWITCH(N_, ...)                                     \
    switch (N_) {                                                 \
    case 32: { constexpr int NQ = 2; __VA_ARGS__; } break;        \
    case 64: { constexpr int NQ = 4; __VA_ARGS__; } break;        \
    case 128: { constexpr int NQ = 8; __VA_ARGS__; } break;       \
    default: return hipErrorInvalidValue;                         \
    }
#define DN_NBP_SWITCH(nbp_, ...)                                  \
    switch (nbp_) {                                               \
    case 8: { constexpr int NBP = 8; __VA_ARGS__; } break;        \
    case 16: { constexpr int NBP = 16; __VA_ARGS__; } break;      \
    case 24: { constexpr int NBP = 24; __VA_ARGS__; } break;      \
    default: return hipErrorInvalidValue;                         \
    }
#define DN_SWITCH(ch, S_, N_, nbp_, ...) \
    DN_CH_SWITCH(ch, DN_S_SWITCH(S_, DN_NQ_SWITCH(N_, DN_NBP_SWITCH(nbp_, __VA_ARGS__))))

// copies of a layer: Wr, Wt, then (S = 3) Wt's and Wr's low pieces
struct DnW {
    const hw *r, *t, *rl, *tl;
};
DnW dn_w(const void *wdn, LayerShape ls, int S)
{
    const size_t e = (size_t)kpad_of(ls) * ls.wout;
    const hw *b = static_cast<const hw *>(wdn);
    DnW w{b, b + e, nullptr, nullptr};
    if (S == 3) {
        w.tl = b + 2 * e;
        w.rl = b + 3 * e;
    }
    return w;
}

}  // namespace

// LDS of the largest instantiation a layer shape can take (5 channels, S = 3)
static size_t dn_lds_worst(LayerShape ls)
{
    size_t m = 0;
    auto f = [&](auto nq, auto nbp) {
        constexpr int NQ = decltype(nq)::value, NBP = decltype(nbp)::value;
        m = std::max({FwdDn<2, 2, 3, NQ, NBP>::lds(), DxDn<2, 2, 3, NQ, NBP>::lds(),
                      DwDn<2, 2, 3, NQ, NBP>::lds(), DwDn<0, 0, 3, NQ, NBP>::lds()});
        return hipSuccess;
    };
    auto g = [&]() -> hipError_t {
        DN_NQ_SWITCH(ls.wout, DN_NBP_SWITCH(nbp_of(ls.nb),
                     f(std::integral_constant<int, NQ>{}, std::integral_constant<int, NBP>{})));
        return hipSuccess;
    };
    if (g() != hipSuccess) return ~(size_t)0;
    return m;
}

bool dn_supported(LayerShape ls, bool first)
{
    return !first && ls.win >= 4 && (ls.wout == 32 || ls.wout == 64 || ls.wout == 128) && ls.nb >= 4 &&
           ls.nb <= 24 && dn_lds_worst(ls) <= (size_t)DN_LDS_MAX;
}

size_t dn_w_bytes(LayerShape ls, int S)
{
    const size_t e = (size_t)kpad_of(ls) * ls.wout;
    return (size_t)(S == 3 ? 4 : 2) * e * sizeof(hw);
}

hipError_t launch_w_prep_dn(const float *W, void *wdn, LayerShape ls, int S, hipStream_t st)
{
    const int kpad = kpad_of(ls);
    const int64_t tot = (int64_t)kpad * ls.wout;
    hw *b = static_cast<hw *>(wdn);
    const size_t e = (size_t)tot;
    k_w_prep<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(W, b, b + e, S == 3 ? b + 3 * e : nullptr,
                                                          S == 3 ? b + 2 * e : nullptr, ls.win, ls.nb,
                                                          nbp_of(ls.nb), ls.wout, kpad);
    return hipGetLastError();
}

hipError_t launch_fwd_dn(ChanCfg ch, const float *zin, const void *wdn, float *zout, int64_t n, LayerShape ls,
                         const GridP<float> &g, int S, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const DnW w = dn_w(wdn, ls, S);
    const float zoff = -g.lo * g.inv_w;
    const unsigned blocks = (unsigned)((n + DN_P - 1) / DN_P);
    DN_SWITCH(ch, S, ls.wout, nbp_of(ls.nb), {
        auto kf = k_fwd_dn<O0, O1, S, NQ, NBP>;
        const size_t lds = FwdDn<O0, O1, S, NQ, NBP>::lds();
        set_lds_limit((const void *)kf);
        kf<<<blocks, DN_T, lds, st>>>(zin, w.t, w.tl, zout, n, ls.win, kpad_of(ls), g.inv_w, zoff);
    });
    return hipGetLastError();
}

hipError_t launch_dx_dn(ChanCfg ch, const float *zin, const float *ybar, const void *wdn, float *zbar,
                        int64_t n, LayerShape ls, const GridP<float> &g, int S, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const DnW w = dn_w(wdn, ls, S);
    const float zoff = -g.lo * g.inv_w;
    const unsigned blocks = (unsigned)((n + DN_P - 1) / DN_P);
    DN_SWITCH(ch, S, ls.wout, nbp_of(ls.nb), {
        auto kf = k_dx_dn<O0, O1, S, NQ, NBP>;
        const size_t lds = DxDn<O0, O1, S, NQ, NBP>::lds();
        set_lds_limit((const void *)kf);
        kf<<<blocks, DN_T, lds, st>>>(zin, ybar, w.r, w.rl, zbar, n, ls.win, g.inv_w, zoff);
    });
    return hipGetLastError();
}

int dw_dn_row_blocks(LayerShape ls) { return (ls.win + 2 * (DW_T / 64) - 1) / (2 * (DW_T / 64)); }

int dw_dn_splits(int64_t n, LayerShape ls)
{
    if (n <= 0) return 0;
    // about 2048 blocks, slices of at least 256 points, a multiple of 8
    // slices when there are 8 or more (the XCD-aware order)
    const int nkb = dw_dn_row_blocks(ls);
    int64_t s = std::max<int64_t>(1, 2048 / nkb);
    s = std::min<int64_t>(s, std::max<int64_t>(1, n / 256));
    if (s >= 8) s = s / 8 * 8;
    return (int)s;
}

hipError_t launch_dw_dn(ChanCfg ch, const float *zin, const float *ybar, float *part, int nsplit, int64_t n,
                        LayerShape ls, const GridP<float> &g, int S, hipStream_t st)
{
    if (n <= 0 || nsplit <= 0) return hipSuccess;
    const float zoff = -g.lo * g.inv_w;
    const int nkb = dw_dn_row_blocks(ls);
    const unsigned blocks = (unsigned)(nkb * nsplit);
    DN_SWITCH(ch, S, ls.wout, nbp_of(ls.nb), {
        auto kf = k_dw_dn<O0, O1, S, NQ, NBP>;
        const size_t lds = DwDn<O0, O1, S, NQ, NBP>::lds();
        set_lds_limit((const void *)kf);
        kf<<<blocks, DW_T, lds, st>>>(zin, ybar, part, n, ls.win, ls.nb, nsplit, nkb, g.inv_w, zoff);
    });
    return hipGetLastError();
}

}  // namespace hrk
