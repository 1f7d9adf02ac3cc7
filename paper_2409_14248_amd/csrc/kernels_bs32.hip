// kernels_bs32.hip -- FP32 matrix-core kernels of one KAN layer for the
// paper's HR basis with k = 3 supports and order m = 4.
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
// Window: in the scaled coordinate zt (supports of width 2, knots at
// multiples of 0.5) a point in interval q = floor(2 zt) has live functions
// q..q+3 clipped to 0..nb-1. Every kernel uses the 4-row window
// qa..qa+3 with qa = clamp(q, 0, nb-4), which holds all live functions, and
// evaluates each window row's bump directly (zero off its support), so row
// addresses are fixed offsets from one base and no lane needs a select.
#include <algorithm>
#include <cstdlib>

#include "internal.h"
#include "kernels_bs.h"

namespace hrk {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;                 // threads of the 4-wave kernels
constexpr int NT8 = 512;                // threads of the 8-wave kernels
constexpr int PW = 16;                  // points per wave
constexpr int TP = 8 * PW;              // points per tile of an 8-wave block
// inputs per staged jet chunk: both inputs of a first layer, else 8 (4 for
// 5-channel sets, whose chunks are larger); hidden widths are multiples of 8
constexpr int kj_of(bool first, int C) { return first ? 2 : (C <= 4 ? 8 : 4); }
constexpr int LDS_FWD = 80 * 1024;      // per 8-wave block: two blocks per CU

// Output groups of the 8-wave kernels: the waves of a block split the outputs
// into OG groups (tiles of 128/OG points), so that a lane holds at most 8
// output quads; single-channel sets (boundary values) always split in 4, which
// gives their small point counts 4 times as many tiles.
constexpr int og_of(int C, int NQ) { return C == 1 ? 4 : NQ / 8; }

// Waves per SIMD the 8-wave kernels are compiled for: two blocks per CU
// (registers <= 128) when a point's channels fit one 4-row group.
template <int O0, int O1, int NQ> constexpr int fwd_waves() { return Ch<O0, O1>::C <= 4 ? 4 : 2; }

// Broadcast lane T of each quad (DPP quad_perm [T,T,T,T]).
template <int T>
__device__ __forceinline__ float qbcast(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), T * 0x55, 0xF, 0xF, true));
}

// Sum over the 4 lanes of each quad (result in every lane of the quad).
__device__ __forceinline__ float quad_sum(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));
    return v;
}

// Window start clamp(floor(2 zt), 0, nb - 4); a NaN coordinate gives 0 so
// that the bumps evaluated there carry the NaN. Needs nb >= 4.
__device__ __forceinline__ int window_k3(float zt, int nb)
{
    return (int)fminf(fmaxf(2.f * zt, 0.f), (float)(nb - 4));
}

// Bump b (k = 3, m = 4) at scaled coordinate zt, derivatives up to ND (in
// the unscaled coordinate): a = zt - (b-3)/2 and be = 2 - a are the
// distances to the support ends; with t = a be and d = be - a,
//   v = t^4, v' = 4 w t^3 d, v'' = 4 w^2 t^2 (3 d^2 - 2 t),
//   v''' = 24 w^3 t d (d^2 - 3 t),   w = inv_w,
// and zero off the open support (a NaN coordinate propagates).
template <int ND>
__device__ __forceinline__ void bump_k3m4(float zt, int b, float inv_w, float *v)
{
    const float a = zt - 0.5f * (float)b + 1.5f;
    const float be = 2.f - a;
    const bool in = !(a <= 0.f) && !(be <= 0.f);
    const float t = a * be, d = be - a, t2 = t * t;
    v[0] = in ? t2 * t2 : 0.f;
    v[1] = in ? (4.f * inv_w) * (t2 * t) * d : 0.f;
    if constexpr (ND >= 2) v[2] = in ? (4.f * inv_w * inv_w) * t2 * (3.f * d * d - 2.f * t) : 0.f;
    if constexpr (ND >= 3) v[3] = in ? (24.f * inv_w * inv_w * inv_w) * t * d * (d * d - 3.f * t) : 0.f;
}

// Feature of channel c as a0 v + a1 v' + a2 v'' (the chain rule of the jets):
//   U: (1, -, -)  X: (0, X, -)  XX: (0, XX, X^2)  Y: (0, Y, -)  YY: (0, YY, Y^2)
// src1 / src2 are the jet channels that give a1 and sqrt(a2); C (one past the
// last channel) names a staged zero row.
template <int O0, int O1>
__device__ __forceinline__ void channel_sources(int c, float &a0, int &src1, int &src2)
{
    using CH = Ch<O0, O1>;
    constexpr int C = CH::C;
    a0 = (c == CH::U) ? 1.f : 0.f;
    src1 = C;
    src2 = C;
    if (c == CH::X || c == CH::XX || c == CH::Y || c == CH::YY) src1 = c;
    if (CH::XX >= 0 && c == CH::XX) src2 = CH::X;
    if (CH::YY >= 0 && c == CH::YY) src2 = CH::Y;
}

// Stage weight rows [r0, r0 + nrows) (N floats each) into LDS, row stride NS.
template <int BLK>
__device__ __forceinline__ void stage_rows(float *sW, const float *__restrict__ W, int r0, int nrows,
                                           int N, int NS)
{
    const int n4 = N / 4;
    for (int e = threadIdx.x; e < nrows * n4; e += BLK) {
        const int r = e / n4, c4 = e % n4;
        *reinterpret_cast<f4 *>(sW + r * NS + 4 * c4) =
            *reinterpret_cast<const f4 *>(W + (size_t)(r0 + r) * N + 4 * c4);
    }
}

// ---------------------------------------------------------------------------
// BF16 products (S > 0). A product a*b of FP32 values is taken as S BF16
// matrix-core products with FP32 accumulation: a = a_hi + a_lo and
// b = b_hi + b_lo (round to nearest even), S = 1: a_hi b_hi; S = 2: adds
// a_lo b_hi; S = 3: adds a_hi b_lo. In the forward and input-bar
// contractions b is the weight; in the weight gradient a is the feature and
// b the output bar. The 4x4x4 BF16 MFMA takes K = 4 per block: the 4 window
// rows (forward), 4 outputs (input bars) or 4 jet channels (gradient).
// ---------------------------------------------------------------------------
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// {a, b} rounded to BF16, a in the low half.
__device__ __forceinline__ unsigned int pk_bf16(float a, float b)
{
    return __builtin_bit_cast(unsigned int, __builtin_convertvector((f2){a, b}, bf2));
}
__device__ __forceinline__ float bf16_lo_f(unsigned int w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi_f(unsigned int w) { return __uint_as_float(w & 0xffff0000u); }

// hi and lo BF16 pieces of 4 FP32 values, packed as MFMA operands
__device__ __forceinline__ void split4(const float *v, s4 &hi, s4 &lo)
{
    const unsigned int h0 = pk_bf16(v[0], v[1]), h1 = pk_bf16(v[2], v[3]);
    const unsigned int l0 = pk_bf16(v[0] - bf16_lo_f(h0), v[1] - bf16_hi_f(h0));
    const unsigned int l1 = pk_bf16(v[2] - bf16_lo_f(h1), v[3] - bf16_hi_f(h1));
    hi = __builtin_bit_cast(s4, (u2){h0, h1});
    lo = __builtin_bit_cast(s4, (u2){l0, l1});
}
__device__ __forceinline__ s4 hi4(const float *v)
{
    return __builtin_bit_cast(s4, (u2){pk_bf16(v[0], v[1]), pk_bf16(v[2], v[3])});
}
__device__ __forceinline__ s4 mk4(unsigned int a, unsigned int b) { return __builtin_bit_cast(s4, (u2){a, b}); }

__device__ __forceinline__ f4 mfma_bf16(s4 a, s4 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, c, 0, 0, 0);
}

// Stage weight rows of `nin` inputs starting at input i0 as BF16 row pairs:
// word (il, b, j) = {W[(i0+il)*nb + b][j], W[(i0+il)*nb + b + 1][j]} for
// b = 0..nb-2, row stride NS words. LO = true stores the low pieces
// W - bf16(W) instead.
template <int BLK, bool LO>
__device__ __forceinline__ void stage_pairs(unsigned int *sP, const float *__restrict__ W, int i0, int nin,
                                            int nb, int N, int NS)
{
    const int n4 = N / 4, np = nb - 1;
    for (int e = threadIdx.x; e < nin * np * n4; e += BLK) {
        const int c4 = e % n4, r = e / n4;
        const int il = r / np, b = r % np;
        const float *w0 = W + (size_t)((i0 + il) * nb + b) * N + 4 * c4;
        const f4 a = *reinterpret_cast<const f4 *>(w0);
        const f4 c = *reinterpret_cast<const f4 *>(w0 + N);
        u4 o;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const unsigned int h = pk_bf16(a[q], c[q]);
            o[q] = LO ? pk_bf16(a[q] - bf16_lo_f(h), c[q] - bf16_hi_f(h)) : h;
        }
        *reinterpret_cast<u4 *>(sP + (il * np + b) * NS + 4 * c4) = o;
    }
}

// Stage weight rows [r0, r0 + nrows) as BF16, row-major, NSH halfwords per
// row (LO: the low pieces).
template <int BLK, bool LO>
__device__ __forceinline__ void stage_rows_bf16(unsigned short *sH, const float *__restrict__ W, int r0,
                                                int nrows, int N, int NSH)
{
    const int n4 = N / 4;
    for (int e = threadIdx.x; e < nrows * n4; e += BLK) {
        const int r = e / n4, c4 = e % n4;
        const f4 a = *reinterpret_cast<const f4 *>(W + (size_t)(r0 + r) * N + 4 * c4);
        unsigned int h0 = pk_bf16(a[0], a[1]), h1 = pk_bf16(a[2], a[3]);
        if (LO) {
            h0 = pk_bf16(a[0] - bf16_lo_f(h0), a[1] - bf16_hi_f(h0));
            h1 = pk_bf16(a[2] - bf16_lo_f(h1), a[3] - bf16_hi_f(h1));
        }
        *reinterpret_cast<u2 *>(sH + r * NSH + 4 * c4) = (u2){h0, h1};
    }
}

// A chunk of KJ inputs' jets for a tile of TPC points, prefetched into
// registers one chunk ahead and stored to LDS as [input][channel][point] with
// C + 1 channel rows per input (the last one stays zero).
template <int O0, int O1, bool FIRST, int BLK, int TPC, int KJ>
struct JetChunk {
    static constexpr int C = Ch<O0, O1>::C;
    static constexpr int CS = (C + 1) * TPC;     // floats per staged input
    static constexpr int E = KJ * C * TPC;
    static constexpr int R = (E + BLK - 1) / BLK;
    float r[R];

    __device__ __forceinline__ void load(const float *__restrict__ zin, int64_t n, int win,
                                         int64_t tile, int jc)
    {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int e = threadIdx.x + k * BLK;
            const int pp = e % TPC, rest = e / TPC, c = rest % C, il = rest / C;
            const int i = jc * KJ + il;
            const int64_t p = tile * TPC + pp;
            const bool ok = e < E && i < win && p < n;
            const int ic = ok ? i : 0;
            const int64_t pc = ok ? p : 0;
            float v;
            if constexpr (FIRST) {
                float zj[C];
                input_jets<float, O0, O1>(zin, pc, ic, zj);
                v = zj[c];
            } else {
                v = zin[(int64_t)(c * win + ic) * n + pc];
            }
            r[k] = ok ? v : 0.f;
        }
    }
    __device__ __forceinline__ void store(float *sZ) const
    {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int e = threadIdx.x + k * BLK;
            if (e < E) sZ[e + (e / (C * TPC)) * TPC] = r[k];
        }
    }
    __device__ __forceinline__ static void zero_rows(float *sZ)
    {
        for (int e = threadIdx.x; e < KJ * TPC; e += BLK) sZ[(e / TPC) * CS + C * TPC + e % TPC] = 0.f;
    }
};

// ---------------------------------------------------------------------------
// forward: zout[c][j][p] = sum_i sum_t W[i*nb + qa + t][j] * A_c(p, i, t)
// Persistent 8-wave blocks walk tiles of points, 16 per wave; for N > 32
// the waves also split the outputs into OG = N/32 groups (tiles of 128/OG
// points), so a lane always holds 8 output quads. The block's weight rows
// are staged once when they fit (KI >= win), else per chunk of KI inputs.
// Block column s owns outputs j = og*32 + s*8 + k.
// S = 0: FP32, one 4x4x1 MFMA per window row t (K = 1). S > 0: BF16, one
// 4x4x4 MFMA per product term with K = the 4 window rows; the weights are
// staged as BF16 row pairs, so a lane's B operand for output j is the two
// words (qa, qa+1) and (qa+2, qa+3) of column j.
// ---------------------------------------------------------------------------
template <int O0, int O1, bool FIRST, int NQ, int S>
__global__ __launch_bounds__(NT8, (fwd_waves<O0, O1, NQ>())) void k_fwd_bs(const float *__restrict__ zin,
                                                   const float *__restrict__ W,
                                                   float *__restrict__ zout, int64_t n, int win,
                                                   int KI, GridP<float> g, BatchMap bm)
{
    constexpr int C = Ch<O0, O1>::C;
    constexpr int RG = (C + 3) / 4;
    constexpr int N = 4 * NQ;
    constexpr int NS = N + 4;
    constexpr int OG = og_of(C, NQ);         // output groups: the waves split the outputs
    constexpr int NQW = NQ / OG;             // output quads per lane
    constexpr int VW = NQW >= 4 ? 4 : 2;     // outputs per LDS weight read
    constexpr int TPK = TP / OG;             // points per tile
    constexpr int KJ = kj_of(FIRST, C);
    using JCk = JetChunk<O0, O1, FIRST, NT8, TPK, KJ>;
    constexpr int CS = JCk::CS;
    extern __shared__ __align__(16) float smem[];
    const int nb = g.nb;
    const float inv_w = g.inv_w, zoff = -g.lo * g.inv_w;
    // FP32: KI*nb rows of NS floats; BF16: KI*(nb-1) pair rows of NS words (x2 for S = 3)
    const int wrows = S == 0 ? nb : nb - 1;
    float *sW = smem;
    unsigned int *sP = reinterpret_cast<unsigned int *>(smem);
    unsigned int *sPl = sP + KI * wrows * NS;
    float *sZ = smem + KI * wrows * NS * (S == 3 ? 2 : 1);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int bl = lane >> 2, s = lane & 3;
    const int og = wv % OG, pt = (wv / OG) * PW + bl;
    const int col0 = og * 4 * NQW + s * NQW;   // this lane's first output
    const int64_t ntiles = (n + TPK - 1) / TPK;
    const int njc = win / KJ;                // win is a multiple of KJ
    const bool single = KI >= win;
    // batched: the weights of the tile's instance, restaged when it changes
    const bool batched = bm.tile_inst != nullptr;
    const float *Wc = W;
    int cur_inst = -1;
    auto stage = [&](int i0, int nin) {
        if constexpr (S == 0) {
            stage_rows<NT8>(sW, Wc, i0 * nb, nin * nb, N, NS);
        } else {
            stage_pairs<NT8, false>(sP, Wc, i0, nin, nb, N, NS);
            if constexpr (S == 3) stage_pairs<NT8, true>(sPl, Wc, i0, nin, nb, N, NS);
        }
    };
    JCk::zero_rows(sZ);

    // this lane's channel rows: coefficient sources (offsets in a staged input)
    float a0[RG];
    int off1[RG], off2[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
        int s1, s2;
        channel_sources<O0, O1>(4 * r + s, a0[r], s1, s2);
        off1[r] = s1 * TPK + pt;
        off2[r] = s2 * TPK + pt;
    }

    JCk pre;
    int64_t tile = blockIdx.x;
    int jc = 0;
    if (tile < ntiles) pre.load(zin, n, win, tile, 0);   // in flight while the weights are staged
    if (single && !batched) stage(0, win);
    f4 acc[RG][NQW];
    while (tile < ntiles) {
        if (jc == 0) {
#pragma unroll
            for (int r = 0; r < RG; ++r)
#pragma unroll
                for (int k = 0; k < NQW; ++k) acc[r][k] = (f4){0.f, 0.f, 0.f, 0.f};
        }
        const int ib = jc * KJ;
        const int iW = single ? 0 : (ib / KI) * KI;
        bool restage = false;
        if (batched && jc == 0) {
            const int inst = bm.tile_inst[(tile * TPK) >> 7];
            restage = inst != cur_inst;
            cur_inst = inst;
            Wc = W + (int64_t)inst * bm.w_stride;
        }
        __syncthreads();
        pre.store(sZ);
        if ((!single && ib % KI == 0) || restage) stage(iW, min(KI, win - iW));
        __syncthreads();
        const int64_t cur_tile = tile;
        if (++jc == njc) {
            jc = 0;
            tile += gridDim.x;
        }
        if (tile < ntiles) pre.load(zin, n, win, tile, jc);

#pragma unroll
        for (int il = 0; il < KJ; ++il) {
            const int i = ib + il;
            const float *zc = sZ + il * CS;
            const float zt = zc[pt] * inv_w + zoff;
            const int qa = window_k3(zt, nb);
            float v[3];
            bump_k3m4<2>(zt, qa + s, inv_w, v);        // this lane: window row t = s
            float vt[4][3];
            vt[0][0] = qbcast<0>(v[0]); vt[0][1] = qbcast<0>(v[1]); vt[0][2] = qbcast<0>(v[2]);
            vt[1][0] = qbcast<1>(v[0]); vt[1][1] = qbcast<1>(v[1]); vt[1][2] = qbcast<1>(v[2]);
            vt[2][0] = qbcast<2>(v[0]); vt[2][1] = qbcast<2>(v[1]); vt[2][2] = qbcast<2>(v[2]);
            vt[3][0] = qbcast<3>(v[0]); vt[3][1] = qbcast<3>(v[1]); vt[3][2] = qbcast<3>(v[2]);
            float a1[RG], a2[RG];
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                a1[r] = zc[off1[r]];
                const float x2 = zc[off2[r]];
                a2[r] = x2 * x2;
            }
            if constexpr (S == 0) {
                const float *wr = sW + ((i - iW) * nb + qa) * NS + col0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    float bw[NQW];
#pragma unroll
                    for (int k = 0; k < NQW; k += VW) {
                        if constexpr (VW == 4) {
                            const f4 w4 = *reinterpret_cast<const f4 *>(wr + t * NS + k);
                            bw[k + 0] = w4[0];
                            bw[k + 1] = w4[1];
                            bw[k + 2] = w4[2];
                            bw[k + 3] = w4[3];
                        } else {
                            const f2 w2 = *reinterpret_cast<const f2 *>(wr + t * NS + k);
                            bw[k + 0] = w2[0];
                            bw[k + 1] = w2[1];
                        }
                    }
#pragma unroll
                    for (int r = 0; r < RG; ++r) {
                        const float A = a0[r] * vt[t][0] + a1[r] * vt[t][1] + a2[r] * vt[t][2];
#pragma unroll
                        for (int k = 0; k < NQW; ++k)
                            acc[r][k] = __builtin_amdgcn_mfma_f32_4x4x1f32(A, bw[k], acc[r][k], 0, 0, 0);
                    }
                }
            } else {
                // A operand: this lane's channel row over the 4 window rows
                s4 ah[RG], al[RG];
#pragma unroll
                for (int r = 0; r < RG; ++r) {
                    float At[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) At[t] = a0[r] * vt[t][0] + a1[r] * vt[t][1] + a2[r] * vt[t][2];
                    if constexpr (S >= 2)
                        split4(At, ah[r], al[r]);
                    else
                        ah[r] = hi4(At);
                }
                const int prow = ((i - iW) * (nb - 1) + qa) * NS + col0;
#pragma unroll
                for (int k0 = 0; k0 < NQW; k0 += VW) {
                    unsigned int p01[VW], p23[VW], q01[VW], q23[VW];
                    auto ld = [&](const unsigned int *src, unsigned int *dst) {
                        if constexpr (VW == 4) {
                            const u4 v = *reinterpret_cast<const u4 *>(src);
                            dst[0] = v[0]; dst[1] = v[1]; dst[2] = v[2]; dst[3] = v[3];
                        } else {
                            const u2 v = *reinterpret_cast<const u2 *>(src);
                            dst[0] = v[0]; dst[1] = v[1];
                        }
                    };
                    ld(sP + prow + k0, p01);
                    ld(sP + prow + 2 * NS + k0, p23);
                    if constexpr (S == 3) {
                        ld(sPl + prow + k0, q01);
                        ld(sPl + prow + 2 * NS + k0, q23);
                    }
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        const int k = k0 + e;
                        const s4 bh = mk4(p01[e], p23[e]);
#pragma unroll
                        for (int r = 0; r < RG; ++r) {
                            acc[r][k] = mfma_bf16(ah[r], bh, acc[r][k]);
                            if constexpr (S >= 2) acc[r][k] = mfma_bf16(al[r], bh, acc[r][k]);
                            if constexpr (S == 3) acc[r][k] = mfma_bf16(ah[r], mk4(q01[e], q23[e]), acc[r][k]);
                        }
                    }
                }
            }
        }
        const int64_t p = cur_tile * TPK + pt;
        if (jc == 0 && p < n) {                 // the tile is complete
#pragma unroll
            for (int r = 0; r < RG; ++r)
#pragma unroll
                for (int k = 0; k < NQW; ++k)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = 4 * r + e;
                        if (c < C) zout[(int64_t)(c * N + col0 + k) * n + p] = acc[r][k][e];
                    }
        }
    }
}

// ---------------------------------------------------------------------------
// input bars: Ab_c(p,i,t) = sum_j W[i*nb + qa + t][j] * ybar[c][j][p]; then
// the adjoint of the features through v..v''' gives zbar[.][i][p].
// Block row = channel, block column = window row t. S = 0: FP32, K = one
// output per 4x4x1 MFMA; S > 0: BF16, K = 4 outputs per 4x4x4 MFMA, the
// bars split once per tile and the weights staged as BF16 rows. Output quads
// accumulate in up to 4 separate chains (added in order at the end) so
// consecutive MFMAs are independent.
// ---------------------------------------------------------------------------
template <int O0, int O1, int NQ, int S>
__global__ __launch_bounds__(NT8, (fwd_waves<O0, O1, NQ>())) void k_dx_bs(const float *__restrict__ zin,
                                                  const float *__restrict__ ybar,
                                                  const float *__restrict__ W,
                                                  float *__restrict__ zbar, int64_t n, int win,
                                                  int KI, GridP<float> g, BatchMap bm)
{
    constexpr int C = Ch<O0, O1>::C;
    constexpr int RG = (C + 3) / 4;
    constexpr int N = 4 * NQ;
    constexpr int NS = N + 4;                // FP32 row stride (floats)
    constexpr int NSH = N + 8;               // BF16 row stride (halfwords)
    constexpr int SA = S >= 2 ? 2 : 1;       // pieces of the bar operand
    constexpr int OG = og_of(C, NQ);         // output groups: the waves split the outputs
    constexpr int NQW = NQ / OG;             // output quads per wave
    constexpr int TPK = TP / OG;             // points per tile
    constexpr int KJ = kj_of(false, C);
    using JCk = JetChunk<O0, O1, false, NT8, TPK, KJ>;
    constexpr int CS = JCk::CS;
    extern __shared__ __align__(16) float smem[];
    const int nb = g.nb;
    const float inv_w = g.inv_w, zoff = -g.lo * g.inv_w;
    float *sW = smem;
    unsigned short *sH = reinterpret_cast<unsigned short *>(smem);
    unsigned short *sHl = sH + KI * nb * NSH;
    const int wfloats = S == 0 ? KI * nb * NS : KI * nb * NSH / 2 * (S == 3 ? 2 : 1);
    float *sZ = smem + wfloats;
    float *sRed = sZ + KJ * CS;              // [OG][KJ][C][TPK] partial input bars (OG > 1)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int bl = lane >> 2, s = lane & 3;
    const int og = wv % OG, pt = (wv / OG) * PW + bl;
    const int jb = og * 4 * NQW;             // this wave's first output
    const int64_t ntiles = (n + TPK - 1) / TPK;
    const int njc = win / KJ;                // win is a multiple of KJ
    const bool single = KI >= win;
    const bool batched = bm.tile_inst != nullptr;
    const float *Wc = W;
    int cur_inst = -1;
    auto stage = [&](int i0, int nin) {
        if constexpr (S == 0) {
            stage_rows<NT8>(sW, Wc, i0 * nb, nin * nb, N, NS);
        } else {
            stage_rows_bf16<NT8, false>(sH, Wc, i0 * nb, nin * nb, N, NSH);
            if constexpr (S == 3) stage_rows_bf16<NT8, true>(sHl, Wc, i0 * nb, nin * nb, N, NSH);
        }
    };
    JCk pre;
    int64_t tile = blockIdx.x;
    int jc = 0;
    if (tile < ntiles) pre.load(zin, n, win, tile, 0);   // in flight while the weights are staged
    if (single && !batched) stage(0, win);
    // the output bars of this lane's channel rows: FP32 (S = 0) or BF16 pieces
    float yb[S == 0 ? RG : 1][S == 0 ? 4 * NQW : 1];
    s4 ybp[S == 0 ? 1 : RG][S == 0 ? 1 : NQW][SA];
    while (tile < ntiles) {
        const int64_t cur_tile = tile;
        const int64_t p = cur_tile * TPK + pt;
        const bool ok = p < n;
        if (jc == 0) {
            const int64_t pc = ok ? p : 0;
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                const int c = 4 * r + s;
                const int cc = c < C ? c : 0;
#pragma unroll
                for (int j4 = 0; j4 < NQW; ++j4) {
                    float y[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float v = ybar[(int64_t)(cc * N + jb + 4 * j4 + e) * n + pc];
                        y[e] = (ok && c < C) ? v : 0.f;
                    }
                    if constexpr (S == 0) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) yb[r][4 * j4 + e] = y[e];
                    } else if constexpr (SA == 2) {
                        split4(y, ybp[r][j4][0], ybp[r][j4][1]);
                    } else {
                        ybp[r][j4][0] = hi4(y);
                    }
                }
            }
        }
        const int ib = jc * KJ;
        const int iW = single ? 0 : (ib / KI) * KI;
        bool restage = false;
        if (batched && jc == 0) {
            const int inst = bm.tile_inst[(cur_tile * TPK) >> 7];
            restage = inst != cur_inst;
            cur_inst = inst;
            Wc = W + (int64_t)inst * bm.w_stride;
        }
        __syncthreads();
        pre.store(sZ);
        if ((!single && ib % KI == 0) || restage) stage(iW, min(KI, win - iW));
        __syncthreads();
        if (++jc == njc) {
            jc = 0;
            tile += gridDim.x;
        }
        if (tile < ntiles) pre.load(zin, n, win, tile, jc);

#pragma unroll
        for (int il = 0; il < KJ; ++il) {
            const int i = ib + il;
            const float *zc = sZ + il * CS + pt;
            float zj[C];
#pragma unroll
            for (int c = 0; c < C; ++c) zj[c] = zc[c * TPK];
            const float zt = zj[0] * inv_w + zoff;
            const int qa = window_k3(zt, nb);
            constexpr int NCH = S == 0 ? 4 : (NQW >= 4 ? 4 : NQW);   // independent accumulation chains
            f4 ab[NCH][RG];
#pragma unroll
            for (int h = 0; h < NCH; ++h)
#pragma unroll
                for (int r = 0; r < RG; ++r) ab[h][r] = (f4){0.f, 0.f, 0.f, 0.f};
            if constexpr (S == 0) {
                // this lane (column t = s) reads window row qa + s
                const float *wr = sW + ((i - iW) * nb + qa + s) * NS + jb;
#pragma unroll
                for (int j4 = 0; j4 < NQW; ++j4) {
                    const f4 w4 = *reinterpret_cast<const f4 *>(wr + 4 * j4);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
#pragma unroll
                        for (int r = 0; r < RG; ++r)
                            ab[e % NCH][r] = __builtin_amdgcn_mfma_f32_4x4x1f32(yb[r][4 * j4 + e], w4[e],
                                                                                ab[e % NCH][r], 0, 0, 0);
                }
            } else {
                const int hrow = ((i - iW) * nb + qa + s) * NSH + jb;
#pragma unroll
                for (int j4 = 0; j4 < NQW; ++j4) {
                    const s4 wh = __builtin_bit_cast(s4, *reinterpret_cast<const u2 *>(sH + hrow + 4 * j4));
                    s4 wl;
                    if constexpr (S == 3)
                        wl = __builtin_bit_cast(s4, *reinterpret_cast<const u2 *>(sHl + hrow + 4 * j4));
#pragma unroll
                    for (int r = 0; r < RG; ++r) {
                        f4 &a = ab[j4 % NCH][r];
                        a = mfma_bf16(ybp[r][j4][0], wh, a);
                        if constexpr (S >= 2) a = mfma_bf16(ybp[r][j4][SA - 1], wh, a);
                        if constexpr (S == 3) a = mfma_bf16(ybp[r][j4][0], wl, a);
                    }
                }
            }
            // lane (block, t): ab[.][r][e] = Abar of channel 4r+e for row t = s
            float v[4];
            bump_k3m4<3>(zt, qa + s, inv_w, v);
            float Ab[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float t = ab[0][c / 4][c % 4];
#pragma unroll
                for (int h = 1; h < NCH; ++h) t += ab[h][c / 4][c % 4];
                Ab[c] = t;
            }
            float zb[C];
#pragma unroll
            for (int c = 0; c < C; ++c) zb[c] = 0.f;
            features_adjoint<float, O0, O1>(v, zj, Ab, zb);
#pragma unroll
            for (int c = 0; c < C; ++c) zb[c] = quad_sum(zb[c]);
            if constexpr (OG == 1) {
                if (ok) {
#pragma unroll
                    for (int r = 0; r < RG; ++r) {
                        const int c = 4 * r + s;
                        float val = zb[0];
#pragma unroll
                        for (int cc = 1; cc < C; ++cc) val = (c == cc) ? zb[cc] : val;
                        if (c < C) zbar[(int64_t)(c * win + i) * n + p] = val;
                    }
                }
            } else if (s == 0) {
                // this wave's part of the sum over outputs; the groups are
                // added in order once the chunk is done
#pragma unroll
                for (int c = 0; c < C; ++c) sRed[((og * KJ + il) * C + c) * TPK + pt] = zb[c];
            }
        }
        if constexpr (OG > 1) {
            __syncthreads();
            for (int e = threadIdx.x; e < KJ * C * TPK; e += NT8) {
                const int pp = e % TPK, c = (e / TPK) % C, il = e / (TPK * C);
                const int64_t pq = cur_tile * TPK + pp;
                float v = sRed[((0 * KJ + il) * C + c) * TPK + pp];
#pragma unroll
                for (int o = 1; o < OG; ++o) v += sRed[((o * KJ + il) * C + c) * TPK + pp];
                if (pq < n) zbar[(int64_t)(c * win + ib + il) * n + pq] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient, block-sparse:
//   gW[i*nb + qa + t][j] += sum_c A_c(p, i, t) * ybar[c][j][p]
// One 4x4x1 MFMA block is (input feature, chunk of 4 outputs) of ONE point:
// rows = window row t, columns = 4 outputs, K = one jet channel (C MFMAs
// accumulate the channels). Each lane then adds its 4 results to rows
// qa..qa+3 of its input in an LDS copy of the gradient. A wave owns II
// inputs (disjoint gradient rows) and walks its points in a fixed order: each
// LDS word has a single writer and the sums are deterministic. Points go in
// pairs, so one point's matrix products overlap the other's
// read-add-write. The 4 waves of a block are WI input groups times WP = 4/WI
// point groups (WI < 4 when the layer has few inputs); each point group
// takes every WP-th point of the slice into its own gradient copy, and the
// copies are summed in order at the end. A block owns WI*II inputs and all
// N outputs of one slice; the next chunk of points is loaded while the
// current one is computed.
// ---------------------------------------------------------------------------
// points per staged chunk (a divisor of the block size): short per-point
// work (2 inputs per wave) takes larger chunks so the global loads stay ahead
// of the compute -- 32 points for 32-output layers (64 would double the
// block's LDS and halve its blocks per CU: no faster on 65,536 points, slower
// on 4,096); else 16, or 8 for wide 5-channel tiles (LDS)
constexpr int dw_pc_of(int NQ, int II, int C)
{
    return NQ >= 32 ? ((II == 2 && C <= 4) ? 16 : 8) : (II == 2 && NQ <= 8) ? 32 : 16;
}
template <int NQ, int II, int C> constexpr int dw_pc() { return dw_pc_of(NQ, II, C); }

template <int O0, int O1, bool FIRST, int NQ, int II, int S>
__global__ __launch_bounds__(NT) void k_dw_bs(const float *__restrict__ zin,
                                              const float *__restrict__ ybar,
                                              float *__restrict__ part, int64_t n, int win,
                                              int nsplit, int WI, GridP<float> g, BatchMap bm)
{
    constexpr int C = Ch<O0, O1>::C;
    constexpr int CP = C <= 4 ? 4 : 8;       // padded channel stride in LDS
    constexpr int N = 4 * NQ;
    constexpr int GS = N;                    // gradient row stride
    // input stride: 4*JC words of padding put the 8 blocks of a half-wave
    // (8/JC inputs x JC output chunks x 4 columns) on 32 distinct banks
    // whatever their rows
    constexpr int IB = 4 * II;               // staged inputs (WI * II of them real)
    constexpr int JC = 16 / II;              // 4-output chunks per MFMA
    constexpr int PASSES = NQ / JC;
    constexpr int PC = dw_pc<NQ, II, C>();
    constexpr int JS = IB * CP + 4;          // staged jets: stride per point
    constexpr int YS = N * CP + 4;           // staged bars: stride per point
    constexpr int EJ = C * IB * PC, EY = C * N * PC;
    constexpr int RJ = (EJ + NT - 1) / NT, RY = (EY + NT - 1) / NT;
    static_assert(PASSES >= 1 && JC * PASSES == NQ, "tile shape");
    extern __shared__ __align__(16) float smem[];
    const int nb = g.nb;
    const float inv_w = g.inv_w, zoff = -g.lo * g.inv_w;
    const int IS = nb * GS + 4 * JC;
    float *sG = smem;                                  // [WP][WI*II][IS]
    float *sJ = sG + IB * IS;                          // [PC][JS]
    float *sY = sJ + PC * JS;                          // [PC][YS]

    const int WP = 4 / WI, IBe = WI * II;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int blk = lane >> 2, s = lane & 3;
    const int wi = wv % WI, wp = wv / WI;
    const int ii = wi * II + blk / JC, jc = blk % JC;  // block-local input of this lane
    const int i0 = blockIdx.x * IBe;
    const int split = blockIdx.y;
    const int64_t per = ((n + nsplit - 1) / nsplit + PC - 1) / PC * PC;
    int64_t ps = (int64_t)split * per, pe = min(n, ps + per);
    if (bm.slices) {
        const int4 sl = bm.slices[split];
        ps = sl.y;
        pe = sl.z;
    }
    for (int e = threadIdx.x; e < IB * IS; e += NT) sG[e] = 0.f;
    float *gbase = sG + (wp * IBe + ii) * IS + 4 * jc + s;

    // staging: each thread's loads of a chunk start at fixed offsets from the
    // chunk's first point (computed once); LDS targets likewise
    const float *jsrc[RJ];
    int jdst[RJ], jpp[RJ];
    bool jok[RJ];
#pragma unroll
    for (int k = 0; k < RJ; ++k) {
        const int e = threadIdx.x + k * NT;
        const int pp = e % PC, rest = e / PC, il = rest % IB, c = rest / IB;
        jok[k] = e < EJ && il < IBe && i0 + il < win;
        const int ic = jok[k] ? i0 + il : 0;
        jpp[k] = pp;
        jdst[k] = pp * JS + il * CP + c;
        if constexpr (FIRST)
            jsrc[k] = zin + 2 * (int64_t)pp + ic;            // x[2p + i]; channel c from input_jets
        else
            jsrc[k] = zin + (int64_t)((jok[k] ? c : 0) * win + ic) * n + pp;
    }
    // bars: element e = threadIdx.x + k NT is point pp = e % PC (the same for
    // every k, PC dividing NT) of row e / PC = c N + j, so the k-th load is
    // the first one plus k (NT / PC) rows
    static_assert(NT % PC == 0, "chunk size must divide the block");
    // a launch may split the outputs over gridDim.z blocks: this block takes
    // outputs J0 .. J0 + N - 1 of NTOT
    const int NTOT = N * (int)gridDim.z, J0 = N * (int)blockIdx.z;
    const int ypp = threadIdx.x % PC, yrow0 = threadIdx.x / PC;
    float rj[RJ], ry[RY];
    auto load = [&](int64_t pc) {
#pragma unroll
        for (int k = 0; k < RJ; ++k) {
            const bool ok = jok[k] && pc + jpp[k] < pe;
            const int64_t o = ok ? pc : -(int64_t)jpp[k];   // a dead lane reads its row's first element
            float v;
            if constexpr (FIRST) {
                // input layer: jets of x_i are (x_i, d/dx0 = [i == 0], ..., d/dx1 = [i == 1], ...)
                const int e = threadIdx.x + k * NT;
                const int rest = e / PC, il = rest % IB, c = rest / IB;
                float zj[C];
                input_jets<float, O0, O1>(zin, ok ? pc + jpp[k] : 0, ok ? i0 + il : 0, zj);
                v = zj[c < C ? c : 0];
            } else {
                v = jsrc[k][o];
            }
            rj[k] = ok ? v : 0.f;
        }
        const bool yin = pc + ypp < pe;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const bool ok = yin && threadIdx.x + k * NT < EY;
            // this block's row c N + j is row c NTOT + J0 + j of the bars
            const int row = yrow0 + k * (NT / PC);
            const int grow = row + (row / N) * (NTOT - N) + J0;
            const float y = ybar[ok ? (int64_t)grow * n + ypp + pc : 0];   // a dead lane reads the first element
            ry[k] = ok ? y : 0.f;
        }
    };
    // one point's operands for this lane's input: window, features (row t = s)
    // and the output bars of this lane's columns
    struct Pt {
        int qa;
        float A[C];
        float yv[PASSES][CP];
    };
    auto prepare = [&](int pp, Pt &o) {
        float zj[CP];
#pragma unroll
        for (int c4 = 0; c4 < CP / 4; ++c4) {
            const f4 z4 = *reinterpret_cast<const f4 *>(sJ + pp * JS + ii * CP + 4 * c4);
            zj[4 * c4 + 0] = z4[0]; zj[4 * c4 + 1] = z4[1]; zj[4 * c4 + 2] = z4[2]; zj[4 * c4 + 3] = z4[3];
        }
        const float zt = zj[0] * inv_w + zoff;
        o.qa = window_k3(zt, nb);
        float v[3];
        bump_k3m4<2>(zt, o.qa + s, inv_w, v);
        features<float, O0, O1>(v, zj, o.A);
#pragma unroll
        for (int q = 0; q < PASSES; ++q)
#pragma unroll
            for (int c4 = 0; c4 < CP / 4; ++c4) {
                const f4 y4 = *reinterpret_cast<const f4 *>(sY + pp * YS + (4 * (q * JC + jc) + s) * CP + 4 * c4);
                o.yv[q][4 * c4 + 0] = y4[0]; o.yv[q][4 * c4 + 1] = y4[1];
                o.yv[q][4 * c4 + 2] = y4[2]; o.yv[q][4 * c4 + 3] = y4[3];
            }
    };
    // rows qa..qa+3 of this lane's input: the stored sums enter the MFMAs as
    // accumulators (no separate additions) and the results are written back;
    // the passes are interleaved so that consecutive MFMAs are independent
    auto rd = [&](const float *gp, f4 *d) {
#pragma unroll
        for (int q = 0; q < PASSES; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) d[q][r] = gp[r * GS + 4 * q * JC];
    };
    auto wr = [&](float *gp, const f4 *d) {
#pragma unroll
        for (int q = 0; q < PASSES; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) gp[r * GS + 4 * q * JC] = d[q][r];
    };
    auto mm = [&](const Pt &o, f4 *d) {
        if constexpr (S == 0) {
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int q = 0; q < PASSES; ++q)
                    d[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(o.A[c], o.yv[q][c], d[q], 0, 0, 0);
        } else {
            // K = 4 channels per 4x4x4 MFMA (channels beyond C are zero)
            constexpr int CG = CP / 4;
            s4 fh[CG], fl[CG];
#pragma unroll
            for (int g4 = 0; g4 < CG; ++g4) {
                float a4[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) a4[e] = (4 * g4 + e < C) ? o.A[(4 * g4 + e) < C ? 4 * g4 + e : 0] : 0.f;
                if constexpr (S >= 2)
                    split4(a4, fh[g4], fl[g4]);
                else
                    fh[g4] = hi4(a4);
            }
#pragma unroll
            for (int g4 = 0; g4 < CG; ++g4)
#pragma unroll
                for (int q = 0; q < PASSES; ++q) {
                    float y4[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) y4[e] = (4 * g4 + e < C) ? o.yv[q][4 * g4 + e] : 0.f;
                    s4 yh, yl;
                    if constexpr (S == 3)
                        split4(y4, yh, yl);
                    else
                        yh = hi4(y4);
                    d[q] = mfma_bf16(fh[g4], yh, d[q]);
                    if constexpr (S >= 2) d[q] = mfma_bf16(fl[g4], yh, d[q]);
                    if constexpr (S == 3) d[q] = mfma_bf16(fh[g4], yl, d[q]);
                }
        }
    };
    auto update = [&](const Pt &o) {
        f4 d[PASSES];
        float *g = gbase + o.qa * GS;
        rd(g, d);
        mm(o, d);
        wr(g, d);
    };

    if (ps < pe) load(ps);
    for (int64_t pc = ps; pc < pe; pc += PC) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RJ; ++k)
            if (threadIdx.x + k * NT < EJ) sJ[jdst[k]] = rj[k];
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int row = yrow0 + k * (NT / PC), j = row % N, c = row / N;
            if (threadIdx.x + k * NT < EY) sY[ypp * YS + j * CP + c] = ry[k];
        }
        __syncthreads();
        if (pc + PC < pe) load(pc + PC);         // next chunk in flight during this one
        const int npts = (int)min<int64_t>(PC, pe - pc);
        int pp = wp;
        // wide layers with one point group: points in fours, so that the
        // next points' operands are prepared while earlier ones update
        // (Poisson [2,64,64,64,1], 262,144 points: 2.02 -> 1.93 ms per
        // launch). Narrow layers keep pairs: the
        // registers of four points would halve the blocks per CU of their
        // smaller-LDS instances.
        if constexpr (NQ >= 16)
            if (WP == 1)
                for (; pp + 3 < npts; pp += 4) {
                    Pt a, b, c, d;
                    prepare(pp, a);
                    prepare(pp + 1, b);
                    prepare(pp + 2, c);
                    prepare(pp + 3, d);
                    update(a);
                    update(b);
                    update(c);
                    update(d);
                }
        for (; pp + WP < npts; pp += 2 * WP) {
            Pt a, b;
            prepare(pp, a);
            prepare(pp + WP, b);
            update(a);
            update(b);
        }
        if (pp < npts) {
            Pt a;
            prepare(pp, a);
            update(a);
        }
    }
    __syncthreads();
    const int64_t KN = (int64_t)win * nb * NTOT;
    const int gcopy = IBe * IS;
    for (int e = threadIdx.x; e < IBe * nb * N; e += NT) {
        const int row = e / N, col = e % N;
        const int il = row / nb, b = row % nb;
        if (i0 + il >= win) continue;
        const int at = il * IS + b * GS + col;
        float sum = sG[at];
        for (int w = 1; w < WP; ++w) sum += sG[w * gcopy + at];
        part[split * KN + (int64_t)(i0 * nb + row) * NTOT + J0 + col] = sum;
    }
}

static size_t dw_bs_lds(int C, int nb, int N, int II)
{
    const int CP = C <= 4 ? 4 : 8, IB = 4 * II, JC = 16 / II;
    const int PC = dw_pc_of(N / 4, II, C);
    return sizeof(float) *
           ((size_t)IB * (nb * N + 4 * JC) + (size_t)PC * (IB * CP + 4) + (size_t)PC * (N * CP + 4));
}

// ---------------------------------------------------------------------------
// last layer (one output): plain vector-ALU kernels
//
// They work with sums over the 4 window rows b = qa + r of one (point, input)
// in the support-midpoint form: u_r = clamp(zt + 1/2 - b/2, -1, 1) and
// t_r = 1 - u_r^2 (= a (2 - a) with a = u_r + 1; exactly zero off the
// support, so no row needs a select), d = -2 u_r, and with weights w_r
//   P0 = sum w t^4,  P1 = sum w t^3 u,  P2 = sum w t^2 (u^2 - 1/7),
//   P3 = sum w t u (u^2 - 3/7),
// the weighted sums of the bump and its derivatives are
//   sum w v = P0,  sum w dv = -8 iw P1,  sum w d2v = 56 iw^2 P2,
//   sum w d3v = -336 iw^3 P3   (iw = inv_w, dv = v', d2v = v'', d3v = v'''),
// so the chain rule of the jets is applied once per (point, input), not per
// row. A NaN coordinate is carried by adding it to t (sn = 1 + NaN).
// ---------------------------------------------------------------------------
template <int NP>
__device__ __forceinline__ void window_sums(float zt, float sn, int qa, const float *w4, float *P)
{
    const float c0 = zt + 0.5f - 0.5f * (float)qa;
#pragma unroll
    for (int k = 0; k < NP; ++k) P[k] = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float u = fminf(fmaxf(c0 - 0.5f * (float)r, -1.f), 1.f);
        const float u2 = u * u;
        const float t = sn - u2;
        const float t2 = t * t;
        P[0] = fmaf(w4[r], t2 * t2, P[0]);
        if constexpr (NP >= 2) P[1] = fmaf(w4[r], t2 * t * u, P[1]);
        if constexpr (NP >= 3) P[2] = fmaf(w4[r], t2 * (u2 - (1.f / 7.f)), P[2]);
        if constexpr (NP >= 4) P[3] = fmaf(w4[r], t * u * (u2 - (3.f / 7.f)), P[3]);
    }
}

__device__ __forceinline__ float nan_carrier(float zt) { return 1.f + (__builtin_isnan(zt) ? zt : 0.f); }

// u_c[p] = sum_i sum_r W[i*nb + qa + r] * A_c(p, i, r); 4 threads per point
// (consecutive lanes), each taking every 4th input with all its loads in
// flight, the 4 partial sums added across the quad.
constexpr int FL_U = 8;   // inputs per thread whose loads are in flight together
template <int O0, int O1>
__global__ __launch_bounds__(NT) void k_fwd_last(const float *__restrict__ zin,
                                                 const float *__restrict__ W,
                                                 float *__restrict__ out, int64_t n, int win,
                                                 GridP<float> g, BatchMap bm)
{
    using CH = Ch<O0, O1>;
    constexpr int C = CH::C;
    constexpr int NP = C > 1 ? 3 : 1;
    extern __shared__ float sW[];
    const int nb = g.nb;
    const float inv_w = g.inv_w, zoff = -g.lo * g.inv_w;
    const float k1 = -8.f * inv_w, k2 = 56.f * inv_w * inv_w;
    const float *Wb = W;
    if (bm.tile_inst) Wb += (int64_t)bm.tile_inst[((int64_t)blockIdx.x * (NT / 4)) >> 7] * bm.w_stride;
    for (int e = threadIdx.x; e < win * nb; e += NT) sW[e] = Wb[e];
    __syncthreads();
    const int qt = threadIdx.x & 3;
    const int64_t p = (int64_t)blockIdx.x * (NT / 4) + (threadIdx.x >> 2);
    const int64_t pc = p < n ? p : 0;
    float acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.f;
    for (int i0 = qt; i0 < win; i0 += 4 * FL_U) {
        float zj[FL_U][C];
#pragma unroll
        for (int u = 0; u < FL_U; ++u)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int i = i0 + 4 * u;
                zj[u][c] = i < win ? zin[((int64_t)c * win + i) * n + pc] : 0.f;
            }
#pragma unroll
        for (int u = 0; u < FL_U; ++u) {
            const int i = i0 + 4 * u;
            if (i >= win) break;
            const float zt = zj[u][CH::U] * inv_w + zoff;
            const int qa = window_k3(zt, nb);
            const float *wr = sW + i * nb + qa;
            const float w4[4] = {wr[0], wr[1], wr[2], wr[3]};
            float P[NP];
            window_sums<NP>(zt, nan_carrier(zt), qa, w4, P);
            acc[CH::U] += P[0];
            if constexpr (C > 1) {
                const float s1 = k1 * P[1], s2 = k2 * P[2];
                if constexpr (CH::X >= 0) acc[CH::X] = fmaf(zj[u][CH::X], s1, acc[CH::X]);
                if constexpr (CH::XX >= 0)
                    acc[CH::XX] += fmaf(zj[u][CH::X] * zj[u][CH::X], s2, zj[u][CH::XX] * s1);
                if constexpr (CH::Y >= 0) acc[CH::Y] = fmaf(zj[u][CH::Y], s1, acc[CH::Y]);
                if constexpr (CH::YY >= 0)
                    acc[CH::YY] += fmaf(zj[u][CH::Y] * zj[u][CH::Y], s2, zj[u][CH::YY] * s1);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = quad_sum(acc[c]);
    if (qt == 0 && p < n) {
#pragma unroll
        for (int c = 0; c < C; ++c) out[(int64_t)c * n + p] = acc[c];
    }
}

// The input bars of a point and input of a 1-output layer from its jets zj,
// the output bars yb and the window sums P (window_sums): with
// S1..S3 the weighted sums of dv, d2v, d3v (the feature bars are w_r ubar_c),
//   zbar_U  = ubar_U S1 + sum_d [ubar_d S2 zd + ubar_dd (S3 zd^2 + S2 zdd)]
//   zbar_d  = ubar_d S1 + 2 ubar_dd S2 zd,   zbar_dd = ubar_dd S1
template <int O0, int O1>
__device__ __forceinline__ void dx_last_bars(const float *zj, const float *yb, const float *P, float inv_w, float *zb)
{
    using CH = Ch<O0, O1>;
    constexpr int C = CH::C;
    const float S1 = (-8.f * inv_w) * P[1];
    float z0 = yb[CH::U] * S1;
    if constexpr (C > 1) {
        const float S2 = (56.f * inv_w * inv_w) * P[2];
        const float S3 = (-336.f * inv_w * inv_w * inv_w) * P[3];
        if constexpr (CH::X >= 0) {
            z0 = fmaf(yb[CH::X] * zj[CH::X], S2, z0);
            zb[CH::X] = yb[CH::X] * S1;
        }
        if constexpr (CH::XX >= 0) {
            z0 = fmaf(yb[CH::XX], fmaf(zj[CH::X] * zj[CH::X], S3, zj[CH::XX] * S2), z0);
            zb[CH::X] = fmaf(2.f * yb[CH::XX] * zj[CH::X], S2, zb[CH::X]);
            zb[CH::XX] = yb[CH::XX] * S1;
        }
        if constexpr (CH::Y >= 0) {
            z0 = fmaf(yb[CH::Y] * zj[CH::Y], S2, z0);
            zb[CH::Y] = yb[CH::Y] * S1;
        }
        if constexpr (CH::YY >= 0) {
            z0 = fmaf(yb[CH::YY], fmaf(zj[CH::Y] * zj[CH::Y], S3, zj[CH::YY] * S2), z0);
            zb[CH::Y] = fmaf(2.f * yb[CH::YY] * zj[CH::Y], S2, zb[CH::Y]);
            zb[CH::YY] = yb[CH::YY] * S1;
        }
    }
    zb[CH::U] = z0;
}

// zbar[c][i][p] from ubar[c][p]; one thread per (point, input)
// (dx_last_bars).
template <int O0, int O1>
__global__ __launch_bounds__(NT) void k_dx_last(const float *__restrict__ zin,
                                                const float *__restrict__ ybar,
                                                const float *__restrict__ W,
                                                float *__restrict__ zbar, int64_t n, int win,
                                                GridP<float> g, BatchMap bm)
{
    using CH = Ch<O0, O1>;
    constexpr int C = CH::C;
    constexpr int NP = C > 1 ? 4 : 2;
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= n * win) return;
    const int i = (int)(e / n);
    const int64_t p = e % n;
    if (bm.tile_inst) W += (int64_t)bm.tile_inst[p >> 7] * bm.w_stride;
    const int nb = g.nb;
    const float inv_w = g.inv_w, zoff = -g.lo * g.inv_w;
    float zj[C], yb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        zj[c] = zin[((int64_t)c * win + i) * n + p];
        yb[c] = ybar[(int64_t)c * n + p];
    }
    const float zt = zj[CH::U] * inv_w + zoff;
    const int qa = window_k3(zt, nb);
    const float *wr = W + i * nb + qa;
    const float w4[4] = {wr[0], wr[1], wr[2], wr[3]};
    float P[NP];
    window_sums<NP>(zt, nan_carrier(zt), qa, w4, P);
    float zb[C];
    dx_last_bars<O0, O1>(zj, yb, P, inv_w, zb);
#pragma unroll
    for (int c = 0; c < C; ++c) zbar[((int64_t)c * win + i) * n + p] = zb[c];
}

// gW[i*nb + b] for one point slice; thread (i, lane-slot) owns a private
// accumulator row in LDS, so every sum has a fixed order. Row r of a
// (point, input) adds sum_c A_c ubar_c = t^4 ubar_U + t^3 u G1 + t^2 (u^2 -
// 1/7) G2 with G1 = -8 iw sum_d (zd ubar_d + zdd ubar_dd) and
// G2 = 56 iw^2 sum_d zd^2 ubar_dd.
// DX: the same pass also writes the input bars zbar[c][i][p] of each point
// it visits (what k_dx_last computes), so the layer's jets are read once for
// both.
constexpr int DL_SL = 8;   // point lanes per input
// SL: point lanes per input (DL_SL, or 64 for DX, whose bar stores then
// cover 64 consecutive points of one input per wave)
template <int O0, int O1, bool DX, int SL = DL_SL>
__global__ __launch_bounds__(NT) void k_dw_last(const float *__restrict__ zin,
                                                const float *__restrict__ ybar,
                                                float *__restrict__ part, int64_t n, int win,
                                                int nsplit, GridP<float> g, BatchMap bm,
                                                const float *__restrict__ W, float *__restrict__ zbar)
{
    using CH = Ch<O0, O1>;
    constexpr int C = CH::C;
    constexpr int IB = NT / SL;           // inputs per block
    __shared__ float sacc[NT][33];
    const int nb = g.nb;
    const float inv_w = g.inv_w, zoff = -g.lo * g.inv_w;
    const float k1 = -8.f * inv_w, k2 = 56.f * inv_w * inv_w;
    const int li = threadIdx.x / SL, sl = threadIdx.x % SL;
    const int i = blockIdx.x * IB + li;
    const int split = blockIdx.y;
    const int64_t per = (n + nsplit - 1) / nsplit;
    int64_t ps = (int64_t)split * per, pe = min(n, ps + per);
    if (bm.slices) {
        const int4 sl = bm.slices[split];
        ps = sl.y;
        pe = sl.z;
        if (DX) W += (int64_t)sl.x * bm.w_stride;   // a slice lies within one instance
    }
    for (int b = 0; b < nb; ++b) sacc[threadIdx.x][b] = 0.f;
    if (i < win) {
        constexpr int U = 4;                    // points whose loads are in flight together
        for (int64_t p0 = ps + sl; p0 < pe; p0 += U * SL) {
            float zj[U][C], yb[U][C];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t p = p0 + (int64_t)u * SL;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    zj[u][c] = p < pe ? zin[((int64_t)c * win + i) * n + p] : 0.f;
                    yb[u][c] = p < pe ? ybar[(int64_t)c * n + p] : 0.f;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (p0 + (int64_t)u * SL >= pe) break;
                const float zt = zj[u][CH::U] * inv_w + zoff;
                const float sn = nan_carrier(zt);
                const int qa = window_k3(zt, nb);
                float G1 = 0.f, G2 = 0.f;
                if constexpr (CH::X >= 0) G1 = fmaf(zj[u][CH::X], yb[u][CH::X], G1);
                if constexpr (CH::XX >= 0) {
                    G1 = fmaf(zj[u][CH::XX], yb[u][CH::XX], G1);
                    G2 = fmaf(zj[u][CH::X] * zj[u][CH::X], yb[u][CH::XX], G2);
                }
                if constexpr (CH::Y >= 0) G1 = fmaf(zj[u][CH::Y], yb[u][CH::Y], G1);
                if constexpr (CH::YY >= 0) {
                    G1 = fmaf(zj[u][CH::YY], yb[u][CH::YY], G1);
                    G2 = fmaf(zj[u][CH::Y] * zj[u][CH::Y], yb[u][CH::YY], G2);
                }
                G1 *= k1;
                G2 *= k2;
                const float c0 = zt + 0.5f - 0.5f * (float)qa;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float uu = fminf(fmaxf(c0 - 0.5f * (float)r, -1.f), 1.f);
                    const float u2 = uu * uu;
                    const float t = sn - u2;
                    const float t2 = t * t;
                    float sum = t2 * t2 * yb[u][CH::U];
                    if constexpr (C > 1) {
                        sum = fmaf(t2 * t * uu, G1, sum);
                        sum = fmaf(t2 * (u2 - (1.f / 7.f)), G2, sum);
                    }
                    sacc[threadIdx.x][qa + r] += sum;
                }
                if constexpr (DX) {
                    constexpr int NP = C > 1 ? 4 : 2;
                    const int64_t p = p0 + (int64_t)u * SL;
                    const float *wr = W + i * nb + qa;
                    const float w4[4] = {wr[0], wr[1], wr[2], wr[3]};
                    float P[NP];
                    window_sums<NP>(zt, sn, qa, w4, P);
                    float zb[C];
                    dx_last_bars<O0, O1>(zj[u], yb[u], P, inv_w, zb);
#pragma unroll
                    for (int c = 0; c < C; ++c) zbar[((int64_t)c * win + i) * n + p] = zb[c];
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
        for (int k = 0; k < SL; ++k) sum += sacc[l2 * SL + k][b];
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

#define HRK_II_SWITCH(II_, ...)                                   \
    switch (II_) {                                                \
    case 2: { constexpr int II = 2; __VA_ARGS__; } break;         \
    case 4: { constexpr int II = 4; __VA_ARGS__; } break;         \
    case 8: { constexpr int II = 8; __VA_ARGS__; } break;         \
    default: return hipErrorInvalidValue;                         \
    }

constexpr size_t LDS_MAX = 160 * 1024;

// Inputs per wave of the weight-gradient kernel: the largest of 8, 4, 2 whose
// block fits two blocks per CU (else one), with at least one output chunk
// per pass. HRKAN_DW_II (2, 4 or 8) overrides it for tile tuning.
static int dw_ii(LayerShape ls, int C)
{
    static int forced = -1;
    if (forced < 0) {
        const char *e = getenv("HRKAN_DW_II");
        forced = (e && (atoi(e) == 2 || atoi(e) == 4 || atoi(e) == 8)) ? atoi(e) : 0;
    }
    const int NQ = ls.wout / 4;
    if (forced && 16 / forced <= NQ && dw_bs_lds(C, ls.nb, ls.wout, forced) <= LDS_MAX) return forced;
    for (size_t cap : {LDS_MAX / 2, LDS_MAX})
        for (int ii : {8, 4, 2})
            if (16 / ii <= NQ && dw_bs_lds(C, ls.nb, ls.wout, ii) <= cap) return ii;
    return 0;
}

bool bs32_supported(LayerShape ls, bool first)
{
    // the forward and input-bar kernels take their inputs in whole chunks
    if (first ? ls.win != 2 : ls.win % 8 != 0) return false;
    if (ls.nb < 4 || ls.nb > 32) return false;
    if (ls.wout == 1) return true;
    if (ls.wout != 32 && ls.wout != 64 && ls.wout != 128) return false;
    return dw_ii(ls, 5) > 0 && dw_ii(ls, 4) > 0 && dw_ii(ls, 1) > 0;
}

// Raise a kernel's dynamic-LDS limit once (outside any graph capture: the
// first launch of each kernel happens eagerly).
static void set_lds_limit(const void *kf)
{
    static const void *done[256];
    static int ndone = 0;
    for (int k = 0; k < ndone; ++k)
        if (done[k] == kf) return;
    (void)hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX);
    if (ndone < 256) done[ndone++] = kf;
}

static int grid_blocks(int64_t tiles, int cap) { return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, cap)); }

// inputs whose weight rows are staged at once (a multiple of KJ, or all of
// them), and the LDS bytes of those rows plus one chunk of jets
// Inputs whose weight rows are staged at once (a multiple of KJ, or all of
// them), and the LDS bytes of those rows plus one chunk of jets. Forward
// BF16 stages nb-1 row pairs of N+4 words per input, input-bar BF16 nb rows
// of N+8 halfwords, FP32 nb rows of N+4 floats; S = 3 stages the low
// pieces as well.
static void w_stage(LayerShape ls, int C, int S, bool fwd, int KJ, int &KI, size_t &bytes)
{
    size_t per_in;
    if (S == 0)
        per_in = (size_t)ls.nb * (ls.wout + 4) * sizeof(float);
    else if (fwd)
        per_in = (size_t)(ls.nb - 1) * (ls.wout + 4) * sizeof(unsigned int);
    else
        per_in = (size_t)ls.nb * (ls.wout + 8) * sizeof(unsigned short);
    if (S == 3) per_in *= 2;
    const int og = og_of(C, ls.wout / 4);           // output groups (tiles of 128/og points)
    size_t jets = (size_t)KJ * (C + 1) * (TP / og) * sizeof(float);
    if (!fwd && og > 1) jets += (size_t)og * KJ * C * (TP / og) * sizeof(float);
    size_t ki = (LDS_FWD - jets) / per_in;
    if (ki >= (size_t)ls.win)
        ki = ls.win;
    else
        ki = std::max<size_t>(KJ, ki / KJ * KJ);
    KI = (int)ki;
    bytes = per_in * ki + jets;
}

// BF16 kernels are built for the channel sets of the PDE residuals (Poisson,
// Burgers) and of boundary values.
#define HRK_CH_SWITCH_BF(ch, ...)                                 \
    switch ((ch).o0 * 3 + (ch).o1) {                              \
    case 0: { constexpr int O0 = 0, O1 = 0; __VA_ARGS__; } break; \
    case 7: { constexpr int O0 = 2, O1 = 1; __VA_ARGS__; } break; \
    case 8: { constexpr int O0 = 2, O1 = 2; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                         \
    }

#define HRK_S_SWITCH(S_, ...)                                     \
    switch (S_) {                                                 \
    case 1: { constexpr int S = 1; __VA_ARGS__; } break;          \
    case 2: { constexpr int S = 2; __VA_ARGS__; } break;          \
    case 3: { constexpr int S = 3; __VA_ARGS__; } break;          \
    default: return hipErrorInvalidValue;                         \
    }

// FP32 (S = 0) over every channel set, BF16 (S = 1..3) over HRK_CH_SWITCH_BF's
#define HRK_CH_S_SWITCH(ch, S_, ...)                                                          \
    if ((S_) == 0) {                                                                          \
        HRK_CH_SWITCH32(ch, { constexpr int S = 0; __VA_ARGS__; });                           \
    } else {                                                                                  \
        HRK_CH_SWITCH_BF(ch, { HRK_S_SWITCH(S_, __VA_ARGS__); });                             \
    }

hipError_t launch_fwd_bs32(ChanCfg ch, bool first, const float *zin, const float *W, float *zout,
                           int64_t n, LayerShape ls, const GridP<float> &g, int cu_blocks, int S,
                           hipStream_t st, const BatchMap &bm)
{
    if (n <= 0) return hipSuccess;
    if (ls.wout == 1) {
        const size_t sh = sizeof(float) * ls.win * ls.nb;
        HRK_CH_SWITCH32(ch, {
            k_fwd_last<O0, O1><<<(unsigned)((n + NT / 4 - 1) / (NT / 4)), NT, sh, st>>>(zin, W, zout, n, ls.win, g,
                                                                                    bm);
        });
        return hipGetLastError();
    }
    if (!bs32_supported(ls, first)) return hipErrorInvalidValue;
    int KI;
    size_t sh;
    w_stage(ls, ch.C(), S, true, kj_of(first, ch.C()), KI, sh);
    const int tpk = TP / og_of(ch.C(), ls.wout / 4);
    const int grid = grid_blocks((n + tpk - 1) / tpk, cu_blocks);
    HRK_CH_S_SWITCH(ch, S, {
        HRK_NQ_SWITCH(ls.wout, {
            if (first) {
                auto kf = k_fwd_bs<O0, O1, true, NQ, S>;
                set_lds_limit((const void *)kf);
                kf<<<grid, NT8, sh, st>>>(zin, W, zout, n, ls.win, KI, g, bm);
            } else {
                auto kf = k_fwd_bs<O0, O1, false, NQ, S>;
                set_lds_limit((const void *)kf);
                kf<<<grid, NT8, sh, st>>>(zin, W, zout, n, ls.win, KI, g, bm);
            }
        });
    });
    return hipGetLastError();
}

hipError_t launch_dx_bs32(ChanCfg ch, const float *zin, const float *ybar, const float *W, float *zbar,
                          int64_t n, LayerShape ls, const GridP<float> &g, int cu_blocks, int S,
                          hipStream_t st, const BatchMap &bm)
{
    if (n <= 0) return hipSuccess;
    if (ls.wout == 1) {
        HRK_CH_SWITCH32(ch, {
            k_dx_last<O0, O1><<<(unsigned)((n * ls.win + NT - 1) / NT), NT, 0, st>>>(zin, ybar, W, zbar, n,
                                                                                   ls.win, g, bm);
        });
        return hipGetLastError();
    }
    if (!bs32_supported(ls, false)) return hipErrorInvalidValue;
    int KI;
    size_t sh;
    w_stage(ls, ch.C(), S, false, kj_of(false, ch.C()), KI, sh);
    const int tpk = TP / og_of(ch.C(), ls.wout / 4);
    const int grid = grid_blocks((n + tpk - 1) / tpk, cu_blocks);
    HRK_CH_S_SWITCH(ch, S, {
        HRK_NQ_SWITCH(ls.wout, {
            auto kf = k_dx_bs<O0, O1, NQ, S>;
            set_lds_limit((const void *)kf);
            kf<<<grid, NT8, sh, st>>>(zin, ybar, W, zbar, n, ls.win, KI, g, bm);
        });
    });
    return hipGetLastError();
}

// Weight-gradient tile: II inputs per wave, WI waves along inputs. Few
// inputs (the first layer has 2) take a small II and WI < 4, and the spare
// waves split the points instead.
struct DwTile {
    int II, WI;
};
static DwTile dw_tile(LayerShape ls, int C, int ii_override = 0)
{
    int ii = dw_ii(ls, C);
    if (ii == 0) return {0, 0};
    if (ii_override && 16 / ii_override <= ls.wout / 4 && dw_bs_lds(C, ls.nb, ls.wout, ii_override) <= LDS_MAX)
        ii = ii_override;
    while (ii > 2 && ii / 2 >= ls.win && 16 / (ii / 2) <= ls.wout / 4) ii /= 2;
    const int groups = (ls.win + ii - 1) / ii;
    const int wi = groups >= 4 ? 4 : groups >= 2 ? 2 : 1;
    return {ii, wi};
}

// Output blocks of the weight-gradient launch: a layer of 64 or 128 outputs
// is split over two blocks (grid z) of half the outputs each, which halves a
// block's LDS gradient copy and staged bars (128 outputs: two blocks per CU
// instead of one; 128 outputs over 1,048,576 points 33.2 -> 24.5 ms, 64
// outputs over 262,144 points 1.99 -> 1.90 ms per launch), at the cost of
// evaluating the features twice.
static int dw_jsplit(LayerShape ls) { return ls.wout >= 64 ? 2 : 1; }
static LayerShape dw_block_shape(LayerShape ls)
{
    ls.wout /= dw_jsplit(ls);
    return ls;
}

hipError_t launch_back_last(ChanCfg ch, const float *zin, const float *ybar, const float *W, float *zbar, float *part,
                            int nsplit, int64_t n, LayerShape ls, const GridP<float> &g, hipStream_t st,
                            const BatchMap &bm)
{
    if (n <= 0) return hipSuccess;
    if (ls.wout != 1 || nsplit < 1) return hipErrorInvalidValue;
    constexpr int SL = 64;
    dim3 grid((unsigned)((ls.win + NT / SL - 1) / (NT / SL)), (unsigned)nsplit);
    HRK_CH_SWITCH32(ch, {
        k_dw_last<O0, O1, true, SL><<<grid, NT, 0, st>>>(zin, ybar, part, n, ls.win, nsplit, g, bm, W, zbar);
    });
    return hipGetLastError();
}

int dw_bs32_splits(int64_t n, LayerShape ls)
{
    if (n <= 0) return 0;
    // about two blocks per CU, with at least 32 points per slice
    const int64_t maxs = std::max<int64_t>(1, n / 32);
    int64_t tiles;
    if (ls.wout == 1) {
        tiles = (ls.win + NT / DL_SL - 1) / (NT / DL_SL);
    } else {
        const DwTile t = dw_tile(dw_block_shape(ls), 4);
        const int ib = std::max(1, t.II * t.WI);
        tiles = (ls.win + ib - 1) / ib;
    }
    const int64_t s = (512 + tiles - 1) / tiles;
    return (int)std::max<int64_t>(1, std::min<int64_t>(std::min(s, maxs), 1024));
}

hipError_t launch_dw_bs32(ChanCfg ch, bool first, const float *zin, const float *ybar, float *part,
                          int nsplit, int64_t n, LayerShape ls, const GridP<float> &g, int S, hipStream_t st,
                          const BatchMap &bm, int dw_ii_override)
{
    if (ls.wout == 1) {
        dim3 grid((unsigned)((ls.win + NT / DL_SL - 1) / (NT / DL_SL)), (unsigned)nsplit);
        HRK_CH_SWITCH32(ch, {
            k_dw_last<O0, O1, false><<<grid, NT, 0, st>>>(zin, ybar, part, n, ls.win, nsplit, g, bm, nullptr,
                                                          nullptr);
        });
        return hipGetLastError();
    }
    const LayerShape lb = dw_block_shape(ls);
    const DwTile tl = dw_tile(lb, ch.C(), dw_ii_override);
    if (tl.II == 0) return hipErrorInvalidValue;
    const int ibe = tl.II * tl.WI;
    const dim3 grid((unsigned)((ls.win + ibe - 1) / ibe), (unsigned)nsplit, (unsigned)dw_jsplit(ls));
    const int wi = tl.WI;
    HRK_CH_S_SWITCH(ch, S, {
        HRK_NQ_SWITCH(lb.wout, {
            HRK_II_SWITCH(tl.II, {
                if constexpr (16 / II <= NQ) {
                    const size_t sh = dw_bs_lds(ch.C(), lb.nb, lb.wout, II);
                    if (first) {
                        auto kf = k_dw_bs<O0, O1, true, NQ, II, S>;
                        set_lds_limit((const void *)kf);
                        kf<<<grid, NT, sh, st>>>(zin, ybar, part, n, ls.win, nsplit, wi, g, bm);
                    } else {
                        auto kf = k_dw_bs<O0, O1, false, NQ, II, S>;
                        set_lds_limit((const void *)kf);
                        kf<<<grid, NT, sh, st>>>(zin, ybar, part, n, ls.win, nsplit, wi, g, bm);
                    }
                }
            });
        });
    });
    return hipGetLastError();
}

}  // namespace hrk
