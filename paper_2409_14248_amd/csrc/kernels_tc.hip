// kernels_tc.hip -- tile-coherent FP32 matrix-core kernels of one hidden KAN
// layer for the HR basis with k = 3 supports and order m = 4 (Eq. 2).
//
// A wave takes a tile of 16 consecutive points. When the point set is
// ordered along a space-filling curve, the points of a tile lie close
// together in the domain, so each of a hidden layer's inputs takes nearby
// values on them and only a few basis rows are non-zero on the whole tile:
// the union of the tile's 4-row windows, rows r0_i .. r1_i of input i. The
// tile's K axis is the concatenation of those rows over the inputs (a few
// more than the 4 live rows per point and input; rows outside a point's own
// support give a zero feature), and the contraction runs on the 16x16x4
// FP32 MFMA with the 16 points as the M axis: the weight row of a K entry is
// the B operand of all 16 points at once. The kernels are correct for any
// point order; the order only sets how long the K axis is.
//
// The basis and its derivatives are evaluated in FP64 from the offsets of the
// FP32 input to the support ends, a = z - s_b and be = e_b - z (knots in
// FP64), and each feature is rounded to FP32 once: on a deep network the
// error of the first layers' features is amplified by the later ones, and
// FP32 evaluation (several roundings per feature, and z - s_b taken at the
// magnitude of the scaled coordinate) would put the step's error well above
// what FP32 storage of the features alone costs. The first layer (inputs
// are the coordinates, jets (1, 0) and (0, 1)) runs on the same kernels.
//
// MFMA lane layout (16x16x4 FP32, wave of 64): lane l, r16 = l % 16,
// g = l / 16: A[r16][g], B[g][r16], D[4 g + r][r16] (r = 0..3).
#include <algorithm>

#include "internal.h"
#include "kernels_tc.h"

namespace hrk {

typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int TNT = 256;            // threads per block: 4 independent waves
constexpr int TW = TNT / 64;
constexpr int TPT = 16;             // points per wave tile
constexpr int TKJ = 16;             // inputs per chunk
constexpr int MAXNB = 32;           // basis rows per input (n_b) at most

// Rows of a chunk's K list: up to TKJ * MAXNB entries, padded to 4.
constexpr int MAXK = TKJ * MAXNB;

template <int O0, int O1>
struct TcLds {
    static constexpr int C = 1 + O0 + O1;
    float z[C][TKJ][TPT];               // the chunk's jets of the tile
    unsigned short ent[MAXK];           // K entry: input (high byte) and row (low byte)
    int nent;
};

// v, v', v'' of bump b at FP32 input z, in FP64 (derivatives in z units:
// inv_w per order); zero off the open support, a NaN input carried.
__device__ __forceinline__ void bump3d(double2 kn, float z, double inv_w, double &v0, double &v1, double &v2)
{
    const double zd = (double)z;
    const double a = (zd - kn.x) * inv_w, be = (kn.y - zd) * inv_w;
    const bool in = !(a <= 0.0) && !(be <= 0.0);
    const double t = a * be, d = be - a, t2 = t * t;
    v0 = in ? t2 * t2 : 0.0;
    v1 = in ? (4.0 * inv_w) * (t2 * t) * d : 0.0;
    v2 = in ? (4.0 * inv_w * inv_w) * t2 * (3.0 * d * d - 2.0 * t) : 0.0;
}

// Feature of channel c from the bump and the point's jets of the input,
// computed in FP64 and rounded once.
template <int O0, int O1>
__device__ __forceinline__ float feature(int c, double v0, double v1, double v2, const float *zj)
{
    using CH = Ch<O0, O1>;
    if (c == CH::U) return (float)v0;
    if (c == CH::X) return (float)(v1 * (double)zj[CH::X]);
    if (c == CH::XX) return (float)(v2 * ((double)zj[CH::X] * (double)zj[CH::X]) + v1 * (double)zj[CH::XX]);
    if (c == CH::Y) return (float)(v1 * (double)zj[CH::Y]);
    return (float)(v2 * ((double)zj[CH::Y] * (double)zj[CH::Y]) + v1 * (double)zj[CH::YY]);
}

// Knot b as FP32 pairs (s_hi, s_lo, e_hi, e_lo) with s = s_hi + s_lo and e =
// e_hi + e_lo to within FP64 rounding, and the basis scales in FP32, for the
// weight gradient and the input bars: there the offsets of z to the knots are
// (z - s_hi) - s_lo and (e_hi - z) + e_lo, each rounded to FP32 (the
// subtraction of the nearby s_hi loses no leading bits), and the rest of the
// basis is FP32: a few FP32 units relative, for features and adjoint terms
// that enter only FP32 sums of their own layer, not the later layers.
__device__ __forceinline__ float4 split_knot(double s, double e)
{
    const float sh = (float)s, eh = (float)e;
    return make_float4(sh, (float)(s - (double)sh), eh, (float)(e - (double)eh));
}

struct BasisScale {
    float w, k1, k2, k3;   // inv_w, 4 inv_w, 4 inv_w^2, 24 inv_w^3
};
__device__ __forceinline__ BasisScale basis_scale(double inv_w)
{
    return BasisScale{(float)inv_w, (float)(4.0 * inv_w), (float)(4.0 * inv_w * inv_w),
                      (float)(24.0 * inv_w * inv_w * inv_w)};
}

// v, v', v'' of bump b at z, zero off the open support, a NaN input carried
__device__ __forceinline__ void bump3f(float4 kn, float z, const BasisScale &bs, float &v0, float &v1, float &v2)
{
    const float a = ((z - kn.x) - kn.y) * bs.w, be = ((kn.z - z) + kn.w) * bs.w;
    const bool in = !(a <= 0.f) && !(be <= 0.f);
    const float t = a * be, d = be - a, t2 = t * t;
    v0 = in ? t2 * t2 : 0.f;
    v1 = in ? bs.k1 * (t2 * t) * d : 0.f;
    v2 = in ? bs.k2 * t2 * (3.f * d * d - 2.f * t) : 0.f;
}

template <int O0, int O1>
__device__ __forceinline__ float feature_f(int c, float v0, float v1, float v2, const float *zj)
{
    using CH = Ch<O0, O1>;
    if (c == CH::U) return v0;
    if (c == CH::X) return v1 * zj[CH::X];
    if (c == CH::XX) return v2 * (zj[CH::X] * zj[CH::X]) + v1 * zj[CH::XX];
    if (c == CH::Y) return v1 * zj[CH::Y];
    return v2 * (zj[CH::Y] * zj[CH::Y]) + v1 * zj[CH::YY];
}

// Jets of a chunk's input il at point p: a hidden layer reads its saved
// jets [C][win][n]; the first layer the coordinates x [n][2] (input il is
// coordinate il, with unit first derivative along its own direction).
// NT: a non-temporal load (the value streams through once, so L2 keeps what
// is re-read, such as weight rows).
template <int O0, int O1, bool FIRST, bool NT = false>
__device__ __forceinline__ float jet_in(const float *__restrict__ zin, int c, int i, int win, int64_t n, int64_t p)
{
    if constexpr (FIRST) {
        using CH = Ch<O0, O1>;
        if (c == CH::U) return zin[2 * p + i];
        if (c == CH::X) return i == 0 ? 1.f : 0.f;
        if (c == CH::Y) return i == 1 ? 1.f : 0.f;
        return 0.f;
    } else if constexpr (NT) {
        return __builtin_nontemporal_load(zin + (int64_t)(c * win + i) * n + p);
    } else {
        return zin[(int64_t)(c * win + i) * n + p];
    }
}

// jet_in at point p of input i when ok, else zero; the load is always issued
// (at a valid point and input), so no load sits in a divergent branch, whose
// join would make the compiler wait for every load in flight.
template <int O0, int O1, bool FIRST>
__device__ __forceinline__ float jet_sel(const float *__restrict__ zin, int c, int i, int win, int64_t n, int64_t p,
                                         bool ok)
{
    const float v = jet_in<O0, O1, FIRST>(zin, c, ok ? i : 0, win, n, ok ? p : 0);
    return ok ? v : 0.f;
}

// lo = min(lo, lo of the lane M below), hi likewise with max, within a DPP
// row of 16 lanes (row_shr:M; a lane whose source lies before the row start
// keeps its own value)
template <int M>
__device__ __forceinline__ void row_shr_minmax(int &lo, int &hi)
{
    lo = min(lo, __builtin_amdgcn_update_dpp(lo, lo, 0x110 + M, 0xf, 0xf, false));
    hi = max(hi, __builtin_amdgcn_update_dpp(hi, hi, 0x110 + M, 0xf, 0xf, false));
}

// Build the K list of the tile's chunk of inputs [i0, i0 + TKJ): each lane
// group g (16 lanes, one per point) takes inputs g, g + 4, g + 8, g + 12 and
// reduces the window starts over the tile's live points; then every lane
// reads the 16 row counts and writes its share of the entries.
template <int KJ>
__device__ __forceinline__ void build_klist(const float (*zv)[TPT], int lane, int64_t p0, int64_t n, float lo,
                                            float inv_w, int nb, int *r0s, int *cnts, int nin = KJ)
{
    const int p = lane & 15, g = lane >> 4;
    const bool pt_ok = p0 + p < n;
#pragma unroll
    for (int q = 0; q < KJ / 4; ++q) {
        const int il = g + 4 * q;
        const bool in_ok = il < nin;               // inputs nin.. of the capacity: no rows
        const float zt = ((in_ok ? zv[il][p] : 0.f) - lo) * inv_w;
        // live: inside the extended grid (-1.5, nb/2) in the scaled coordinate, or NaN
        const bool live = in_ok && pt_ok && !(zt <= -1.5f) && !(zt >= 0.5f * (float)nb);
        const int qa = (int)fminf(fmaxf(2.f * zt, 0.f), (float)(nb - 4));
        int lo_q = live ? qa : 1 << 20, hi_q = live ? qa : -1;
        // min and max over the 16 lanes (one DPP row): after shifts by 1, 2,
        // 4 and 8 lanes within the row, lane 15 has seen every lane of it (a
        // lane whose source would lie before the row start keeps its value)
        row_shr_minmax<1>(lo_q, hi_q);
        row_shr_minmax<2>(lo_q, hi_q);
        row_shr_minmax<4>(lo_q, hi_q);
        row_shr_minmax<8>(lo_q, hi_q);
        if (p == 15) {
            r0s[il] = hi_q < 0 ? 0 : lo_q;
            cnts[il] = hi_q < 0 ? 0 : min(hi_q + 3, nb - 1) - lo_q + 1;
        }
    }
}

// The K list from the row counts: entries e = lane, lane + 64, .. get
// (input << 8 | row); returns the number of entries.
template <int KJ>
__device__ __forceinline__ int write_entries(unsigned short *ent, int lane, const int *r0s, const int *cnts)
{
    int tot = 0;
    int offs[KJ];
#pragma unroll
    for (int il = 0; il < KJ; ++il) {
        offs[il] = tot;
        tot += cnts[il];
    }
    for (int e = lane; e < tot; e += 64) {
        int il = 0, base = 0;
#pragma unroll
        for (int q = 1; q < KJ; ++q)
            if (e >= offs[q]) {
                il = q;
                base = offs[q];
            }
        ent[e] = (unsigned short)((il << 8) | (r0s[il] + e - base));
    }
    return tot;
}

// v', v'', v''' of bump b at z (v[0] unused), for the adjoint of the
// features in the input bars (split knots, FP32: see split_knot); zero off
// the open support, a NaN input carried.
__device__ __forceinline__ void bump_d123f(float4 kn, float z, const BasisScale &bs, float *v)
{
    const float a = ((z - kn.x) - kn.y) * bs.w, be = ((kn.z - z) + kn.w) * bs.w;
    const bool in = !(a <= 0.f) && !(be <= 0.f);
    const float t = a * be, d = be - a, t2 = t * t;
    v[0] = 0.f;
    v[1] = in ? bs.k1 * (t2 * t) * d : 0.f;
    v[2] = in ? bs.k2 * t2 * (3.f * d * d - 2.f * t) : 0.f;
    v[3] = in ? bs.k3 * t * d * (d * d - 3.f * t) : 0.f;
}

// ---------------------------------------------------------------------------
// forward: zout[c][j][p] = sum over the tile's K entries (i, b) of
// A_c(p, i, b) W[i nb + b][j]. A wave takes a tile and all its outputs; each
// lane owns output columns j = col * NT16 + ot (ot < NT16), so its B operands
// of one K entry are NT16 consecutive floats of the weight row, loaded a step
// ahead.
// ---------------------------------------------------------------------------
// waves per SIMD the forward and input-bar kernels are built for: a
// 128-output layer keeps all its accumulators in one wave's registers
template <int NT16> constexpr int tc_waves() { return 2; }

template <int O0, int O1, bool FIRST, int NT16>
__global__ __launch_bounds__(TNT, tc_waves<NT16>()) void k_fwd_tc(const float *__restrict__ zin, const float *__restrict__ W,
                                                float *__restrict__ zout, int64_t n, int win, TcGrid gr)
{
    constexpr int C = 1 + O0 + O1;
    constexpr int N = 16 * NT16;
    constexpr int NTW = NT16;                       // 16-output tiles per wave
    constexpr int WPT = NT16 / NTW;                 // waves per tile
    constexpr int TPB = TW / WPT;                   // tiles per block round
    __shared__ TcLds<O0, O1> lds[TW];
    __shared__ double2 knots[MAXNB];
    __shared__ int r0s_s[TW][TKJ], cnt_s[TW][TKJ];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    TcLds<O0, O1> &L = lds[wv];
    int *r0s = r0s_s[wv], *cnts = cnt_s[wv];
    const int nb = gr.nb;
    const float inv_w = gr.inv_w, lo = gr.lo;
    const double inv_wd = gr.inv_w_d;
    if (threadIdx.x < nb) knots[threadIdx.x] = make_double2(gr.s[threadIdx.x], gr.e[threadIdx.x]);
    __syncthreads();
    const int64_t ntiles = (n + TPT - 1) / TPT;
    const int nchunk = FIRST ? 1 : win / TKJ;
    const int nin = FIRST ? win : TKJ;

    const int oh = wv % WPT;                        // this wave's output part
    const int64_t tfirst = (int64_t)blockIdx.x * TPB + wv / WPT;
    const int64_t tstride = (int64_t)gridDim.x * TPB;

    for (int64_t tile = tfirst; tile < ntiles; tile += tstride) {
        const int64_t p0 = tile * TPT;
        f4 acc[C][NTW];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int o = 0; o < NTW; ++o) acc[c][o] = (f4){0.f, 0.f, 0.f, 0.f};

        for (int ch = 0; ch < nchunk; ++ch) {
            const int i0 = ch * TKJ;
            // the chunk's jets: lane (r16 = point, g) loads inputs g, g + 4, ..
            // Past the last point or the layer's inputs the lane reads point 0
            // / input 0 instead and no value is selected: the K list takes
            // neither (build_klist masks them), and a padding point's row of
            // the products is its own and never stored. So each load goes
            // straight to its register, all are issued before the first LDS
            // write (the scheduling barrier), and one wait covers them.
            {
                const int64_t p = p0 + r16;
                const bool ok = p < n;
                float zr[C][TKJ / 4];
#pragma unroll
                for (int c = 0; c < C; ++c)
#pragma unroll
                    for (int q = 0; q < TKJ / 4; ++q) {
                        const int il = g + 4 * q;
                        const bool okq = ok && il < nin;
                        zr[c][q] = jet_in<O0, O1, FIRST>(zin, c, i0 + (okq ? il : 0), win, n, okq ? p : 0);
                    }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int c = 0; c < C; ++c)
#pragma unroll
                    for (int q = 0; q < TKJ / 4; ++q) L.z[c][g + 4 * q][r16] = zr[c][q];
            }
            __builtin_amdgcn_wave_barrier();
            build_klist<TKJ>(L.z[0], lane, p0, n, lo, inv_w, nb, r0s, cnts, nin);
            __builtin_amdgcn_wave_barrier();
            // the same count in every lane: taken as a scalar, so the loop
            // branches are uniform and no load waits at a divergent join
            const int tot = __builtin_amdgcn_readfirstlane(write_entries<TKJ>(L.ent, lane, r0s, cnts));
            __builtin_amdgcn_wave_barrier();
            const int nsteps = (tot + 3) / 4;
            // B operands of step s: this lane's NTW columns of the row of
            // entry 4 s + g (padding entries past tot read the last entry's
            // row, their A operand is zero); no divergent branch, so the
            // loads stay in flight across the MFMAs
            auto load_b = [&](int s, float *bw) {
                const int e = min(4 * s + g, tot - 1);
                const int en = L.ent[e];
                const int row = (i0 + (en >> 8)) * nb + (en & 0xFF);
                const float *src = W + (int64_t)row * N + oh * 16 * NTW + r16 * NTW;
                if constexpr (NTW % 4 == 0) {
#pragma unroll
                    for (int o = 0; o < NTW; o += 4) {
                        const f4 w4 = *reinterpret_cast<const f4 *>(src + o);
                        bw[o] = w4[0];
                        bw[o + 1] = w4[1];
                        bw[o + 2] = w4[2];
                        bw[o + 3] = w4[3];
                    }
                } else {
                    static_assert(NTW == 2, "32, 64 or 128 outputs");
                    const float2 w2 = *reinterpret_cast<const float2 *>(src);
                    bw[0] = w2.x;
                    bw[1] = w2.y;
                }
            };
            // A operands of step s: point r16, entry 4 s + g (zero past tot)
            auto comp_a = [&](int s, float *A) {
                const int e = 4 * s + g;
                const int en = L.ent[min(e, tot - 1)];
                const int il = en >> 8, b = en & 0xFF;
                float zj[C];
#pragma unroll
                for (int c = 0; c < C; ++c) zj[c] = L.z[c][il][r16];
                double v0, v1, v2;
                bump3d(knots[b], zj[0], inv_wd, v0, v1, v2);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float f = feature<O0, O1>(c, v0, v1, v2, zj);
                    A[c] = e < tot ? f : 0.f;
                }
            };
            // two B buffers used in turn: the loads of a step stay in flight
            // while the previous step computes (no copies between them)
            float b0[NTW], b1[NTW], a[C];
            auto mma = [&](const float *bw) {
#pragma unroll
                for (int c = 0; c < C; ++c)
#pragma unroll
                    for (int o = 0; o < NTW; ++o)
                        acc[c][o] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], bw[o], acc[c][o], 0, 0, 0);
            };
            // steps in pairs; the prefetches past the last step read the last
            // entry's row again and a step past it multiplies zeros, so every
            // load is unconditional and the waits count loads exactly
            if (nsteps > 0) load_b(0, b0);
            for (int s = 0; s < nsteps; s += 2) {
                load_b(s + 1, b1);
                comp_a(s, a);
                mma(b0);
                load_b(s + 2, b0);
                comp_a(s + 1, a);
                mma(b1);
            }
            __builtin_amdgcn_wave_barrier();
        }
        // D[4 g + r][r16] of tile o: point p0 + 4 g + r, output
        // oh 16 NTW + r16 NTW + o; the lane's 4 values are consecutive points
        // of one output row
        const int64_t pg = p0 + 4 * g;
        const bool vec = (n % 4 == 0) && pg + 3 < n;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int o = 0; o < NTW; ++o) {
                const int j = oh * 16 * NTW + r16 * NTW + o;
                float *dst = zout + (int64_t)(c * N + j) * n + pg;
                if (vec) {
                    *reinterpret_cast<f4 *>(dst) = acc[c][o];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (pg + r < n) dst[r] = acc[c][o][r];
                }
            }
    }
}

// ---------------------------------------------------------------------------
// input bars: Abar_c(p, i, b) = sum_j W[i nb + b][j] ybar[c][j][p] over the
// tile's K entries (i, b), on the 16x16x4 FP32 MFMA with the entries as the
// M axis (A = 16 weight rows), the points as the N axis (B = the output bars)
// and the outputs as the reduction axis. Lane (g, r16) holds the B operands
// ybar[c][16 s + 4 g + q][p0 + r16] of its pass's outputs in registers (at
// most 64 outputs per pass, 32 for four or five channels of a 64-output
// layer; every pass after the first adds to the result); the matching A
// operand is the weight
// W[row][16 s + 4 g + q], four consecutive floats of the row per s.
// The adjoint of each feature through v', v'', v''' gives the entry's terms
// of zbar[.][i][p]; they are staged per entry block and summed per input in
// entry order, so every sum has one fixed order.
// ---------------------------------------------------------------------------
template <int O0, int O1>
struct TcDxLds {
    static constexpr int C = 1 + O0 + O1;
    float z[C][TKJ][TPT];
    float zb[C][TKJ][TPT];              // the chunk's input bars, summed over entries
    float tm[16][C][TPT];               // the terms of one entry block
    unsigned short ent[MAXK];
};

template <int O0, int O1, int NT16>
__global__ __launch_bounds__(TNT, tc_waves<NT16>()) void k_dx_tc(const float *__restrict__ zin, const float *__restrict__ ybar,
                                                  const float *__restrict__ W, float *__restrict__ zbar, int64_t n,
                                                  int win, TcGrid gr)
{
    constexpr int C = 1 + O0 + O1;
    constexpr int N = 16 * NT16;
    // 16-output groups per pass (the registers of a pass's bars stay within
    // two waves per SIMD) and passes over the outputs
    constexpr int NS = NT16 > 4 ? 4 : (NT16 == 4 && C >= 4 ? 2 : NT16);
    constexpr int NP = NT16 / NS;
    __shared__ TcDxLds<O0, O1> lds[TW];
    __shared__ float4 knots[MAXNB];    // split knots (split_knot)
    __shared__ int r0s_s[TW][TKJ], cnt_s[TW][TKJ];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    TcDxLds<O0, O1> &L = lds[wv];
    int *r0s = r0s_s[wv], *cnts = cnt_s[wv];
    const int nb = gr.nb;
    const float inv_w = gr.inv_w, lo = gr.lo;
    if (threadIdx.x < nb) knots[threadIdx.x] = split_knot(gr.s[threadIdx.x], gr.e[threadIdx.x]);
    const BasisScale bsc = basis_scale(gr.inv_w_d);
    __syncthreads();
    const int64_t ntiles = (n + TPT - 1) / TPT;
    const int nchunk = win / TKJ;

    const int64_t tstride = (int64_t)gridDim.x * TW;
    // a chunk's jets in registers, the next chunk's loaded during the current one
    float pz[C][TKJ / 4];
    // Past the last point (or the last tile) a lane reads point 0 and keeps
    // that value: the K list never takes such a point, and its column of the
    // products, its adjoint terms and its sums are its own and never stored.
    // Without a value select each load lands in its own register. Jets and
    // bars stream through once per pass (non-temporal loads), so that L2
    // keeps the weight rows the entry blocks read.
    auto load_chunk = [&](int64_t tl, int chn) {
        const int64_t p = tl * TPT + r16;
        const bool ok = tl < ntiles && p < n;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int q = 0; q < TKJ / 4; ++q)
                pz[c][q] = jet_in<O0, O1, false, true>(zin, c, chn * TKJ + g + 4 * q, win, n, ok ? p : 0);
    };
    load_chunk((int64_t)blockIdx.x * TW + wv, 0);

    for (int64_t tile = (int64_t)blockIdx.x * TW + wv; tile < ntiles; tile += tstride) {
        const int64_t p0 = tile * TPT;
        const int64_t pl = p0 + r16;
        const bool pl_ok = pl < n;
#pragma unroll 1
        for (int pass = 0; pass < NP; ++pass) {
            const int j0 = pass * 16 * NS;
            float yb[C][NS][4];
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int sg = 0; sg < NS; ++sg)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                    {
                        yb[c][sg][q] = __builtin_nontemporal_load(ybar + (int64_t)(c * N + j0 + 16 * sg + 4 * g + q) * n + (pl_ok ? pl : 0));
                    }

#pragma unroll 1
            for (int chn = 0; chn < nchunk; ++chn) {
                const int i0 = chn * TKJ;
#pragma unroll
                for (int c = 0; c < C; ++c)
#pragma unroll
                    for (int q = 0; q < TKJ / 4; ++q) {
                        const int il = g + 4 * q;
                        L.z[c][il][r16] = pz[c][q];
                        L.zb[c][il][r16] = 0.f;
                    }
                if (chn + 1 < nchunk)
                    load_chunk(tile, chn + 1);
                else if (pass + 1 < NP)
                    load_chunk(tile, 0);
                else
                    load_chunk(tile + tstride, 0);
                __builtin_amdgcn_wave_barrier();
                build_klist<TKJ>(L.z[0], lane, p0, n, lo, inv_w, nb, r0s, cnts);
                __builtin_amdgcn_wave_barrier();
                const int tot = __builtin_amdgcn_readfirstlane(write_entries<TKJ>(L.ent, lane, r0s, cnts));
                __builtin_amdgcn_wave_barrier();
                const int nblk = (tot + 15) / 16;
                // A operands (weight rows) of entry block eb: entry eb*16 + r16,
                // past tot the last entry's row (multiplied as zero); the next
                // block's are loaded during the current block's work
                auto load_w = [&](int eb_, f4 *w) {
                    const int en = L.ent[min(eb_ * 16 + r16, tot - 1)];
                    const int wrow = (i0 + (en >> 8)) * nb + (en & 0xFF);
                    const float *wsrc = W + (int64_t)wrow * N + j0 + 4 * g;
#pragma unroll
                    for (int sg = 0; sg < NS; ++sg) w[sg] = *reinterpret_cast<const f4 *>(wsrc + 16 * sg);
                };
                f4 wcur[NS], wnxt[NS];
                if (nblk > 0) load_w(0, wcur);
#pragma unroll 1
                for (int eb = 0; eb < nblk; ++eb) {
                    load_w(eb + 1, wnxt);            // past the last block: the last entry's row again
                    const bool em_ok = eb * 16 + r16 < tot;
                    f4 acc[C];
#pragma unroll
                    for (int c = 0; c < C; ++c) acc[c] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int sg = 0; sg < NS; ++sg) {
                        const f4 w4 = em_ok ? wcur[sg] : (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int q = 0; q < 4; ++q)
#pragma unroll
                            for (int c = 0; c < C; ++c)
                                acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4[q], yb[c][sg][q], acc[c], 0, 0, 0);
                    }
#pragma unroll
                    for (int sg = 0; sg < NS; ++sg) wcur[sg] = wnxt[sg];
                    // acc[c][r] = Abar_c(point r16, entry eb*16 + 4 g + r):
                    // the entry's terms of the input bars
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int e = eb * 16 + 4 * g + r;
                        const int en = L.ent[min(e, tot - 1)];
                        const int il = en >> 8, b = en & 0xFF;
                        float zj[C], Ab[C], v[4], zd[C];
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            zj[c] = L.z[c][il][r16];
                            Ab[c] = acc[c][r];
                            zd[c] = 0.f;
                        }
                        bump_d123f(knots[b], zj[0], bsc, v);
                        features_adjoint<float, O0, O1>(v, zj, Ab, zd);
#pragma unroll
                        for (int c = 0; c < C; ++c) L.tm[4 * g + r][c][r16] = e < tot ? zd[c] : 0.f;
                    }
                    __builtin_amdgcn_wave_barrier();
                    // per (channel, point): the block's entries in order, one
                    // running sum per input. The entries' inputs are the same
                    // for every lane: taken once into scalar registers, so the
                    // branches are uniform and the 16 term reads independent.
                    const int ne = min(16, tot - eb * 16);
                    const int my_in = L.ent[min(eb * 16 + r16, tot - 1)] >> 8;
                    int ein[16];
#pragma unroll
                    for (int e = 0; e < 16; ++e) ein[e] = __builtin_amdgcn_readlane(my_in, e);
                    for (int cp = lane; cp < C * TPT; cp += 64) {
                        const int c = cp / TPT, p = cp % TPT;
                        float tv[16];
#pragma unroll
                        for (int e = 0; e < 16; ++e) tv[e] = L.tm[e][c][p];
                        int cur = ein[0];
                        float run = 0.f;
#pragma unroll
                        for (int e = 0; e < 16; ++e) {
                            if (e < ne) {
                                if (ein[e] != cur) {
                                    L.zb[c][cur][p] += run;
                                    run = 0.f;
                                    cur = ein[e];
                                }
                                run += tv[e];
                            }
                        }
                        L.zb[c][cur][p] += run;
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                // the chunk's input bars (the second pass adds to the first's)
                if (pl_ok)
#pragma unroll
                    for (int c = 0; c < C; ++c)
#pragma unroll
                        for (int q = 0; q < TKJ / 4; ++q) {
                            const int il = g + 4 * q;
                            float *dst = zbar + (int64_t)(c * win + i0 + il) * n + pl;
                            const float v = L.zb[c][il][r16];
                            *dst = pass == 0 ? v : *dst + v;
                        }
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: gW[i nb + b][j] = sum_p sum_c A_c(p, i, b) ybar[c][j][p].
// A block takes TDI inputs and one slice of the points; wave w takes the 32
// outputs 32 (w % OG) .. + 31 (OG = N / 32 output groups) and every
// (4 / OG)-th tile of the slice. For a tile, the entries of the block's
// inputs (its K list) form the M axis in blocks of 16, the outputs the N
// axis, and the 16 points the reduction axis in 4 steps of 4 (lane group g
// takes point 4 g + s in step s), on the 16x16x4 FP32 MFMA; each entry
// block's 16 x 32 result is added into the wave's LDS copy of the block's
// gradient rows (every element by one lane, so in a fixed order). At the
// end the copies of the waves that share outputs are summed in wave order
// and written as the slice's partial rows (reduced over slices in FP64).
// ---------------------------------------------------------------------------
constexpr int TDI = 6;              // inputs per gradient block
constexpr int TDJ = 8;              // lane-group capacity of the K list builder (>= TDI)

template <int O0, int O1>
struct alignas(16) TcDwLds {
    static constexpr int C = 1 + O0 + O1;
    float z[C][TDI][TPT];
    unsigned short ent[TDI * MAXNB];    // entry blocks of 16 (TDI * MAXNB is a multiple of 16)
};

template <int O0, int O1, bool FIRST, int NT16, bool VEC>
__global__ __launch_bounds__(TNT, 2) void k_dw_tc(const float *__restrict__ zin, const float *__restrict__ ybar,
                                                  float *__restrict__ part, int64_t n, int win, int nsplit,
                                                  int64_t slice_pts, int nib, bool xcd_map, TcGrid gr)
{
    constexpr int C = 1 + O0 + O1;
    constexpr int N = 16 * NT16;
    constexpr int OG = NT16 / 2;                // 32-output groups
    constexpr int TPH = TW / OG;                // waves per output group (tile phases)
    extern __shared__ __align__(16) float dsm[];
    __shared__ TcDwLds<O0, O1> lds[TW];
    __shared__ float4 knots[MAXNB];    // split knots (split_knot)
    __shared__ int r0s_s[TW][TDJ], cnt_s[TW][TDJ];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    const int og = wv % OG, ph = wv / OG;
    TcDwLds<O0, O1> &L = lds[wv];
    int *r0s = r0s_s[wv], *cnts = cnt_s[wv];
    const int nb = gr.nb;
    const float inv_w = gr.inv_w, lo = gr.lo;
    // this block's input group and point slice. Blocks are dealt to the 8
    // XCDs in turn (block b to XCD b % 8); with xcd_map every input group of
    // a slice runs on one XCD, one after the other in its dispatch order, so
    // that the slice's bars, which each group reads, are shared in that
    // XCD's L2 (nsplit is then a multiple of 8)
    int ib, sl;
    if (xcd_map) {
        const int k = (int)(blockIdx.x >> 3);
        ib = k % nib;
        sl = (k / nib) * 8 + (int)(blockIdx.x & 7);
    } else {
        ib = (int)(blockIdx.x % nib);
        sl = (int)(blockIdx.x / nib);
    }
    const int i0 = ib * TDI;
    const int nin = min(TDI, win - i0);
    const int rows = nin * nb;
    float *grad = dsm + (size_t)wv * TDI * nb * 32;        // [row][32]
    if (threadIdx.x < nb) knots[threadIdx.x] = split_knot(gr.s[threadIdx.x], gr.e[threadIdx.x]);
    const BasisScale bsc = basis_scale(gr.inv_w_d);
    for (int e = lane; e < TDI * nb * 32; e += 64) grad[e] = 0.f;
    __syncthreads();
    const int64_t ps = (int64_t)sl * slice_pts;
    const int64_t pe = min(n, ps + slice_pts);
    const int64_t ntl = ps < pe ? (pe - ps + TPT - 1) / TPT : 0;
    // VEC: n is a multiple of 4, so a lane's 4 points of a tile are one aligned 16-byte load

    // a tile's jets of the block's inputs and its B operands
    // ybar[c][32 og + 16 ot + r16][p0 + 4 g + s] (s = 0..3), in registers;
    // the next tile's are loaded while the current one computes. Every load
    // is issued at an in-range place; which values are real (not past the
    // slice end or the block's inputs) is kept as masks and applied when the
    // tile is used, a loop iteration later, so that no load is sunk into a
    // branch (where the branches join the compiler would wait for every
    // load in flight).
    constexpr int NQ = (TDI + 3) / 4;
    float pz[C][NQ];
    f4 py[C][2];
    unsigned zmask = 0, ymask = 0;    // bit q: jet slot q real; bit s: point 4 g + s real
    auto load_tile = [&](int64_t t_) {
        const bool tok = t_ < ntl;
        const int64_t p0_ = ps + t_ * TPT;
        const int64_t p = p0_ + r16;
        const bool ok = tok && p < pe;
        zmask = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int il = g + 4 * q;
            const bool okq = ok && il < nin;
            zmask |= okq ? 1u << q : 0u;
#pragma unroll
            for (int c = 0; c < C; ++c) pz[c][q] = jet_in<O0, O1, FIRST>(zin, c, i0 + (okq ? il : 0), win, n, okq ? p : 0);
        }
        const int64_t pg = p0_ + 4 * g;
        ymask = 0;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) ymask |= (tok && pg + s4 < pe) ? 1u << s4 : 0u;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int ot = 0; ot < 2; ++ot) {
                const float *row = ybar + (int64_t)(c * N + 32 * og + 16 * ot + r16) * n;
                if constexpr (VEC) {
                    // n and pg are multiples of 4: pg <= n - 4 whenever pg < n
                    const int64_t pc = tok ? min(pg, n - 4) : 0;
                    py[c][ot] = *reinterpret_cast<const f4 *>(row + pc);
                } else {
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) py[c][ot][s4] = row[((ymask >> s4) & 1u) ? pg + s4 : 0];
                }
            }
    };
    load_tile(ph);

#pragma unroll 1
    for (int64_t t = ph; t < ntl; t += TPH) {
        const int64_t p0 = ps + t * TPT;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (g + 4 * q < TDI) L.z[c][g + 4 * q][r16] = ((zmask >> q) & 1u) ? pz[c][q] : 0.f;
        f4 yv[C][2];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int ot = 0; ot < 2; ++ot)
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) yv[c][ot][s4] = ((ymask >> s4) & 1u) ? py[c][ot][s4] : 0.f;
        load_tile(t + TPH);
        __builtin_amdgcn_wave_barrier();
        build_klist<TDJ>(L.z[0], lane, p0, pe, lo, inv_w, nb, r0s, cnts, nin);
        __builtin_amdgcn_wave_barrier();
        // the same count in every lane: a scalar, so the loops below branch
        // uniformly
        const int tot = __builtin_amdgcn_readfirstlane(write_entries<TDJ>(L.ent, lane, r0s, cnts));
        __builtin_amdgcn_wave_barrier();
        const int nblk = (tot + 15) / 16;
        // this lane's A row of entry block eb_ (entry eb_*16 + r16; past tot
        // the last entry, multiplied as zero)
        struct Ent {
            int il;
            float4 kn;
            bool ok;
        };
        auto ent_of = [&](int eb_) {
            const int em = eb_ * 16 + r16;
            const int en = L.ent[min(em, tot - 1)];
            return Ent{en >> 8, knots[en & 0xFF], em < tot};
        };
        // features of the 4 steps (points 4 g + s) of an entry block: the
        // lane's 4 points of each channel are one 16-byte LDS read, and the 4
        // FP64 basis evaluations are independent of each other
        auto comp_blk = [&](const Ent &E, float (*A)[C]) {
            f4 zz[C];
#pragma unroll
            for (int c = 0; c < C; ++c) zz[c] = *reinterpret_cast<const f4 *>(&L.z[c][E.il][4 * g]);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                float zj[C];
#pragma unroll
                for (int c = 0; c < C; ++c) zj[c] = zz[c][s];
                float v0, v1, v2;
                bump3f(E.kn, zj[0], bsc, v0, v1, v2);
#pragma unroll
                for (int c = 0; c < C; ++c) A[s][c] = E.ok ? feature_f<O0, O1>(c, v0, v1, v2, zj) : 0.f;
            }
        };
        if (nblk > 0) {
            // one software pipeline over the entry blocks: the next block's
            // features are computed while the current block's products run,
            // then the current block's gradient rows are read, added to and
            // written (the K list holds each (input, row) once, so the 4 rows
            // of a lane are distinct and all reads may precede the writes)
            Ent cur = ent_of(0);
            float Ac[4][C], An[4][C];
            comp_blk(cur, Ac);
#pragma unroll 1
            for (int eb = 0; eb < nblk; ++eb) {
                // this lane's 4 accumulator entries (one 8-byte read; past tot
                // unused) and its entry of the next block, read before the
                // products so that their latency is hidden behind them
                const int eq = eb * 16 + 4 * g;
                const uint2 e4 = *reinterpret_cast<const uint2 *>(&L.ent[eq]);
                const bool more = eb + 1 < nblk;
                const int en_nx = L.ent[min((eb + 1) * 16 + r16, tot - 1)];
                f4 acc[2] = {(f4){0.f, 0.f, 0.f, 0.f}, (f4){0.f, 0.f, 0.f, 0.f}};
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int c = 0; c < C; ++c)
#pragma unroll
                        for (int ot = 0; ot < 2; ++ot)
                            acc[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ac[s][c], yv[c][ot][s], acc[ot], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                // acc[ot][r] = D[entry eb*16 + 4 g + r][output 16 ot + r16]
                int rw[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int en = (int)((r < 2 ? e4.x : e4.y) >> (16 * (r & 1))) & 0xFFFF;
                    rw[r] = eq + r < tot ? (en >> 8) * nb + (en & 0xFF) : 0;
                }
                if (more) {
                    const int em = (eb + 1) * 16 + r16;
                    cur = Ent{en_nx >> 8, knots[en_nx & 0xFF], em < tot};
                    comp_blk(cur, An);
                }
                float old[4][2];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int ot = 0; ot < 2; ++ot) old[r][ot] = grad[rw[r] * 32 + 16 * ot + r16];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (eq + r < tot)
#pragma unroll
                        for (int ot = 0; ot < 2; ++ot) grad[rw[r] * 32 + 16 * ot + r16] = old[r][ot] + acc[ot][r];
                if (more)
#pragma unroll
                    for (int s = 0; s < 4; ++s)
#pragma unroll
                        for (int c = 0; c < C; ++c) Ac[s][c] = An[s][c];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // the slice's partial rows: the tile phases of each output group summed
    // in wave order
    float *dst = part + (int64_t)sl * ((int64_t)win * nb * N) + (int64_t)i0 * nb * N;
    for (int e = threadIdx.x; e < rows * N; e += TNT) {
        const int row = e / N, j = e % N;
        const int o = j / 32, jj = j % 32;
        float v = 0.f;
#pragma unroll
        for (int q = 0; q < TPH; ++q) v += dsm[(size_t)(q * OG + o) * TDI * nb * 32 + row * 32 + jj];
        dst[(int64_t)row * N + j] = v;
    }
}

#define HRK_TC_CH_SWITCH(ch, ...)                                  \
    switch ((ch).o0 * 3 + (ch).o1) {                               \
    case 0: { constexpr int O0 = 0, O1 = 0; __VA_ARGS__; } break;  \
    case 4: { constexpr int O0 = 1, O1 = 1; __VA_ARGS__; } break;  \
    case 6: { constexpr int O0 = 2, O1 = 0; __VA_ARGS__; } break;  \
    case 7: { constexpr int O0 = 2, O1 = 1; __VA_ARGS__; } break;  \
    case 8: { constexpr int O0 = 2, O1 = 2; __VA_ARGS__; } break;  \
    default: return hipErrorInvalidValue;                          \
    }

#define HRK_TC_N_SWITCH(N, ...)                                    \
    switch (N) {                                                   \
    case 32: { constexpr int NT16 = 2; __VA_ARGS__; } break;       \
    case 64: { constexpr int NT16 = 4; __VA_ARGS__; } break;       \
    case 128: { constexpr int NT16 = 8; __VA_ARGS__; } break;      \
    default: return hipErrorInvalidValue;                          \
    }

int grid_of(int64_t n, int cu_blocks, int tiles_per_block = TW)
{
    const int64_t tiles = (n + TPT - 1) / TPT;
    const int64_t blocks = (tiles + tiles_per_block - 1) / tiles_per_block;
    const int64_t cap = (int64_t)cu_blocks * 4;
    return (int)std::max<int64_t>(1, std::min(blocks, cap));
}

}  // namespace

bool tc_supported(ChanCfg ch, LayerShape ls, int k, int m, bool first)
{
    const int cs = ch.o0 * 3 + ch.o1;
    const bool chan_ok = cs == 0 || cs == 4 || cs == 6 || cs == 7 || cs == 8;
    const bool in_ok = first ? ls.win == 2 : ls.win % TKJ == 0;
    return chan_ok && in_ok && k == 3 && m == 4 && ls.nb >= 4 && ls.nb <= MAXNB &&
           (ls.wout == 32 || ls.wout == 64 || ls.wout == 128);
}

TcGrid make_tc_grid(double lo, double hi, int G, int k)
{
    TcGrid t{};
    const int nb = G + k;
    const double h = (hi - lo) / G;
    t.nb = nb;
    t.lo = (float)lo;
    t.inv_w = (float)(2.0 / ((k + 1) * h));
    t.inv_w_d = 2.0 / ((k + 1) * h);
    for (int b = 0; b < nb && b < MAXNB; ++b) {
        t.s[b] = lo + (b - k) * h;
        t.e[b] = lo + (b + 1) * h;
    }
    return t;
}

hipError_t launch_fwd_tc(ChanCfg ch, bool first, const float *zin, const float *W, float *zout, int64_t n,
                         LayerShape ls, const TcGrid &gr, int cu_blocks, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (!tc_supported(ch, ls, 3, 4, first)) return hipErrorInvalidValue;
    const int grid = grid_of(n, cu_blocks);
    HRK_TC_CH_SWITCH(ch, {
        HRK_TC_N_SWITCH(ls.wout, {
            if (first)
                hipLaunchKernelGGL((k_fwd_tc<O0, O1, true, NT16>), dim3(grid), dim3(TNT), 0, st, zin, W, zout, n,
                                   ls.win, gr);
            else
                hipLaunchKernelGGL((k_fwd_tc<O0, O1, false, NT16>), dim3(grid), dim3(TNT), 0, st, zin, W, zout, n,
                                   ls.win, gr);
        });
    });
    return hipGetLastError();
}



hipError_t launch_dx_tc(ChanCfg ch, const float *zin, const float *ybar, const float *W, float *zbar, int64_t n,
                        LayerShape ls, const TcGrid &gr, int cu_blocks, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (!tc_supported(ch, ls, 3, 4, false)) return hipErrorInvalidValue;
    const int grid = grid_of(n, cu_blocks);
    HRK_TC_CH_SWITCH(ch, {
        HRK_TC_N_SWITCH(ls.wout, {
            hipLaunchKernelGGL((k_dx_tc<O0, O1, NT16>), dim3(grid), dim3(TNT), 0, st, zin, ybar, W, zbar, n,
                               ls.win, gr);
        });
    });
    return hipGetLastError();
}

size_t dw_tc_lds_bytes(int nb) { return sizeof(float) * (size_t)TW * TDI * nb * 32; }

// Raise a kernel's dynamic-LDS limit to `bytes` when its last setting is
// lower (the first launch of each kernel and size happens eagerly, outside
// any graph capture). Kernels are told apart by their address.
hipError_t raise_lds(int, const void *kf, size_t bytes)
{
    static const void *fn[64];
    static size_t lim[64];
    static int nfn = 0;
    int k = 0;
    while (k < nfn && fn[k] != kf) ++k;
    if (k < nfn && lim[k] >= bytes) return hipSuccess;
    if (bytes <= 64 * 1024) return hipSuccess;         // the default limit
    const hipError_t e = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    if (k == nfn && nfn < 64) fn[nfn++] = kf;
    if (k < 64) lim[k] = bytes;
    return hipSuccess;
}

namespace {
// blocks of the weight-gradient kernel one XCD holds at a time: two per CU
int dw_xcd_slots()
{
    static int cached = 0;
    if (!cached) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 8)
            cus = 256;
        cached = 2 * (cus / 8);
    }
    return cached;
}
}  // namespace

int dw_tc_splits(int64_t n, LayerShape ls)
{
    if (n <= 0) return 0;
    const int64_t groups = (ls.win + TDI - 1) / TDI;
    const int64_t maxs = std::max<int64_t>(1, n / 256);     // at least 256 points per slice
    // XCD-aware (a multiple of 8 slices, every group of a slice on one XCD):
    // the fewest slices per XCD, m, that give at least 12 rounds of the XCD's
    // blocks (else at least 2) with the last round at least 95% full, at
    // 2,048 points per slice or more (a block's partial rows stay small
    // beside its reads). On the 128-wide hidden layers of 1,048,576 points
    // (22 groups, 64 blocks per XCD at a time) 13 to 17 rounds took 14.5 ms
    // per launch, 9 to 10 rounds 14.7 to 14.9, 5 rounds 15.1, 3 rounds 16.1
    // (smaller slices keep the groups of a slice closer together in time, so
    // more of their reads of the bars hit in L2; the slices' partial rows
    // grow with their number, 1.5 MB each there)
    const int64_t slots = dw_xcd_slots();
    for (const int64_t min_rounds : {12, 2})
        for (int64_t m = 1; m <= 64 && 8 * m <= n / 2048; ++m) {
            const int64_t blocks = groups * m;
            if (blocks < min_rounds * slots) continue;
            const int64_t rounds = (blocks + slots - 1) / slots;
            if (blocks * 100 >= rounds * slots * 95) return (int)(8 * m);
        }
    // otherwise two rounds of two blocks per CU over the input groups and
    // point slices (rounded down, so the last round is not a sliver)
    const int64_t s = std::max<int64_t>(1, 16 * slots / groups);
    return (int)std::max<int64_t>(1, std::min<int64_t>(std::min(s, maxs), 4096));
}

hipError_t launch_dw_tc(ChanCfg ch, bool first, const float *zin, const float *ybar, float *part, int nsplit,
                        int64_t n, LayerShape ls, const TcGrid &gr, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (!tc_supported(ch, ls, 3, 4, first) || nsplit < 1) return hipErrorInvalidValue;
    int64_t slice = (n + nsplit - 1) / nsplit;
    slice = (slice + TPT - 1) / TPT * TPT;
    const int nib = (ls.win + TDI - 1) / TDI;
    const dim3 grid((unsigned)(nib * nsplit));
    const bool xcd_map = nsplit % 8 == 0;
    const size_t sh = dw_tc_lds_bytes(ls.nb);
    HRK_TC_CH_SWITCH(ch, {
        HRK_TC_N_SWITCH(ls.wout, {
            const bool vec = n % 4 == 0;
            auto kf = first ? (vec ? k_dw_tc<O0, O1, true, NT16, true> : k_dw_tc<O0, O1, true, NT16, false>)
                            : (vec ? k_dw_tc<O0, O1, false, NT16, true> : k_dw_tc<O0, O1, false, NT16, false>);
            const hipError_t e = raise_lds(first ? 1 : 0, (const void *)kf, sh);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kf, grid, dim3(TNT), sh, st, zin, ybar, part, n, ls.win, nsplit, slice, nib, xcd_map,
                               gr);
        });
    });
    return hipGetLastError();
}

}  // namespace hrk
