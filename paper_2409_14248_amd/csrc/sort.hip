// sort.hip -- deterministic reordering of a collocation point set along a
// Z-order (Morton) curve, so that consecutive points of the reordered set lie
// close together in the domain. A training step's loss and weight gradient
// are sums over points, so they do not depend on the order (up to rounding);
// neighbouring points have nearby hidden-layer values, so a tile of
// consecutive points needs few basis rows per input (the tile-coherent
// kernels multiply only those).
//
// Key: 8 bits per coordinate over the set's bounding box, interleaved into a
// 16-bit Morton code. Sort: two stable least-significant-digit radix passes
// of 8 bits (per-chunk histograms, one exclusive scan, stable scatter with
// wave-level digit matching), then one gather of the points (and boundary
// targets) in the new order. No atomics on global memory; the result is the
// same on every run.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "sort.h"

namespace hrk {

namespace {

constexpr int SB = 512;                 // threads per sort block (8 waves)
constexpr int PER = 16;                 // keys per thread
constexpr int CHUNK = SB * PER;         // keys per block
constexpr int NBINS = 256;
constexpr int MAX_BBOX_BLOCKS = 256;

__host__ __device__ int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Per-block min and max of both coordinates (NaN coordinates are skipped:
// fminf / fmaxf return the other operand).
__global__ __launch_bounds__(SB) void k_bbox_part(const float *__restrict__ x, int64_t n, float4 *__restrict__ part)
{
    __shared__ float4 red[SB];
    float4 b = make_float4(FLT_MAX, -FLT_MAX, FLT_MAX, -FLT_MAX);
    for (int64_t p = (int64_t)blockIdx.x * SB + threadIdx.x; p < n; p += (int64_t)gridDim.x * SB) {
        const float2 v = reinterpret_cast<const float2 *>(x)[p];
        b.x = fminf(b.x, v.x);
        b.y = fmaxf(b.y, v.x);
        b.z = fminf(b.z, v.y);
        b.w = fmaxf(b.w, v.y);
    }
    red[threadIdx.x] = b;
    __syncthreads();
    for (int s = SB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const float4 o = red[threadIdx.x + s];
            float4 &m = red[threadIdx.x];
            m.x = fminf(m.x, o.x);
            m.y = fmaxf(m.y, o.y);
            m.z = fminf(m.z, o.z);
            m.w = fmaxf(m.w, o.w);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__device__ __forceinline__ uint32_t spread8(uint32_t v)
{
    v = (v | (v << 4)) & 0x0F0Fu;
    v = (v | (v << 2)) & 0x3333u;
    v = (v | (v << 1)) & 0x5555u;
    return v;
}

__device__ __forceinline__ uint32_t quant8(float v, float lo, float scale)
{
    const float q = (v - lo) * scale;
    if (!(q > 0.f)) return 0u;            // also NaN
    return q >= 255.f ? 255u : (uint32_t)q;
}

// Morton key of every point of the block's chunk and the chunk's histogram
// of the low key byte; counts are stored bin-major: counts[bin * nblk + blk].
__global__ __launch_bounds__(SB) void k_keys_hist(const float *__restrict__ x, int64_t n,
                                                  const float4 *__restrict__ bpart, int nbp,
                                                  uint32_t *__restrict__ keys, uint32_t *__restrict__ counts,
                                                  int nblk)
{
    __shared__ float4 red[SB];
    __shared__ uint32_t hist[NBINS];
    float4 b = make_float4(FLT_MAX, -FLT_MAX, FLT_MAX, -FLT_MAX);
    if (threadIdx.x < nbp) b = bpart[threadIdx.x];
    red[threadIdx.x] = b;
    if (threadIdx.x < NBINS) hist[threadIdx.x] = 0u;
    __syncthreads();
    for (int s = SB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const float4 o = red[threadIdx.x + s];
            float4 &m = red[threadIdx.x];
            m.x = fminf(m.x, o.x);
            m.y = fmaxf(m.y, o.y);
            m.z = fminf(m.z, o.z);
            m.w = fmaxf(m.w, o.w);
        }
        __syncthreads();
    }
    const float4 bb = red[0];
    const float sx = (bb.y > bb.x) ? 256.f / (bb.y - bb.x) : 0.f;
    const float sy = (bb.w > bb.z) ? 256.f / (bb.w - bb.z) : 0.f;
    const int64_t base = (int64_t)blockIdx.x * CHUNK;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t e = base + j * SB + threadIdx.x;
        if (e < n) {
            const float2 v = reinterpret_cast<const float2 *>(x)[e];
            const uint32_t key = (spread8(quant8(v.x, bb.x, sx)) << 1) | spread8(quant8(v.y, bb.z, sy));
            keys[e] = key;
            atomicAdd(&hist[key & 0xFFu], 1u);      // LDS counter: the count does not depend on the order
        }
    }
    __syncthreads();
    if (threadIdx.x < NBINS) counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = hist[threadIdx.x];
}

// Histogram of key byte `shift / 8` of every chunk of an array of keys.
__global__ __launch_bounds__(SB) void k_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                             uint32_t *__restrict__ counts, int nblk)
{
    __shared__ uint32_t hist[NBINS];
    if (threadIdx.x < NBINS) hist[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * CHUNK;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int64_t e = base + j * SB + threadIdx.x;
        if (e < n) atomicAdd(&hist[(keys[e] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    if (threadIdx.x < NBINS) counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = hist[threadIdx.x];
}

// Exclusive scan of m counts in place by one block of 1024 threads, row by
// row of 1024 consecutive entries (coalesced), each row scanned with wave
// shuffles and the 16 wave totals, plus the carry of the rows before it.
constexpr int SCAN_T = 1024;
__global__ __launch_bounds__(SCAN_T) void k_scan(uint32_t *__restrict__ c, int64_t m)
{
    __shared__ uint32_t wsum[SCAN_T / 64];
    __shared__ uint32_t carry_s;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0u;
    const int64_t rows = cdiv(m, SCAN_T);
    uint32_t nxt = threadIdx.x < m ? c[threadIdx.x] : 0u;
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t i = r * SCAN_T + threadIdx.x;
        const uint32_t v = nxt;
        const int64_t i2 = i + SCAN_T;
        nxt = i2 < m ? c[i2] : 0u;                    // next row in flight
        uint32_t inc = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t u = __shfl_up(inc, off, 64);
            if (lane >= off) inc += u;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t before = carry_s;
        for (int q = 0; q < w; ++q) before += wsum[q];
        if (i < m) c[i] = before + inc - v;
        __syncthreads();
        if (threadIdx.x == SCAN_T - 1) carry_s = before + inc;
        __syncthreads();
    }
}

// Stable scatter of one radix pass. The chunk's keys are taken in the order
// (wave, round, lane): wave w owns chunk positions [64 PER w, 64 PER (w + 1))
// in PER rounds of 64. In a round, the lanes holding the same digit find each other
// by 8 ballots; their rank is the number of such lanes below them plus the
// wave's running count of that digit (one lane per digit group updates it).
// Afterwards the waves' counts give each wave's base within the chunk's
// share of every digit. idx_in null: the element's own position.
__global__ __launch_bounds__(SB) void k_scatter(const uint32_t *__restrict__ keys_in,
                                                const uint32_t *__restrict__ idx_in, int64_t n, int shift,
                                                const uint32_t *__restrict__ offs, int nblk,
                                                uint32_t *__restrict__ keys_out, uint32_t *__restrict__ idx_out)
{
    constexpr int NW = SB / 64;
    __shared__ uint32_t cnt[NW][NBINS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int d = lane; d < NBINS; d += 64) cnt[w][d] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * CHUNK + (int64_t)w * (PER * 64);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t key[PER], dig[PER], rank[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int64_t e = base + r * 64 + lane;
        const bool ok = e < n;
        key[r] = ok ? keys_in[e] : 0u;
        const uint32_t d = (key[r] >> shift) & 0xFFu;
        dig[r] = d;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t m = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        const uint32_t old = ok ? cnt[w][d] : 0u;
        const uint32_t below_cnt = (uint32_t)__popcll(peers & below);
        if (ok && below_cnt == 0u) cnt[w][d] = old + (uint32_t)__popcll(peers);
        rank[r] = old + below_cnt;
    }
    __syncthreads();
    // base of each wave within the chunk's run of digit d
    for (int d = threadIdx.x; d < NBINS; d += SB) {
        uint32_t acc = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const uint32_t v = cnt[q][d];
            cnt[q][d] = acc;
            acc += v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int64_t e = base + r * 64 + lane;
        if (e < n) {
            const uint32_t d = dig[r];
            const uint32_t pos = offs[(int64_t)d * nblk + blockIdx.x] + cnt[w][d] + rank[r];
            if (pos < (uint64_t)n) {            // always true for consistent counts
                keys_out[pos] = key[r];
                idx_out[pos] = idx_in ? idx_in[e] : (uint32_t)e;
            }
        }
    }
}

__global__ __launch_bounds__(SB) void k_gather_points(const float *__restrict__ x, const float *__restrict__ g,
                                                      const uint32_t *__restrict__ idx, int64_t n,
                                                      float *__restrict__ xs, float *__restrict__ gs)
{
    for (int64_t p = (int64_t)blockIdx.x * SB + threadIdx.x; p < n; p += (int64_t)gridDim.x * SB) {
        const uint32_t q = idx[p];
        if (q >= (uint64_t)n) continue;          // never, for a permutation
        reinterpret_cast<float2 *>(xs)[p] = reinterpret_cast<const float2 *>(x)[q];
        if (g) gs[p] = g[q];
    }
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t sort_ws_bytes(int64_t n)
{
    if (n <= 0) return 0;
    const int64_t nblk = cdiv(n, CHUNK);
    return 4 * up256(sizeof(uint32_t) * (size_t)n) + up256(sizeof(uint32_t) * NBINS * (size_t)nblk) +
           up256(sizeof(float4) * MAX_BBOX_BLOCKS);
}

hipError_t launch_sort_points(const float *x, const float *g, int64_t n, void *ws, float *xs, float *gs,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int nblk = (int)cdiv(n, CHUNK);
    char *w = (char *)ws;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *p = w + o;
        o += up256(bytes);
        return p;
    };
    uint32_t *k0 = (uint32_t *)take(sizeof(uint32_t) * (size_t)n);
    uint32_t *i0 = (uint32_t *)take(sizeof(uint32_t) * (size_t)n);
    uint32_t *k1 = (uint32_t *)take(sizeof(uint32_t) * (size_t)n);
    uint32_t *i1 = (uint32_t *)take(sizeof(uint32_t) * (size_t)n);
    uint32_t *cnt = (uint32_t *)take(sizeof(uint32_t) * NBINS * (size_t)nblk);
    float4 *bpart = (float4 *)take(sizeof(float4) * MAX_BBOX_BLOCKS);
    const int nbp = (int)(cdiv(n, CHUNK) < MAX_BBOX_BLOCKS ? cdiv(n, CHUNK) : MAX_BBOX_BLOCKS);
    const int64_t m = (int64_t)NBINS * nblk;
    hipLaunchKernelGGL(k_bbox_part, dim3(nbp), dim3(SB), 0, st, x, n, bpart);
    hipLaunchKernelGGL(k_keys_hist, dim3(nblk), dim3(SB), 0, st, x, n, bpart, nbp, k0, cnt, nblk);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(SCAN_T), 0, st, cnt, m);
    hipLaunchKernelGGL(k_scatter, dim3(nblk), dim3(SB), 0, st, k0, (const uint32_t *)nullptr, n, 0, cnt, nblk,
                       k1, i1);
    hipLaunchKernelGGL(k_hist, dim3(nblk), dim3(SB), 0, st, k1, n, 8, cnt, nblk);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(SCAN_T), 0, st, cnt, m);
    hipLaunchKernelGGL(k_scatter, dim3(nblk), dim3(SB), 0, st, k1, i1, n, 8, cnt, nblk, k0, i0);
    const int gb = (int)(cdiv(n, SB) < 4096 ? cdiv(n, SB) : 4096);
    hipLaunchKernelGGL(k_gather_points, dim3(gb), dim3(SB), 0, st, x, g, i0, n, xs, gs);
    return hipGetLastError();
}

}  // namespace hrk
