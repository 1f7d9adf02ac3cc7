// kernels_batch.hip -- kernels of the batched step that differ from the
// single-instance ones: gathering every instance's points onto one
// concatenated axis, the residual / seeds / loss per instance, and the
// per-instance reduction of the weight-gradient slices.
//
// Concatenated axis: instance q's points occupy [off_q, off_q + n_q); every
// off_q is a multiple of 256 and the gap up to the next instance holds
// padding points (coordinates 0, target 0) whose seeds are zero, so they add
// nothing to any gradient or loss.
#include "batch.h"

namespace hrk {

namespace {

constexpr int NTB = 256;

__device__ __forceinline__ double wave_sum_b(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 256-thread block in a fixed order; valid in thread 0.
__device__ __forceinline__ double block_sum_b(double v, double *sh)
{
    v = wave_sum_b(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

// Copies each instance's points and targets onto the concatenated axes
// (interior [n_int_tot][2], boundary [n_bc_tot][2] and [n_bc_tot]).
__global__ __launch_bounds__(NTB) void k_gather(const BatchInst *__restrict__ inst,
                                                const int *__restrict__ ginst_int,
                                                const int *__restrict__ ginst_bc, int64_t n_int_tot,
                                                int64_t n_bc_tot, float *__restrict__ x_int,
                                                float *__restrict__ x_bc, float *__restrict__ g_bc)
{
    const int64_t p = (int64_t)blockIdx.x * NTB + threadIdx.x;
    if (p < n_int_tot) {
        const BatchInst &q = inst[ginst_int[p >> 7]];
        const int64_t l = p - q.off_int;
        float2 v = make_float2(0.f, 0.f);
        if (l < q.n_int) v = reinterpret_cast<const float2 *>(q.x_int)[l];
        reinterpret_cast<float2 *>(x_int)[p] = v;
    }
    if (p < n_bc_tot) {
        const BatchInst &q = inst[ginst_bc[p >> 7]];
        const int64_t l = p - q.off_bc;
        float2 v = make_float2(0.f, 0.f);
        float gv = 0.f;
        if (l < q.n_bc) {
            v = reinterpret_cast<const float2 *>(q.x_bc)[l];
            gv = q.g_bc[l];
        }
        reinterpret_cast<float2 *>(x_bc)[p] = v;
        g_bc[p] = gv;
    }
}

__device__ __forceinline__ float sin_pi_f(float v) { return sinpif(v); }

// Blocks [0, nblk_int) cover the interior axis, the rest the boundary axis;
// each 256-point block lies in one instance. Residual and seeds per point
// with that instance's coefficients; one loss partial per block.
template <int KIND>
__global__ __launch_bounds__(NTB) void k_residual_batched(
    const BatchInst *__restrict__ inst, const int *__restrict__ ginst_int,
    const int *__restrict__ ginst_bc, const float *__restrict__ jets,
    const float *__restrict__ x_int, int64_t n_int_tot, const float *__restrict__ u_bc,
    const float *__restrict__ g_bc, int64_t n_bc_tot, int nblk_int, float *__restrict__ seed_int,
    float *__restrict__ seed_bc, double *__restrict__ partials)
{
    __shared__ double sh[4];
    double e = 0.0;
    if ((int)blockIdx.x < nblk_int) {
        const int64_t p = (int64_t)blockIdx.x * NTB + threadIdx.x;
        const int64_t n = n_int_tot;
        const BatchInst &q = inst[ginst_int[p >> 7]];
        const bool live = p - q.off_int < q.n_int;
        float r;
        if constexpr (KIND == HRKAN_POISSON2D) {
            const float uxx = jets[2 * n + p], uyy = jets[4 * n + p];
            const float x = x_int[2 * p], y = x_int[2 * p + 1];
            r = uxx + uyy + 19.739208802178716f * sin_pi_f(x) * sin_pi_f(y);
            const float rho = live ? q.sc_int * r : 0.f;
            seed_int[0 * n + p] = 0.f;
            seed_int[1 * n + p] = 0.f;
            seed_int[2 * n + p] = rho;
            seed_int[3 * n + p] = 0.f;
            seed_int[4 * n + p] = rho;
        } else {
            const float u = jets[p], ux = jets[n + p], uxx = jets[2 * n + p], ut = jets[3 * n + p];
            r = ut + q.adv * u * ux - q.nu * uxx;
            const float rho = live ? q.sc_int * r : 0.f;
            seed_int[0 * n + p] = rho * q.adv * ux;
            seed_int[1 * n + p] = rho * q.adv * u;
            seed_int[2 * n + p] = -rho * q.nu;
            seed_int[3 * n + p] = rho;
        }
        if (live) e = (double)r * (double)r;
    } else {
        const int64_t p = (int64_t)(blockIdx.x - nblk_int) * NTB + threadIdx.x;
        const BatchInst &q = inst[ginst_bc[p >> 7]];
        const bool live = p - q.off_bc < q.n_bc;
        const float d = u_bc[p] - g_bc[p];
        seed_bc[p] = live ? q.sc_bc * d : 0.f;
        if (live) e = (double)d * (double)d;
    }
    const double s = block_sum_b(e, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
    (void)n_bc_tot;
}

// One block per instance: its interior and boundary block partials summed
// in a fixed order, loss_out[q][3] = {L, L_pde, L_bc}.
__global__ __launch_bounds__(NTB) void k_loss_batched(const BatchInst *__restrict__ inst,
                                                      const double *__restrict__ partials,
                                                      int nblk_int, double *__restrict__ loss_out,
                                                      uint32_t *__restrict__ status)
{
    __shared__ double sh[4];
    const BatchInst &q = inst[blockIdx.x];
    const int bi0 = (int)(q.off_int / NTB), bi1 = bi0 + q.blk_int;
    const int bb0 = nblk_int + (int)(q.off_bc / NTB), bb1 = bb0 + q.blk_bc;
    double a = 0.0, b = 0.0;
    for (int i = bi0 + threadIdx.x; i < bi1; i += NTB) a += partials[i];
    for (int i = bb0 + threadIdx.x; i < bb1; i += NTB) b += partials[i];
    const double sa = block_sum_b(a, sh);
    const double sb = block_sum_b(b, sh);
    if (threadIdx.x == 0) {
        const double lpde = q.n_int > 0 ? sa / (double)q.n_int : 0.0;
        const double lbc = q.n_bc > 0 ? sb / (double)q.n_bc : 0.0;
        const double L = q.alpha * lpde + lbc;
        loss_out[3 * blockIdx.x + 0] = L;
        loss_out[3 * blockIdx.x + 1] = lpde;
        loss_out[3 * blockIdx.x + 2] = lbc;
        if (!isfinite(L)) status[0] |= HRKAN_STATUS_NONFINITE;
    }
}

// gW of instance blockIdx.y, layer elements [32 blockIdx.x, +32): the sum of
// its interior slices then its boundary slices (in index order), each of
// 8 slice lanes summing a strided subset, the lanes added in order.
constexpr int RB_EB = 32, RB_SL = NTB / RB_EB;
__global__ __launch_bounds__(NTB) void k_reduce_batched(const BatchInst *__restrict__ inst,
                                                        const float *__restrict__ part,
                                                        int64_t count, int nsl_int,
                                                        float *__restrict__ gW, int64_t w_stride)
{
    __shared__ double sh[RB_SL][RB_EB];
    const BatchInst &q = inst[blockIdx.y];
    const int el = threadIdx.x % RB_EB, sl = threadIdx.x / RB_EB;
    const int64_t e = (int64_t)blockIdx.x * RB_EB + el;
    double s = 0.0;
    if (e < count) {
        const int ranges[2][2] = {{q.sl_int0, q.sl_int0 + q.nsl_int},
                                  {nsl_int + q.sl_bc0, nsl_int + q.sl_bc0 + q.nsl_bc}};
        for (int r = 0; r < 2; ++r) {
            int k = ranges[r][0] + sl;
            for (; k + 7 * RB_SL < ranges[r][1]; k += 8 * RB_SL) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(k + u * RB_SL) * count + e];
#pragma unroll
                for (int u = 0; u < 8; ++u) s += (double)v[u];
            }
            for (; k < ranges[r][1]; k += RB_SL) s += (double)part[(int64_t)k * count + e];
        }
    }
    sh[sl][el] = s;
    __syncthreads();
    if (sl == 0 && e < count) {
        double t = 0.0;
        for (int k = 0; k < RB_SL; ++k) t += sh[k][el];
        gW[(int64_t)blockIdx.y * w_stride + e] = (float)t;
    }
}

}  // namespace

hipError_t launch_gather(const BatchDev &b, hipStream_t st)
{
    const int64_t n = std::max(b.n_int_tot, b.n_bc_tot);
    if (n <= 0) return hipSuccess;
    k_gather<<<(unsigned)((n + NTB - 1) / NTB), NTB, 0, st>>>(b.inst, b.ginst_int, b.ginst_bc, b.n_int_tot,
                                                           b.n_bc_tot, b.x_int, b.x_bc, b.g_bc);
    return hipGetLastError();
}

hipError_t launch_residual_batched(int kind, const BatchDev &b, const float *jets, const float *u_bc,
                                   float *seed_int, float *seed_bc, double *partials, hipStream_t st)
{
    const int nbi = (int)(b.n_int_tot / NTB), nbb = (int)(b.n_bc_tot / NTB);
    if (nbi + nbb == 0) return hipSuccess;
    if (kind == HRKAN_POISSON2D)
        k_residual_batched<HRKAN_POISSON2D><<<nbi + nbb, NTB, 0, st>>>(
            b.inst, b.ginst_int, b.ginst_bc, jets, b.x_int, b.n_int_tot, u_bc, b.g_bc, b.n_bc_tot, nbi,
            seed_int, seed_bc, partials);
    else
        k_residual_batched<HRKAN_BURGERS1D><<<nbi + nbb, NTB, 0, st>>>(
            b.inst, b.ginst_int, b.ginst_bc, jets, b.x_int, b.n_int_tot, u_bc, b.g_bc, b.n_bc_tot, nbi,
            seed_int, seed_bc, partials);
    return hipGetLastError();
}

hipError_t launch_loss_batched(const BatchDev &b, int n_inst, const double *partials, double *loss_out,
                               uint32_t *status, hipStream_t st)
{
    k_loss_batched<<<n_inst, NTB, 0, st>>>(b.inst, partials, (int)(b.n_int_tot / NTB), loss_out, status);
    return hipGetLastError();
}

hipError_t launch_reduce_batched(const BatchDev &b, int n_inst, const float *part, int64_t count,
                                 int nsl_int, float *gW, int64_t w_stride, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const dim3 grid((unsigned)((count + RB_EB - 1) / RB_EB), (unsigned)n_inst);
    k_reduce_batched<<<grid, NTB, 0, st>>>(b.inst, part, count, nsl_int, gW, w_stride);
    return hipGetLastError();
}

}  // namespace hrk
