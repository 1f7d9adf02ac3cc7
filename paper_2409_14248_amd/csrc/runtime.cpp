// runtime.cpp -- host side of the HRKAN C ABI: argument validation, workspace
// layout, and the sequence of kernel launches of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "hrkan.h"
#include "internal.h"
#include "kernels_bs.h"
#include "kernels_tc.h"
#include "sort.h"
#include "kernels_dn.h"
#include "runtime_internal.h"

namespace hrk {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(HRKAN_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int check_net(const hrkan_net_desc *d, NetInfo *ni)
{
    if (!d) return fail(HRKAN_ERR_INVALID_ARG, "net is NULL");
    if (d->n_layers < 1 || d->n_layers > HRKAN_MAX_LAYERS)
        return fail(HRKAN_ERR_INVALID_ARG, "n_layers=%d outside 1..%d", d->n_layers, HRKAN_MAX_LAYERS);
    if (d->widths[0] != 2) return fail(HRKAN_ERR_INVALID_ARG, "widths[0]=%d, must be 2", d->widths[0]);
    if (d->widths[d->n_layers] != 1)
        return fail(HRKAN_ERR_INVALID_ARG, "widths[n_layers]=%d, must be 1", d->widths[d->n_layers]);
    int maxw = 0;
    for (int l = 0; l <= d->n_layers; ++l) {
        if (d->widths[l] < 1 || d->widths[l] > HRKAN_MAX_WIDTH)
            return fail(HRKAN_ERR_INVALID_ARG, "widths[%d]=%d outside 1..%d", l, d->widths[l], HRKAN_MAX_WIDTH);
        maxw = std::max(maxw, d->widths[l]);
    }
    if (d->G < 1 || d->G > 4096) return fail(HRKAN_ERR_INVALID_ARG, "G=%d outside 1..4096", d->G);
    if (d->k < 0 || d->k > 8) return fail(HRKAN_ERR_INVALID_ARG, "k=%d outside 0..8", d->k);
    if (d->m < 2 || d->m > 8) return fail(HRKAN_ERR_UNSUPPORTED, "m=%d outside 2..8", d->m);
    if (!std::isfinite(d->lo) || !std::isfinite(d->hi) || !(d->hi > d->lo))
        return fail(HRKAN_ERR_INVALID_ARG, "grid [%g, %g] is not a finite interval", d->lo, d->hi);
    if (d->dtype != HRKAN_F64 && d->dtype != HRKAN_F32 && d->dtype != HRKAN_BF16)
        return fail(HRKAN_ERR_INVALID_ARG, "dtype=%d unknown", d->dtype);
    if (d->dtype == HRKAN_BF16 && (d->bf16_split < 1 || d->bf16_split > 3))
        return fail(HRKAN_ERR_INVALID_ARG, "bf16_split=%d outside 1..3", d->bf16_split);
    if (d->k + 1 > 4)
        return fail(HRKAN_ERR_UNSUPPORTED, "k=%d: at most 4 live basis functions per input (k <= 3)", d->k);
    ni->L = d->n_layers;
    for (int l = 0; l <= d->n_layers; ++l) ni->w[l] = d->widths[l];
    ni->G = d->G;
    ni->k = d->k;
    ni->m = d->m;
    ni->nb = d->G + d->k;
    ni->lo = d->lo;
    ni->hi = d->hi;
    ni->dtype = d->dtype;
    ni->S = d->dtype == HRKAN_BF16 ? d->bf16_split : 1;
    ni->elem = d->dtype == HRKAN_F64 ? 8 : 4;
    ni->maxw = maxw;
    if (ni->nb > 32) return fail(HRKAN_ERR_UNSUPPORTED, "n_b = G + k = %d > 32", ni->nb);
    if (d->dtype == HRKAN_BF16) {
        if (d->k != 3 || d->m != 4)
            return fail(HRKAN_ERR_UNSUPPORTED, "HRKAN_BF16 needs k = 3 and m = 4 (k=%d, m=%d)", d->k, d->m);
        for (int l = 0; l < d->n_layers; ++l)
            if (!bs32_supported(LayerShape{d->widths[l], d->widths[l + 1], ni->nb}, l == 0))
                return fail(HRKAN_ERR_UNSUPPORTED, "HRKAN_BF16: layer %d shape %d x %d (n_b %d) not supported",
                            l, d->widths[l], d->widths[l + 1], ni->nb);
    }
    ni->n_params = 0;
    for (int l = 0; l < ni->L; ++l) ni->n_params += (int64_t)ni->w[l] * ni->nb * ni->w[l + 1];
    ni->cw = 5;
    ni->mc = true;
    return HRKAN_OK;
}

// The channel sets the matrix-core kernels take.
static bool mc_channels(ChanCfg ch)
{
    return (ch.o0 == 0 && ch.o1 == 0) || (ch.o0 == 1 && ch.o1 == 1) ||
           (ch.o0 == 2 && ch.o1 <= 2);
}

int apply_channels(NetInfo *ni, ChanCfg ch)
{
    ni->cw = std::max(5, ch.C());
    ni->mc = mc_channels(ch);
    if (!ni->mc && ni->dtype == HRKAN_BF16)
        return fail(HRKAN_ERR_UNSUPPORTED,
                    "HRKAN_BF16 runs the jet orders (%d, %d) on no kernel: the BF16 matrix-core kernels take "
                    "at most second derivatives (U; U,X,Y; U,X,XX; U,X,XX,Y; U,X,XX,Y,YY)", ch.o0, ch.o1);
    return HRKAN_OK;
}

// The derivative bits of each coordinate, by order 1..5.
static const uint32_t XBITS[HRKAN_MAX_ORDER] = {HRKAN_CH_X, HRKAN_CH_XX, HRKAN_CH_X3, HRKAN_CH_X4, HRKAN_CH_X5};
static const uint32_t YBITS[HRKAN_MAX_ORDER] = {HRKAN_CH_Y, HRKAN_CH_YY, HRKAN_CH_Y3, HRKAN_CH_Y4, HRKAN_CH_Y5};

// Order of the derivatives of one coordinate in a mask: the bits of orders
// 1..o and no other; -1 if there is a gap.
static int axis_order(uint32_t mask, const uint32_t *bits)
{
    int o = 0;
    while (o < HRKAN_MAX_ORDER && (mask & bits[o])) ++o;
    for (int k = o; k < HRKAN_MAX_ORDER; ++k)
        if (mask & bits[k]) return -1;
    return o;
}

int mask_cfg(uint32_t mask, ChanCfg *ch)
{
    uint32_t all = HRKAN_CH_U;
    for (int k = 0; k < HRKAN_MAX_ORDER; ++k) all |= XBITS[k] | YBITS[k];
    if (!(mask & HRKAN_CH_U) || (mask & ~all))
        return fail(HRKAN_ERR_INVALID_ARG, "channel mask 0x%x: must contain U and only the HRKAN_CH_* bits", mask);
    const int ox = axis_order(mask, XBITS), oy = axis_order(mask, YBITS);
    if (ox < 0 || oy < 0)
        return fail(HRKAN_ERR_INVALID_ARG,
                    "channel mask 0x%x: the derivatives of a coordinate must be those of order 1..o", mask);
    *ch = {ox, oy};
    return HRKAN_OK;
}

template <typename T>
GridP<T> make_grid(const NetInfo &ni)
{
    const double h = (ni.hi - ni.lo) / ni.G;
    GridP<T> g;
    g.lo = (T)ni.lo;
    g.inv_w = (T)(2.0 / ((ni.k + 1) * h));
    g.kappa = (T)(2.0 / (ni.k + 1));
    g.inv_kappa = (T)((ni.k + 1) / 2.0);
    g.k = ni.k;
    g.nb = ni.nb;
    g.m = ni.m;
    return g;
}
template GridP<float> make_grid<float>(const NetInfo &);
template GridP<double> make_grid<double>(const NetInfo &);

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

int64_t saved_elems(const NetInfo &ni, int C, int64_t n)
{
    int64_t e = 0;
    for (int l = 1; l < ni.L; ++l) e += (int64_t)C * ni.w[l] * n;
    return e;
}

// Slices of the weight-gradient reduction for n points at layer l.
// The FP32 and BF16 arrays go through the matrix-core kernels where the
// layer shape allows it; FP64 (and other shapes) through the generic ones.
bool use_bs32(const NetInfo &ni, int l)
{
    return ni.mc && ni.dtype != HRKAN_F64 && ni.m == 4 && ni.k == 3 &&
           bs32_supported(LayerShape{ni.w[l], ni.w[l + 1], ni.nb}, l == 0);
}

// Hidden BF16 layers with 32, 64 or 128 outputs run on the dense BF16
// kernels (HRKAN_BF16_DENSE=0 in the environment keeps them on the
// block-sparse ones); the input and output layers stay block-sparse.
bool use_dn(const NetInfo &ni, int l)
{
    static const bool enabled = [] {
        const char *e = getenv("HRKAN_BF16_DENSE");
        return !(e && e[0] == '0');
    }();
    return enabled && ni.mc && ni.dtype == HRKAN_BF16 && ni.m == 4 && ni.k == 3 &&
           dn_supported(LayerShape{ni.w[l], ni.w[l + 1], ni.nb}, l == 0);
}


// FP32 layers with 32, 64 or 128 outputs run on the tile-coherent kernels
// (HRKAN_TC=0 in the environment keeps them on the block-sparse ones).
bool tc_enabled()
{
    static const bool enabled = [] {
        const char *e = getenv("HRKAN_TC");
        return !(e && e[0] == '0');
    }();
    return enabled;
}

// Where the tile-coherent kernels beat the block-sparse ones, measured per
// stage on the FP32 steps (ms per launch, sets ordered along the curve):
//  - 32-output layers (Burgers [2,32,32,1], 65,536 + 4,096 points): never:
//    the point ordering alone (0.12 ms) costs more than they save (at
//    1,048,576 points they save 0.4 ms of 4.5 per step, the ordering costing
//    0.24);
//  - 64 outputs (Poisson [2,64,64,64,1], 262,144 points): forward (0.61
//    against 1.33) and weight gradient (1.05 to 1.20 against 1.89), not the
//    input bars (1.55 and 1.80 for the two hidden layers against 1.60 and
//    1.60: the second layer's K lists are longer);
//  - 128 outputs (Burgers [2,128,128,128,1], 1,048,576 points): every stage
//    (forward 6.1 against 18.2, input bars 11.3 against 20.9, weight
//    gradient 14.5 against 24.3).
// stage: 'f' forward, 'x' input bars, 'w' weight gradient.
bool use_tc(const NetInfo &ni, int l, char stage)
{
    if (!(tc_enabled() && ni.mc && ni.dtype == HRKAN_F32 &&
          tc_supported(ChanCfg{2, 2}, LayerShape{ni.w[l], ni.w[l + 1], ni.nb}, ni.k, ni.m, l == 0)))
        return false;
    const int N = ni.w[l + 1];
    return stage == 'x' ? N >= 128 : N >= 64;
}

// A training step orders each point set along a Z-order curve first (in the
// workspace) when its hidden layers run on the tile-coherent kernels and the
// sets run separately (not merged).
bool sorted_sets(const NetInfo &ni, int64_t n_int, int64_t n_bc)
{
    if (merged_sets(ni, n_int, n_bc) || n_int > ((int64_t)1 << 24) || n_bc > ((int64_t)1 << 24)) return false;
    for (int l = 0; l < ni.L; ++l)
        if (use_tc(ni, l, 'f') || use_tc(ni, l, 'x') || use_tc(ni, l, 'w')) return true;
    return false;
}

size_t wdn_offset(const NetInfo &ni, int l)
{
    size_t o = 0;
    for (int q = 0; q < l; ++q)
        if (use_dn(ni, q)) o += up256(dn_w_bytes(LayerShape{ni.w[q], ni.w[q + 1], ni.nb}, ni.S));
    return o;
}

// The padded BF16 weight copies the dense kernels read, for every such layer.
int prep_dense(const NetInfo &ni, const float *const *W, char *wdn, hipStream_t st)
{
    for (int l = 0; l < ni.L; ++l) {
        if (!use_dn(ni, l)) continue;
        const hipError_t e =
            launch_w_prep_dn(W[l], wdn + wdn_offset(ni, l), LayerShape{ni.w[l], ni.w[l + 1], ni.nb}, ni.S, st);
        if (e != hipSuccess) return hip_fail(e, "weight copy launch");
    }
    return HRKAN_OK;
}

// BF16 product terms of the matrix-core kernels (0: FP32 products). check_net
// admits HRKAN_BF16 only where every layer runs on them.
int bf16_terms(const NetInfo &ni) { return ni.dtype == HRKAN_BF16 ? ni.S : 0; }

int dw_splits(const NetInfo &ni, int l, int64_t n)
{
    if (n <= 0) return 0;
    const LayerShape ls{ni.w[l], ni.w[l + 1], ni.nb};
    if (use_dn(ni, l)) return dw_dn_splits(n, ls);
    if (use_tc(ni, l, 'w')) return dw_tc_splits(n, ls);
    return use_bs32(ni, l) ? dw_bs32_splits(n, ls) : dw_generic_splits(n, ls);
}

int cu_blocks()
{
    static int cached = 0;
    if (!cached) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached = 2 * cus;
    }
    return cached;
}

// How a training step runs its interior and boundary sets, by the interior
// points times the widest hidden layer (measured on the FP32 kernels):
//  - up to MERGE_MAX_WORK (the paper's instances, 1,024 x 8): as one set, the
//    boundary points as more rows of the interior set with the interior's jet
//    channels (their derivative channels get zero seeds, so they add no term
//    to the loss or the gradient). The boundary set's own launches would cost
//    more than its points do there.
//  - up to OVERLAP_MAX_WORK (65,536 x 32): the boundary set on a side stream,
//    beside the interior set, which hides launch gaps.
//  - above it (262,144 x 64) one after the other on the caller's stream: a
//    hidden-layer launch of such a set fills the GPU in one round of blocks,
//    and a kernel beside it pushes some of those blocks into a second round,
//    which costs more than the overlap gains.
constexpr int64_t MERGE_MAX_WORK = (int64_t)1 << 20;
constexpr int64_t OVERLAP_MAX_WORK = (int64_t)4 << 20;

static int64_t set_work(const NetInfo &ni, int64_t n_int)
{
    int wmax = 0;
    for (int l = 1; l < ni.L; ++l) wmax = std::max(wmax, ni.w[l]);
    return n_int * (int64_t)wmax;
}

bool merged_sets(const NetInfo &ni, int64_t n_int, int64_t n_bc)
{
    return n_int > 0 && n_bc > 0 && set_work(ni, n_int) <= MERGE_MAX_WORK;
}

static bool overlap_sets(const NetInfo &ni, int64_t n_int, int64_t n_bc)
{
    return n_int > 0 && n_bc > 0 && !merged_sets(ni, n_int, n_bc) && set_work(ni, n_int) <= OVERLAP_MAX_WORK;
}

// A second stream per (device, caller stream), for overlap_sets: created on
// first use and kept for the life of the process, at the default priority.
int get_fork(hipStream_t st, Fork **out)
{
    struct Entry {
        int dev;
        hipStream_t st;
        Fork f;
    };
    static std::mutex mu;
    static Entry tab[64];
    static int ntab = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(mu);
    for (int k = 0; k < ntab; ++k)
        if (tab[k].dev == dev && tab[k].st == st) {
            *out = &tab[k].f;
            return HRKAN_OK;
        }
    if (ntab == 64) {
        *out = nullptr;
        return HRKAN_OK;
    }
    Entry &en = tab[ntab];
    en.dev = dev;
    en.st = st;
    if ((e = hipStreamCreateWithFlags(&en.f.side, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "side stream");
    if ((e = hipEventCreateWithFlags(&en.f.fork, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&en.f.join, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "fork events");
    ++ntab;
    *out = &en.f;
    return HRKAN_OK;
}

int fork_to(Fork *f, hipStream_t st)
{
    hipError_t e = hipEventRecord(f->fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(f->side, f->fork, 0);
    return e == hipSuccess ? HRKAN_OK : hip_fail(e, "stream fork");
}

int join_from(Fork *f, hipStream_t st)
{
    hipError_t e = hipEventRecord(f->join, f->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, f->join, 0);
    return e == hipSuccess ? HRKAN_OK : hip_fail(e, "stream join");
}

// Weight-gradient partial slices of layer l for point sets of n_a and n_b
// points (elements). Every layer has a region of its own, so that the two
// sets' reverse passes can run concurrently and reduce at the end.
int64_t part_layer_elems(const NetInfo &ni, int l, int64_t n_a, int64_t n_b)
{
    const int64_t kn = (int64_t)ni.w[l] * ni.nb * ni.w[l + 1];
    return (int64_t)(dw_splits(ni, l, n_a) + dw_splits(ni, l, n_b)) * kn;
}

static int64_t part_elems_total(const NetInfo &ni, int64_t n_a, int64_t n_b)
{
    int64_t m = 0;
    for (int l = 0; l < ni.L; ++l) m += part_layer_elems(ni, l, n_a, n_b);
    return m;
}

// Workspace regions, in bytes from the start of ws. Sizes use ni.cw channels
// (at least 5) for interior sets, so one layout serves the Poisson and
// Burgers kinds and every call of either. A merged step keeps its one set in
// the interior regions.
WsLayout layout(const NetInfo &ni, int64_t n_int, int64_t n_bc)
{
    WsLayout L{};
    const size_t E = ni.elem;
    L.merged = merged_sets(ni, n_int, n_bc);
    const int64_t na = L.merged ? n_int + n_bc : n_int, nbs = L.merged ? 0 : n_bc;
    const int64_t nmax = std::max<int64_t>(std::max(na, nbs), 1);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += up256(bytes); return at; };
    L.status = take(256);
    L.nres = residual_blocks(n_int, n_bc);
    L.loss_part = take(sizeof(double) * 2 * (size_t)L.nres);
    L.xall = take(L.merged ? E * 2 * (size_t)na : 0);
    const size_t cw = (size_t)ni.cw;
    L.sv_int = take(E * (size_t)saved_elems(ni, ni.cw, na));
    L.jets_int = take(E * cw * (size_t)na);
    L.sv_bc = take(E * (size_t)saved_elems(ni, 1, nbs));
    L.ubc = take(E * (size_t)nbs);
    L.seed_int = take(E * cw * (size_t)na);
    L.seed_bc = take(E * (size_t)nbs);
    L.bars0 = take(E * cw * (size_t)ni.maxw * nmax);
    L.bars1 = take(E * cw * (size_t)ni.maxw * nmax);
    L.bbars0 = take(E * (size_t)ni.maxw * nbs);
    L.bbars1 = take(E * (size_t)ni.maxw * nbs);
    L.part_elems = part_elems_total(ni, na, nbs);
    L.part = take(E * (size_t)L.part_elems);
    L.wdn = take(wdn_offset(ni, ni.L));
    L.sorted = sorted_sets(ni, n_int, n_bc);
    L.xs_int = take(L.sorted ? sizeof(float) * 2 * (size_t)n_int : 0);
    L.xs_bc = take(L.sorted ? sizeof(float) * 2 * (size_t)n_bc : 0);
    L.gs_bc = take(L.sorted ? sizeof(float) * (size_t)n_bc : 0);
    L.sort_ws = take(L.sorted ? sort_ws_bytes(std::max(n_int, n_bc)) : 0);
    L.total = o;
    return L;
}

int check_pde(const hrkan_pde_desc *pde)
{
    if (!pde) return fail(HRKAN_ERR_INVALID_ARG, "pde is NULL");
    if (pde->kind != HRKAN_POISSON2D && pde->kind != HRKAN_BURGERS1D && pde->kind != HRKAN_LINEAR2D)
        return fail(HRKAN_ERR_INVALID_ARG, "pde kind %d unknown", pde->kind);
    if (!std::isfinite(pde->nu) || !std::isfinite(pde->alpha) || !std::isfinite(pde->adv))
        return fail(HRKAN_ERR_INVALID_ARG, "pde coefficients must be finite");
    if (pde->kind == HRKAN_LINEAR2D) {
        bool ok = std::isfinite(pde->c0);
        for (int k = 0; k < HRKAN_MAX_ORDER; ++k) ok = ok && std::isfinite(pde->cx[k]) && std::isfinite(pde->cy[k]);
        if (!ok) return fail(HRKAN_ERR_INVALID_ARG, "linear pde coefficients must be finite");
    }
    return HRKAN_OK;
}

// Highest derivative order with a non-zero coefficient along x / y.
static void linear_orders(const hrkan_pde_desc *pde, int *ox, int *oy)
{
    *ox = *oy = 0;
    for (int k = 1; k <= HRKAN_MAX_ORDER; ++k) {
        if (pde->cx[k - 1] != 0.0) *ox = k;
        if (pde->cy[k - 1] != 0.0) *oy = k;
    }
}

uint32_t pde_mask(const hrkan_pde_desc *pde)
{
    if (pde->kind == HRKAN_POISSON2D) return HRKAN_MASK_POISSON;
    if (pde->kind == HRKAN_BURGERS1D) return HRKAN_MASK_BURGERS;
    int ox, oy;
    linear_orders(pde, &ox, &oy);
    return hrkan_mask_of_orders(ox, oy);
}

PdeParams pde_params(const hrkan_pde_desc *pde)
{
    PdeParams p{};
    p.kind = pde->kind;
    p.nu = pde->nu;
    p.alpha = pde->alpha;
    p.adv = pde->adv;
    if (pde->kind == HRKAN_LINEAR2D) {
        p.c0 = pde->c0;
        for (int k = 0; k < HRKAN_MAX_ORDER; ++k) {
            p.cx[k] = pde->cx[k];
            p.cy[k] = pde->cy[k];
        }
        linear_orders(pde, &p.ox, &p.oy);
    }
    return p;
}


}  // namespace hrk

using namespace hrk;

// ---------------------------------------------------------------------------
// forward / backward bodies (array type T)
// ---------------------------------------------------------------------------
namespace {

template <typename T>
int forward_impl(const NetInfo &ni, ChanCfg ch, const T *const *W, const T *x, int64_t n,
                 T *jets_out, T *saved, T *tmp0, T *tmp1, hipStream_t st, bool bc = false,
                 const char *wdn = nullptr)
{
    const GridP<T> g = make_grid<T>(ni);
    const int C = ch.C();
    const T *zin = x;
    int64_t soff = 0;
    for (int l = 0; l < ni.L; ++l) {
        T *zout;
        if (l == ni.L - 1)
            zout = jets_out;
        else if (saved) {
            zout = saved + soff;
            soff += (int64_t)C * ni.w[l + 1] * n;
        } else
            zout = (l % 2 == 0) ? tmp0 : tmp1;
        hipError_t e;
        {
            ProfScope ps("fwd", l, st, bc);
            const LayerShape ls{ni.w[l], ni.w[l + 1], ni.nb};
            if constexpr (std::is_same<T, float>::value) {
                if (use_dn(ni, l))
                    e = launch_fwd_dn(ch, zin, wdn + wdn_offset(ni, l), zout, n, ls, g, ni.S, st);
                else if (use_tc(ni, l, 'f'))
                    e = launch_fwd_tc(ch, l == 0, zin, W[l], zout, n, ls, make_tc_grid(ni.lo, ni.hi, ni.G, ni.k),
                                      cu_blocks(), st);
                else if (use_bs32(ni, l))
                    e = launch_fwd_bs32(ch, l == 0, zin, W[l], zout, n, ls, g, cu_blocks(), bf16_terms(ni), st);
                else
                    e = launch_fwd_generic<T>(ch, l == 0, zin, W[l], zout, n, ls, g, st);
            } else {
                e = launch_fwd_generic<T>(ch, l == 0, zin, W[l], zout, n, ls, g, st);
            }
        }
        if (e != hipSuccess) return hip_fail(e, "forward layer launch");
        zin = zout;
    }
    return HRKAN_OK;
}

// Input jets of layer l (x for l = 0, else a block of `saved`).
template <typename T>
const T *layer_input(const NetInfo &ni, int C, int l, const T *x, const T *saved, int64_t n)
{
    if (l == 0) return x;
    int64_t off = 0;
    for (int q = 1; q < l; ++q) off += (int64_t)C * ni.w[q] * n;
    return saved + off;
}

// Reverse pass of up to two point sets sharing W: set A (channels chA) and
// optionally set B (chB), each with its own seeds, saved jets and bar
// buffers. Their weight gradients are summed into gW (fixed order: all
// slices of A, then of B).
template <typename T>
struct RevSet {
    ChanCfg ch;
    const T *x;
    int64_t n;
    const T *seed;
    const T *saved;
    T *bar0, *bar1;
};

// Reverse pass of one point set: per layer (last to first) the weight-gradient
// slices into that layer's partial region at offset off[l], then the input
// bars of the layer below.
#define TRY(x)                          \
    do {                                \
        int rc_ = (x);                  \
        if (rc_ != HRKAN_OK) return rc_; \
    } while (0)

template <typename T>
int reverse_set(const NetInfo &ni, const T *const *W, const RevSet<T> &S, const int64_t *off, T *part,
                hipStream_t st, bool bc, const char *wdn)
{
    const GridP<T> g = make_grid<T>(ni);
    const T *ybar = S.seed;
    for (int l = ni.L - 1; l >= 0; --l) {
        const LayerShape ls{ni.w[l], ni.w[l + 1], ni.nb};
        const int ns = dw_splits(ni, l, S.n);
        const T *zin = layer_input<T>(ni, S.ch.C(), l, S.x, S.saved, S.n);
        hipError_t e;
        if constexpr (std::is_same<T, float>::value) {
            // a 1-output layer below which there are layers: its weight
            // gradient and input bars in one pass over its jets
            if (l > 0 && ls.wout == 1 && use_bs32(ni, l)) {
                T *zbar = (ybar == S.bar0) ? S.bar1 : S.bar0;
                {
                    ProfScope ps("dwx", l, st, bc);
                    e = launch_back_last(S.ch, zin, ybar, W[l], zbar, part + off[l], ns, S.n, ls, g, st);
                }
                if (e != hipSuccess) return hip_fail(e, "last-layer gradient launch");
                ybar = zbar;
                continue;
            }
        }
        {
            ProfScope ps("dw", l, st, bc);
            T *dst = part + off[l];
            if constexpr (std::is_same<T, float>::value) {
                if (use_dn(ni, l))
                    e = launch_dw_dn(S.ch, zin, ybar, dst, ns, S.n, ls, g, ni.S, st);
                else if (use_tc(ni, l, 'w'))
                    e = launch_dw_tc(S.ch, l == 0, zin, ybar, dst, ns, S.n, ls, make_tc_grid(ni.lo, ni.hi, ni.G, ni.k),
                                     st);
                else if (use_bs32(ni, l))
                    e = launch_dw_bs32(S.ch, l == 0, zin, ybar, dst, ns, S.n, ls, g, bf16_terms(ni), st);
                else
                    e = launch_dw_generic<T>(S.ch, l == 0, zin, ybar, dst, ns, S.n, ls, g, st);
            } else {
                e = launch_dw_generic<T>(S.ch, l == 0, zin, ybar, dst, ns, S.n, ls, g, st);
            }
        }
        if (e != hipSuccess) return hip_fail(e, "weight-gradient launch");
        if (l == 0) break;
        T *zbar = (ybar == S.bar0) ? S.bar1 : S.bar0;
        {
            ProfScope ps("dx", l, st, bc);
            if constexpr (std::is_same<T, float>::value) {
                if (use_dn(ni, l))
                    e = launch_dx_dn(S.ch, zin, ybar, wdn + wdn_offset(ni, l), zbar, S.n, ls, g, ni.S, st);
                else if (use_tc(ni, l, 'x'))
                    e = launch_dx_tc(S.ch, zin, ybar, W[l], zbar, S.n, ls, make_tc_grid(ni.lo, ni.hi, ni.G, ni.k),
                                     cu_blocks(), st);
                else if (use_bs32(ni, l))
                    e = launch_dx_bs32(S.ch, zin, ybar, W[l], zbar, S.n, ls, g, cu_blocks(), bf16_terms(ni), st);
                else
                    e = launch_dx_generic<T>(S.ch, zin, ybar, W[l], zbar, S.n, ls, g, st);
            } else {
                e = launch_dx_generic<T>(S.ch, zin, ybar, W[l], zbar, S.n, ls, g, st);
            }
        }
        if (e != hipSuccess) return hip_fail(e, "input-bar launch");
        ybar = zbar;
    }
    return HRKAN_OK;
}

// Loss partials to be summed by the gradient-reduction launch.
struct LossTail {
    const double *part;
    int nblk;
    double inv_int, inv_bc, alpha;
    double *out;
    uint32_t *status;
};

// Reverse pass of up to two point sets sharing W: set 0 on st, set 1 on st1
// (st itself, or the side stream of `fk`, which then starts from fk->fork as
// recorded by the caller and is joined back before the reduction). Layer l's
// partial region holds all slices of set 0, then all of set 1. Every layer is
// reduced in one launch at the end, each element summed over its slices in
// that fixed order; with `loss`, one more block of the same launch sums the
// loss partials.
template <typename T>
int reverse_impl(const NetInfo &ni, const T *const *W, const RevSet<T> *sets, int nsets,
                 T *const *gW, int accumulate, T *part, hipStream_t st, hipStream_t st1, Fork *fk,
                 const char *wdn, const LossTail *loss)
{
    const int64_t n0 = nsets > 0 ? sets[0].n : 0, n1 = nsets > 1 ? sets[1].n : 0;
    int64_t base[HRKAN_MAX_LAYERS], off0[HRKAN_MAX_LAYERS], off1[HRKAN_MAX_LAYERS];
    int tot[HRKAN_MAX_LAYERS];
    int64_t o = 0;
    for (int l = 0; l < ni.L; ++l) {
        const int64_t kn = (int64_t)ni.w[l] * ni.nb * ni.w[l + 1];
        const int s0 = dw_splits(ni, l, n0), s1 = dw_splits(ni, l, n1);
        base[l] = o;
        off0[l] = o;
        off1[l] = o + (int64_t)s0 * kn;
        tot[l] = s0 + s1;
        o += part_layer_elems(ni, l, n0, n1);
    }
    if (n0 > 0) TRY(reverse_set<T>(ni, W, sets[0], off0, part, st, false, wdn));
    if (st1 != st) {
        const hipError_t e = hipStreamWaitEvent(st1, fk->fork, 0);
        if (e != hipSuccess) return hip_fail(e, "stream wait");
    }
    if (n1 > 0) TRY(reverse_set<T>(ni, W, sets[1], off1, part, st1, true, wdn));
    if (st1 != st) TRY(join_from(fk, st));
    // a layer without slices gets zeros, or is left as it is when accumulating
    ReduceTable<T> tab{};
    tab.L = ni.L;
    for (int l = 0; l < ni.L; ++l) {
        tab.part[l] = part + base[l];
        tab.nsplit[l] = tot[l];
        tab.count[l] = (int64_t)ni.w[l] * ni.nb * ni.w[l + 1];
        tab.out[l] = gW[l];
    }
    if (loss) {
        tab.loss_part = loss->part;
        tab.loss_nblk = loss->nblk;
        tab.inv_int = loss->inv_int;
        tab.inv_bc = loss->inv_bc;
        tab.alpha = loss->alpha;
        tab.loss_out = loss->out;
        tab.status = loss->status;
    }
    hipError_t e;
    {
        ProfScope ps("reduce", -1, st);
        e = launch_reduce_layers<T>(tab, accumulate, st);
    }
    if (e != hipSuccess) return hip_fail(e, "gradient reduction launch");
    return HRKAN_OK;
}

int check_ws(void *ws, size_t ws_bytes, size_t need)
{
    if (!ws) return fail(HRKAN_ERR_INVALID_ARG, "ws is NULL");
    if (!aligned(ws, 256)) return fail(HRKAN_ERR_INVALID_ARG, "ws is not 256-byte aligned");
    if (ws_bytes < need)
        return fail(HRKAN_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    return HRKAN_OK;
}

int check_weights(const NetInfo &ni, const void *const *W, const char *what)
{
    if (!W) return fail(HRKAN_ERR_INVALID_ARG, "%s array is NULL", what);
    for (int l = 0; l < ni.L; ++l) {
        if (!W[l]) return fail(HRKAN_ERR_INVALID_ARG, "%s[%d] is NULL", what, l);
        if (!aligned(W[l], 16)) return fail(HRKAN_ERR_INVALID_ARG, "%s[%d] is not 16-byte aligned", what, l);
    }
    return HRKAN_OK;
}


}  // namespace

extern "C" {

int hrkan_version(void) { return 200; }

const char *hrkan_status_string(int code)
{
    switch (code) {
    case HRKAN_OK: return "ok";
    case HRKAN_ERR_INVALID_ARG: return "invalid argument";
    case HRKAN_ERR_UNSUPPORTED: return "unsupported configuration";
    case HRKAN_ERR_WORKSPACE: return "workspace too small";
    case HRKAN_ERR_DEVICE: return "HIP device error";
    case HRKAN_ERR_PLAN_MISMATCH: return "plan mismatch";
    case HRKAN_ERR_HOST_MEMORY: return "host memory exhausted";
    default: return "unknown status";
    }
}

const char *hrkan_last_error(void) { return g_err.c_str(); }

int hrkan_net_init(hrkan_net_desc *net)
{
    if (!net) return fail(HRKAN_ERR_INVALID_ARG, "net is NULL");
    std::memset(net, 0, sizeof *net);
    net->n_layers = 2;
    net->widths[0] = 2;
    net->widths[1] = 2;
    net->widths[2] = 1;
    net->G = 5;
    net->k = 3;
    net->m = 4;
    net->lo = -1.0;
    net->hi = 1.0;
    net->dtype = HRKAN_F32;
    net->bf16_split = 2;
    return HRKAN_OK;
}

int hrkan_pde_init(hrkan_pde_desc *pde, int32_t kind)
{
    if (!pde) return fail(HRKAN_ERR_INVALID_ARG, "pde is NULL");
    if (kind != HRKAN_POISSON2D && kind != HRKAN_BURGERS1D && kind != HRKAN_LINEAR2D)
        return fail(HRKAN_ERR_INVALID_ARG, "pde kind %d unknown", kind);
    std::memset(pde, 0, sizeof *pde);
    pde->kind = kind;
    pde->alpha = 0.05;
    pde->adv = 1.0;
    pde->nu = kind == HRKAN_BURGERS1D ? 0.01 / 3.14159265358979323846 : 0.0;
    return HRKAN_OK;
}

int hrkan_mask_channels(uint32_t channel_mask)
{
    ChanCfg ch;
    TRY(mask_cfg(channel_mask, &ch));
    return ch.C();
}

uint32_t hrkan_mask_of_orders(int32_t ox, int32_t oy)
{
    if (ox < 0 || oy < 0 || ox > HRKAN_MAX_ORDER || oy > HRKAN_MAX_ORDER) return 0u;
    uint32_t m = HRKAN_CH_U;
    for (int k = 0; k < ox; ++k) m |= XBITS[k];
    for (int k = 0; k < oy; ++k) m |= YBITS[k];
    return m;
}

int hrkan_saved_bytes(const hrkan_net_desc *net, int64_t n, uint32_t channel_mask, size_t *bytes)
{
    NetInfo ni;
    ChanCfg ch;
    TRY(check_net(net, &ni));
    TRY(mask_cfg(channel_mask, &ch));
    if (n < 0) return fail(HRKAN_ERR_INVALID_ARG, "n < 0");
    if (!bytes) return fail(HRKAN_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = ni.elem * (size_t)saved_elems(ni, ch.C(), n);
    return HRKAN_OK;
}

int hrkan_workspace_bytes(const hrkan_net_desc *net, const hrkan_pde_desc *pde, int64_t n_int,
                          int64_t n_bc, size_t *bytes)
{
    NetInfo ni;
    ChanCfg chi;
    TRY(check_net(net, &ni));
    TRY(check_pde(pde));
    TRY(mask_cfg(pde_mask(pde), &chi));
    TRY(apply_channels(&ni, chi));
    if (n_int < 0 || n_bc < 0) return fail(HRKAN_ERR_INVALID_ARG, "negative point count");
    if (!bytes) return fail(HRKAN_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = layout(ni, n_int, n_bc).total;
    return HRKAN_OK;
}

int hrkan_forward_jets(const hrkan_net_desc *net, const void *const *W, const void *x, int64_t n,
                       uint32_t channel_mask, void *jets_out, void *saved, void *ws, size_t ws_bytes,
                       hipStream_t stream)
{
    NetInfo ni;
    ChanCfg ch;
    TRY(check_net(net, &ni));
    TRY(mask_cfg(channel_mask, &ch));
    TRY(apply_channels(&ni, ch));
    if (n < 0) return fail(HRKAN_ERR_INVALID_ARG, "n < 0");
    TRY(check_weights(ni, W, "W"));
    if (n > 0 && (!x || !jets_out)) return fail(HRKAN_ERR_INVALID_ARG, "x or jets_out is NULL");
    if (x && !aligned(x, ni.elem)) return fail(HRKAN_ERR_INVALID_ARG, "x misaligned");
    const WsLayout L = layout(ni, n, 0);
    TRY(check_ws(ws, ws_bytes, L.total));
    if (n == 0) return HRKAN_OK;
    char *w = (char *)ws;
    if (ni.dtype == HRKAN_F64)
        return forward_impl<double>(ni, ch, (const double *const *)W, (const double *)x, n,
                                    (double *)jets_out, (double *)saved, (double *)(w + L.bars0),
                                    (double *)(w + L.bars1), stream);
    TRY(prep_dense(ni, (const float *const *)W, w + L.wdn, stream));
    return forward_impl<float>(ni, ch, (const float *const *)W, (const float *)x, n,
                               (float *)jets_out, (float *)saved, (float *)(w + L.bars0),
                               (float *)(w + L.bars1), stream, false, w + L.wdn);
}

int hrkan_residual(const hrkan_pde_desc *pde, int32_t dtype, const void *jets_int, const void *u_bc,
                   const hrkan_points *pts, void *r_out, double *loss_out, void *seed_int,
                   void *seed_bc, void *ws, size_t ws_bytes, hipStream_t stream)
{
    TRY(check_pde(pde));
    if (dtype != HRKAN_F64 && dtype != HRKAN_F32)
        return fail(HRKAN_ERR_INVALID_ARG, "residual dtype must be HRKAN_F64 or HRKAN_F32");
    if (!pts) return fail(HRKAN_ERR_INVALID_ARG, "pts is NULL");
    if (pts->n_int < 0 || pts->n_bc < 0) return fail(HRKAN_ERR_INVALID_ARG, "negative point count");
    if (pts->n_int > 0 && (!jets_int || !pts->x_int))
        return fail(HRKAN_ERR_INVALID_ARG, "jets_int or x_int is NULL");
    if (pts->n_bc > 0 && (!u_bc || !pts->g_bc)) return fail(HRKAN_ERR_INVALID_ARG, "u_bc or g_bc is NULL");
    if (!loss_out) return fail(HRKAN_ERR_INVALID_ARG, "loss_out is NULL");
    const int nblk = residual_blocks(pts->n_int, pts->n_bc);
    const size_t need = 256 + up256(sizeof(double) * 2 * nblk);
    TRY(check_ws(ws, ws_bytes, need));
    char *w = (char *)ws;
    double *partials = (double *)(w + 256);
    const PdeParams pp = pde_params(pde);
    const int C = hrkan_mask_channels(pde_mask(pde));
    hipError_t e;
    if (dtype == HRKAN_F64)
        e = launch_residual<double>(pp, C, (const double *)jets_int, (const double *)pts->x_int,
                                    pts->n_int, (const double *)u_bc, (const double *)pts->g_bc,
                                    pts->n_bc, (double *)r_out, (double *)seed_int,
                                    (double *)seed_bc, partials, nblk, stream);
    else
        e = launch_residual<float>(pp, C, (const float *)jets_int, (const float *)pts->x_int,
                                   pts->n_int, (const float *)u_bc, (const float *)pts->g_bc,
                                   pts->n_bc, (float *)r_out, (float *)seed_int, (float *)seed_bc,
                                   partials, nblk, stream);
    if (e != hipSuccess) return hip_fail(e, "residual launch");
    e = launch_loss_final(partials, nblk, pts->n_int, pts->n_bc, pde->alpha, loss_out,
                          (uint32_t *)w, stream);
    if (e != hipSuccess) return hip_fail(e, "loss launch");
    return HRKAN_OK;
}

int hrkan_backward(const hrkan_net_desc *net, const void *const *W, const void *x, int64_t n,
                   uint32_t channel_mask, const void *seed, const void *saved, void *const *gW_out,
                   int32_t accumulate, void *ws, size_t ws_bytes, hipStream_t stream)
{
    NetInfo ni;
    ChanCfg ch;
    TRY(check_net(net, &ni));
    TRY(mask_cfg(channel_mask, &ch));
    TRY(apply_channels(&ni, ch));
    if (n < 0) return fail(HRKAN_ERR_INVALID_ARG, "n < 0");
    TRY(check_weights(ni, W, "W"));
    TRY(check_weights(ni, (const void *const *)gW_out, "gW_out"));
    if (n > 0 && (!x || !seed)) return fail(HRKAN_ERR_INVALID_ARG, "x or seed is NULL");
    if (n > 0 && ni.L > 1 && !saved) return fail(HRKAN_ERR_INVALID_ARG, "saved is NULL");
    const WsLayout L = layout(ni, n, 0);
    TRY(check_ws(ws, ws_bytes, L.total));
    char *w = (char *)ws;
    if (ni.dtype == HRKAN_F64) {
        RevSet<double> s{ch, (const double *)x, n, (const double *)seed, (const double *)saved,
                         (double *)(w + L.bars0), (double *)(w + L.bars1)};
        return reverse_impl<double>(ni, (const double *const *)W, &s, 1, (double *const *)gW_out,
                                    accumulate, (double *)(w + L.part), stream, stream, nullptr, nullptr, nullptr);
    }
    RevSet<float> s{ch, (const float *)x, n, (const float *)seed, (const float *)saved,
                    (float *)(w + L.bars0), (float *)(w + L.bars1)};
    if (n > 0) TRY(prep_dense(ni, (const float *const *)W, w + L.wdn, stream));
    return reverse_impl<float>(ni, (const float *const *)W, &s, 1, (float *const *)gW_out, accumulate,
                               (float *)(w + L.part), stream, stream, nullptr, w + L.wdn, nullptr);
}

int hrkan_step(const hrkan_net_desc *net, const hrkan_pde_desc *pde, const void *const *W,
               const hrkan_points *pts, double *loss_out, void *const *gW_out, void *ws,
               size_t ws_bytes, hipStream_t stream)
{
    return step_impl(net, pde, W, pts, loss_out, gW_out, ws, ws_bytes, stream, true);
}

}  // extern "C"

namespace hrk {

int step_impl(const hrkan_net_desc *net, const hrkan_pde_desc *pde, const void *const *W,
              const hrkan_points *pts, double *loss_out, void *const *gW_out, void *ws,
              size_t ws_bytes, hipStream_t stream, bool allow_fork)
{
    NetInfo ni;
    ChanCfg chi, chb;
    TRY(check_net(net, &ni));
    TRY(check_pde(pde));
    TRY(mask_cfg(pde_mask(pde), &chi));
    TRY(mask_cfg(HRKAN_MASK_VALUE, &chb));
    TRY(apply_channels(&ni, chi));
    TRY(check_weights(ni, W, "W"));
    TRY(check_weights(ni, (const void *const *)gW_out, "gW_out"));
    if (!pts) return fail(HRKAN_ERR_INVALID_ARG, "pts is NULL");
    if (pts->n_int < 0 || pts->n_bc < 0) return fail(HRKAN_ERR_INVALID_ARG, "negative point count");
    if (pts->n_int > 0 && !pts->x_int) return fail(HRKAN_ERR_INVALID_ARG, "x_int is NULL");
    if (pts->n_bc > 0 && (!pts->x_bc || !pts->g_bc)) return fail(HRKAN_ERR_INVALID_ARG, "x_bc or g_bc is NULL");
    if (!loss_out) return fail(HRKAN_ERR_INVALID_ARG, "loss_out is NULL");
    for (const void *p : {pts->x_int, pts->x_bc, pts->g_bc})
        if (p && !aligned(p, ni.elem)) return fail(HRKAN_ERR_INVALID_ARG, "point array misaligned");
    size_t need = 0;
    TRY(hrkan_workspace_bytes(net, pde, pts->n_int, pts->n_bc, &need));
    TRY(check_ws(ws, ws_bytes, need));
    const WsLayout L = layout(ni, pts->n_int, pts->n_bc);
    char *w = (char *)ws;
    const int64_t ni_ = pts->n_int, nb_ = pts->n_bc;
    const PdeParams pp = pde_params(pde);

    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        T *sv_int = (T *)(w + L.sv_int), *jets = (T *)(w + L.jets_int);
        T *sv_bc = (T *)(w + L.sv_bc), *ubc = (T *)(w + L.ubc);
        T *seed_int = (T *)(w + L.seed_int), *seed_bc = (T *)(w + L.seed_bc);
        char *wdn = w + L.wdn;
        if constexpr (std::is_same<T, float>::value)
            if (ni_ + nb_ > 0) TRY(prep_dense(ni, (const float *const *)W, wdn, stream));
        double *partials = (double *)(w + L.loss_part);
        hipError_t e;
        if (L.merged) {
            // one set: interior points, then boundary points (merged_sets)
            const int64_t na = ni_ + nb_;
            T *xa = (T *)(w + L.xall);
            e = launch_concat_points<T>((const T *)pts->x_int, ni_, (const T *)pts->x_bc, nb_, xa, stream);
            if (e != hipSuccess) return hip_fail(e, "point concatenation launch");
            TRY(forward_impl<T>(ni, chi, (const T *const *)W, xa, na, jets, sv_int, nullptr, nullptr, stream,
                                false, wdn));
            const int rb = residual_blocks_of(na);
            {
                ProfScope ps("residual", -1, stream);
                e = launch_residual_merged<T>(pp, chi.C(), jets, (const T *)pts->x_int, ni_,
                                              (const T *)pts->g_bc, nb_, seed_int, partials, rb, stream);
            }
            if (e != hipSuccess) return hip_fail(e, "residual launch");
            const LossTail lt{partials, rb, 1.0 / (double)ni_, 1.0 / (double)nb_, pde->alpha, loss_out,
                              (uint32_t *)w};
            const RevSet<T> s{chi, xa, na, seed_int, sv_int, (T *)(w + L.bars0), (T *)(w + L.bars1)};
            return reverse_impl<T>(ni, (const T *const *)W, &s, 1, (T *const *)gW_out, 0, (T *)(w + L.part),
                                   stream, stream, nullptr, wdn, &lt);
        }
        // two sets: the boundary set on a side stream (overlap_sets; not while
        // per-launch profiling is on, whose events then time each launch
        // alone), forked before the forward pass and again after the
        // residual, joined after each pass. The interior set's launches are
        // enqueued first: it is the longer chain.
        const T *x_int = (const T *)pts->x_int, *x_bc = (const T *)pts->x_bc, *g_bc = (const T *)pts->g_bc;
        if constexpr (std::is_same<T, float>::value) {
            if (L.sorted) {
                float *xs = (float *)(w + L.xs_int), *xb = (float *)(w + L.xs_bc), *gb = (float *)(w + L.gs_bc);
                {
                    ProfScope ps("sort", -1, stream);
                    e = launch_sort_points(x_int, nullptr, ni_, w + L.sort_ws, xs, nullptr, stream);
                    if (e == hipSuccess) e = launch_sort_points(x_bc, g_bc, nb_, w + L.sort_ws, xb, gb, stream);
                }
                if (e != hipSuccess) return hip_fail(e, "point ordering launch");
                x_int = xs;
                x_bc = xb;
                g_bc = gb;
            }
        }
        Fork *fk = nullptr;
        if (allow_fork && overlap_sets(ni, ni_, nb_) && !prof_on()) TRY(get_fork(stream, &fk));
        hipStream_t sb = fk ? fk->side : stream;
        // no gradient needs the loss value: the gradient reduction's launch
        // sums it too
        const LossTail lt{partials,
                          L.nres,
                          ni_ > 0 ? 1.0 / (double)ni_ : 0.0,
                          nb_ > 0 ? 1.0 / (double)nb_ : 0.0,
                          pde->alpha,
                          loss_out,
                          (uint32_t *)w};
        RevSet<T> sets[2] = {
            {chi, x_int, ni_, seed_int, sv_int, (T *)(w + L.bars0), (T *)(w + L.bars1)},
            {chb, x_bc, nb_, seed_bc, sv_bc, (T *)(w + L.bbars0), (T *)(w + L.bbars1)},
        };
        if (fk) TRY(fork_to(fk, stream));
        if (ni_ > 0)
            TRY(forward_impl<T>(ni, chi, (const T *const *)W, x_int, ni_, jets, sv_int, nullptr, nullptr, stream,
                                false, wdn));
        if (nb_ > 0)
            TRY(forward_impl<T>(ni, chb, (const T *const *)W, x_bc, nb_, ubc, sv_bc, nullptr, nullptr, sb, true,
                                wdn));
        if (fk) TRY(join_from(fk, stream));
        {
            ProfScope ps("residual", -1, stream);
            e = launch_residual<T>(pp, chi.C(), jets, x_int, ni_, ubc, g_bc, nb_, nullptr, seed_int, seed_bc,
                                   partials, L.nres, stream);
        }
        if (e != hipSuccess) return hip_fail(e, "residual launch");
        if (fk) {
            if ((e = hipEventRecord(fk->fork, stream)) != hipSuccess) return hip_fail(e, "event record");
        }
        return reverse_impl<T>(ni, (const T *const *)W, sets, 2, (T *const *)gW_out, 0,
                               (T *)(w + L.part), stream, sb, fk, wdn, &lt);
    };
    if (ni.dtype == HRKAN_F64) return run(double{});
    return run(float{});
}

}  // namespace hrk

extern "C" {

int hrkan_adam(const hrkan_net_desc *net, void *const *W, const void *const *gW, void *const *m,
               void *const *v, int64_t *step_dev, double lr, double beta1, double beta2, double eps,
               hipStream_t stream)
{
    NetInfo ni;
    TRY(check_net(net, &ni));
    TRY(check_weights(ni, (const void *const *)W, "W"));
    TRY(check_weights(ni, gW, "gW"));
    TRY(check_weights(ni, (const void *const *)m, "m"));
    TRY(check_weights(ni, (const void *const *)v, "v"));
    if (!step_dev) return fail(HRKAN_ERR_INVALID_ARG, "step_dev is NULL");
    if (!aligned(step_dev, 8)) return fail(HRKAN_ERR_INVALID_ARG, "step_dev misaligned");
    if (!(lr >= 0.0) || !std::isfinite(lr)) return fail(HRKAN_ERR_INVALID_ARG, "lr must be finite and >= 0");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return fail(HRKAN_ERR_INVALID_ARG, "betas must lie in [0, 1)");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(HRKAN_ERR_INVALID_ARG, "eps must be finite and > 0");
    hipError_t e;
    auto run = [&](auto tag) {
        using T = decltype(tag);
        AdamTable<T> tab{};
        tab.L = ni.L;
        for (int l = 0; l < ni.L; ++l) {
            tab.W[l] = (T *)W[l];
            tab.g[l] = (const T *)gW[l];
            tab.m[l] = (T *)m[l];
            tab.v[l] = (T *)v[l];
            tab.count[l] = (int64_t)ni.w[l] * ni.nb * ni.w[l + 1];
        }
        return launch_adam<T>(tab, step_dev, lr, beta1, beta2, eps, stream);
    };
    e = ni.dtype == HRKAN_F64 ? run(double{}) : run(float{});
    if (e != hipSuccess) return hip_fail(e, "adam launch");
    return HRKAN_OK;
}

int hrkan_read_status(void *ws, size_t ws_bytes, hipStream_t stream, uint32_t *flags)
{
    if (!flags) return fail(HRKAN_ERR_INVALID_ARG, "flags is NULL");
    TRY(check_ws(ws, ws_bytes, 256));
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, ws, sizeof v, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemsetAsync(ws, 0, sizeof v, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "status read");
    *flags = v;
    return HRKAN_OK;
}

}  // extern "C"
