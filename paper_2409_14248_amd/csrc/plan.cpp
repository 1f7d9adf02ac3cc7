// plan.cpp -- batched step: many independent instances of one network shape,
// each with its own weights, PDE coefficients and point counts, laid out on
// one concatenated point axis (each instance padded to a multiple of 256
// points). Every stage is one launch over all instances (the forward and
// input-bar kernels persistent over the tiles of every instance, the
// weight-gradient kernel over every instance's point slices), and the whole
// step is captured once into a HIP graph, so an execute is one graph launch.
// An autotuner times candidate tile shapes (points per gradient slice,
// inputs per wave of the gradient kernel) on the caller's buffers first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "autotune.h"
#include "batch.h"
#include "kernels_bs.h"
#include "runtime_internal.h"

using namespace hrk;

namespace {

constexpr int PAD = 256;                        // instance alignment on the point axis
constexpr int SLICES[] = {1024, 2048, 4096};    // candidate points per gradient slice
constexpr int MIN_SLICE = 1024;
constexpr int DW_II[] = {0, 4};                 // candidate inputs per wave (0: automatic)

int64_t pad_to(int64_t n) { return (n + PAD - 1) / PAD * PAD; }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

struct PlanCfg {
    int slice_pts, dw_ii, blocks;
};

struct PlanLayout {
    size_t status, inst, ginst_int, ginst_bc, sl_int, sl_bc, x_int, x_bc, g_bc;
    size_t sv_int, jets, sv_bc, ubc, seed_int, seed_bc, bars0, bars1, bbars0, bbars1, partials, part;
    size_t total;
    int64_t n_int_tot, n_bc_tot;
    int64_t part_elems;
};

int64_t slices_of(int64_t n, int P) { return n > 0 ? cdiv(n, P) : 0; }

PlanLayout plan_layout(const NetInfo &ni, int n_inst, const hrkan_points *pts)
{
    PlanLayout L{};
    int64_t si = 0, sb = 0;
    for (int q = 0; q < n_inst; ++q) {
        L.n_int_tot += pad_to(pts[q].n_int);
        L.n_bc_tot += pad_to(pts[q].n_bc);
        si += slices_of(pts[q].n_int, MIN_SLICE);
        sb += slices_of(pts[q].n_bc, MIN_SLICE);
    }
    const int64_t ni_ = std::max<int64_t>(L.n_int_tot, 1), nb_ = std::max<int64_t>(L.n_bc_tot, 1);
    L.part_elems = 0;
    for (int l = 0; l < ni.L; ++l) L.part_elems += (si + sb) * (int64_t)ni.w[l] * ni.nb * ni.w[l + 1];
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += round256(bytes);
        return at;
    };
    L.status = take(256);
    L.inst = take(sizeof(BatchInst) * n_inst);
    L.ginst_int = take(sizeof(int) * (size_t)(ni_ / 128 + 1));
    L.ginst_bc = take(sizeof(int) * (size_t)(nb_ / 128 + 1));
    L.sl_int = take(sizeof(int4) * (size_t)std::max<int64_t>(si, 1));
    L.sl_bc = take(sizeof(int4) * (size_t)std::max<int64_t>(sb, 1));
    L.x_int = take(sizeof(float) * 2 * (size_t)ni_);
    L.x_bc = take(sizeof(float) * 2 * (size_t)nb_);
    L.g_bc = take(sizeof(float) * (size_t)nb_);
    L.sv_int = take(sizeof(float) * (size_t)saved_elems(ni, 5, ni_));
    L.jets = take(sizeof(float) * 5 * (size_t)ni_);
    L.sv_bc = take(sizeof(float) * (size_t)saved_elems(ni, 1, nb_));
    L.ubc = take(sizeof(float) * (size_t)nb_);
    L.seed_int = take(sizeof(float) * 5 * (size_t)ni_);
    L.seed_bc = take(sizeof(float) * (size_t)nb_);
    L.bars0 = take(sizeof(float) * 5 * (size_t)ni.maxw * ni_);
    L.bars1 = take(sizeof(float) * 5 * (size_t)ni.maxw * ni_);
    L.bbars0 = take(sizeof(float) * (size_t)ni.maxw * nb_);
    L.bbars1 = take(sizeof(float) * (size_t)ni.maxw * nb_);
    L.partials = take(sizeof(double) * (size_t)(ni_ / PAD + nb_ / PAD + 2));
    L.part = take(sizeof(float) * (size_t)std::max<int64_t>(L.part_elems, 1));
    L.total = o;
    return L;
}

int check_plan_net(const hrkan_net_desc *net, NetInfo *ni)
{
    int rc = check_net(net, ni);
    if (rc != HRKAN_OK) return rc;
    if (ni->dtype == HRKAN_F64) return fail(HRKAN_ERR_UNSUPPORTED, "batched plans run HRKAN_F32 or HRKAN_BF16");
    for (int l = 0; l < ni->L; ++l)
        if (!use_bs32(*ni, l))
            return fail(HRKAN_ERR_UNSUPPORTED, "batched plans need k = 3, m = 4 and matrix-core layer shapes");
    return HRKAN_OK;
}

int check_points(int n_inst, const hrkan_points *pts)
{
    if (n_inst < 1) return fail(HRKAN_ERR_INVALID_ARG, "n_inst=%d, must be >= 1", n_inst);
    if (!pts) return fail(HRKAN_ERR_INVALID_ARG, "pts is NULL");
    int64_t ti = 0, tb = 0;
    for (int q = 0; q < n_inst; ++q) {
        const hrkan_points &p = pts[q];
        if (p.n_int < 0 || p.n_bc < 0) return fail(HRKAN_ERR_INVALID_ARG, "instance %d: negative point count", q);
        ti += pad_to(p.n_int);
        tb += pad_to(p.n_bc);
    }
    // slice bounds and 128-point group indices are 32-bit on the device
    if (ti >= ((int64_t)1 << 31) || tb >= ((int64_t)1 << 31))
        return fail(HRKAN_ERR_UNSUPPORTED, "batched plans hold fewer than 2^31 points per set");
    return HRKAN_OK;
}

}  // namespace

struct hrkan_plan {
    NetInfo ni;
    int n_inst;
    int kind;
    ChanCfg chi, chb;
    std::vector<hrkan_points> pts;
    std::vector<hrkan_pde_desc> pdes;
    const float *W;
    float *gW;
    double *loss;
    char *ws;
    size_t ws_bytes;
    PlanLayout L;
    PlanCfg cfg;
    int nsl_int, nsl_bc;
    int64_t woff[HRKAN_MAX_LAYERS];
    int dev;
    bool from_cache;     // the configuration came from the autotune cache
    double tune_ms;      // its measured step time (ms)
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

// Host tables for one slice size, copied into the workspace.
int upload_tables(hrkan_plan *p, int P)
{
    const PlanLayout &L = p->L;
    std::vector<BatchInst> inst(p->n_inst);
    std::vector<int> gi((size_t)(L.n_int_tot / 128) + 1, 0), gb((size_t)(L.n_bc_tot / 128) + 1, 0);
    std::vector<int4> si, sb;
    int64_t oi = 0, ob = 0;
    for (int q = 0; q < p->n_inst; ++q) {
        const hrkan_points &pt = p->pts[q];
        const hrkan_pde_desc &pd = p->pdes[q];
        BatchInst &b = inst[q];
        b.x_int = (const float *)pt.x_int;
        b.x_bc = (const float *)pt.x_bc;
        b.g_bc = (const float *)pt.g_bc;
        b.off_int = oi;
        b.n_int = pt.n_int;
        b.off_bc = ob;
        b.n_bc = pt.n_bc;
        b.nu = (float)pd.nu;
        b.adv = (float)pd.adv;
        b.alpha = pd.alpha;
        b.sc_int = pt.n_int > 0 ? (float)(2.0 * pd.alpha / (double)pt.n_int) : 0.f;
        b.sc_bc = pt.n_bc > 0 ? (float)(2.0 / (double)pt.n_bc) : 0.f;
        const int64_t pi = pad_to(pt.n_int), pb = pad_to(pt.n_bc);
        b.blk_int = (int)(pi / PAD);
        b.blk_bc = (int)(pb / PAD);
        for (int64_t g = oi / 128; g < (oi + pi) / 128; ++g) gi[(size_t)g] = q;
        for (int64_t g = ob / 128; g < (ob + pb) / 128; ++g) gb[(size_t)g] = q;
        b.sl_int0 = (int)si.size();
        for (int64_t s = 0; s < pt.n_int; s += P)
            si.push_back(make_int4(q, (int)(oi + s), (int)(oi + std::min<int64_t>(s + P, pt.n_int)), 0));
        b.nsl_int = (int)si.size() - b.sl_int0;
        b.sl_bc0 = (int)sb.size();
        for (int64_t s = 0; s < pt.n_bc; s += P)
            sb.push_back(make_int4(q, (int)(ob + s), (int)(ob + std::min<int64_t>(s + P, pt.n_bc)), 0));
        b.nsl_bc = (int)sb.size() - b.sl_bc0;
        oi += pi;
        ob += pb;
    }
    p->nsl_int = (int)si.size();
    p->nsl_bc = (int)sb.size();
    hipError_t e = hipMemcpy(p->ws + L.inst, inst.data(), sizeof(BatchInst) * inst.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->ws + L.ginst_int, gi.data(), sizeof(int) * gi.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->ws + L.ginst_bc, gb.data(), sizeof(int) * gb.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !si.empty())
        e = hipMemcpy(p->ws + L.sl_int, si.data(), sizeof(int4) * si.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !sb.empty())
        e = hipMemcpy(p->ws + L.sl_bc, sb.data(), sizeof(int4) * sb.size(), hipMemcpyHostToDevice);
    return e == hipSuccess ? HRKAN_OK : hip_fail(e, "plan tables");
}

#define PTRY(x)                                  \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess) return hip_fail(e_, #x); \
    } while (0)

// Enqueue one batched step with configuration cfg (tables already uploaded).
int enqueue(const hrkan_plan *p, const PlanCfg &cfg, hipStream_t st)
{
    const NetInfo &ni = p->ni;
    const PlanLayout &L = p->L;
    char *w = p->ws;
    const GridP<float> g = make_grid<float>(ni);
    BatchDev b;
    b.inst = (const BatchInst *)(w + L.inst);
    b.ginst_int = (const int *)(w + L.ginst_int);
    b.ginst_bc = (const int *)(w + L.ginst_bc);
    b.n_int_tot = L.n_int_tot;
    b.n_bc_tot = L.n_bc_tot;
    b.x_int = (float *)(w + L.x_int);
    b.x_bc = (float *)(w + L.x_bc);
    b.g_bc = (float *)(w + L.g_bc);
    BatchMap bmi, bmb;
    bmi.tile_inst = b.ginst_int;
    bmi.w_stride = ni.n_params;
    bmi.slices = (const int4 *)(w + L.sl_int);
    bmb.tile_inst = b.ginst_bc;
    bmb.w_stride = ni.n_params;
    bmb.slices = (const int4 *)(w + L.sl_bc);
    float *sv_int = (float *)(w + L.sv_int), *jets = (float *)(w + L.jets);
    float *sv_bc = (float *)(w + L.sv_bc), *ubc = (float *)(w + L.ubc);
    float *seed_int = (float *)(w + L.seed_int), *seed_bc = (float *)(w + L.seed_bc);
    float *part = (float *)(w + L.part);

    PTRY(launch_gather(b, st));

    auto forward = [&](ChanCfg ch, const float *x, int64_t n, float *saved, float *out,
                       const BatchMap &bm) -> int {
        if (n <= 0) return HRKAN_OK;
        const float *zin = x;
        int64_t soff = 0;
        for (int l = 0; l < ni.L; ++l) {
            float *zout = (l == ni.L - 1) ? out : saved + soff;
            if (l < ni.L - 1) soff += (int64_t)ch.C() * ni.w[l + 1] * n;
            const LayerShape ls{ni.w[l], ni.w[l + 1], ni.nb};
            PTRY(launch_fwd_bs32(ch, l == 0, zin, p->W + p->woff[l], zout, n, ls, g, cfg.blocks, bf16_terms(ni), st,
                                 bm));
            zin = zout;
        }
        return HRKAN_OK;
    };
    int rc = forward(p->chi, b.x_int, L.n_int_tot, sv_int, jets, bmi);
    if (rc == HRKAN_OK) rc = forward(p->chb, b.x_bc, L.n_bc_tot, sv_bc, ubc, bmb);
    if (rc != HRKAN_OK) return rc;

    double *partials = (double *)(w + L.partials);
    PTRY(launch_residual_batched(p->kind, b, jets, ubc, seed_int, seed_bc, partials, st));
    PTRY(launch_loss_batched(b, p->n_inst, partials, p->loss, (uint32_t *)w, st));

    // layer l's slice region: interior slices, then boundary slices
    int64_t base[HRKAN_MAX_LAYERS], kn[HRKAN_MAX_LAYERS];
    int64_t o = 0;
    for (int l = 0; l < ni.L; ++l) {
        kn[l] = (int64_t)ni.w[l] * ni.nb * ni.w[l + 1];
        base[l] = o;
        o += (int64_t)(p->nsl_int + p->nsl_bc) * kn[l];
    }
    auto reverse = [&](ChanCfg ch, const float *x, int64_t n, const float *saved, const float *seed,
                       float *bar0, float *bar1, int nsl, int slot0, const BatchMap &bm) -> int {
        if (n <= 0 || nsl == 0) return HRKAN_OK;
        const float *ybar = seed;
        for (int l = ni.L - 1; l >= 0; --l) {
            const LayerShape ls{ni.w[l], ni.w[l + 1], ni.nb};
            int64_t off = 0;
            for (int q = 1; q < l; ++q) off += (int64_t)ch.C() * ni.w[q] * n;
            const float *zin = l == 0 ? x : saved + off;
            if (l > 0 && ls.wout == 1) {
                // the 1-output layer's weight gradient and input bars in one pass
                float *zbar = (ybar == bar0) ? bar1 : bar0;
                PTRY(launch_back_last(ch, zin, ybar, p->W + p->woff[l], zbar, part + base[l] + (int64_t)slot0 * kn[l], nsl,
                                      n, ls, g, st, bm));
                ybar = zbar;
                continue;
            }
            PTRY(launch_dw_bs32(ch, l == 0, zin, ybar, part + base[l] + (int64_t)slot0 * kn[l], nsl, n, ls, g, bf16_terms(ni),
                                st, bm, cfg.dw_ii));
            if (l == 0) break;
            float *zbar = (ybar == bar0) ? bar1 : bar0;
            PTRY(launch_dx_bs32(ch, zin, ybar, p->W + p->woff[l], zbar, n, ls, g, cfg.blocks, bf16_terms(ni), st, bm));
            ybar = zbar;
        }
        return HRKAN_OK;
    };
    rc = reverse(p->chi, b.x_int, L.n_int_tot, sv_int, seed_int, (float *)(w + L.bars0), (float *)(w + L.bars1),
                 p->nsl_int, 0, bmi);
    if (rc == HRKAN_OK)
        rc = reverse(p->chb, b.x_bc, L.n_bc_tot, sv_bc, seed_bc, (float *)(w + L.bbars0), (float *)(w + L.bbars1),
                     p->nsl_bc, p->nsl_int, bmb);
    if (rc != HRKAN_OK) return rc;
    for (int l = 0; l < ni.L; ++l)
        PTRY(launch_reduce_batched(b, p->n_inst, part + base[l], kn[l], p->nsl_int, p->gW + p->woff[l],
                                   ni.n_params, st));
    return HRKAN_OK;
}

// Average time of `reps` enqueues of cfg (after one untimed), in ms. The two
// events are released on every path.
int time_cfg(hrkan_plan *p, const PlanCfg &cfg, hipStream_t st, int reps, float *ms)
{
    int rc = enqueue(p, cfg, st);
    if (rc != HRKAN_OK) return rc;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = hipEventRecord(ev[0], st);
    for (int r = 0; r < reps && e == hipSuccess && rc == HRKAN_OK; ++r) rc = enqueue(p, cfg, st);
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, ev[0], ev[1]);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(e, "plan timing events");
    *ms /= reps;
    return rc;
}

void release(hrkan_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
}

}  // namespace

extern "C" {

int hrkan_plan_workspace_bytes(const hrkan_net_desc *net, int32_t n_inst, const hrkan_points *pts, size_t *bytes)
{
    NetInfo ni;
    int rc = check_plan_net(net, &ni);
    if (rc != HRKAN_OK) return rc;
    rc = check_points(n_inst, pts);
    if (rc != HRKAN_OK) return rc;
    if (!bytes) return fail(HRKAN_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = plan_layout(ni, n_inst, pts).total;
    return HRKAN_OK;
}

static int plan_build(hrkan_plan *p, const NetInfo &ni, int32_t n_inst, const hrkan_pde_desc *pdes,
                      const void *W_packed, const hrkan_points *pts, double *loss_out, void *gW_packed, void *ws,
                      size_t ws_bytes, const PlanLayout &L, hipStream_t stream);

static int plan_create(hrkan_plan **out, const hrkan_net_desc *net, int32_t n_inst, const hrkan_pde_desc *pdes,
                       const void *W_packed, const hrkan_points *pts, double *loss_out, void *gW_packed, void *ws,
                       size_t ws_bytes, hipStream_t stream)
{
    if (!out) return fail(HRKAN_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    NetInfo ni;
    int rc = check_plan_net(net, &ni);
    if (rc != HRKAN_OK) return rc;
    rc = check_points(n_inst, pts);
    if (rc != HRKAN_OK) return rc;
    if (!pdes) return fail(HRKAN_ERR_INVALID_ARG, "pdes is NULL");
    for (int q = 0; q < n_inst; ++q) {
        rc = check_pde(&pdes[q]);
        if (rc != HRKAN_OK) return rc;
        if (pdes[q].kind != HRKAN_BURGERS1D && pdes[q].kind != HRKAN_POISSON2D)
            return fail(HRKAN_ERR_UNSUPPORTED, "instance %d: a plan takes Burgers or Poisson instances", q);
        if (pdes[q].kind != pdes[0].kind) return fail(HRKAN_ERR_INVALID_ARG, "instance %d: another PDE kind", q);
        const hrkan_points &p = pts[q];
        if ((p.n_int > 0 && !p.x_int) || (p.n_bc > 0 && (!p.x_bc || !p.g_bc)))
            return fail(HRKAN_ERR_INVALID_ARG, "instance %d: point array is NULL", q);
        for (const void *a : {p.x_int, p.x_bc})
            if (a && ((uintptr_t)a % 8)) return fail(HRKAN_ERR_INVALID_ARG, "instance %d: points not 8-byte aligned", q);
        if (p.g_bc && ((uintptr_t)p.g_bc % 4)) return fail(HRKAN_ERR_INVALID_ARG, "instance %d: g_bc misaligned", q);
    }
    if (!W_packed || !gW_packed || !loss_out) return fail(HRKAN_ERR_INVALID_ARG, "W_packed, gW_packed or loss_out is NULL");
    // every instance's layer arrays must be 16-byte aligned
    if ((uintptr_t)W_packed % 16 || (uintptr_t)gW_packed % 16)
        return fail(HRKAN_ERR_INVALID_ARG, "W_packed and gW_packed must be 16-byte aligned");
    int64_t o = 0;
    for (int l = 0; l < ni.L; ++l) {
        if (o % 4) return fail(HRKAN_ERR_UNSUPPORTED, "layer %d starts at a non-multiple of 4 floats", l);
        o += (int64_t)ni.w[l] * ni.nb * ni.w[l + 1];
    }
    if (ni.n_params % 4) return fail(HRKAN_ERR_UNSUPPORTED, "parameters per instance not a multiple of 4");
    const PlanLayout L = plan_layout(ni, n_inst, pts);
    if (!ws || (uintptr_t)ws % 256) return fail(HRKAN_ERR_INVALID_ARG, "ws is NULL or not 256-byte aligned");
    if (ws_bytes < L.total) return fail(HRKAN_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);

    hrkan_plan *p = new hrkan_plan();
    p->graph = nullptr;
    p->exec = nullptr;
    try {
        rc = plan_build(p, ni, n_inst, pdes, W_packed, pts, loss_out, gW_packed, ws, ws_bytes, L, stream);
    } catch (...) {
        release(p);
        throw;
    }
    if (rc != HRKAN_OK) {
        release(p);
        return rc;
    }
    *out = p;
    return HRKAN_OK;
}

// Fill a new plan: tables, autotuned configuration, captured graph.
static int plan_build(hrkan_plan *p, const NetInfo &ni, int32_t n_inst, const hrkan_pde_desc *pdes,
                      const void *W_packed, const hrkan_points *pts, double *loss_out, void *gW_packed, void *ws,
                      size_t ws_bytes, const PlanLayout &L, hipStream_t stream)
{
    int rc = HRKAN_OK;
    p->ni = ni;
    p->n_inst = n_inst;
    p->kind = pdes[0].kind;
    rc = mask_cfg(pde_mask(&pdes[0]), &p->chi);
    if (rc == HRKAN_OK) rc = mask_cfg(HRKAN_MASK_VALUE, &p->chb);
    p->pts.assign(pts, pts + n_inst);
    p->pdes.assign(pdes, pdes + n_inst);
    p->W = (const float *)W_packed;
    p->gW = (float *)gW_packed;
    p->loss = loss_out;
    p->ws = (char *)ws;
    p->ws_bytes = ws_bytes;
    p->L = L;
    int64_t o = 0;
    for (int l = 0; l < ni.L; ++l) {
        p->woff[l] = o;
        o += (int64_t)ni.w[l] * ni.nb * ni.w[l + 1];
    }
    if (rc == HRKAN_OK && hipGetDevice(&p->dev) != hipSuccess) rc = fail(HRKAN_ERR_DEVICE, "hipGetDevice");

    // autotune: the cached choice for this kind of batch (device
    // architecture, network, dtype, PDE kind, instance and point counts in
    // powers of two), else every candidate timed on the caller's buffers and
    // the winner stored in the cache
    PlanCfg best{SLICES[0], 0, cu_blocks()};
    float best_ms = INFINITY;
    char arch[256] = "";
    hipDeviceProp_t prop;
    if (rc == HRKAN_OK && hipGetDeviceProperties(&prop, p->dev) == hipSuccess)
        snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    int64_t total = 0;
    for (int q = 0; q < n_inst; ++q) total += pts[q].n_int;
    const std::string path = tune_cache_path();
    const std::string key = tune_key(arch, ni, p->kind, n_inst, total);
    TunedCfg tc{};
    p->from_cache = rc == HRKAN_OK && tune_lookup(path, key, &tc) &&
                    std::find(std::begin(SLICES), std::end(SLICES), tc.slice_pts) != std::end(SLICES) &&
                    std::find(std::begin(DW_II), std::end(DW_II), tc.dw_ii) != std::end(DW_II);
    if (p->from_cache) {
        best = PlanCfg{tc.slice_pts, tc.dw_ii, cu_blocks()};
        best_ms = (float)tc.ms;
    } else {
        for (int P : SLICES) {
            if (rc != HRKAN_OK) break;
            rc = upload_tables(p, P);
            for (int ii : DW_II) {
                if (rc != HRKAN_OK) break;
                const PlanCfg c{P, ii, cu_blocks()};
                float ms = 0.f;
                rc = time_cfg(p, c, stream, 2, &ms);
                if (rc == HRKAN_OK && ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        }
        if (rc == HRKAN_OK) tune_store(path, key, TunedCfg{best.slice_pts, best.dw_ii, (double)best_ms});
    }
    if (rc == HRKAN_OK) rc = upload_tables(p, best.slice_pts);
    p->cfg = best;
    p->tune_ms = best_ms;
    // capture one step into a graph, on a private stream (the caller's may be
    // the null stream, which cannot be captured); nothing runs during capture
    if (rc == HRKAN_OK) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
        hipStream_t cs = nullptr;
        if (rc == HRKAN_OK && (e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
            rc = hip_fail(e, "capture stream");
        if (rc == HRKAN_OK) {
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) rc = hip_fail(e, "hipStreamBeginCapture");
            if (rc == HRKAN_OK) {
                const int erc = enqueue(p, best, cs);
                e = hipStreamEndCapture(cs, &p->graph);
                if (erc != HRKAN_OK) rc = erc;
                else if (e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
            }
            if (rc == HRKAN_OK) {
                e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
            }
        }
        if (cs) (void)hipStreamDestroy(cs);
    }
    return rc;
}

int hrkan_plan_create(hrkan_plan **out, const hrkan_net_desc *net, int32_t n_inst, const hrkan_pde_desc *pdes,
                      const void *W_packed, const hrkan_points *pts, double *loss_out, void *gW_packed, void *ws,
                      size_t ws_bytes, hipStream_t stream)
{
    try {
        return plan_create(out, net, n_inst, pdes, W_packed, pts, loss_out, gW_packed, ws, ws_bytes, stream);
    } catch (const std::bad_alloc &) {
        if (out) *out = nullptr;
        return fail(HRKAN_ERR_HOST_MEMORY, "host memory exhausted while building the plan");
    }
}

int hrkan_plan_execute(hrkan_plan *plan, hipStream_t stream)
{
    if (!plan || !plan->exec) return fail(HRKAN_ERR_PLAN_MISMATCH, "plan is NULL or not built");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->dev)
        return fail(HRKAN_ERR_PLAN_MISMATCH, "plan built on device %d, current device %d", plan->dev, dev);
    const hipError_t e = hipGraphLaunch(plan->exec, stream);
    return e == hipSuccess ? HRKAN_OK : hip_fail(e, "hipGraphLaunch");
}

int hrkan_plan_config(const hrkan_plan *plan, int32_t *tile_points, int32_t *blocks)
{
    if (!plan) return fail(HRKAN_ERR_PLAN_MISMATCH, "plan is NULL");
    if (tile_points) *tile_points = plan->cfg.slice_pts;
    if (blocks) *blocks = plan->cfg.blocks;
    return HRKAN_OK;
}

int hrkan_plan_autotune_info(const hrkan_plan *plan, int32_t *from_cache, double *step_ms)
{
    if (!plan) return fail(HRKAN_ERR_PLAN_MISMATCH, "plan is NULL");
    if (from_cache) *from_cache = plan->from_cache ? 1 : 0;
    if (step_ms) *step_ms = plan->tune_ms;
    return HRKAN_OK;
}

void hrkan_plan_destroy(hrkan_plan *plan) { release(plan); }

}  // extern "C"
