// internal.h -- interface between the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hr_device.h"
#include "hrkan.h"

namespace hrk {

// Channel configuration of a call: orders of differentiation along x0, x1.
struct ChanCfg {
    int o0, o1;
    int C() const { return 1 + o0 + o1; }
};

// One layer's shapes.
struct LayerShape {
    int win, wout, nb;
};

// Many independent instances on one concatenated point axis (batched plans).
// Each instance's points start at a multiple of 256, so every 128-point
// group, 256-point block and tile belongs to one instance. Null tile_inst:
// a single instance.
struct BatchMap {
    const int *tile_inst = nullptr;   // instance of each 128-point group
    int64_t w_stride = 0;             // elements between consecutive instances' weights
    const int4 *slices = nullptr;     // weight-gradient slices {instance, p_begin, p_end, -}
};

// ---- generic kernels (any supported dtype as T = float / double) ----------
template <typename T>
hipError_t launch_fwd_generic(ChanCfg ch, bool first, const T *zin, const T *W, T *zout,
                              int64_t n, LayerShape ls, const GridP<T> &g, hipStream_t st);

template <typename T>
hipError_t launch_dx_generic(ChanCfg ch, const T *zin, const T *ybar, const T *W, T *zbar,
                             int64_t n, LayerShape ls, const GridP<T> &g, hipStream_t st);

// Partial weight gradients of `nsplit` point slices into part[nsplit][K*N].
template <typename T>
hipError_t launch_dw_generic(ChanCfg ch, bool first, const T *zin, const T *ybar, T *part,
                             int nsplit, int64_t n, LayerShape ls, const GridP<T> &g,
                             hipStream_t st);
int dw_generic_splits(int64_t n, LayerShape ls);
size_t dw_generic_lds_bytes(int elem, int C, int nb);


// gW[l][e] (+)= sum_s part_l[s][e] for every layer of a network in one
// launch, each element's slices summed in a fixed order in FP64 (blk0 is
// filled in by the launcher).
template <typename T>
struct ReduceTable {
    int L;
    const T *part[HRKAN_MAX_LAYERS];
    int nsplit[HRKAN_MAX_LAYERS];
    int64_t count[HRKAN_MAX_LAYERS];
    T *out[HRKAN_MAX_LAYERS];
    int64_t blk0[HRKAN_MAX_LAYERS + 1];
    // optional: one more block sums the loss partials as k_loss_final does
    const double *loss_part;     // [loss_nblk][2], or null
    int loss_nblk;
    double inv_int, inv_bc, alpha;
    double *loss_out;
    uint32_t *status;
};
template <typename T>
hipError_t launch_reduce_layers(ReduceTable<T> tab, int accumulate, hipStream_t st);

// Adam update of every layer in one launch, then the device step count
// advanced (blk0 filled in by the launcher).
template <typename T>
struct AdamTable {
    int L;
    T *W[HRKAN_MAX_LAYERS];
    const T *g[HRKAN_MAX_LAYERS];
    T *m[HRKAN_MAX_LAYERS];
    T *v[HRKAN_MAX_LAYERS];
    int64_t count[HRKAN_MAX_LAYERS];
    int64_t blk0[HRKAN_MAX_LAYERS + 1];
};
template <typename T>
hipError_t launch_adam(AdamTable<T> tab, int64_t *tdev, double lr, double b1, double b2, double eps,
                       hipStream_t st);

// Residual, seeds and per-block loss partials; then the final reduction.
struct PdeParams {
    int kind;
    double nu, alpha, adv;
    double c0, cx[HRKAN_MAX_ORDER], cy[HRKAN_MAX_ORDER];   // HRKAN_LINEAR2D
    int ox, oy;                                            // its jet orders
};
template <typename T>
hipError_t launch_residual(const PdeParams &pde, int C, const T *jets, const T *x_int,
                           int64_t n_int, const T *u_bc, const T *g_bc, int64_t n_bc, T *r_out,
                           T *seed_int, T *seed_bc, double *partials, int nblk, hipStream_t st);
// The interior and boundary sets as one set (training steps of small sets):
// points concatenated, and the residual with the boundary misfit on the value
// channel of rows n_int.. of [C][n_int + n_bc] jets and seeds.
template <typename T>
hipError_t launch_concat_points(const T *x_int, int64_t n_int, const T *x_bc, int64_t n_bc, T *out,
                                hipStream_t st);
template <typename T>
hipError_t launch_residual_merged(const PdeParams &pde, int C, const T *jets, const T *x_int, int64_t n_int,
                                  const T *g_bc, int64_t n_bc, T *seed, double *partials, int nblk,
                                  hipStream_t st);
int residual_blocks(int64_t n_int, int64_t n_bc);   // partial slots for both sets
int residual_blocks_of(int64_t n);                  // blocks of one set's residual launch
hipError_t launch_loss_final(const double *partials, int nblk, int64_t n_int, int64_t n_bc,
                             double alpha, double *loss_out, uint32_t *status, hipStream_t st);

}  // namespace hrk
