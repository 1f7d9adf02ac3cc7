// batch.h -- device tables and launchers of the batched step (many
// independent instances of one network shape on one concatenated point axis).
#pragma once

#include <algorithm>

#include "internal.h"

namespace hrk {

// One instance, as the batched kernels read it (device memory).
struct BatchInst {
    const float *x_int, *x_bc, *g_bc;   // the caller's arrays ([n,2], [n,2], [n])
    int64_t off_int, n_int;             // interior points on the concatenated axis
    int64_t off_bc, n_bc;               // boundary points
    float nu, adv, sc_int, sc_bc;       // PDE coefficients; seed scales 2 alpha / n_int, 2 / n_bc
    double alpha;                       // loss weight of the residual term
    int blk_int, blk_bc;                // 256-point blocks of the padded ranges
    int sl_int0, nsl_int;               // weight-gradient slices of the interior set
    int sl_bc0, nsl_bc;                 // and of the boundary set
};

// Device view of a batched workspace.
struct BatchDev {
    const BatchInst *inst;
    const int *ginst_int, *ginst_bc;    // instance of each 128-point group
    int64_t n_int_tot, n_bc_tot;        // padded lengths of the two axes (multiples of 256)
    float *x_int, *x_bc, *g_bc;         // concatenated points and targets
};

hipError_t launch_gather(const BatchDev &b, hipStream_t st);
hipError_t launch_residual_batched(int kind, const BatchDev &b, const float *jets, const float *u_bc,
                                   float *seed_int, float *seed_bc, double *partials, hipStream_t st);
hipError_t launch_loss_batched(const BatchDev &b, int n_inst, const double *partials, double *loss_out,
                               uint32_t *status, hipStream_t st);
hipError_t launch_reduce_batched(const BatchDev &b, int n_inst, const float *part, int64_t count,
                                 int nsl_int, float *gW, int64_t w_stride, hipStream_t st);

}  // namespace hrk
