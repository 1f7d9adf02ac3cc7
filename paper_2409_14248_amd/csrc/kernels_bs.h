// kernels_bs.h -- launchers of the matrix-core layer kernels.
#pragma once

#include "internal.h"

namespace hrk {

// Matrix-core kernels for k = 3, m = 4: block-sparse MFMA for the forward,
// input-bar and weight-gradient contractions (one collocation point per
// 4x4 block), vector-ALU kernels for a one-output layer.
// Layer shapes the matrix-core kernels take (first: the network's input layer).
bool bs32_supported(LayerShape ls, bool first);
// S = 0: FP32 products; S = 1..3: BF16 products with S terms (hrkan.h,
// bf16_split), FP32 accumulation. BF16 covers the Poisson, Burgers and
// boundary-value channel sets.
// With a BatchMap (batched plans) the point axis holds many instances: the
// forward and input-bar kernels take each tile's weights at
// W + instance * bm.w_stride, and the weight-gradient kernels take their
// point slices from bm.slices (nsplit of them). dw_ii_override (0 = automatic)
// picks the inputs per wave of the gradient kernel (tile tuning).
hipError_t launch_fwd_bs32(ChanCfg ch, bool first, const float *zin, const float *W, float *zout,
                           int64_t n, LayerShape ls, const GridP<float> &g, int cu_blocks, int S,
                           hipStream_t st, const BatchMap &bm = BatchMap{});
hipError_t launch_dx_bs32(ChanCfg ch, const float *zin, const float *ybar, const float *W, float *zbar,
                          int64_t n, LayerShape ls, const GridP<float> &g, int cu_blocks, int S,
                          hipStream_t st, const BatchMap &bm = BatchMap{});
int dw_bs32_splits(int64_t n, LayerShape ls);
// The weight-gradient slices of a 1-output layer (as launch_dw_bs32) and, in
// the same pass over its jets, its input bars (as launch_dx_bs32).
hipError_t launch_back_last(ChanCfg ch, const float *zin, const float *ybar, const float *W, float *zbar, float *part,
                            int nsplit, int64_t n, LayerShape ls, const GridP<float> &g, hipStream_t st,
                            const BatchMap &bm = BatchMap{});
hipError_t launch_dw_bs32(ChanCfg ch, bool first, const float *zin, const float *ybar, float *part,
                          int nsplit, int64_t n, LayerShape ls, const GridP<float> &g, int S,
                          hipStream_t st, const BatchMap &bm = BatchMap{}, int dw_ii_override = 0);

}  // namespace hrk
