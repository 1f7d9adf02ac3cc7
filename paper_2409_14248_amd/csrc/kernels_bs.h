// kernels_bs.h -- launchers of the matrix-core layer kernels.
#pragma once

#include "internal.h"

namespace hrk {

// Matrix-core kernels for k = 3, m = 4: block-sparse MFMA for the forward,
// input-bar and weight-gradient contractions (one collocation point per
// 4x4 block), vector-ALU kernels for a one-output layer.
bool bs32_supported(LayerShape ls);
// S = 0: FP32 products; S = 1..3: BF16 products with S terms (hrkan.h,
// bf16_split), FP32 accumulation. BF16 covers the Poisson, Burgers and
// boundary-value channel sets.
hipError_t launch_fwd_bs32(ChanCfg ch, bool first, const float *zin, const float *W, float *zout,
                           int64_t n, LayerShape ls, const GridP<float> &g, int cu_blocks, int S,
                           hipStream_t st);
hipError_t launch_dx_bs32(ChanCfg ch, const float *zin, const float *ybar, const float *W, float *zbar,
                          int64_t n, LayerShape ls, const GridP<float> &g, int cu_blocks, int S,
                          hipStream_t st);
int dw_bs32_splits(int64_t n, LayerShape ls);
hipError_t launch_dw_bs32(ChanCfg ch, bool first, const float *zin, const float *ybar, float *part,
                          int nsplit, int64_t n, LayerShape ls, const GridP<float> &g, int S,
                          hipStream_t st);

}  // namespace hrk
