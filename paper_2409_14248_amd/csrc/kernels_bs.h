// kernels_bs.h -- launchers of the matrix-core layer kernels.
#pragma once

#include "internal.h"

namespace hrk {

// FP32 kernels: block-sparse 4x4x1 MFMA for the forward and input-bar
// contractions, dense 32x32x2 MFMA for the weight gradient, vector-ALU
// kernels for a one-output layer.
bool bs32_supported(LayerShape ls);
hipError_t launch_fwd_bs32(ChanCfg ch, bool first, const float *zin, const float *W, float *zout,
                           int64_t n, LayerShape ls, const GridP<float> &g, int cu_blocks,
                           hipStream_t st);
hipError_t launch_dx_bs32(ChanCfg ch, const float *zin, const float *ybar, const float *W, float *zbar,
                          int64_t n, LayerShape ls, const GridP<float> &g, int cu_blocks,
                          hipStream_t st);
int dw_bs32_splits(int64_t n, LayerShape ls);
hipError_t launch_dw_bs32(ChanCfg ch, bool first, const float *zin, const float *ybar, float *part,
                          int nsplit, int64_t n, LayerShape ls, const GridP<float> &g, hipStream_t st);

}  // namespace hrk
