// kernels_dn.h -- launchers of the dense BF16 matrix-core kernels of hidden
// layers (k = 3, m = 4, BF16 products with S = 1..3 terms).
#pragma once

#include "internal.h"

namespace hrk {

// Hidden layers (not the network's input layer) with 32, 64 or 128 outputs
// and at most 24 basis functions per input.
bool dn_supported(LayerShape ls, bool first);

// Bytes of a layer's padded BF16 weight copies (written by launch_w_prep_dn,
// read by the forward and input-bar kernels; 256-byte alignment suffices).
size_t dn_w_bytes(LayerShape ls, int S);
hipError_t launch_w_prep_dn(const float *W, void *wdn, LayerShape ls, int S, hipStream_t st);

hipError_t launch_fwd_dn(ChanCfg ch, const float *zin, const void *wdn, float *zout, int64_t n, LayerShape ls,
                         const GridP<float> &g, int S, hipStream_t st);
hipError_t launch_dx_dn(ChanCfg ch, const float *zin, const float *ybar, const void *wdn, float *zbar,
                        int64_t n, LayerShape ls, const GridP<float> &g, int S, hipStream_t st);
// Partial weight gradients of nsplit point slices into part[nsplit][win*nb*N].
int dw_dn_splits(int64_t n, LayerShape ls);
hipError_t launch_dw_dn(ChanCfg ch, const float *zin, const float *ybar, float *part, int nsplit, int64_t n,
                        LayerShape ls, const GridP<float> &g, int S, hipStream_t st);

}  // namespace hrk
