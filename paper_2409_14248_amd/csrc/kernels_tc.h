// kernels_tc.h -- launchers of the tile-coherent FP32 hidden-layer kernels
// (kernels_tc.hip): 16-point tiles, K axis = the union of the tile's basis
// windows per input, 16x16x4 FP32 MFMA.
#pragma once

#include "internal.h"

namespace hrk {

// Grid of the tile-coherent kernels: the knots of every basis row in FP64
// (s_b, e_b), the grid start and the support scale 2 / ((k+1) h) in FP32
// (window selection) and FP64 (basis).
struct TcGrid {
    int nb;
    float lo, inv_w;
    double inv_w_d;
    double s[32], e[32];
};
TcGrid make_tc_grid(double lo, double hi, int G, int k);

// Layer shapes and channel sets the kernels take: k = 3, m = 4, n_b <= 32,
// 32 / 64 / 128 outputs, inputs a multiple of 16 (hidden layers) or the two
// coordinates (first layer); every channel set of hrkan_mask_channels.
bool tc_supported(ChanCfg ch, LayerShape ls, int k, int m, bool first);

// zout[c][j][p] = sum_{i, b} A_c(p, i, b) W[i nb + b][j] (zin [C][win][n]
// for a hidden layer, the points [n][2] for the first, W [win nb][wout],
// zout [C][wout][n]).
hipError_t launch_fwd_tc(ChanCfg ch, bool first, const float *zin, const float *W, float *zout, int64_t n,
                         LayerShape ls, const TcGrid &gr, int cu_blocks, hipStream_t st);

// zbar[c][i][p] = d(sum over the layer's outputs of ybar . zout)/d(zin[c][i][p])
// for a hidden layer (zin [C][win][n] its saved input jets, ybar [C][wout][n]
// the bars of its outputs); hidden layers of tc_supported.
hipError_t launch_dx_tc(ChanCfg ch, const float *zin, const float *ybar, const float *W, float *zbar, int64_t n,
                        LayerShape ls, const TcGrid &gr, int cu_blocks, hipStream_t st);

// Partial weight gradients of a hidden layer over `nsplit` point slices:
// part[s][K * wout] (K = win * nb), slice s the points
// [s * P, min(n, (s + 1) * P)) with P = ceil(n / nsplit) rounded up to 16.
int dw_tc_splits(int64_t n, LayerShape ls);
size_t dw_tc_lds_bytes(int nb);
hipError_t launch_dw_tc(ChanCfg ch, bool first, const float *zin, const float *ybar, float *part, int nsplit,
                        int64_t n, LayerShape ls, const TcGrid &gr, hipStream_t st);

}  // namespace hrk
