// kernels_generic_f64.hip -- the FP64 instances of the vector-ALU layer
// kernels (generic_layers.h): the forward with jets, the input bars and the
// weight gradient for every pair of jet orders.
#include "generic_layers.h"

namespace hrk {

template hipError_t launch_fwd_generic<double>(ChanCfg, bool, const double *, const double *, double *, int64_t,
                                               LayerShape, const GridP<double> &, hipStream_t);
template hipError_t launch_dx_generic<double>(ChanCfg, const double *, const double *, const double *, double *,
                                              int64_t, LayerShape, const GridP<double> &, hipStream_t);
template hipError_t launch_dw_generic<double>(ChanCfg, bool, const double *, const double *, double *, int,
                                              int64_t, LayerShape, const GridP<double> &, hipStream_t);

}  // namespace hrk
