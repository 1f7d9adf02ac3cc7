// bf16_path.cpp -- BF16 matrix-core path (not yet available).
#include "runtime_internal.h"

namespace hrk {

size_t extra_ws_bytes(const NetInfo &, int64_t, int64_t) { return 0; }

int bf16_forward(const NetInfo &, ChanCfg, const void *const *, const float *, int64_t, float *,
                 float *, void *, size_t, hipStream_t)
{
    return fail(HRKAN_ERR_UNSUPPORTED, "HRKAN_BF16 is not available in this build");
}
int bf16_backward(const NetInfo &, ChanCfg, const void *const *, const float *, int64_t,
                  const float *, const float *, float *const *, int, void *, size_t, hipStream_t)
{
    return fail(HRKAN_ERR_UNSUPPORTED, "HRKAN_BF16 is not available in this build");
}
int bf16_step(const NetInfo &, const hrkan_pde_desc *, const void *const *, const hrkan_points *,
              double *, void *const *, void *, size_t, hipStream_t)
{
    return fail(HRKAN_ERR_UNSUPPORTED, "HRKAN_BF16 is not available in this build");
}

}  // namespace hrk
