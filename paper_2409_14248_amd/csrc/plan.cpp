// plan.cpp -- batched persistent step (not yet available).
#include "runtime_internal.h"

using namespace hrk;

struct hrkan_plan {
    int dummy;
};

extern "C" {
int hrkan_plan_workspace_bytes(const hrkan_net_desc *, int32_t, const hrkan_points *, size_t *)
{
    return fail(HRKAN_ERR_UNSUPPORTED, "batched plans are not available in this build");
}
int hrkan_plan_create(hrkan_plan **, const hrkan_net_desc *, int32_t, const hrkan_pde_desc *,
                      const void *, const hrkan_points *, double *, void *, void *, size_t,
                      hipStream_t)
{
    return fail(HRKAN_ERR_UNSUPPORTED, "batched plans are not available in this build");
}
int hrkan_plan_execute(hrkan_plan *, hipStream_t)
{
    return fail(HRKAN_ERR_PLAN_MISMATCH, "no plan");
}
int hrkan_plan_config(const hrkan_plan *, int32_t *, int32_t *)
{
    return fail(HRKAN_ERR_PLAN_MISMATCH, "no plan");
}
void hrkan_plan_destroy(hrkan_plan *) {}
}
