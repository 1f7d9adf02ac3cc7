// sort.h -- reordering of a point set along a Z-order curve (sort.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hrk {

// Scratch bytes of launch_sort_points for n points.
size_t sort_ws_bytes(int64_t n);

// xs[p] = x[q(p)] (and gs[p] = g[q(p)] when g is not null) for the stable
// permutation q that orders the points [n][2] by the 16-bit Morton code of
// their coordinates quantised to 256 steps over the set's bounding box. The
// result depends only on the input. ws: sort_ws_bytes(n) bytes, 256-aligned.
hipError_t launch_sort_points(const float *x, const float *g, int64_t n, void *ws, float *xs, float *gs,
                              hipStream_t st);

}  // namespace hrk
