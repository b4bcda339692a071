// Work items of the gridder (shared by the plan builder and the (de)gridding kernels).
#pragma once

#include <cstdint>

namespace frmi {

// One work item of the gridder: the visibilities [start, start + count) of the
// sorted record arrays share a uv tile and a first w-plane.
struct WorkItem {
    int32_t tu, tv;   // tile origin in cells
    int32_t p0;       // first w-plane touched (0 when coplanar)
    int32_t chan;
    int64_t start;
    int32_t count;
    int32_t rows;     // gridding items: tile rows touched (halo included), first | last << 16
};

}  // namespace frmi
