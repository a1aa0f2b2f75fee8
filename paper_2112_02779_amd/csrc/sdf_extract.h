// Surface extraction from a fused SDF volume (sdf_extract.hip): the zero
// crossings along the grid edges of the dense block grid of rir_ops.h.
#pragma once

#include "rir_ops.h"

namespace rir {

struct SdfExtractArgs {
    const float *vox;            // (sdf, weight) per voxel, block layout of SdfArgs
    int nbx, nby, nbz;
    float min_weight;
    double max_jump;
    double origin[3], voxel;
    float *pts;                  // [max_pts][3]
    long long max_pts;
    unsigned long long *count;   // crossings found (may exceed max_pts)
};

// Zero crossings of a fused volume (count zeroed first, then one launch).
hipError_t launch_sdf_extract(const SdfExtractArgs &a, hipStream_t stream);

}  // namespace rir
