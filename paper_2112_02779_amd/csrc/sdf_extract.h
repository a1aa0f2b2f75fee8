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
    // sparse volume: block b is pool slot b at blocks[b].xyz; nbr[3 b + a]
    // the slot of its +x / +y / +z neighbour (a = 0, 1, 2; -1: none)
    const int4 *blocks;
    const int *nbr;
    int n_blocks;
};

// Zero crossings of a fused volume (count zeroed first, then one launch).
hipError_t launch_sdf_extract(const SdfExtractArgs &a, bool hashed, hipStream_t stream);

}  // namespace rir
