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
    float *pts;                  // [max_pts][3] points (extraction) or [max_pts][9] triangles (mesh)
    long long max_pts;
    unsigned long long *count;   // crossings / triangles found (may exceed max_pts)
    // sparse volume: block b is pool slot b at blocks[b].xyz; nbr[7 b + d]
    // the slot of its neighbour d = +x, +y, +z, +x+y, +x+z, +y+z, +x+y+z
    // (-1: none)
    const int4 *blocks;
    const int *nbr;
    int n_blocks;
};

constexpr int kNbrPerBlock = 7;

// Zeroes a device counter (a kernel, so that the call can be captured).
hipError_t launch_zero_count(unsigned long long *count, hipStream_t stream);
// Zero crossings of a fused volume (count zeroed first, then one launch).
hipError_t launch_sdf_extract(const SdfExtractArgs &a, bool hashed, hipStream_t stream);
// Level-set triangles of a fused volume (sdf_mesh.hip; count zeroed first).
hipError_t launch_sdf_mesh(const SdfExtractArgs &a, bool hashed, hipStream_t stream);

}  // namespace rir
