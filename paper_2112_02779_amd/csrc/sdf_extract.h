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

// Exclusive prefix sum of v over a workgroup of 256 threads in thread order,
// and the workgroup's total: inclusive sums within each wavefront by lane
// exchanges, then the totals of the wavefronts before (s_wsum: 4 ints of
// shared memory; two barriers, all threads must call).
__device__ __forceinline__ int block_scan256(int *s_wsum, int v, int &total)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(inc, off, 64);
        inc += lane >= off ? u : 0;
    }
    __syncthreads();  // earlier readers of s_wsum are done
    if (lane == 63)
        s_wsum[wv] = inc;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int t = s_wsum[w];
        before += w < wv ? t : 0;
        total += t;
    }
    return before + inc - v;
}

// Zeroes a device counter (a kernel, so that the call can be captured).
hipError_t launch_zero_count(unsigned long long *count, hipStream_t stream);
// Zero crossings of a fused volume (count zeroed first, then one launch).
hipError_t launch_sdf_extract(const SdfExtractArgs &a, bool hashed, hipStream_t stream);
// Level-set triangles of a fused volume (sdf_mesh.hip; count zeroed first).
hipError_t launch_sdf_mesh(const SdfExtractArgs &a, bool hashed, hipStream_t stream);

}  // namespace rir
