// Zero crossings of a fused SDF volume on gfx950 (Dong et al., Sec. 4.2: the
// level set that the paper meshes with marching cubes; here its vertices).
#include "sdf_extract.h"

namespace rir {

// Zero crossings of the fused SDF along the grid edges (the vertices of the
// level set that Sec. 4.2 meshes with marching cubes).  One workgroup per
// block, thread (x, y) walks its column; each voxel tests its +x, +y and +z
// edges (the neighbour may sit in the next block).  A crossing needs both
// weights >= min_weight, SDF values on different sides of zero (s_a > 0 >= s_b
// or the reverse) and |s_a - s_b| <= max_jump; its point a + t (b - a),
// t = s_a / (s_a - s_b), is formed in FP64 and appended through an atomic
// counter (so the order of the points is not defined).
__device__ __forceinline__ size_t vox_index(int nbx, int nby, int i, int j, int k)
{
    const size_t blk = ((size_t)(k >> 4) * nby + (j >> 4)) * nbx + (i >> 4);
    return blk * (kSdfEdge * kSdfEdge * kSdfEdge) + (size_t)(((k & 15) * kSdfEdge + (j & 15)) * kSdfEdge + (i & 15));
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

__global__ __launch_bounds__(256) void k_sdf_extract(const SdfExtractArgs a)
{
    const int b = blockIdx.x;
    const int bx = b % a.nbx, byz = b / a.nbx;
    const int by = byz % a.nby, bz = byz / a.nby;
    const int tid = threadIdx.x;
    const int i = bx * kSdfEdge + (tid & 15), j = by * kSdfEdge + (tid >> 4);
    const int NX = a.nbx * kSdfEdge, NY = a.nby * kSdfEdge, NZ = a.nbz * kSdfEdge;
    const float2 *vox = reinterpret_cast<const float2 *>(a.vox);
    for (int kz = 0; kz < kSdfEdge; ++kz) {
        const int k = bz * kSdfEdge + kz;
        const float2 A = vox[vox_index(a.nbx, a.nby, i, j, k)];
        if (!(A.y >= a.min_weight))
            continue;
        for (int ax = 0; ax < 3; ++ax) {
            const int di = ax == 0, dj = ax == 1, dk = ax == 2;
            if (i + di >= NX || j + dj >= NY || k + dk >= NZ)
                continue;
            const float2 B = vox[vox_index(a.nbx, a.nby, i + di, j + dj, k + dk)];
            if (!(B.y >= a.min_weight) || (A.x > 0.f) == (B.x > 0.f) || fabs((double)A.x - (double)B.x) > a.max_jump)
                continue;
            const double t = (double)A.x / ((double)A.x - (double)B.x);
            const unsigned long long n = atomicAdd(a.count, 1ull);
            if (n < (unsigned long long)a.max_pts) {
                a.pts[3 * n] = (float)(a.origin[0] + a.voxel * ((double)i + t * di));
                a.pts[3 * n + 1] = (float)(a.origin[1] + a.voxel * ((double)j + t * dj));
                a.pts[3 * n + 2] = (float)(a.origin[2] + a.voxel * ((double)k + t * dk));
            }
        }
    }
}

hipError_t launch_sdf_extract(const SdfExtractArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, stream, a.count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sdf_extract, dim3(a.nbx * a.nby * a.nbz), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace rir
