// Zero crossings of a fused SDF volume on gfx950 (Dong et al., Sec. 4.2: the
// level set that the paper meshes with marching cubes; here its vertices).
#include "sdf_extract.h"

namespace rir {

// Zero crossings of the fused SDF along the grid edges (the vertices of the
// level set that Sec. 4.2 meshes with marching cubes).  One workgroup per
// block: the block's 16^3 voxels and the first plane of its +x, +y and +z
// neighbour blocks are staged in shared memory with independent loads
// (outside the volume: weight -inf, no crossing); thread (x, y) then tests
// the +x, +y and +z edges of every voxel of its column.  A crossing needs both
// weights >= min_weight, SDF values on different sides of zero (s_a > 0 >=
// s_b or the reverse) and |s_a - s_b| <= max_jump; its point
// a + t (b - a), t = s_a / (s_a - s_b), is formed in FP64.  The workgroup
// counts its crossings (a block without any stops there), takes one range of
// the output with one atomic add, and writes its points there in thread
// order (so the order of the points across blocks is not defined).
__device__ __forceinline__ size_t vox_index(int nbx, int nby, int i, int j, int k)
{
    const size_t blk = ((size_t)(k >> 4) * nby + (j >> 4)) * nbx + (i >> 4);
    return blk * (kSdfEdge * kSdfEdge * kSdfEdge) + (size_t)(((k & 15) * kSdfEdge + (j & 15)) * kSdfEdge + (i & 15));
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

constexpr int kE1 = kSdfEdge + 1;  // staged edge: the block plus one plane

__device__ __forceinline__ bool crossing(const SdfExtractArgs &a, float2 A, float2 B)
{
    return B.y >= a.min_weight && (A.x > 0.f) != (B.x > 0.f) && !(fabs((double)A.x - (double)B.x) > a.max_jump);
}

template <bool HASHED>
__global__ __launch_bounds__(256) void k_sdf_extract(const SdfExtractArgs a)
{
    __shared__ float2 s_v[kE1][kE1][kE1];  // [z][y][x]
    __shared__ int s_wsum[4];
    __shared__ unsigned long long s_base;
    const int b = blockIdx.x;
    int bx, by, bz;
    if constexpr (HASHED) {
        const int4 B = a.blocks[b];
        bx = B.x;
        by = B.y;
        bz = B.z;
    } else {
        bx = b % a.nbx;
        const int byz = b / a.nbx;
        by = byz % a.nby;
        bz = byz / a.nby;
    }
    const int tid = threadIdx.x;
    const float2 *vox = reinterpret_cast<const float2 *>(a.vox);
    const float2 none = make_float2(0.f, -INFINITY);
    // the block: 4096 voxels, contiguous, two per 16-byte load
    const float4 *blk = reinterpret_cast<const float4 *>(vox + (size_t)b * (kSdfEdge * kSdfEdge * kSdfEdge));
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int f = q * 256 + tid;  // voxels 2f, 2f + 1: same row
        const float4 w = blk[f];
        const int x = (2 * f) & 15, y = ((2 * f) >> 4) & 15, z = (2 * f) >> 8;
        s_v[z][y][x] = make_float2(w.x, w.y);
        s_v[z][y][x + 1] = make_float2(w.z, w.w);
    }
    // first planes of the +x, +y and +z neighbour blocks
    {
        const int u = tid & 15, w = tid >> 4;
        const int i0 = bx * kSdfEdge, j0 = by * kSdfEdge, k0 = bz * kSdfEdge;
        float2 fx = none, fy = none, fz = none;
        if constexpr (HASHED) {
            // the neighbour's first plane: (0, u, w), (u, 0, w), (u, w, 0)
            constexpr size_t kB = kSdfEdge * kSdfEdge * kSdfEdge;
            const int nx = a.nbr[kNbrPerBlock * b], ny = a.nbr[kNbrPerBlock * b + 1],
                      nz = a.nbr[kNbrPerBlock * b + 2];
            if (nx >= 0)
                fx = vox[(size_t)nx * kB + (size_t)((w * kSdfEdge + u) * kSdfEdge)];
            if (ny >= 0)
                fy = vox[(size_t)ny * kB + (size_t)(w * kSdfEdge * kSdfEdge + u)];
            if (nz >= 0)
                fz = vox[(size_t)nz * kB + (size_t)(w * kSdfEdge + u)];
        } else {
            if (bx + 1 < a.nbx)
                fx = vox[vox_index(a.nbx, a.nby, i0 + kSdfEdge, j0 + u, k0 + w)];
            if (by + 1 < a.nby)
                fy = vox[vox_index(a.nbx, a.nby, i0 + u, j0 + kSdfEdge, k0 + w)];
            if (bz + 1 < a.nbz)
                fz = vox[vox_index(a.nbx, a.nby, i0 + u, j0 + w, k0 + kSdfEdge)];
        }
        s_v[w][u][kSdfEdge] = fx;
        s_v[w][kSdfEdge][u] = fy;
        s_v[kSdfEdge][w][u] = fz;
    }
    __syncthreads();
    const int x = tid & 15, y = tid >> 4;
    // pass 1: this thread's crossings
    int cnt = 0;
    for (int z = 0; z < kSdfEdge; ++z) {
        const float2 A = s_v[z][y][x];
        if (!(A.y >= a.min_weight))
            continue;
        cnt += crossing(a, A, s_v[z][y][x + 1]) ? 1 : 0;
        cnt += crossing(a, A, s_v[z][y + 1][x]) ? 1 : 0;
        cnt += crossing(a, A, s_v[z + 1][y][x]) ? 1 : 0;
    }
    // a block without crossings (most of the volume) ends here
    if (!__syncthreads_or(cnt))
        return;
    int total;
    const int before = block_scan256(s_wsum, cnt, total);
    if (tid == 0)
        s_base = atomicAdd(a.count, (unsigned long long)total);
    __syncthreads();
    if (cnt == 0)
        return;
    // pass 2: write the points
    unsigned long long n = s_base + (unsigned long long)before;
    const int i = bx * kSdfEdge + x, j = by * kSdfEdge + y;
    for (int z = 0; z < kSdfEdge; ++z) {
        const float2 A = s_v[z][y][x];
        if (!(A.y >= a.min_weight))
            continue;
        const int k = bz * kSdfEdge + z;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const float2 B = ax == 0 ? s_v[z][y][x + 1] : (ax == 1 ? s_v[z][y + 1][x] : s_v[z + 1][y][x]);
            if (!crossing(a, A, B))
                continue;
            const double t = (double)A.x / ((double)A.x - (double)B.x);
            if (n < (unsigned long long)a.max_pts) {
                a.pts[3 * n] = (float)(a.origin[0] + a.voxel * ((double)i + t * (ax == 0)));
                a.pts[3 * n + 1] = (float)(a.origin[1] + a.voxel * ((double)j + t * (ax == 1)));
                a.pts[3 * n + 2] = (float)(a.origin[2] + a.voxel * ((double)k + t * (ax == 2)));
            }
            ++n;
        }
    }
}

hipError_t launch_zero_count(unsigned long long *count, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, stream, count);
    return hipGetLastError();
}

hipError_t launch_sdf_extract(const SdfExtractArgs &a, bool hashed, hipStream_t stream)
{
    hipError_t e = launch_zero_count(a.count, stream);
    if (e != hipSuccess)
        return e;
    if (hashed) {
        if (a.n_blocks > 0)
            hipLaunchKernelGGL(k_sdf_extract<true>, dim3(a.n_blocks), dim3(256), 0, stream, a);
    } else {
        hipLaunchKernelGGL(k_sdf_extract<false>, dim3(a.nbx * a.nby * a.nbz), dim3(256), 0, stream, a);
    }
    return hipGetLastError();
}

}  // namespace rir
