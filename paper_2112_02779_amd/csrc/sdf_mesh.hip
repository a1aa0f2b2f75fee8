// Level-set triangles of a fused SDF volume on gfx950 (Sec. 4.2 meshes the
// fused SDF with marching cubes; this is its tetrahedral form, consistent
// without the ambiguous cube cases), for the dense block grid and for the
// sparse volume's block list.
//
// One workgroup per block: the block's 16^3 voxels and the first planes,
// edges and corner of its +x, +y, +z neighbours (17^3 voxels) are staged in
// shared memory with independent loads (outside the volume or in a block
// that is not active: weight -inf, no triangle).  The cubes whose (0, 0, 0)
// voxel lies in the block and whose voxels lie on both sides of zero (the
// only ones with triangles) are compacted into a work list that the 256
// threads share out evenly; each cube is split into the six tetrahedra around
// its 000-111 diagonal, and each
// tetrahedron whose four voxels are observed (weight >= min_weight) and whose
// sign-changing edges step by at most max_jump gives one triangle (one
// vertex on its own side) or two (two and two), turned so that its normal
// points towards positive SDF; vertices by linear interpolation in FP64.
// The workgroup counts its triangles, takes one output range with one
// atomic add, and writes them (the order across blocks is not defined).
#include "sdf_extract.h"

namespace rir {

namespace {

constexpr int kM1 = kSdfEdge + 1;
// the second and third vertex of tetrahedron t: path 000 -> e_p -> e_p + e_q -> 111
constexpr int kTetP[6] = {0, 0, 1, 1, 2, 2};
constexpr int kTetQ[6] = {1, 2, 0, 2, 0, 1};

struct D3 {
    double x, y, z;
};

template <typename V>
__device__ __forceinline__ V sel4(int i, V v0, V v1, V v2, V v3)
{
    return i == 0 ? v0 : (i == 1 ? v1 : (i == 2 ? v2 : v3));
}

// Triangles (0, 1 or 2) of tetrahedron t (0..5; unrolled by the callers, so
// that its vertex offsets are constants) of the cube c whose (0, 0, 0) voxel
// is g (global voxel index).  With out != nullptr also writes them, 9 floats
// each, triangle k at out + 9 k if first + k < cap.  Everything stays in
// registers: vertex data is picked by index with selects.
__device__ __forceinline__ int tet_triangles(const SdfExtractArgs &a, const float2 (&c)[2][2][2], const int (&g)[3],
                                             int t, float *out, unsigned long long first, unsigned long long cap)
{
    const int P = kTetP[t], Q = kTetQ[t];
    const int o1[3] = {P == 0, P == 1, P == 2};
    const int o2[3] = {P == 0 || Q == 0, P == 1 || Q == 1, P == 2 || Q == 2};
    const float2 v0 = c[0][0][0], v1 = c[o1[2]][o1[1]][o1[0]], v2 = c[o2[2]][o2[1]][o2[0]], v3 = c[1][1][1];
    if (!(v0.y >= a.min_weight && v1.y >= a.min_weight && v2.y >= a.min_weight && v3.y >= a.min_weight))
        return 0;
    const bool b0 = v0.x > 0.f, b1 = v1.x > 0.f, b2 = v2.x > 0.f, b3 = v3.x > 0.f;
    const int np = (int)b0 + (int)b1 + (int)b2 + (int)b3;
    if (np == 0 || np == 4)
        return 0;
    auto jump = [&](bool ba, float sa, bool bb, float sb) {
        return ba != bb && fabs((double)sa - (double)sb) > a.max_jump;
    };
    if (jump(b0, v0.x, b1, v1.x) || jump(b0, v0.x, b2, v2.x) || jump(b0, v0.x, b3, v3.x) ||
        jump(b1, v1.x, b2, v2.x) || jump(b1, v1.x, b3, v3.x) || jump(b2, v2.x, b3, v3.x))
        return 0;
    const int ntri = np == 2 ? 2 : 1;
    if (!out)
        return ntri;
    // edges (vertex pairs) of the triangles: triangle k has (ea[k][w], eb[k][w])
    int ea0, eb0, ea1, eb1, ea2, eb2, fa1, fb1, fa2, fb2;  // second triangle: (ea0, eb0), (fa1, fb1), (fa2, fb2)
    if (np != 2) {
        const bool want = np == 1;  // the lone vertex is the positive one
        const int lone = b0 == want ? 0 : (b1 == want ? 1 : (b2 == want ? 2 : 3));
        ea0 = ea1 = ea2 = lone;
        eb0 = lone == 0 ? 1 : 0;
        eb1 = lone <= 1 ? 2 : 1;
        eb2 = lone <= 2 ? 3 : 2;
        fa1 = fb1 = fa2 = fb2 = 0;
    } else {
        // positive p0 < p1 and non-positive n0 < n1 (tetrahedron order)
        const int p0 = b0 ? 0 : (b1 ? 1 : 2);
        const int p1 = b3 ? 3 : (b2 ? 2 : 1);
        const int n0 = !b0 ? 0 : (!b1 ? 1 : 2);
        const int n1 = !b3 ? 3 : (!b2 ? 2 : 1);
        // quadrilateral p0n0, p0n1, p1n1, p1n0 as (0, 1, 2) and (0, 2, 3)
        ea0 = p0, eb0 = n0;
        ea1 = p0, eb1 = n1;
        ea2 = p1, eb2 = n1;
        fa1 = p1, fb1 = n1;
        fa2 = p1, fb2 = n0;
    }
    auto pos = [&](int q) -> D3 {
        const int dx = q == 3 ? 1 : (q == 1 ? o1[0] : (q == 2 ? o2[0] : 0));
        const int dy = q == 3 ? 1 : (q == 1 ? o1[1] : (q == 2 ? o2[1] : 0));
        const int dz = q == 3 ? 1 : (q == 1 ? o1[2] : (q == 2 ? o2[2] : 0));
        return {a.origin[0] + a.voxel * (double)(g[0] + dx), a.origin[1] + a.voxel * (double)(g[1] + dy),
                a.origin[2] + a.voxel * (double)(g[2] + dz)};
    };
    const D3 x0 = pos(0), x1 = pos(1), x2 = pos(2), x3 = pos(3);
    auto crossing = [&](int i0, int i1) -> D3 {
        const double sa = (double)sel4(i0, v0.x, v1.x, v2.x, v3.x), sb = (double)sel4(i1, v0.x, v1.x, v2.x, v3.x);
        const D3 xa = sel4(i0, x0, x1, x2, x3), xb = sel4(i1, x0, x1, x2, x3);
        const double tt = sa / (sa - sb);
        return {xa.x + tt * (xb.x - xa.x), xa.y + tt * (xb.y - xa.y), xa.z + tt * (xb.z - xa.z)};
    };
    // from the non-positive towards the positive vertices: mean against mean,
    // scaled by np (4 - np) > 0 (only the sign of its product with the
    // normal is used)
    const double wp = (double)(4 - np), wn = (double)np;
    const D3 gd = {wp * ((b0 ? x0.x : 0.0) + (b1 ? x1.x : 0.0) + (b2 ? x2.x : 0.0) + (b3 ? x3.x : 0.0)) -
                       wn * ((b0 ? 0.0 : x0.x) + (b1 ? 0.0 : x1.x) + (b2 ? 0.0 : x2.x) + (b3 ? 0.0 : x3.x)),
                   wp * ((b0 ? x0.y : 0.0) + (b1 ? x1.y : 0.0) + (b2 ? x2.y : 0.0) + (b3 ? x3.y : 0.0)) -
                       wn * ((b0 ? 0.0 : x0.y) + (b1 ? 0.0 : x1.y) + (b2 ? 0.0 : x2.y) + (b3 ? 0.0 : x3.y)),
                   wp * ((b0 ? x0.z : 0.0) + (b1 ? x1.z : 0.0) + (b2 ? x2.z : 0.0) + (b3 ? x3.z : 0.0)) -
                       wn * ((b0 ? 0.0 : x0.z) + (b1 ? 0.0 : x1.z) + (b2 ? 0.0 : x2.z) + (b3 ? 0.0 : x3.z))};
    auto emit = [&](int k, const D3 &p0, const D3 &p1, const D3 &p2) {
        if (first + (unsigned long long)k >= cap)
            return;
        const double u1x = p1.x - p0.x, u1y = p1.y - p0.y, u1z = p1.z - p0.z;
        const double u2x = p2.x - p0.x, u2y = p2.y - p0.y, u2z = p2.z - p0.z;
        const double nx = u1y * u2z - u1z * u2y, ny = u1z * u2x - u1x * u2z, nz = u1x * u2y - u1y * u2x;
        const bool flip = nx * gd.x + ny * gd.y + nz * gd.z < 0.0;
        const D3 q1 = flip ? p2 : p1, q2 = flip ? p1 : p2;
        float *o = out + 9 * k;
        o[0] = (float)p0.x, o[1] = (float)p0.y, o[2] = (float)p0.z;
        o[3] = (float)q1.x, o[4] = (float)q1.y, o[5] = (float)q1.z;
        o[6] = (float)q2.x, o[7] = (float)q2.y, o[8] = (float)q2.z;
    };
    const D3 c0 = crossing(ea0, eb0), c1 = crossing(ea1, eb1), c2 = crossing(ea2, eb2);
    emit(0, c0, c1, c2);
    if (ntri == 2)
        emit(1, c0, crossing(fa1, fb1), crossing(fa2, fb2));
    return ntri;
}

}  // namespace

template <bool HASHED>
__global__ __launch_bounds__(256) void k_sdf_mesh(const SdfExtractArgs a)
{
    __shared__ float2 s_v[kM1][kM1][kM1];  // [z][y][x]
    __shared__ int s_wsum[4];
    __shared__ uint16_t s_list[kSdfEdge * kSdfEdge * kSdfEdge];
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
    constexpr size_t kB = kSdfEdge * kSdfEdge * kSdfEdge;
    const float2 *vox = reinterpret_cast<const float2 *>(a.vox);
    const float2 none = make_float2(0.f, -INFINITY);
    const float4 *blk = reinterpret_cast<const float4 *>(vox + (size_t)b * kB);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int f = q * 256 + tid;  // voxels 2f, 2f + 1: same row
        const float4 w = blk[f];
        const int x = (2 * f) & 15, y = ((2 * f) >> 4) & 15, z = (2 * f) >> 8;
        s_v[z][y][x] = make_float2(w.x, w.y);
        s_v[z][y][x + 1] = make_float2(w.z, w.w);
    }
    // voxel (lx, ly, lz) of the staged region with some coordinate = 16: in
    // the +x / +y / +z neighbour (faces, edges, corner)
    auto far = [&](int lx, int ly, int lz) -> float2 {
        const int dx = lx >> 4, dy = ly >> 4, dz = lz >> 4;
        if constexpr (HASHED) {
            // neighbour order: +x, +y, +z, +x+y, +x+z, +y+z, +x+y+z
            const int dir = dx + dy + dz == 1 ? (dx ? 0 : (dy ? 1 : 2))
                                              : (dx + dy + dz == 3 ? 6 : (!dz ? 3 : (!dy ? 4 : 5)));
            const int slot = a.nbr[kNbrPerBlock * b + dir];
            if (slot < 0)
                return none;
            return vox[(size_t)slot * kB + (size_t)((((lz & 15) * kSdfEdge) + (ly & 15)) * kSdfEdge + (lx & 15))];
        } else {
            const int gi = bx * kSdfEdge + lx, gj = by * kSdfEdge + ly, gk = bz * kSdfEdge + lz;
            if (gi >= kSdfEdge * a.nbx || gj >= kSdfEdge * a.nby || gk >= kSdfEdge * a.nbz)
                return none;
            const size_t blkid = ((size_t)(gk >> 4) * a.nby + (gj >> 4)) * a.nbx + (gi >> 4);
            return vox[blkid * kB + (size_t)(((gk & 15) * kSdfEdge + (gj & 15)) * kSdfEdge + (gi & 15))];
        }
    };
    {
        const int u = tid & 15, w = tid >> 4;
        s_v[w][u][kSdfEdge] = far(kSdfEdge, u, w);
        s_v[w][kSdfEdge][u] = far(u, kSdfEdge, w);
        s_v[kSdfEdge][w][u] = far(u, w, kSdfEdge);
        if (tid < kSdfEdge) {
            s_v[tid][kSdfEdge][kSdfEdge] = far(kSdfEdge, kSdfEdge, tid);
            s_v[kSdfEdge][tid][kSdfEdge] = far(kSdfEdge, tid, kSdfEdge);
            s_v[kSdfEdge][kSdfEdge][tid] = far(tid, kSdfEdge, kSdfEdge);
        }
        if (tid == 0)
            s_v[kSdfEdge][kSdfEdge][kSdfEdge] = far(kSdfEdge, kSdfEdge, kSdfEdge);
    }
    __syncthreads();
    // the cubes with voxels on both sides of zero (the only ones with
    // triangles) as a work list in shared memory: thread (x, y) marks those of
    // its column, then the workgroup compacts them (cube index z << 8 | y << 4
    // | x, in thread order, then z)
    const int x = tid & 15, y = tid >> 4;
    uint32_t mask = 0;
    for (int z = 0; z < kSdfEdge; ++z) {
        int npos = 0;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx)
                    npos += s_v[z + dz][y + dy][x + dx].x > 0.f ? 1 : 0;
        if (npos != 0 && npos != 8)
            mask |= 1u << z;
    }
    const int nmine = __builtin_popcount(mask);
    if (!__syncthreads_or(nmine))
        return;  // no surface in this block (most of the volume)
    int n_cubes;
    const int first = block_scan256(s_wsum, nmine, n_cubes);
    for (int z = 0, k = first; z < kSdfEdge; ++z)
        if (mask & (1u << z))
            s_list[k++] = (uint16_t)((z << 8) | (y << 4) | x);
    __syncthreads();
    auto load_cube = [&](int id, float2 (&c)[2][2][2], int (&g)[3]) {
        const int cx = id & 15, cy = (id >> 4) & 15, cz = id >> 8;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx)
                    c[dz][dy][dx] = s_v[cz + dz][cy + dy][cx + dx];
        g[0] = bx * kSdfEdge + cx;
        g[1] = by * kSdfEdge + cy;
        g[2] = bz * kSdfEdge + cz;
    };
    // pass 1: triangles of this thread's cubes (list entries tid, tid + 256, ...)
    int cnt = 0;
    for (int i = tid; i < n_cubes; i += 256) {
        float2 c[2][2][2];
        int g[3];
        load_cube(s_list[i], c, g);
#pragma unroll
        for (int t = 0; t < 6; ++t)
            cnt += tet_triangles(a, c, g, t, nullptr, 0, 0);
    }
    int total;
    const int before = block_scan256(s_wsum, cnt, total);
    if (tid == 0)
        s_base = total > 0 ? atomicAdd(a.count, (unsigned long long)total) : 0ull;
    __syncthreads();
    if (cnt == 0)
        return;
    // pass 2: write them
    unsigned long long n = s_base + (unsigned long long)before;
    for (int i = tid; i < n_cubes; i += 256) {
        float2 c[2][2][2];
        int g[3];
        load_cube(s_list[i], c, g);
#pragma unroll
        for (int t = 0; t < 6; ++t)
            n += (unsigned long long)tet_triangles(a, c, g, t, a.max_pts > 0 ? a.pts + 9 * n : nullptr, n,
                                                   (unsigned long long)a.max_pts);
    }
}

hipError_t launch_sdf_mesh(const SdfExtractArgs &a, bool hashed, hipStream_t stream)
{
    hipError_t e = launch_zero_count(a.count, stream);
    if (e != hipSuccess)
        return e;
    if (hashed) {
        if (a.n_blocks > 0)
            hipLaunchKernelGGL(k_sdf_mesh<true>, dim3(a.n_blocks), dim3(256), 0, stream, a);
    } else {
        hipLaunchKernelGGL(k_sdf_mesh<false>, dim3(a.nbx * a.nby * a.nbz), dim3(256), 0, stream, a);
    }
    return hipGetLastError();
}

}  // namespace rir
