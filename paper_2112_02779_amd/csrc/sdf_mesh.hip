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

struct Corner {
    float s, w;
    int d[3];  // offset in the cube
};

// Triangles (0, 1 or 2) of tetrahedron t of the cube whose (0, 0, 0) voxel is
// g (global voxel index); with out != nullptr also writes them, 9 floats each.
__device__ __forceinline__ int tet_triangles(const SdfExtractArgs &a, const float2 (&c)[2][2][2], const int (&g)[3],
                                             int t, float *out)
{
    Corner v[4];
    int off[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
    off[1][kTetP[t]] = 1;
    off[2][kTetP[t]] = 1;
    off[2][kTetQ[t]] = 1;
    int np = 0;
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float2 cv = c[off[q][2]][off[q][1]][off[q][0]];
        v[q].s = cv.x;
        v[q].w = cv.y;
        v[q].d[0] = off[q][0];
        v[q].d[1] = off[q][1];
        v[q].d[2] = off[q][2];
        ok = ok && cv.y >= a.min_weight;
        np += cv.x > 0.f ? 1 : 0;
    }
    if (!ok || np == 0 || np == 4)
        return 0;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = p + 1; q < 4; ++q)
            if ((v[p].s > 0.f) != (v[q].s > 0.f) && fabs((double)v[p].s - (double)v[q].s) > a.max_jump)
                return 0;
    // edges (vertex pairs) of the triangles
    int e[2][3][2];
    int ntri;
    if (np == 1 || np == 3) {
        int lone = 0;
        for (int q = 0; q < 4; ++q)
            if ((v[q].s > 0.f) == (np == 1))
                lone = q;
        int m = 0;
        for (int q = 0; q < 4; ++q)
            if (q != lone) {
                e[0][m][0] = lone;
                e[0][m][1] = q;
                ++m;
            }
        ntri = 1;
    } else {
        int P[2], N[2], mp = 0, mn = 0;
        for (int q = 0; q < 4; ++q) {
            if (v[q].s > 0.f)
                P[mp++] = q;
            else
                N[mn++] = q;
        }
        // quadrilateral P0N0, P0N1, P1N1, P1N0 as (0, 1, 2) and (0, 2, 3)
        e[0][0][0] = P[0], e[0][0][1] = N[0];
        e[0][1][0] = P[0], e[0][1][1] = N[1];
        e[0][2][0] = P[1], e[0][2][1] = N[1];
        e[1][0][0] = P[0], e[1][0][1] = N[0];
        e[1][1][0] = P[1], e[1][1][1] = N[1];
        e[1][2][0] = P[1], e[1][2][1] = N[0];
        ntri = 2;
    }
    if (!out)
        return ntri;
    double x[4][3];
    for (int q = 0; q < 4; ++q)
        for (int k = 0; k < 3; ++k)
            x[q][k] = a.origin[k] + a.voxel * (double)(g[k] + v[q].d[k]);
    // from the non-positive towards the positive vertices: mean against mean,
    // scaled by np (4 - np) > 0 (only the sign of its product with the
    // normal is used)
    double gdir[3];
    for (int k = 0; k < 3; ++k) {
        double sp = 0.0, sn = 0.0;
        for (int q = 0; q < 4; ++q) {
            if (v[q].s > 0.f)
                sp += x[q][k];
            else
                sn += x[q][k];
        }
        gdir[k] = (double)(4 - np) * sp - (double)np * sn;
    }
    for (int tr = 0; tr < ntri; ++tr) {
        double p[3][3];
        for (int w = 0; w < 3; ++w) {
            const int i0 = e[tr][w][0], i1 = e[tr][w][1];
            const double sa = (double)v[i0].s, sb = (double)v[i1].s;
            const double tt = sa / (sa - sb);
            for (int k = 0; k < 3; ++k)
                p[w][k] = x[i0][k] + tt * (x[i1][k] - x[i0][k]);
        }
        const double u1[3] = {p[1][0] - p[0][0], p[1][1] - p[0][1], p[1][2] - p[0][2]};
        const double u2[3] = {p[2][0] - p[0][0], p[2][1] - p[0][1], p[2][2] - p[0][2]};
        const double nn[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2],
                              u1[0] * u2[1] - u1[1] * u2[0]};
        const bool flip = nn[0] * gdir[0] + nn[1] * gdir[1] + nn[2] * gdir[2] < 0.0;
        float *o = out + 9 * tr;
        const int order[3] = {0, flip ? 2 : 1, flip ? 1 : 2};
        for (int w = 0; w < 3; ++w)
            for (int k = 0; k < 3; ++k)
                o[3 * w + k] = (float)p[order[w]][k];
    }
    return ntri;
}

// Exclusive prefix sum of v over the 256 threads of the workgroup
// (Hillis-Steele in shared memory); s_scan then holds the inclusive sums.
__device__ __forceinline__ int block_exclusive_scan(int *s_scan, int v)
{
    const int tid = threadIdx.x;
    __syncthreads();
    s_scan[tid] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int u = tid >= off ? s_scan[tid - off] : 0;
        __syncthreads();
        s_scan[tid] += u;
        __syncthreads();
    }
    return s_scan[tid] - v;
}

}  // namespace

template <bool HASHED>
__global__ __launch_bounds__(256) void k_sdf_mesh(const SdfExtractArgs a)
{
    __shared__ float2 s_v[kM1][kM1][kM1];  // [z][y][x]
    __shared__ int s_scan[256];
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
    const int first = block_exclusive_scan(s_scan, nmine);
    const int n_cubes = s_scan[255];  // inclusive total, left by the scan
    __syncthreads();
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
            cnt += tet_triangles(a, c, g, t, nullptr);
    }
    const int before = block_exclusive_scan(s_scan, cnt);
    if (tid == 255)
        s_base = s_scan[255] > 0 ? atomicAdd(a.count, (unsigned long long)s_scan[255]) : 0ull;
    __syncthreads();
    if (cnt == 0)
        return;
    // pass 2: write them
    unsigned long long n = s_base + (unsigned long long)before;
    for (int i = tid; i < n_cubes; i += 256) {
        float2 c[2][2][2];
        int g[3];
        load_cube(s_list[i], c, g);
        for (int t = 0; t < 6; ++t) {
            const int k = tet_triangles(a, c, g, t, nullptr);
            if (k == 0)
                continue;
            if (n + (unsigned long long)k <= (unsigned long long)a.max_pts) {
                tet_triangles(a, c, g, t, a.pts + 9 * n);
            } else if (n < (unsigned long long)a.max_pts) {
                float tmp[18];
                tet_triangles(a, c, g, t, tmp);
                for (int q = 0; q < 9; ++q)
                    a.pts[9 * n + q] = tmp[q];
            }
            n += (unsigned long long)k;
        }
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
