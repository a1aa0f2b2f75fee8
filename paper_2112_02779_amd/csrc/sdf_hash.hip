// Sparse voxel-block volume of Sec. 4.2 on gfx950: the 16^3-voxel blocks near
// the returns of each scan are activated in an open-addressing hash table
// keyed by block coordinates, and only activated blocks are fused (the
// fusion and extraction kernels of sdf.hip / sdf_extract.hip, run over the
// table's block list).
//
// Activation: one thread per return.  The return is unprojected in FP64
// (Eq. (1)) and moved to the world frame, x = R^T (x_s - t); every block whose
// cell o + [E b, E (b + 1)) (o: the volume origin) meets the cube
// [x - radius, x + radius] is looked up
// and, if absent, inserted (64-bit compare-and-swap on the key, then a slot of
// the block pool from a counter).  Each table entry keeps the first scan that
// activated it (atomic minimum), so that fusion can apply a scan only to the
// blocks that scan or an earlier one activated, as if every scan were
// activated and then fused in turn.  Neighbouring lanes mostly produce the
// same cube: a lane whose scan and block range equal those of the lane below
// it leaves the inserts to that lane.
#include "sdf_extract.h"
#include "sdf_hash.h"

namespace rir {

__device__ __forceinline__ uint64_t bvol_key(int bx, int by, int bz)
{
    return ((uint64_t)(uint32_t)(bx + kBvolBias) << 42) | ((uint64_t)(uint32_t)(by + kBvolBias) << 21) |
           (uint64_t)(uint32_t)(bz + kBvolBias);
}

// SplitMix64 finaliser (Steele, Lea and Flood, 2014): a bijective 64-bit mix.
__device__ __forceinline__ uint32_t bvol_hash(uint64_t k)
{
    k = (k ^ (k >> 30)) * 0xbf58476d1ce4e5b9ull;
    k = (k ^ (k >> 27)) * 0x94d049bb133111ebull;
    return (uint32_t)(k ^ (k >> 31));
}

__device__ __forceinline__ bool bvol_in_range(int b) { return b > -kBvolBias && b < kBvolBias; }

// Finds or inserts block (bx, by, bz) and lowers its entry's first scan to
// `frame`.  Once the pool is full no key is added (the call then fails and
// the volume must be reset), so the table stays below about half full and
// every probe sequence ends at a free entry.
__device__ __forceinline__ void bvol_insert(const BvolDev &t, int bx, int by, int bz, int frame)
{
    const unsigned long long key = bvol_key(bx, by, bz);
    uint32_t h = bvol_hash(key) & t.mask;
    for (uint32_t probe = 0; probe <= t.mask; ++probe) {
        unsigned long long k = __hip_atomic_load(t.keys + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == kBvolEmpty) {
            if (__hip_atomic_load(t.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= t.max_blocks) {
                atomicOr(t.flags, kBvolFull);
                return;
            }
            k = atomicCAS(t.keys + h, kBvolEmpty, key);
            if (k == kBvolEmpty) {
                const int slot = atomicAdd(t.count, 1);
                if (slot < t.max_blocks) {
                    t.blocks[slot] = make_int4(bx, by, bz, (int)h);
                    t.vals[h] = slot;
                } else {
                    atomicOr(t.flags, kBvolFull);
                }
                atomicMin(t.act + h, frame);
                return;
            }
        }
        if (k == key) {
            if (__hip_atomic_load(t.act + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > frame)
                atomicMin(t.act + h, frame);
            return;
        }
        h = (h + 1) & t.mask;
    }
    atomicOr(t.flags, kBvolFull);
}

__device__ __forceinline__ int bvol_find(const BvolDev &t, int bx, int by, int bz)
{
    if (!bvol_in_range(bx) || !bvol_in_range(by) || !bvol_in_range(bz))
        return -1;
    const unsigned long long key = bvol_key(bx, by, bz);
    uint32_t h = bvol_hash(key) & t.mask;
    for (uint32_t probe = 0; probe <= t.mask; ++probe) {
        const unsigned long long k = t.keys[h];
        if (k == key)
            return t.vals[h];
        if (k == kBvolEmpty)
            return -1;
        h = (h + 1) & t.mask;
    }
    return -1;
}

__global__ __launch_bounds__(256) void k_bvol_activate(const BvolActArgs a)
{
    const int H = cload(&a.tab->H), W = cload(&a.tab->W);
    const double *row = cload(&a.tab->row), *col = cload(&a.tab->col);
    const double r0 = cload(&a.tab->r0);
    const int64_t hw = (int64_t)H * W, n = hw * a.n_frames;
    const int lane = threadIdx.x & 63;
    // whole wavefronts step together (the lane comparison below needs them)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        const int64_t i = base + lane;
        int f = 0, lo[3] = {0, 0, 0}, hi[3] = {-1, -1, -1};
        bool on = false;
        if (i < n) {
            f = (int)(i / hw);
            const int p = (int)(i - (int64_t)f * hw), v = p / W, u = p - v * W;
            const float rf = a.ranges[i];
            on = range_ok(rf) && !(a.clip > 0.0 && (double)rf > a.clip);
            if (on) {
                const V3<double> xs = unproject(row, col, r0, u, v, (double)rf);
                const SdfFrame &F = a.f[f];
                const double d[3] = {xs.x - F.t[0], xs.y - F.t[1], xs.z - F.t[2]};
                for (int j = 0; j < 3; ++j) {
                    const double x = F.R[j] * d[0] + F.R[3 + j] * d[1] + F.R[6 + j] * d[2] - a.origin[j];
                    const double l = floor((x - a.radius) / a.edge), h = floor((x + a.radius) / a.edge);
                    if (!(l > (double)-kBvolBias && h < (double)kBvolBias)) {
                        on = false;  // outside the table's coordinate range
                        break;
                    }
                    lo[j] = (int)l;
                    hi[j] = (int)h;
                }
                if (!on)
                    atomicOr(a.t.flags, kBvolRange);
            }
        }
        // the lane below with the same scan and block range inserts for both
        const int pf = __shfl_up(f, 1), pl0 = __shfl_up(lo[0], 1), pl1 = __shfl_up(lo[1], 1),
                  pl2 = __shfl_up(lo[2], 1), ph0 = __shfl_up(hi[0], 1), ph1 = __shfl_up(hi[1], 1),
                  ph2 = __shfl_up(hi[2], 1);
        const bool pon = __shfl_up(on ? 1 : 0, 1) != 0;
        const bool same = lane > 0 && pon && pf == f && pl0 == lo[0] && pl1 == lo[1] && pl2 == lo[2] &&
                          ph0 == hi[0] && ph1 == hi[1] && ph2 == hi[2];
        if (!on || same)
            continue;
        const int frame = a.frame0 + f;
        for (int bz = lo[2]; bz <= hi[2]; ++bz)
            for (int by = lo[1]; by <= hi[1]; ++by)
                for (int bx = lo[0]; bx <= hi[0]; ++bx)
                    bvol_insert(a.t, bx, by, bz, frame);
    }
}

// Slots of the +x, +y, +z, +x+y, +x+z, +y+z and +x+y+z neighbours of every
// block (-1: not active).
__global__ __launch_bounds__(256) void k_bvol_neighbors(const BvolDev t, int n_blocks, int *nbr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNbrPerBlock * n_blocks)
        return;
    const int b = i / kNbrPerBlock, d = i - kNbrPerBlock * b;
    constexpr int kDx[kNbrPerBlock] = {1, 0, 0, 1, 1, 0, 1}, kDy[kNbrPerBlock] = {0, 1, 0, 1, 0, 1, 1},
                  kDz[kNbrPerBlock] = {0, 0, 1, 0, 1, 1, 1};
    const int4 B = t.blocks[b];
    nbr[i] = bvol_find(t, B.x + kDx[d], B.y + kDy[d], B.z + kDz[d]);
}

// Block coordinates and activation scans of the pool, in slot order.
__global__ __launch_bounds__(256) void k_bvol_export(const BvolDev t, int n_blocks, int4 *out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_blocks)
        return;
    const int4 B = t.blocks[b];
    out[b] = make_int4(B.x, B.y, B.z, t.act[B.w]);
}

hipError_t launch_bvol_activate(const BvolActArgs &a, hipStream_t stream)
{
    const int64_t n = (int64_t)a.n_frames * a.H * a.W;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_bvol_activate, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_bvol_neighbors(const BvolDev &t, int n_blocks, int *nbr, hipStream_t stream)
{
    if (n_blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_bvol_neighbors, dim3((kNbrPerBlock * n_blocks + 255) / 256), dim3(256), 0, stream, t,
                       n_blocks, nbr);
    return hipGetLastError();
}

hipError_t launch_bvol_export(const BvolDev &t, int n_blocks, int4 *out, hipStream_t stream)
{
    if (n_blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_bvol_export, dim3((n_blocks + 255) / 256), dim3(256), 0, stream, t, n_blocks, out);
    return hipGetLastError();
}

}  // namespace rir
