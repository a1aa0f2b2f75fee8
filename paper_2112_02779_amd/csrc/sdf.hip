// Projective SDF fusion (Dong et al., Sec. 4.2, Eq. (8)-(10)) into a dense
// grid of 16^3-voxel blocks on gfx950.
//
// One workgroup of 256 threads owns one block: thread (x, y) walks the 16
// voxels (x, y, 0..15) of its column a few at a time, reading each voxel's
// state once and writing it once per launch whatever the number of scans
// fused into it (up to kSdfFrames).  Per scan and voxel: the sensor-frame position R x + t
// (three FMAs from per-block constants built in FP64), the projection of
// Eq. (3)-(4) at the finest level, one gather of the scan's range, the signed
// distance of Eq. (9) and the running mean of Eq. (10).  A block whose every
// voxel lies beyond the range clip plus the truncation band of a scan (plus
// the receiver radius) is not visited for that scan; a block no scan of the
// launch can reach is neither read nor written.
#include "rir_ops.h"

namespace rir {

namespace {

// Per-scan constants of one block in LDS: columns c0, c1, c2 of voxel * R and
// the sensor-frame position tb of the block's voxel (0, 0, 0), as 12 floats
// c0x c0y c0z c1x | c1y c1z c2x c2y | c2z tbx tby tbz (three 16-byte reads).
constexpr int kFrameWords = 16;
// Voxels of a column each thread processes together.
constexpr int kVox = 4;
// Consecutive blocks one XCD takes at a time.
constexpr int kSdfXcdRun = 8;

}  // namespace

template <bool R0, bool POW2, bool HASHED>
__global__ __launch_bounds__(256) void k_sdf_fuse(const SdfArgs a)
{
    __shared__ __align__(16) float s_fr[kSdfFrames][kFrameWords];
    __shared__ uint32_t s_mask;

    const int nblk = HASHED ? a.n_blocks : a.nbx * a.nby * a.nbz;
    int b = blockIdx.x;
    // XCD-aware order: workgroups go to the 8 XCDs round robin by id; give
    // each XCD runs of kSdfXcdRun consecutive blocks (neighbouring blocks read
    // neighbouring pixels, which then share that XCD's L2), the runs dealt to
    // the XCDs in turn, so that every XCD gets its share of the blocks the
    // scans reach (one contiguous slab per XCD would leave most XCDs idle:
    // the reachable blocks follow the sensor's path).  The grid is a
    // multiple of 8 runs; ids past the last block exit.
    if (a.xcd_remap) {
        const int j = b >> 3;
        b = (j / kSdfXcdRun) * (8 * kSdfXcdRun) + (b & 7) * kSdfXcdRun + j % kSdfXcdRun;
        if (b >= nblk)
            return;
    }
    int bx, by, bz, first = 0;
    if constexpr (HASHED) {
        const int *B = reinterpret_cast<const int *>(a.blocks + b);
        bx = cload(B);
        by = cload(B + 1);
        bz = cload(B + 2);
        first = cload(a.act + cload(B + 3)) - a.frame0;  // the launch's first scan that may update it
    } else {
        bx = b % a.nbx;
        const int byz = b / a.nbx;
        by = byz % a.nby;
        bz = byz / a.nby;
    }
    const int tid = threadIdx.x;

    if (tid < 64) {
        bool act = false;
        if (tid < a.n_frames && (!HASHED || tid >= first)) {
            const SdfFrame &F = a.f[tid];
            const double s = a.voxel;
            const double o[3] = {a.origin[0] + (double)(kSdfEdge * bx) * s, a.origin[1] + (double)(kSdfEdge * by) * s,
                                 a.origin[2] + (double)(kSdfEdge * bz) * s};
            double p[3];
            for (int i = 0; i < 3; ++i)
                p[i] = F.R[3 * i] * o[0] + F.R[3 * i + 1] * o[1] + F.R[3 * i + 2] * o[2] + F.t[i];
            float *dst = s_fr[tid];
            for (int k = 0; k < 3; ++k) {          // column k of s R
                dst[3 * k] = (float)(s * F.R[k]);
                dst[3 * k + 1] = (float)(s * F.R[3 + k]);
                dst[3 * k + 2] = (float)(s * F.R[6 + k]);
            }
            dst[9] = (float)p[0];
            dst[10] = (float)p[1];
            dst[11] = (float)p[2];
            if (a.cull > 0.0) {
                // distance from the sensor to the block centre, minus the
                // block's half diagonal
                const double h = 0.5 * (double)(kSdfEdge - 1) * s;
                double c2 = 0.0;
                for (int i = 0; i < 3; ++i) {
                    const double ci = p[i] + h * (F.R[3 * i] + F.R[3 * i + 1] + F.R[3 * i + 2]);
                    c2 += ci * ci;
                }
                act = sqrt(c2) - h * 1.7320508075688772 <= a.cull;
            } else {
                act = true;
            }
        }
        const uint64_t bal = __ballot(act);
        if (tid == 0)
            s_mask = (uint32_t)bal;
    }
    __syncthreads();
    const uint32_t mask = __builtin_amdgcn_readfirstlane(s_mask);
    if (mask == 0)
        return;

    const LevelView<float> V = level_view(a.tab, 0);
    const int H = V.Hl, W = V.Wl;
    const rsrc_t img = make_rsrc(a.ranges, (uint32_t)a.n_frames * (uint32_t)H * (uint32_t)W * 4u);
    const float x = (float)(tid & (kSdfEdge - 1)), y = (float)(tid >> 4);

    float2 *vb = reinterpret_cast<float2 *>(a.vox) + (size_t)b * (kSdfEdge * kSdfEdge * kSdfEdge) + tid;
    // Voxel-outer order: each thread walks its column kVox voxels at a time
    // (z, z + 16 / kVox, ...) and fuses every scan into them, so few voxel
    // states are live (few registers, many waves in flight) while the kVox
    // independent projection chains overlap their gathers.
    constexpr int kStep = kSdfEdge / kVox;
    for (int z0 = 0; z0 < kStep; ++z0) {
        float sd[kVox], wt[kVox];
        bool chg[kVox];
#pragma unroll
        for (int k = 0; k < kVox; ++k) {
            const float2 st = vb[(z0 + k * kStep) * kSdfEdge * kSdfEdge];
            sd[k] = st.x;
            wt[k] = st.y;
            chg[k] = false;
        }
        for (uint32_t m = mask; m != 0; m &= m - 1) {
            const int f = __builtin_ctz(m);
            const float4 *fr = reinterpret_cast<const float4 *>(s_fr[f]);
            const float4 q0 = fr[0], q1 = fr[1], q2 = fr[2];
            // tb + x c0 + y c1, then + z c2 per voxel
            const float px = fmaf(y, q0.w, fmaf(x, q0.x, q2.y));
            const float py = fmaf(y, q1.x, fmaf(x, q0.y, q2.z));
            const float pz = fmaf(y, q1.y, fmaf(x, q0.z, q2.w));
            const uint32_t fbase = (uint32_t)f * (uint32_t)H;
#pragma unroll
            for (int k = 0; k < kVox; ++k) {
                const float zf = (float)(z0 + k * kStep);
                const float xs = fmaf(zf, q1.z, px), ys = fmaf(zf, q1.w, py), zs = fmaf(zf, q2.x, pz);
                int u, v;
                float r;
                const bool ok = project<float, R0, POW2>(V, xs, ys, zs, u, v, r);
                // u, v are in range even when ok is false: the gather is unconditional
                const float om = bld1<float>(img, ((fbase + (uint32_t)v) * (uint32_t)W + (uint32_t)u) * 4u);
                float d = om - r;
                const bool use = ok && range_ok(om) && om <= a.clip && d >= -a.trunc;
                d = fminf(d, a.trunc);
                const float wn = wt[k] + 1.0f;
                const float sn = fmaf(d - sd[k], d_rcp(wn), sd[k]);
                sd[k] = use ? sn : sd[k];
                wt[k] = use ? wn : wt[k];
                chg[k] = chg[k] || use;
            }
        }
#pragma unroll
        for (int k = 0; k < kVox; ++k)
            if (chg[k])
                vb[(z0 + k * kStep) * kSdfEdge * kSdfEdge] = make_float2(sd[k], wt[k]);
    }
}

template <bool HASHED>
static void launch_sdf_fuse_h(const SdfArgs &a, bool r0, bool pow2, int nblk, hipStream_t stream)
{
    if (r0)
        hipLaunchKernelGGL((k_sdf_fuse<true, false, HASHED>), dim3(nblk), dim3(256), 0, stream, a);
    else if (pow2)
        hipLaunchKernelGGL((k_sdf_fuse<false, true, HASHED>), dim3(nblk), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL((k_sdf_fuse<false, false, HASHED>), dim3(nblk), dim3(256), 0, stream, a);
}

hipError_t launch_sdf_fuse(const SdfArgs &a, bool r0, bool pow2, bool hashed, hipStream_t stream)
{
    const int n = hashed ? a.n_blocks : a.nbx * a.nby * a.nbz, run = 8 * kSdfXcdRun;
    if (n <= 0)
        return hipSuccess;
    const int nblk = a.xcd_remap ? (n + run - 1) / run * run : n;
    if (hashed)
        launch_sdf_fuse_h<true>(a, r0, pow2, nblk, stream);
    else
        launch_sdf_fuse_h<false>(a, r0, pow2, nblk, stream);
    return hipGetLastError();
}

}  // namespace rir
