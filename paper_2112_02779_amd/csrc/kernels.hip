// Kernels of the range-image ICP hot path on gfx950 (Dong et al., Sec. 3-4.1):
//  - geometry entry points (unproject, project, normals);
//  - the prepass: target normal image (cross product of neighbour
//    differences) written at level 0 as (n, n . q) records and subsampled
//    into the strided pyramid levels together with the source and target
//    ranges (Sec. 4.1);
//  - the Gauss-Newton step: per source pixel unprojection, rigid transform,
//    projection, projective association, residual, Jacobian and robust weight
//    (Eq. (5)-(7)), accumulated in registers, reduced across the wavefront by
//    recursive halving and across waves through LDS into one partial record
//    per tile;
//  - the solve: per pair, the tile records summed in FP64 in a fixed order,
//    the 6x6 system solved by Cholesky and the SE(3) update applied.
// No floating-point atomics: results are bitwise reproducible for a fixed
// tuning.
#include <float.h>

#include "rir_internal.h"
#include "rir_mlp_device.h"

namespace rir {

// ----------------------------------------------------------------------------- helpers

// Tile sequence of this workgroup.  With xcd_remap the tile list is cut into 8
// contiguous chunks, one per XCD (workgroups are dealt to the 8 XCDs round
// robin by workgroup id), so neighbouring tiles of a pair share an L2.
struct TileIter {
    int cur, step, end;
};
__device__ __forceinline__ TileIter tile_iter(int n_tiles, int xcd_remap)
{
    const int G = gridDim.x, b = blockIdx.x;
    TileIter it;
    if (xcd_remap && (G & 7) == 0) {
        const int per = G >> 3, x = b & 7, j = b >> 3;
        const int chunk = (n_tiles + 7) >> 3;
        it.cur = x * chunk + j;
        it.step = per;
        it.end = min((x + 1) * chunk, n_tiles);
    } else {
        it.cur = b;
        it.step = G;
        it.end = n_tiles;
    }
    return it;
}

// Stores through global-address-space pointers (the generic form would
// also wait on the LDS counter).
__device__ __forceinline__ void gst4(float *p, V4<float> v)
{
    typedef float vtype __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) vtype gtype;
    *(gtype *)p = vtype{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ void gst4(double *p, V4<double> v)
{
    typedef double vtype __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(1))) vtype gtype;
    ((gtype *)p)[0] = vtype{v.x, v.y};
    ((gtype *)p)[1] = vtype{v.z, v.w};
}
__device__ __forceinline__ void gst1(float *p, float v)
{
    typedef __attribute__((address_space(1))) float gtype;
    *(gtype *)p = v;
}

// Sum of 32 per-lane values over the 64-lane wavefront by recursive halving:
// at step s each lane keeps half of its remaining values and sends the other
// half to the lane whose id differs in bit s, so every exchange moves one
// value instead of all 32.  Lane l < 32 returns the total of value index
// bitrev5(l); lanes l and l + 32 return the same total.
template <typename T>
__device__ __forceinline__ T wave_sum32(T (&v)[kAccum], int lane)
{
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        const int half = 16 >> s;
        const int m = 1 << s;
        const bool up = (lane & m) != 0;
#pragma unroll
        for (int k = 0; k < half; ++k) {
            const T lo = v[k], hi = v[k + half];
            const T send = up ? lo : hi;
            const T keep = up ? hi : lo;
            v[k] = keep + __shfl_xor(send, m, 64);
        }
    }
    return v[0] + __shfl_xor(v[0], 32, 64);
}

__device__ __forceinline__ int bitrev5(int x)
{
    return ((x & 1) << 4) | ((x & 2) << 2) | (x & 4) | ((x & 8) >> 2) | ((x & 16) >> 4);
}

__device__ __forceinline__ int wave_count(bool p) { return __builtin_popcountll(__builtin_amdgcn_ballot_w64(p)); }

// ----------------------------------------------------------------------------- geometry kernels

__global__ void k_unproject(SensorTab<float> S, const float *range, float *xyz, uint8_t *valid)
{
    const int N = S.H * S.W;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int v = i / S.W, u = i - v * S.W;
        const float r = range[i];
        const bool ok = range_ok(r);
        V3<float> p = {0.f, 0.f, 0.f};
        if (ok)
            p = unproject(S, u, v, r);
        xyz[3 * (size_t)i] = p.x;
        xyz[3 * (size_t)i + 1] = p.y;
        xyz[3 * (size_t)i + 2] = p.z;
        valid[i] = ok ? 1 : 0;
    }
}

__global__ void k_project(const SensorTab<float> *tab, int level, const float *xyz, int64_t n, int32_t *uo,
                          int32_t *vo, float *ro, uint8_t *valid)
{
    const LevelView<float> V = level_view(tab, level);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        int u = -1, v = -1;
        float r = sqrtf(x * x + y * y + z * z);
        const bool ok = project(V, x, y, z, u, v, r);
        uo[i] = ok ? u : -1;
        vo[i] = ok ? v : -1;
        ro[i] = ok ? r : sqrtf(x * x + y * y + z * z);
        valid[i] = ok ? 1 : 0;
    }
}

__global__ void k_normals(SensorTab<float> S, const float *range, double edge_rel, float *nrm, uint8_t *valid)
{
    const int N = S.H * S.W;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int v = i / S.W, u = i - v * S.W;
        V3<float> n = {0.f, 0.f, 0.f};
        const bool ok = normal_at(S, range, u, v, edge_rel, n);
        nrm[3 * (size_t)i] = ok ? n.x : 0.f;
        nrm[3 * (size_t)i + 1] = ok ? n.y : 0.f;
        nrm[3 * (size_t)i + 2] = ok ? n.z : 0.f;
        valid[i] = ok ? 1 : 0;
    }
}

__global__ void k_clear(int *flags, int n_flags, rir_level_stats *stats, int n_stats)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
    for (int i = tid; i < n_flags; i += nt)
        flags[i] = 0;
    int *sw = reinterpret_cast<int *>(stats);
    const int nw = n_stats * (int)(sizeof(rir_level_stats) / sizeof(int));
    for (int i = tid; i < nw; i += nt)
        sw[i] = 0;
}

// ----------------------------------------------------------------------------- prepass

// Normal image and pyramid (Sec. 4.1): each wavefront takes kPrepSeg
// segments of target rows at a time, issues all their range loads first
// (centre, row neighbours, rows above and below; bounds-checked buffer
// loads), then computes the normals of their pixels (row factors by scalar
// loads) and writes the (n, n . q) records (0, 0, 0, NaN where the normal is
// invalid) at level 0 and, for rows and columns on the grid of level l, the
// strided copies of the record, the target range and the source range.  With
// init_centroid each tile also records the sums of its valid source and
// target points (reduced per pair by k_centroid); CENTROID instances only.
constexpr int kPrepSeg = 4;

template <typename T, bool CENTROID>
__global__ __launch_bounds__(256) void k_prepass(PrepArgs a)
{
    __shared__ T s_red[4][kAccum];
    const PairDesc<T> *pairs = reinterpret_cast<const PairDesc<T> *>(a.pairs);
    T *psum = reinterpret_cast<T *>(a.psum);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), nwave = blockDim.x >> 6;
    for (TileIter it = tile_iter(a.n_tiles, a.xcd_remap); it.cur < it.end; it.cur += it.step) {
        const int cur = a.tile_base + it.cur;
        const int2 tl = cload(a.tiles + cur);
        const PairDesc<T> *P = pairs + tl.x;
        const SensorTab<T> *S = cload(&P->tab);
        const int H = cload(&P->H), W = cload(&P->W), spr = (W + kSegPx - 1) / kSegPx;
        const int seg_end = min(tl.y + a.tile_seg, H * spr);
        const uint32_t img = (uint32_t)(H * W) * 4u;
        const rsrc_t drs = make_rsrc(cload(&P->dstr[0]), img), srs = make_rsrc(cload(&P->src[0]), img);
        const rsrc_t crs = make_rsrc(cload(&S->col), (uint32_t)(W * 2 * sizeof(T)));
        const T *rowt = cload(&S->row), *nrowt = cload(&S->nrow);
        const T r0 = cload(&S->r0), cos_h = cload(&S->cos_h), sin_h = cload(&S->sin_h);
        T *d40 = cload(&P->dst4[0]);
        T acc[kAccum];
#pragma unroll
        for (int k = 0; k < kAccum; ++k)
            acc[k] = (T)0;
        for (int s0 = tl.y + wave; s0 < seg_end; s0 += kPrepSeg * nwave) {
            int vs[kPrepSeg], us[kPrepSeg];
            bool in[kPrepSeg];
            float rc[kPrepSeg], rs[kPrepSeg], rl[kPrepSeg], rr[kPrepSeg], ru[kPrepSeg], rd[kPrepSeg];
            T ca[kPrepSeg], sa[kPrepSeg];
#pragma unroll
            for (int j = 0; j < kPrepSeg; ++j) {
                const int seg = s0 + j * nwave;
                const bool live = seg < seg_end;
                const int v = live ? seg / spr : 0;
                const int u = (seg - v * spr) * kSegPx + lane;
                const bool ok = live && u < W;
                const bool inner = live && v > 0 && v < H - 1;  // normal rows (uniform)
                const int i = v * W + u;
                const int ul = u == 0 ? W - 1 : u - 1, ur = u == W - 1 ? 0 : u + 1;
                vs[j] = v;
                us[j] = u;
                in[j] = ok;
                rc[j] = bld1<float>(drs, ok ? 4u * (uint32_t)i : kNoLoad);
                rs[j] = bld1<float>(srs, ok ? 4u * (uint32_t)i : kNoLoad);
                bld2(crs, ok ? (uint32_t)u * (uint32_t)(2 * sizeof(T)) : kNoLoad, ca[j], sa[j]);
                rl[j] = bld1<float>(drs, ok && inner ? 4u * (uint32_t)(v * W + ul) : kNoLoad);
                rr[j] = bld1<float>(drs, ok && inner ? 4u * (uint32_t)(v * W + ur) : kNoLoad);
                ru[j] = bld1<float>(drs, ok && inner ? 4u * (uint32_t)(i - W) : kNoLoad);
                rd[j] = bld1<float>(drs, ok && inner ? 4u * (uint32_t)(i + W) : kNoLoad);
            }
#pragma unroll
            for (int j = 0; j < kPrepSeg; ++j) {
                const int v = vs[j], u = us[j];
                const V4<T> rw = sld4(rowt, v);
                V4<T> rec = {(T)0, (T)0, (T)0, quiet_nan<T>()};
                if (a.given_normals) {
                    if (in[j])
                        rec = ld4(d40 + 4 * (size_t)(v * W + u));
                } else if (v > 0 && v < H - 1) {
                    V3<T> n;
                    if (normal_core(ca[j], sa[j], rw, sld4(rowt, v + 1), sld4(rowt, v - 1), sld4(nrowt, 2 * v),
                                    sld4(nrowt, 2 * v + 1), r0, cos_h, sin_h, rc[j], rl[j], rr[j], ru[j], rd[j],
                                    a.edge_rel, n)) {
                        const V3<T> d = ray_dir(rw, ca[j], sa[j]);
                        const T q0 = (T)rc[j] * d.x + r0 * ca[j], q1 = (T)rc[j] * d.y + r0 * sa[j];
                        const T q2 = (T)rc[j] * d.z;
                        rec = V4<T>{n.x, n.y, n.z, n.x * q0 + n.y * q1 + n.z * q2};
                    }
                }
                if (in[j]) {
                    if (!a.given_normals)
                        gst4(d40 + 4 * (size_t)(v * W + u), rec);
                    if constexpr (CENTROID) {
                        const V3<T> d = ray_dir(rw, ca[j], sa[j]);
                        if (range_ok(rs[j])) {
                            acc[0] += (T)rs[j] * d.x + r0 * ca[j];
                            acc[1] += (T)rs[j] * d.y + r0 * sa[j];
                            acc[2] += (T)rs[j] * d.z;
                            acc[3] += (T)1;
                        }
                        if (range_ok(rc[j])) {
                            acc[4] += (T)rc[j] * d.x + r0 * ca[j];
                            acc[5] += (T)rc[j] * d.y + r0 * sa[j];
                            acc[6] += (T)rc[j] * d.z;
                            acc[7] += (T)1;
                        }
                    }
                }
                // pyramid copies: rows on the level grid (uniform test), then columns
                for (int l = 1; l < a.levels && (v & ((1 << l) - 1)) == 0; ++l) {
                    if (in[j] && (u & ((1 << l) - 1)) == 0) {
                        const size_t q = (size_t)(v >> l) * (W >> l) + (u >> l);
                        gst4(cload(&P->dst4[l]) + 4 * q, rec);
                        gst1(cload(&P->dstr[l]) + q, rc[j]);
                        gst1(cload(&P->src[l]) + q, rs[j]);
                    }
                }
            }
        }
        if constexpr (!CENTROID)
            continue;
        const T tot = wave_sum32(acc, lane);
        if (lane < 32)
            s_red[wave][bitrev5(lane)] = tot;
        __syncthreads();
        if (tid < kAccum) {
            T sum = (T)0;
            for (int w = 0; w < nwave; ++w)
                sum += s_red[w][tid];
            psum[(size_t)cur * kAccum + tid] = sum;
        }
        __syncthreads();
    }
}

// Initial pose from the point-set centres (Sec. 4.1): R = I and
// t = mean(valid target points) - mean(valid source points), from the tile
// sums of the prepass, added in FP64 in tile order.  One wave per pair.
template <typename T>
__global__ __launch_bounds__(64) void k_centroid(PrepArgs a)
{
    __shared__ double s_c[8];
    const int pair = a.pair_base + blockIdx.x;
    const PairDesc<T> &P = reinterpret_cast<const PairDesc<T> *>(a.pairs)[pair];
    const T *psum = reinterpret_cast<const T *>(a.psum);
    const int lane = threadIdx.x;
    if (lane < 8) {
        double s = 0.0;
        for (int k = 0; k < P.ntile[0]; ++k)
            s += (double)psum[(size_t)(P.tile0[0] + k) * kAccum + lane];
        s_c[lane] = s;
    }
    __syncthreads();
    if (lane < 16) {
        double *T0 = a.poses + 16 * (size_t)pair;
        double val = (lane % 5 == 0) ? 1.0 : 0.0;
        if ((lane == 3 || lane == 7 || lane == 11) && s_c[3] > 0.0 && s_c[7] > 0.0) {
            const int c = lane / 4;
            val = s_c[4 + c] / s_c[7] - s_c[c] / s_c[3];
        }
        T0[lane] = val;
    }
}

// Neighbour features of the learned weight (PairDesc::nbf) for every target
// pixel of level l of every pair that keeps them: grid (pixel blocks, pair).
// FP32 plans only (the step's features are then read back bit for bit).
__global__ __launch_bounds__(256) void k_nbr_feats(NbrArgs a)
{
    const PairDesc<float> *P = reinterpret_cast<const PairDesc<float> *>(a.pairs) + a.pair_base + blockIdx.y;
    const int l = a.level;
    uint32_t *out = cload(&P->nbf[l]);
    if (!out)
        return;
    const int Hl = cload(&P->H) >> l, Wl = cload(&P->W) >> l, n = Hl * Wl;
    const float *img = cload(&P->dstr[l]);
    const float inv_delta = (float)(1.0 / a.delta);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int vl = i / Wl, ul = i - vl * Wl;
        const uint4 f = neighbour_features<float>(img, Hl, Wl, ul, vl, img[i], inv_delta);
        reinterpret_cast<uint4 *>(out)[i] = f;
    }
}

// ----------------------------------------------------------------------------- solve

// FP64 lane exchange helpers for the wavefront solve.
__device__ __forceinline__ double rlane(double v, int src)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src, 64); }

// Start of row r of the packed upper triangle of a symmetric 6x6 matrix
// (21 entries, row-major): entry (r, c), c >= r, is tri_off(r) + c - r.
__device__ __forceinline__ int tri_off(int r) { return r * 6 - (r * (r - 1)) / 2; }

// The Gauss-Newton update of one pair (Eq. (7)) by one wavefront, each lane
// holding one entry, so that the solve needs few registers and no single
// lane walks the whole factorisation:
//  - lane t < 21 holds entry t of the packed J^T W J; the upper Cholesky
//    factor U (U^T U = J^T W J) is formed in place, right-looking: at step j
//    row j is finished (pivot sqrt, row scaled by its reciprocal) and every
//    later entry (r, c) subtracts U(j, r) U(j, c), so each entry sees its
//    subtractions in ascending j as in the textbook left-looking form.  A
//    pivot not above 1e-12 times the largest diagonal entry fails;
//  - lanes 0..5 solve U^T y = -g, then U xi = y;
//  - lanes 0..11 form T <- Exp(xi) T (left update, Exp(xi) = [R, V tau] with
//    R = I + A K + B K^2, V = I + B K + C K^2, K = [omega]x, A = sin a / a,
//    B = (1 - cos a) / a^2, C = (a - sin a) / a^3, Taylor below a = 1e-6),
//    one pose entry each.
// Then the per-level statistics.  tot: the 30 FP64 sums (J^T W J, J^T W e,
// sum w, sum w e^2, robust cost), cnt: valid, inlier and projection counts.
// Called by all 64 lanes of one wavefront; returns (wave-uniform) whether the
// pose moved, and then leaves the new pose in pose_out[0..11].
__device__ __forceinline__ bool solve_pair_wave(const StepArgs &a, int pair, int *fl, const double *tot,
                                                const long long *cnt, double *pose_out)
{
    int lane = threadIdx.x & 63;
    // opaque to the optimiser, so that the lane-dependent constants below are
    // formed here and not hoisted into (and kept live through) the caller's
    // pixel loop
    asm volatile("" : "+v"(lane));
    const int l = a.level;
    const bool isU = lane < 21;
    int ur = 0, uc = 0;  // (row, column) of this lane's entry
    {
        int t = lane;
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const int len = 6 - r;
            if (t >= 0 && t < len) {
                ur = r;
                uc = r + t;
            }
            t -= len;
        }
    }
    const double tv = lane < 30 ? tot[lane] : 0.0;
    const double sum_w = tot[27], sum_we2 = tot[28], rho = tot[29];
    const int n_valid = (int)cnt[0];
    const bool finite = __builtin_amdgcn_ballot_w64(lane < 30 && !isfinite(tv)) == 0;
    rir_level_stats *out = a.stats + (a.mode == kStepDebug ? 0 : (size_t)pair * a.levels + l);
    if (isU)
        out->JtJ[lane] = tv;
    double U = isU ? tv : 0.0;
    double dmax = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const double d = rlane(U, tri_off(j));
        dmax = d > dmax ? d : dmax;
    }
    bool ok = n_valid >= 6 && finite && dmax > 0.0;
    double rinv = 0.0, v = 0.0;  // lane j < 6: 1 / U(j, j); then y_j, then xi_j
    if (ok) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const double d = rlane(U, tri_off(j));
            ok = ok && d > 1e-12 * dmax;
            const double sd = sqrt(d > 0.0 ? d : 1.0), inv = 1.0 / sd;
            if (lane == j)
                rinv = inv;
            if (isU && ur == j)
                U = uc == j ? sd : U * inv;
            const bool below = isU && ur > j;
            const double ar = shfl_d(U, below ? tri_off(j) + ur - j : 0);
            const double ac = shfl_d(U, below ? tri_off(j) + uc - j : 0);
            if (below)
                U -= ar * ac;
        }
    }
    if (ok) {
        v = -shfl_d(tv, lane < 6 ? 21 + lane : 0);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double yk = rlane(v, k) * rlane(rinv, k);
            const double ukl = shfl_d(U, lane > k && lane < 6 ? tri_off(k) + lane - k : 0);
            if (lane == k)
                v = yk;
            else if (lane > k && lane < 6)
                v -= ukl * yk;
        }
#pragma unroll
        for (int k = 5; k >= 0; --k) {
            const double xk = rlane(v, k) * rlane(rinv, k);
            const double ulk = shfl_d(U, lane < k ? tri_off(lane) + k - lane : 0);
            if (lane == k)
                v = xk;
            else if (lane < k)
                v -= ulk * xk;
        }
    }
    if (a.learned && a.mode == kStepNormal && (!ok || sum_w < 0.1 * (double)n_valid)) {
        // learned weights rejected: the pseudo-Huber pass that follows redoes
        // this iteration and rewrites the statistics
        if (lane == 0)
            fl[kMaxLevels] = 1;
        return false;
    }
    int status = a.mode == kStepFallback ? RIR_LEVEL_FALLBACK_HUBER : RIR_LEVEL_OK;
    if (a.mode == kStepFallback && lane == 0)
        fl[kMaxLevels] = 0;
    double srot = 0.0, stra = 0.0;
    bool moved = false;
    if (!ok) {
        status = finite ? RIR_LEVEL_DEGENERATE : RIR_LEVEL_NONFINITE;
        if (a.mode != kStepDebug && lane == 0)
            fl[l] = 1;
    } else {
        const double w0 = rlane(v, 0), w1 = rlane(v, 1), w2 = rlane(v, 2);
        const double t0 = rlane(v, 3), t1 = rlane(v, 4), t2 = rlane(v, 5);
        srot = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
        stra = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
        if (a.mode != kStepDebug) {
            const double a2 = w0 * w0 + w1 * w1 + w2 * w2, an = sqrt(a2);
            double A, B, C;
            if (an < 1e-6) {
                A = 1.0 - a2 / 6.0;
                B = 0.5 - a2 / 24.0;
                C = 1.0 / 6.0 - a2 / 120.0;
            } else {
                double sn, cs;
                sincos(an, &sn, &cs);
                A = sn / an;
                B = (1.0 - cs) / a2;
                C = (an - sn) / (a2 * an);
            }
            double *Tp = a.poses + 16 * (size_t)pair;
            const int i = (lane >> 2) & 3, j = lane & 3;
            const double wi = i == 0 ? w0 : (i == 1 ? w1 : w2);
            const double w[3] = {w0, w1, w2}, tau[3] = {t0, t1, t2};
            // row i of K = [omega]x
            const double K[3] = {i == 0 ? 0.0 : (i == 1 ? w2 : -w1), i == 0 ? -w2 : (i == 1 ? 0.0 : w0),
                                 i == 0 ? w1 : (i == 1 ? -w0 : 0.0)};
            double Er[3], Et = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double I = i == k ? 1.0 : 0.0;
                const double K2 = wi * w[k] - I * a2;
                Er[k] = I + A * K[k] + B * K2;
                Et += (I + B * K[k] + C * K2) * tau[k];
            }
            double Tn = 0.0;
            if (lane < 12) {
                double acc = j == 3 ? Et : 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    acc += Er[k] * Tp[4 * k + j];
                Tn = acc;
            }
            // every lane has read the old pose (one load instruction per k)
            // before any lane stores
            __builtin_amdgcn_wave_barrier();
            if (lane < 12) {
                Tp[lane] = Tn;
                pose_out[lane] = Tn;
            }
            moved = true;
            // small-step stop: the level's remaining iterations are skipped
            if (a.stop_eps > 0.0 && srot * srot + stra * stra <= a.stop_eps * a.stop_eps && lane == 0)
                fl[l] = 1;
        }
    }
    const double gj = shfl_d(tv, lane < 6 ? 21 + lane : 0);  // all lanes exchange
    if (lane < 6)
        out->Jtr[lane] = gj;
    if (lane == 0) {
        out->status = status;
        out->iters_run = a.iter + 1;
        out->n_valid = n_valid;
        out->n_inlier = (int)cnt[1];
        out->n_proj = (int)cnt[2];
        out->pad = 0;
        out->sum_w = sum_w;
        out->sum_w_e2 = sum_we2;
        out->robust_cost = rho;
        out->step_rot = srot;
        out->step_trans = stra;
    }
    return moved;
}

// Frame of ray rows for pose R (FP64, row-major 3x4): for the row with
// factors rw = (cos phi, sin phi, cos theta, sin theta), g1 = R (A, B, 0),
// g2 = R (-B, A, 0), g3 = sin(phi) R e_z with A = cos(phi) cos(theta),
// B = cos(phi) sin(theta); then three zeros (PairDesc::frames layout).
template <typename T>
__device__ __forceinline__ void frame_row(const T *rw, const double (&R)[12], T *o)
{
    const double cphi = (double)rw[0], sphi = (double)rw[1];
    const double A = cphi * (double)rw[2], B = cphi * (double)rw[3];
    o[0] = (T)(A * R[0] + B * R[1]);
    o[1] = (T)(A * R[4] + B * R[5]);
    o[2] = (T)(A * R[8] + B * R[9]);
    o[3] = (T)(A * R[1] - B * R[0]);
    o[4] = (T)(A * R[5] - B * R[4]);
    o[5] = (T)(A * R[9] - B * R[8]);
    o[6] = (T)(sphi * R[2]);
    o[7] = (T)(sphi * R[6]);
    o[8] = (T)(sphi * R[10]);
    o[9] = o[10] = o[11] = (T)0;
}

// Ray frames of every full-resolution row of one pair for the pose in
// s_pose (the PairDesc::frames layout), written by the threads of one
// workgroup; FP64 arithmetic, stored in T.
template <typename T>
__device__ __forceinline__ void write_frames(const PairDesc<T> *P, const double (&R)[12])
{
    const SensorTab<T> *tab = cload(&P->tab);
    const T *row = cload(&tab->row);
    T *fr = cload(&P->frames);
    const int H = cload(&P->H);
    int v0 = threadIdx.x;
    asm volatile("" : "+v"(v0));  // see solve_pair_wave
    for (int v = v0; v < H; v += blockDim.x)
        frame_row(row + 4 * (size_t)v, R, fr + (size_t)v * kFrame);
}

// ----------------------------------------------------------------------------- step

// The per-pixel work of one Gauss-Newton iteration (Eq. (5)-(7), Sec. 4.1) over
// segments [seg_begin, seg_end) of one pair's level image, by all wavefronts of
// the workgroup: each wavefront takes CHUNK segments at a time (its own
// 64-pixel pieces of CHUNK rows), so that CHUNK source loads, then CHUNK
// target gathers, are in flight together.  A segment's row frame (g1, g2, g3:
// the ray directions of Eq. (1) rotated by the pose) is uniform, so
// unprojection plus the rigid transform is x = r (ca g1 + sa g2 + g3) +
// r0 R (ca, sa, 0) + t.  The target record holds (n, n . q), so
// e = n . x - n . q (NaN, hence invalid, where the record is).  Frames come
// from the pair's full-resolution table in device memory (scalar loads) or,
// with LDS_FRAMES, from a table of the level's rows in shared memory.  Each
// wavefront leaves its sums in s_wave[wave] (kAccum values; [30] the valid
// count) and its inlier / projection counts in s_wcnt[wave][1..2].  LEAN
// instances (StepArgs::lean) leave out the receiver offset, the distance gate,
// the debug dumps and the per-lane row-end test, and wrap columns with a mask
// (the level width is a power of two).
template <typename T, int WMODE, int CHUNK, bool LEAN, bool LDS_FRAMES>
__device__ __forceinline__ void step_segments(const StepArgs &a, const MlpInfer &F, int pair, int seg_begin,
                                              int seg_end, bool stats, const T (&pose)[12], const T *frames,
                                              T (*s_wave)[kAccum], int (*s_wcnt)[4])
{
    const PairDesc<T> *P = reinterpret_cast<const PairDesc<T> *>(a.pairs) + pair;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), nwave = blockDim.x >> 6;
    const int l = a.level, s = 1 << l;
    const T delta = (T)a.delta, inv_delta = (T)(1.0 / a.delta);
    const T mc2 = !LEAN && a.max_corr > 0.0 ? (T)(a.max_corr * a.max_corr) : (T)-1;
    const bool dbg = !LEAN && a.mode == kStepDebug;
    const uint32_t lane4 = 4u * (uint32_t)lane, lane_col = (uint32_t)(lane << l) * (uint32_t)(2 * sizeof(T));
    const LevelView<T> V = level_view(cload(&P->tab), l);
    const LevelImage LI = {cload(&P->dstr[l]), V.Hl, V.Wl};
    const uint32_t *nbf = WMODE == 1 && !dbg ? cload(&P->nbf[l]) : nullptr;
    const T r00 = pose[0], r01 = pose[1], r10 = pose[4], r11 = pose[5], r20 = pose[8], r21 = pose[9];
    const T t0 = pose[3], t1 = pose[7], t2 = pose[11];
    const int Wl = V.Wl, Hl = V.Hl, spr = (Wl + kSegPx - 1) / kSegPx;
    const uint32_t npx = (uint32_t)(Hl * Wl);
    const rsrc_t srs = make_rsrc(cload(&P->src[l]), npx * 4u);
    const rsrc_t drs = make_rsrc(cload(&P->dst4[l]), npx * (uint32_t)(4 * sizeof(T)));
    const T r0 = LEAN ? (T)0 : V.r0;
    const T h1x = r0 * r00, h1y = r0 * r10, h1z = r0 * r20;  // r0 R e_x
    const T h2x = r0 * r01, h2y = r0 * r11, h2z = r0 * r21;  // r0 R e_y
    T acc[kAccum];
#pragma unroll
    for (int k = 0; k < kAccum; ++k)
        acc[k] = (T)0;
    int c_valid = 0, c_in = 0, c_proj = 0;  // lane count, wave counts
    for (int s0 = seg_begin + wave; s0 < seg_end; s0 += CHUNK * nwave) {
        float rs[CHUNK];
        T ca[CHUNK], sa[CHUNK];
        int vs[CHUNK], us[CHUNK];
        bool in[CHUNK];
#pragma unroll
        for (int j = 0; j < CHUNK; ++j) {
            const int seg = s0 + j * nwave;
            const bool live = seg < seg_end;
            const int v = live ? seg / spr : 0;
            const int u0 = (seg - v * spr) * kSegPx, u = u0 + lane;
            vs[j] = v;
            us[j] = u;
            if constexpr (LEAN) {
                // whole segments: uniform base plus the lane's offset
                in[j] = live;
                const uint32_t sb = __builtin_amdgcn_readfirstlane(live ? 4u * (uint32_t)(v * Wl + u0) : kNoLoad);
                const uint32_t cb = __builtin_amdgcn_readfirstlane(
                    live ? (uint32_t)(s * u0) * (uint32_t)(2 * sizeof(T)) : kNoLoad);
                rs[j] = bld1<float>(srs, sb + lane4);
                bld2(V.col, cb + lane_col, ca[j], sa[j]);
            } else {
                in[j] = live && u < Wl;
                rs[j] = bld1<float>(srs, in[j] ? 4u * (uint32_t)(v * Wl + u) : kNoLoad);
                bld2(V.col, in[j] ? (uint32_t)(s * u) * (uint32_t)(2 * sizeof(T)) : kNoLoad, ca[j], sa[j]);
            }
        }
        // A chunk none of whose lanes has a return (sky rows, mostly) adds
        // exact zeros to every sum (e = 0, w = 0, finite J) and counts
        // nothing: the wavefront skips it after the range loads (one
        // wave-uniform branch; debug dumps keep every segment).
        bool any = false;
#pragma unroll
        for (int j = 0; j < CHUNK; ++j)
            any = any || range_ok(rs[j]);
        if (!dbg && __builtin_amdgcn_ballot_w64(any) == 0)
            continue;
        bool proj[CHUNK];
        int ul[CHUNK], vl[CHUNK];
        T xx[CHUNK], xy[CHUNK], xz[CHUNK], xr[CHUNK];
#pragma unroll
        for (int j = 0; j < CHUNK; ++j) {
            V4<T> f0, f1, f2;
            if constexpr (LDS_FRAMES) {
                const T *fr = frames + vs[j] * kFrame;
                f0 = {fr[0], fr[1], fr[2], fr[3]};
                f1 = {fr[4], fr[5], fr[6], fr[7]};
                f2 = {fr[8], fr[9], fr[10], fr[11]};
            } else {
                const T *fr = frames + (size_t)(s * vs[j]) * kFrame;
                f0 = sld4(fr, 0);
                f1 = sld4(fr, 1);
                f2 = sld4(fr, 2);
            }
            // a pixel without a return (0, negative, NaN, infinite) unprojects
            // at r = 0: its point is finite, so its exact-zero terms stay zero
            const bool okr = range_ok(rs[j]);
            const T r = okr ? (T)rs[j] : (T)0, c = ca[j], sn = sa[j], rc = r * c, rsn = r * sn;
            xx[j] = fma(rc, f0.x, fma(rsn, f0.w, fma(r, f1.z, t0)));
            xy[j] = fma(rc, f0.y, fma(rsn, f1.x, fma(r, f1.w, t1)));
            xz[j] = fma(rc, f0.z, fma(rsn, f1.y, fma(r, f2.x, t2)));
            if (!LEAN && r0 > (T)0) {
                xx[j] += c * h1x + sn * h2x;
                xy[j] += c * h1y + sn * h2y;
                xz[j] += c * h1z + sn * h2z;
            }
            proj[j] = project<T, !LEAN, LEAN>(V, xx[j], xy[j], xz[j], ul[j], vl[j], xr[j]) & okr;
        }
        // the gather needs no mask: project() keeps (ul, vl) inside the
        // level image for every lane, and a lane that did not project adds
        // exact zeros below whatever record it reads (w = 0, e = 0, finite J)
        V4<T> D[CHUNK];
#pragma unroll
        for (int j = 0; j < CHUNK; ++j)
            D[j] = bld4<T>(drs, (__umul24((uint32_t)vl[j], (uint32_t)Wl) + (uint32_t)ul[j]) *
                                    (uint32_t)(4 * sizeof(T)));
        // learned weights (FP32): the features' target-side loads go out with
        // the record gather (same pixel), not after it
        constexpr bool kRec = WMODE == 1 && sizeof(T) == 4;
        const bool use_rec = kRec && nbf && a.mode != kStepFallback;
        NbrRec NR[kRec ? CHUNK : 1];
        if constexpr (kRec) {
            if (use_rec) {
#pragma unroll
                for (int j = 0; j < CHUNK; ++j)
                    NR[j] = load_nbr(LI, nbf, proj[j], ul[j], vl[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < CHUNK; ++j) {
            const T n0 = D[j].x, n1 = D[j].y, n2 = D[j].z;
            const T ex = n0 * xx[j] + n1 * xy[j] + n2 * xz[j] - D[j].w;
            bool valid = proj[j] && ex == ex;
            if (mc2 >= (T)0) {
                // Sec. 4.1 correspondence gate: |x - q| against the target point
                const rsrc_t rrs = make_rsrc(LI.rng, npx * 4u);
                const uint32_t pix = (uint32_t)(vl[j] * Wl + ul[j]);
                const T rq = (T)bld1<float>(rrs, valid ? 4u * pix : kNoLoad);
                const V4<T> rw = bld4<T>(V.row, (uint32_t)(s * vl[j]) * (uint32_t)(4 * sizeof(T)));
                T cq, sq;
                bld2(V.col, (uint32_t)(s * ul[j]) * (uint32_t)(2 * sizeof(T)), cq, sq);
                const V3<T> d = ray_dir(rw, cq, sq);
                const T dx = xx[j] - (rq * d.x + r0 * cq), dy = xy[j] - (rq * d.y + r0 * sq);
                const T dz = xz[j] - rq * d.z;
                valid = valid && dx * dx + dy * dy + dz * dz <= mc2;
            }
            const T e = valid ? ex : (T)0;
            const T J0 = xy[j] * n2 - xz[j] * n1;
            const T J1 = xz[j] * n0 - xx[j] * n2;
            const T J2 = xx[j] * n1 - xy[j] * n0;
            const T tq = e * inv_delta;
            const T wh = d_rsqrt((T)1 + tq * tq);
            T w = wh;
            const int i = in[j] ? vs[j] * Wl + us[j] : -1;
            if constexpr (kRec) {
                if (use_rec)
                    w = (T)learned_weight_rec(a, F, NR[j], (float)e, (float)xr[j], (float)n0, (float)n1, (float)n2);
                else if (a.mode != kStepFallback)
                    w = learned_weight<T>(a, F, LI, valid, ul[j], vl[j], e, xr[j], n0, n1, n2,
                                          dbg ? a.dbg_feat : nullptr, i);
            } else if constexpr (WMODE == 1) {
                if (a.mode != kStepFallback)
                    w = learned_weight<T>(a, F, LI, valid, ul[j], vl[j], e, xr[j], n0, n1, n2,
                                          dbg ? a.dbg_feat : nullptr, i);
            }
            w = valid ? w : (T)0;
            c_valid += valid ? 1 : 0;
            if (stats) {
                acc[29] += valid ? e * e * wh * d_rcp(wh + (T)1) : (T)0;
                c_proj += wave_count(proj[j]);
                c_in += wave_count(valid && fabs(e) < delta);
            }
            // an invalid pixel has w = 0, e = 0 and finite J (n = 0 unless the
            // distance gate rejected it), so it adds exact zeros
            const T J[6] = {J0, J1, J2, n0, n1, n2};
            T wJ[6];
#pragma unroll
            for (int k = 0; k < 6; ++k)
                wJ[k] = w * J[k];
            int k = 0;
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int c = r; c < 6; ++c)
                    acc[k++] += wJ[r] * J[c];
#pragma unroll
            for (int r = 0; r < 6; ++r)
                acc[21 + r] += wJ[r] * e;
            acc[27] += w;
            acc[28] += w * e * e;
            if (dbg && i >= 0) {
                if (a.dbg_u) a.dbg_u[i] = proj[j] ? ul[j] : -1;
                if (a.dbg_v) a.dbg_v[i] = proj[j] ? vl[j] : -1;
                if (a.dbg_mask) a.dbg_mask[i] = valid ? 1 : 0;
                if (a.dbg_e) a.dbg_e[i] = (float)e;
                if (a.dbg_w) a.dbg_w[i] = (float)w;
                if (a.dbg_J)
                    for (int q = 0; q < 6; ++q)
                        a.dbg_J[6 * (size_t)i + q] = valid ? (float)J[q] : 0.f;
                if (WMODE == 0 && a.dbg_feat)
                    store_features<T>(a, LI, valid, ul[j], vl[j], e, xr[j], n0, n1, n2,
                                      a.dbg_feat + 14 * (size_t)i);
            }
        }
    }
    acc[30] = (T)c_valid;  // exact: far below 2^24 per wavefront
    const T tot = wave_sum32(acc, lane);
    if (lane < 32)
        s_wave[wave][bitrev5(lane)] = tot;
    if (lane == 0) {
        s_wcnt[wave][1] = c_in;
        s_wcnt[wave][2] = c_proj;
    }
}

template <typename T, bool COHERENT>
__device__ __forceinline__ void solve_from_tiles(const StepArgs &a, int pair, int *fl);

// One Gauss-Newton iteration at level l for every pair of the batch.  Each
// workgroup walks its tiles; a tile is a run of tile_seg segments of one
// pair's level-l image, and its sums go to one record (k_solve reduces them).
// FINE tags the finest-level instance (same code) so that profiles report it
// separately.  FUSED instances (one tile per workgroup) also solve: the
// workgroup that finishes a pair's last tile applies that pair's update.
template <typename T, int WMODE, bool FINE, int CHUNK, bool LEAN, bool FUSED>
__global__ __launch_bounds__(256) void k_icp_step(StepArgs a)
{
    __shared__ T s_wave[4][kAccum];
    __shared__ int s_last;
    __shared__ int s_wcnt[4][4];
    T *psum = reinterpret_cast<T *>(a.psum);
    const int tid = threadIdx.x, nwave = blockDim.x >> 6, l = a.level;
    const bool dbg = !LEAN && a.mode == kStepDebug;
    const PairDesc<T> *pairs = reinterpret_cast<const PairDesc<T> *>(a.pairs);
    MlpInfer F;
    if constexpr (WMODE == 1)
        mlp_infer_load(a.mlp, F);
    auto tile = [&](int cur) {
        const int2 tl = cload(a.tiles + cur);
        const int pair = tl.x;
        const int *fl = a.flags + (size_t)pair * kFlagStride;
        const PairDesc<T> *P = pairs + pair;
        const double *Tp = a.poses + 16 * (size_t)pair;
        // What the tile reads that depends on the pair alone is loaded before
        // the flag tests and waited for once (the empty asm takes it all), so
        // that these loads go out together rather than as a chain of
        // dependent round trips behind the early exits.
        const int f_lvl = cload(fl + l), f_fb = cload(fl + kMaxLevels);
        double Td[12];
#pragma unroll
        for (int k = 0; k < 12; ++k)
            Td[k] = cload(Tp + k);
        const int Hp = cload(&P->H), Wp = cload(&P->W);
        const SensorTab<T> *ptab = cload(&P->tab);
        const float *psrc = cload(&P->src[l]), *pdstr = cload(&P->dstr[l]);
        const T *pdst4 = cload(&P->dst4[l]), *pfr = cload(&P->frames);
        asm volatile("" ::"s"(f_lvl), "s"(f_fb), "s"(Hp), "s"(Wp), "s"(ptab), "s"(psrc), "s"(pdstr), "s"(pdst4),
                     "s"(pfr), "s"(Td[0]), "s"(Td[1]), "s"(Td[2]), "s"(Td[3]), "s"(Td[4]), "s"(Td[5]), "s"(Td[6]),
                     "s"(Td[7]), "s"(Td[8]), "s"(Td[9]), "s"(Td[10]), "s"(Td[11]));
        if (!dbg) {
            if (f_lvl & 1)
                return;
            if (a.mode == kStepFallback && !(f_fb & 1))
                return;
        }
        T pose[12];
#pragma unroll
        for (int k = 0; k < 12; ++k)
            pose[k] = (T)Td[k];
        const int Hl = Hp >> l, spr = ((Wp >> l) + kSegPx - 1) / kSegPx;
        step_segments<T, WMODE, CHUNK, LEAN, false>(a, F, pair, tl.y, min(tl.y + a.tile_seg, Hl * spr),
                                                    a.stats_pass != 0, pose, pfr, s_wave, s_wcnt);
        __syncthreads();
        if (tid < kAccum) {
            T sum = (T)0;
            for (int w = 0; w < nwave; ++w)
                sum += s_wave[w][tid];
            T *dst = psum + (size_t)cur * kAccum + tid;
            if constexpr (FUSED)
                __hip_atomic_store(dst, sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                *dst = sum;
        } else if (tid == kAccum) {
            int4 c = make_int4(0, 0, 0, 0);
            for (int w = 0; w < nwave; ++w) {
                c.x += (int)s_wave[w][30];
                c.y += s_wcnt[w][1];
                c.z += s_wcnt[w][2];
            }
            if constexpr (FUSED) {
                int *dst = reinterpret_cast<int *>(a.pcnt + cur);
                __hip_atomic_store(dst + 0, c.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(dst + 1, c.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(dst + 2, c.z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                a.pcnt[cur] = c;
            }
        }
        if constexpr (FUSED) {
            // The record is written with agent-scope (device-coherent) stores;
            // once they have completed, this tile's ticket is taken.  The
            // workgroup that takes a pair's last ticket has every record of
            // the pair visible to its agent-scope loads and solves the pair
            // (the order of the sum does not depend on which workgroup that
            // is), then resets the pair's ticket count for the next launch.
            // No workgroup waits for another, and no cache is flushed.
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the record stores are complete
            __syncthreads();
            if (tid == 0) {
                const int t = __hip_atomic_fetch_add(a.tickets + pair, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_last = t == cload(&P->ntile[l]) - 1 ? 1 : 0;
            }
            __syncthreads();
            if (s_last) {
                solve_from_tiles<T, true>(a, pair, a.flags + (size_t)pair * kFlagStride);
                if (tid == 0)
                    __hip_atomic_store(a.tickets + pair, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    };
    if constexpr (FUSED) {
        // one tile per workgroup (no tile loop whose invariants the solve's
        // constants could be hoisted out of)
        const TileIter it = tile_iter(a.n_tiles, a.xcd_remap);
        if (it.cur < it.end)
            tile(a.tile_base + it.cur);
    } else {
        for (TileIter it = tile_iter(a.n_tiles, a.xcd_remap); it.cur < it.end; it.cur += it.step)
            tile(a.tile_base + it.cur);
    }
}

// All Gauss-Newton iterations of level l for one pair per workgroup (pairs
// with no tiles at this level: small level images, pseudo-Huber weights, lean
// conditions; the host decides per pair): the workgroup covers the
// pair's whole level image each iteration, reduces its sums in FP64 (wave
// order), solves, and keeps the pose and the level rows' frames in shared
// memory, so that the level needs one launch instead of two per iteration.
// At the end it writes the frames of all full-resolution rows for the pose
// reached (the next level's input).
template <typename T, int CHUNK>
__global__ __launch_bounds__(kPairBlock) void k_icp_level(StepArgs a)
{
    __shared__ T s_wave[kPairBlock / 64][kAccum];
    __shared__ int s_wcnt[kPairBlock / 64][4];
    __shared__ T s_fr[kPairRows * kFrame];
    __shared__ double s_tot[kAccum];
    __shared__ long long s_cnt[4];
    __shared__ double s_pose[12];
    __shared__ int s_go;
    const int pair = a.pair_base + blockIdx.x, tid = threadIdx.x, nwave = blockDim.x >> 6, l = a.level;
    int *fl = a.flags + (size_t)pair * kFlagStride;
    const PairDesc<T> *P = reinterpret_cast<const PairDesc<T> *>(a.pairs) + pair;
    if (cload(&P->ntile[l]) != 0 || (cload(fl + l) & 1))
        return;  // a tiled pair at this level, or the level stopped
    const SensorTab<T> *tab = cload(&P->tab);
    const T *rowt = cload(&tab->row);
    const int Hl = cload(&P->H) >> l, spr = (cload(&P->W) >> l) / kSegPx;
    if (tid < 12)
        s_pose[tid] = a.poses[16 * (size_t)pair + tid];
    __syncthreads();
    MlpInfer F;
    for (int it = 0; it < a.iters; ++it) {
        double R[12];
#pragma unroll
        for (int k = 0; k < 12; ++k)
            R[k] = s_pose[k];
        for (int v = tid; v < Hl; v += blockDim.x)
            frame_row(rowt + 4 * (size_t)(v << l), R, s_fr + v * kFrame);
        T pose[12];
#pragma unroll
        for (int k = 0; k < 12; ++k)
            pose[k] = (T)R[k];
        __syncthreads();
        const bool last = it == a.iters - 1;
        step_segments<T, 0, CHUNK, true, true>(a, F, pair, 0, Hl * spr, last, pose, s_fr, s_wave, s_wcnt);
        __syncthreads();
        if (tid < kAccum) {
            double t = 0.0;
            for (int w = 0; w < nwave; ++w)
                t += (double)s_wave[w][tid];
            s_tot[tid] = t;
        } else if (tid >= 64 && tid < 67) {
            long long c = 0;
            for (int w = 0; w < nwave; ++w)
                c += tid == 64 ? (long long)s_wave[w][30] : (long long)s_wcnt[w][tid - 64];
            s_cnt[tid - 64] = c;
        }
        __syncthreads();
        if (tid < 64) {
            StepArgs b = a;
            b.iter = it;
            b.stats_pass = last ? 1 : 0;
            const bool moved = solve_pair_wave(b, pair, fl, s_tot, s_cnt, s_pose);
            if (tid == 0)
                s_go = moved && !(fl[l] & 1) ? 1 : 0;  // stopped by a small step
        }
        __syncthreads();
        if (!s_go)
            break;
    }
    double R[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
        R[k] = s_pose[k];
    write_frames(P, R);
}

// ----------------------------------------------------------------------------- solve kernels

// Frames for the current poses of all pairs (after the poses are set from
// the host or by the centroid initialisation).  One workgroup per pair.
template <typename T>
__global__ __launch_bounds__(256) void k_frames(StepArgs a)
{
    const int pair = a.pair_base + blockIdx.x;
    const PairDesc<T> *P = reinterpret_cast<const PairDesc<T> *>(a.pairs) + pair;
    double R[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
        R[k] = a.poses[16 * (size_t)pair + k];
    write_frames(P, R);
}

// Sum of one pair's tile records t0 .. t0 + nt - 1 in FP64 in a fixed order
// that does not depend on the batch or the block size: group g (of 8) of 32
// threads, one per record entry, adds tiles g, g + 8, ... in that order (four
// records in flight at a time), then the 8 group sums are added in group
// order.  Leaves the 30 sums in s_tot and the 3 counts in s_cnt; all threads
// of the block (64..256) take part.  COHERENT reads the records with
// agent-scope loads (records written during the same launch by other
// workgroups, see k_icp_step).
template <typename T, bool COHERENT>
__device__ __forceinline__ void reduce_pair_tiles(const StepArgs &a, int t0, int nt, double (*s_part)[kAccum],
                                                  long long (*s_cpart)[4], double *s_tot, long long *s_cnt)
{
    const T *psum = reinterpret_cast<const T *>(a.psum);
    const int *pcnt = reinterpret_cast<const int *>(a.pcnt);
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));  // see solve_pair_wave
    const int comp = tid & 31;
    auto rec = [&](int k) -> T {
        const T *q = psum + (size_t)(t0 + k) * kAccum + comp;
        if constexpr (COHERENT)
            return __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return *q;
    };
    auto cnt_of = [&](int k) -> int {
        const int *q = pcnt + 4 * (size_t)(t0 + k) + comp;
        if constexpr (COHERENT)
            return __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return *q;
    };
    for (int grp = tid >> 5; grp < 8; grp += (int)(blockDim.x >> 5)) {
        double sum = 0.0;
        long long c = 0;
        int k = grp;
        for (; k + 24 < nt; k += 32) {
            const T v0 = rec(k), v1 = rec(k + 8), v2 = rec(k + 16), v3 = rec(k + 24);
            if (comp < 3) {
                const int c0 = cnt_of(k), c1 = cnt_of(k + 8), c2 = cnt_of(k + 16), c3 = cnt_of(k + 24);
                c += c0;
                c += c1;
                c += c2;
                c += c3;
            }
            sum += (double)v0;
            sum += (double)v1;
            sum += (double)v2;
            sum += (double)v3;
        }
        for (; k < nt; k += 8) {
            sum += (double)rec(k);
            if (comp < 3)
                c += cnt_of(k);
        }
        s_part[grp][comp] = sum;
        if (comp < 3)
            s_cpart[grp][comp] = c;
    }
    __syncthreads();
    if (tid < 30) {
        double t = 0.0;
        for (int g = 0; g < 8; ++g)
            t += s_part[g][tid];
        s_tot[tid] = t;
    } else if (tid >= 32 && tid < 35) {
        long long t = 0;
        for (int g = 0; g < 8; ++g)
            t += s_cpart[g][tid - 32];
        s_cnt[tid - 32] = t;
    }
    __syncthreads();
}

// The Gauss-Newton update of one pair from its tile records (Eq. (7)):
// FP64 fixed-order sum, Cholesky solve, T <- Exp(xi) T, per-level
// statistics, then the ray frames of the new pose.  Run by every thread of
// one workgroup.
template <typename T, bool COHERENT>
__device__ __forceinline__ void solve_from_tiles(const StepArgs &a, int pair, int *fl)
{
    __shared__ double s_part[8][kAccum];
    __shared__ long long s_cpart[8][4];
    __shared__ double s_tot[32];
    __shared__ long long s_cnt[4];
    __shared__ double s_pose[12];
    __shared__ int s_moved;
    const PairDesc<T> *P = reinterpret_cast<const PairDesc<T> *>(a.pairs) + pair;
    const int l = a.level;
    reduce_pair_tiles<T, COHERENT>(a, cload(&P->tile0[l]), cload(&P->ntile[l]), s_part, s_cpart, s_tot, s_cnt);
    if (threadIdx.x < 64) {
        const bool m = solve_pair_wave(a, pair, fl, s_tot, s_cnt, s_pose);
        if (threadIdx.x == 0)
            s_moved = m ? 1 : 0;
    }
    __syncthreads();
    if (s_moved) {
        double R[12];
#pragma unroll
        for (int k = 0; k < 12; ++k)
            R[k] = s_pose[k];
        write_frames(P, R);
    }
}

// Reduction of one pair's tile records and the Gauss-Newton update, as a
// launch of its own (one workgroup per pair): the debug pass, whose step
// launch does not solve.
template <typename T>
__global__ __launch_bounds__(256) void k_solve(StepArgs a)
{
    const int pair = a.pair_base + blockIdx.x, l = a.level;
    int *fl = a.flags + (size_t)pair * kFlagStride;
    if (a.mode != kStepDebug) {
        if (fl[l] & 1)
            return;
        if (a.mode == kStepFallback && !(fl[kMaxLevels] & 1))
            return;
    }
    const PairDesc<T> *P = reinterpret_cast<const PairDesc<T> *>(a.pairs) + pair;
    if (cload(&P->ntile[l]) == 0)
        return;  // the pair-resident kernel runs this pair's level
    solve_from_tiles<T, false>(a, pair, fl);
}

// ----------------------------------------------------------------------------- launchers

static int grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

hipError_t launch_unproject(const SensorTab<float> &S, const float *range, float *xyz, uint8_t *valid,
                            hipStream_t stream)
{
    hipLaunchKernelGGL(k_unproject, dim3(grid_for((int64_t)S.H * S.W, 256)), dim3(256), 0, stream, S, range, xyz,
                       valid);
    return hipGetLastError();
}

hipError_t launch_project(const SensorTab<float> *tab, int level, const float *xyz, int64_t n, int32_t *u, int32_t *v,
                          float *r, uint8_t *valid, hipStream_t stream)
{
    hipLaunchKernelGGL(k_project, dim3(grid_for(n, 256)), dim3(256), 0, stream, tab, level, xyz, n, u, v, r, valid);
    return hipGetLastError();
}

hipError_t launch_normals(const SensorTab<float> &S, const float *range, double edge_rel, float *nrm,
                          uint8_t *valid, hipStream_t stream)
{
    hipLaunchKernelGGL(k_normals, dim3(grid_for((int64_t)S.H * S.W, 256)), dim3(256), 0, stream, S, range, edge_rel,
                       nrm, valid);
    return hipGetLastError();
}

hipError_t launch_clear(int *flags, int n_flags, rir_level_stats *stats, int n_stats, hipStream_t stream)
{
    int64_t nw = (int64_t)n_stats * (int64_t)(sizeof(rir_level_stats) / sizeof(int));
    int64_t n = nw > n_flags ? nw : n_flags;
    hipLaunchKernelGGL(k_clear, dim3(grid_for(n, 256)), dim3(256), 0, stream, flags, n_flags, stats, n_stats);
    return hipGetLastError();
}

hipError_t launch_prepass(bool fp64, const PrepArgs &a, int grid, int block, int n_pairs, hipStream_t stream)
{
    if (fp64) {
        if (a.init_centroid)
            hipLaunchKernelGGL((k_prepass<double, true>), dim3(grid), dim3(block), 0, stream, a);
        else
            hipLaunchKernelGGL((k_prepass<double, false>), dim3(grid), dim3(block), 0, stream, a);
    } else {
        if (a.init_centroid)
            hipLaunchKernelGGL((k_prepass<float, true>), dim3(grid), dim3(block), 0, stream, a);
        else
            hipLaunchKernelGGL((k_prepass<float, false>), dim3(grid), dim3(block), 0, stream, a);
    }
    if (a.init_centroid) {
        if (fp64)
            hipLaunchKernelGGL(k_centroid<double>, dim3(n_pairs), dim3(64), 0, stream, a);
        else
            hipLaunchKernelGGL(k_centroid<float>, dim3(n_pairs), dim3(64), 0, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_nbr_feats(const NbrArgs &a, int n_pairs, int max_px, hipStream_t stream)
{
    hipLaunchKernelGGL(k_nbr_feats, dim3(grid_for(max_px, 256), n_pairs), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_solve(bool fp64, const StepArgs &a, int n_pairs, hipStream_t stream)
{
    if (fp64)
        hipLaunchKernelGGL(k_solve<double>, dim3(n_pairs), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(k_solve<float>, dim3(n_pairs), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_frames(bool fp64, const StepArgs &a, int n_pairs, hipStream_t stream)
{
    if (fp64)
        hipLaunchKernelGGL(k_frames<double>, dim3(n_pairs), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL(k_frames<float>, dim3(n_pairs), dim3(256), 0, stream, a);
    return hipGetLastError();
}

template <typename T, int WMODE, int CHUNK, bool LEAN, bool FUSED>
static void launch_step_f(const StepArgs &a, int grid, int block, hipStream_t stream)
{
    if (a.level == 0)
        hipLaunchKernelGGL((k_icp_step<T, WMODE, true, CHUNK, LEAN, FUSED>), dim3(grid), dim3(block), 0, stream, a);
    else
        hipLaunchKernelGGL((k_icp_step<T, WMODE, false, CHUNK, LEAN, FUSED>), dim3(grid), dim3(block), 0, stream, a);
}

template <typename T, int WMODE, int CHUNK, bool LEAN>
static void launch_step_l(const StepArgs &a, int grid, int block, hipStream_t stream)
{
    if (a.fused)
        launch_step_f<T, WMODE, CHUNK, LEAN, true>(a, grid, block, stream);
    else
        launch_step_f<T, WMODE, CHUNK, LEAN, false>(a, grid, block, stream);
}

template <typename T, int WMODE, int CHUNK>
static void launch_step_c(const StepArgs &a, int grid, int block, hipStream_t stream)
{
    if (a.lean)
        launch_step_l<T, WMODE, CHUNK, true>(a, grid, block, stream);
    else
        launch_step_l<T, WMODE, CHUNK, false>(a, grid, block, stream);
}

template <typename T, int WMODE>
static void launch_step_t(const StepArgs &a, int grid, int block, hipStream_t stream)
{
    if (a.chunk >= 4)
        launch_step_c<T, WMODE, 4>(a, grid, block, stream);
    else if (a.chunk == 2)
        launch_step_c<T, WMODE, 2>(a, grid, block, stream);
    else
        launch_step_c<T, WMODE, 1>(a, grid, block, stream);
}

hipError_t launch_level(bool fp64, const StepArgs &a, int n_pairs, hipStream_t stream)
{
    if (fp64)
        return hipErrorInvalidValue;  // FP32 per-pixel arithmetic only
    if (a.chunk >= 4)
        hipLaunchKernelGGL((k_icp_level<float, 4>), dim3(n_pairs), dim3(kPairBlock), 0, stream, a);
    else if (a.chunk == 2)
        hipLaunchKernelGGL((k_icp_level<float, 2>), dim3(n_pairs), dim3(kPairBlock), 0, stream, a);
    else
        hipLaunchKernelGGL((k_icp_level<float, 1>), dim3(n_pairs), dim3(kPairBlock), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_step(bool fp64, int weight_mode, const StepArgs &a, int grid, int block, hipStream_t stream)
{
    if (fp64) {
        if (weight_mode == 1)
            launch_step_t<double, 1>(a, grid, block, stream);
        else
            launch_step_t<double, 0>(a, grid, block, stream);
    } else {
        if (weight_mode == 1)
            launch_step_t<float, 1>(a, grid, block, stream);
        else
            launch_step_t<float, 0>(a, grid, block, stream);
    }
    return hipGetLastError();
}

}  // namespace rir
