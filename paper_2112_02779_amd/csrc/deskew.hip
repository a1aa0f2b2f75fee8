// Re-projection of range images under per-column poses on gfx950: the
// non-rigid model of Dong et al.'s outlook (Sec. 6), with consecutive poses
// assigned to each column as in LOAM.  Column u is captured at sweep time
// s_u = (u + 1/2) / W - 1/2; under a constant twist xi per sweep its pose in
// the mid-sweep frame is Exp(s_u xi).  Every return is unprojected (Eq. (1)),
// moved by its column's pose and projected again (Eq. (3)-(4)); the output
// pixel keeps the nearest range (an atomic minimum on the FP32 bit pattern,
// which orders like the value for positive floats).
//
// All in FP64 (the pose, the point and the projection with the FP64 sensor
// tables), so the output differs from an FP64 reference only where a
// projection lies on a rounding boundary.
#include "rir_ops.h"

namespace rir {

namespace {

constexpr uint32_t kInfBits = 0x7f800000u;

// SE(3) exponential of xi = (omega, tau): R = I + A K + B K^2,
// t = (I + B K + C K^2) tau with K = [omega]x (Rodrigues, series for small
// angles).
__device__ __forceinline__ void exp_twist(const double xi[6], double R[9], double t[3])
{
    const double wx = xi[0], wy = xi[1], wz = xi[2];
    const double a2 = wx * wx + wy * wy + wz * wz;
    double A, B, C;
    if (a2 < 1e-12) {
        A = 1.0 - a2 / 6.0;
        B = 0.5 - a2 / 24.0;
        C = 1.0 / 6.0 - a2 / 120.0;
    } else {
        const double a = sqrt(a2), sn = sin(a), cs = cos(a);
        A = sn / a;
        B = (1.0 - cs) / a2;
        C = (a - sn) / (a2 * a);
    }
    const double K[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    double V[9];
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + A * K[i] + B * K2[i];
        V[i] = I + B * K[i] + C * K2[i];
    }
    for (int i = 0; i < 3; ++i)
        t[i] = V[3 * i] * xi[3] + V[3 * i + 1] * xi[4] + V[3 * i + 2] * xi[5];
}

// Twists of up to kDeskewBatch scans, passed as kernel arguments.
constexpr int kDeskewBatch = 32;
struct Twists {
    double xi[kDeskewBatch][6];
};

}  // namespace

__global__ void k_fill_bits(uint32_t *p, int64_t n, uint32_t bits)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = bits;
}

__global__ void k_inf_to_zero(uint32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (p[i] == kInfBits)
            p[i] = 0u;
}

// Columns per workgroup and row groups (threads per column) of k_deskew.
constexpr int kDeskewCols = 64, kDeskewRowGroups = 4;

// One workgroup per 64 columns of one scan (grid: column blocks x scans of
// the batch); each thread takes one column and every 4th row of it, so a
// column's pose Exp(s_u xi) is formed once per thread instead of once per
// pixel, and the loads of a row are coalesced across the 64 columns.
template <bool R0, bool POW2>
__global__ __launch_bounds__(256) void k_deskew(const SensorTab<double> *tab, const float *in, uint32_t *out,
                                                Twists tw)
{
    const LevelView<double> V = level_view(tab, 0);
    const int H = V.Hl, W = V.Wl;
    const double *row = V.rowp, *col = cload(&tab->col);
    const double r0 = V.r0;
    const int img = blockIdx.y;
    const int u = blockIdx.x * kDeskewCols + (int)(threadIdx.x % kDeskewCols);
    const int v0 = (int)(threadIdx.x / kDeskewCols);
    if (u >= W)
        return;
    const int64_t hw = (int64_t)H * W;
    const float *src = in + (size_t)img * hw;
    uint32_t *dst = out + (size_t)img * hw;
    const double su = ((double)u + 0.5) / (double)W - 0.5;
    double xs[6], R[9], t[3];
    for (int k = 0; k < 6; ++k)
        xs[k] = su * tw.xi[img][k];
    exp_twist(xs, R, t);
    for (int v = v0; v < H; v += kDeskewRowGroups) {
        const float rf = src[(size_t)v * W + u];
        if (!range_ok(rf))
            continue;
        const V3<double> p = unproject(row, col, r0, u, v, (double)rf);
        const double x = R[0] * p.x + R[1] * p.y + R[2] * p.z + t[0];
        const double y = R[3] * p.x + R[4] * p.y + R[5] * p.z + t[1];
        const double z = R[6] * p.x + R[7] * p.y + R[8] * p.z + t[2];
        int u2, v2;
        double r2;
        if (!project<double, R0, POW2>(V, x, y, z, u2, v2, r2))
            continue;
        atomicMin(dst + (size_t)v2 * W + u2, __float_as_uint((float)r2));
    }
}

hipError_t launch_deskew(const SensorTab<double> *tab, int H, int W, bool r0, int n_images, const float *in,
                         const double *twists, float *out, hipStream_t stream)
{
    const int64_t hw = (int64_t)H * W, n = hw * n_images;
    uint32_t *ob = reinterpret_cast<uint32_t *>(out);
    const int gfill = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_bits, dim3(gfill), dim3(256), 0, stream, ob, n, kInfBits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const bool pow2 = (W & (W - 1)) == 0;
    for (int k0 = 0; k0 < n_images; k0 += kDeskewBatch) {
        const int nb = std::min(kDeskewBatch, n_images - k0);
        Twists tw;
        for (int k = 0; k < nb; ++k)
            for (int j = 0; j < 6; ++j)
                tw.xi[k][j] = twists[6 * (k0 + k) + j];
        const float *src = in + hw * k0;
        uint32_t *dst = ob + hw * k0;
        const dim3 g((unsigned)((W + kDeskewCols - 1) / kDeskewCols), (unsigned)nb);
        const dim3 b(kDeskewCols * kDeskewRowGroups);
        if (r0)
            hipLaunchKernelGGL((k_deskew<true, false>), g, b, 0, stream, tab, src, dst, tw);
        else if (pow2)
            hipLaunchKernelGGL((k_deskew<false, true>), g, b, 0, stream, tab, src, dst, tw);
        else
            hipLaunchKernelGGL((k_deskew<false, false>), g, b, 0, stream, tab, src, dst, tw);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_inf_to_zero, dim3(gfill), dim3(256), 0, stream, ob, n);
    return hipGetLastError();
}

}  // namespace rir
