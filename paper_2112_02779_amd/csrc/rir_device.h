// Device-side sensor tables and per-pixel geometry of the range-image model
// (Dong et al., Sec. 3): unprojection Eq. (1)-(2), projection Eq. (3)-(4) with
// an inverse elevation table, and the cross-product normal image (Sec. 4.1).
// Everything is templated on the arithmetic type T (float or double).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rir {

constexpr int kMaxLevels = 8;

// Sensor tables in device memory (pointers) plus scalars, one copy per type.
//  row  [H][4]  cos phi_v, sin phi_v, cos theta_v, sin theta_v
//  col  [W][2]  cos a_u, sin a_u with a_u = 2 pi u / W
//  nrow [H][8]  factors of d(u, v+1) - d(u, v-1) in product form (rows 1..H-2):
//               cos(m+s), sin(m+s), cos(m-s), sin(m-s), sin(dt+dp), sin(dt-dp),
//               2 cos(s) sin(dp), 0 with s, dp the half sum / half difference of
//               the two elevations and m, dt those of the two azimuth offsets
//  theta [H]    azimuth offsets
//  per level l (stride 2^l):
//   mu[l]   [H_l-1] sin of the elevation midpoints between strided rows
//   bins[l] [nbins] first candidate row of each inverse-table bin over sin(phi)
//   uoff[l] [H_l]   theta_lut[s t] * W / (2 pi s) (column offset of each row)
template <typename T>
struct SensorTab {
    int H, W, nlev;
    int nbins[kMaxLevels];
    T r0, s_lo, s_hi, cos_h, sin_h;
    T bin_lo[kMaxLevels], bin_scale[kMaxLevels], kW[kMaxLevels];
    const T *row, *col, *nrow, *theta;
    const T *mu[kMaxLevels];
    const int32_t *bins[kMaxLevels];
    const T *uoff[kMaxLevels];
};

template <typename T>
struct V3 {
    T x, y, z;
};

template <typename T>
struct V4 {
    T x, y, z, w;
};

__device__ __forceinline__ V4<float> ld4(const float *p)
{
    float4 v = *reinterpret_cast<const float4 *>(p);
    return {v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ V4<double> ld4(const double *p)
{
    double2 a = reinterpret_cast<const double2 *>(p)[0];
    double2 b = reinterpret_cast<const double2 *>(p)[1];
    return {a.x, a.y, b.x, b.y};
}
__device__ __forceinline__ void ld2(const float *p, float &a, float &b)
{
    float2 v = *reinterpret_cast<const float2 *>(p);
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void ld2(const double *p, double &a, double &b)
{
    double2 v = *reinterpret_cast<const double2 *>(p);
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void st4(float *p, V4<float> v)
{
    *reinterpret_cast<float4 *>(p) = make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(double *p, V4<double> v)
{
    reinterpret_cast<double2 *>(p)[0] = make_double2(v.x, v.y);
    reinterpret_cast<double2 *>(p)[1] = make_double2(v.z, v.w);
}

__device__ __forceinline__ float d_atan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double d_atan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float d_rsqrt(float x) { return rsqrtf(x); }
__device__ __forceinline__ double d_rsqrt(double x) { return 1.0 / sqrt(x); }
template <typename T>
__device__ __forceinline__ T two_pi();
template <>
__device__ __forceinline__ float two_pi<float>() { return 6.28318530717958647692f; }
template <>
__device__ __forceinline__ double two_pi<double>() { return 6.28318530717958647692; }

__device__ __forceinline__ bool range_ok(float r) { return r > 0.0f && r <= 3.402823466e38f; }

// Ray direction of row `rw` (cos phi, sin phi, cos theta, sin theta) at encoder
// angle (ca, sa): d = (cos phi cos(a + theta), cos phi sin(a + theta), sin phi).
template <typename T>
__device__ __forceinline__ V3<T> ray_dir(V4<T> rw, T ca, T sa)
{
    T cal = ca * rw.z - sa * rw.w;
    T sal = sa * rw.z + ca * rw.w;
    return {rw.x * cal, rw.x * sal, rw.y};
}

// The tables one pyramid level needs, copied out of SensorTab into
// registers once per tile: the per-pixel code then never re-reads the table
// descriptor (which, living in global memory next to the kernel's stores,
// the compiler could not keep in registers).
template <typename T>
struct LevelView {
    const T *row, *col;               // full-resolution factors of Eq. (1)
    const T *mu, *uoff;               // this level's midpoints and column offsets
    const int32_t *bins;
    const SensorTab<T> *tab;          // everything else (receiver-offset search)
    T r0, s_lo, s_hi, kW, bin_lo, bin_scale;
    int Hl, Wl, nb;
};

template <typename T>
__device__ __forceinline__ LevelView<T> level_view(const SensorTab<T> &S, int l)
{
    LevelView<T> V;
    V.row = S.row;
    V.col = S.col;
    V.mu = S.mu[l];
    V.uoff = S.uoff[l];
    V.bins = S.bins[l];
    V.tab = &S;
    V.r0 = S.r0;
    V.s_lo = S.s_lo;
    V.s_hi = S.s_hi;
    V.kW = S.kW[l];
    V.bin_lo = S.bin_lo[l];
    V.bin_scale = S.bin_scale[l];
    V.Hl = S.H >> l;
    V.Wl = S.W >> l;
    V.nb = S.nbins[l];
    return V;
}

// Eq. (1): p = r d(u, v) + r0 (cos a_u, sin a_u, 0) for full-resolution pixel (u, v).
template <typename T>
__device__ __forceinline__ V3<T> unproject(const T *row, const T *col, T r0, int u, int v, T r)
{
    V4<T> rw = ld4(row + 4 * v);
    T ca, sa;
    ld2(col + 2 * u, ca, sa);
    V3<T> d = ray_dir(rw, ca, sa);
    return {r * d.x + r0 * ca, r * d.y + r0 * sa, r * d.z};
}
template <typename T>
__device__ __forceinline__ V3<T> unproject(const SensorTab<T> &S, int u, int v, T r)
{
    return unproject(S.row, S.col, S.r0, u, v, r);
}
template <typename T>
__device__ __forceinline__ V3<T> unproject(const LevelView<T> &V, int u, int v, T r)
{
    return unproject(V.row, V.col, V.r0, u, v, r);
}

// Eq. (4) on sz = sin(phi) over a level's rows: the row t whose elevation is
// nearest (ties to the smaller t), i.e. the number of level midpoints
// strictly above phi.  The inverse table gives a start row; the two bounded
// walks make the result exact whatever the bin rounding.
template <typename T>
__device__ __forceinline__ int elev_index(const T *mu, const int32_t *bins, T bin_lo, T bin_scale, int nb, int Hl,
                                          T sz)
{
    if (Hl <= 1)
        return 0;
    T f = (sz - bin_lo) * bin_scale;
    const T fmaxb = (T)(nb - 1);
    f = f >= (T)0 ? f : (T)0;  // also maps NaN to bin 0
    f = f < fmaxb ? f : fmaxb;
    int v = bins[(int)f];
    while (v < Hl - 1 && mu[v] > sz)
        ++v;
    while (v > 0 && mu[v - 1] <= sz)
        --v;
    return v;
}

// Eq. (3)-(4) at the view's level.  With r0 > 0 the receiver offset is
// compensated exactly (Sec. 3.2 iterates towards the same fixed point): for
// beam v the ray leaving the receiver at encoder angle a reaches p iff, seen
// from the axis, p = r0 (cos a, sin a) + t (cos(a + th_v), sin(a + th_v))
// horizontally, so t = sqrt(rho^2 - r0^2 sin^2 th_v) - r0 cos th_v
// (rho = |p_xy|) and the ray azimuth is atan2(p_y, p_x) - atan2(t sin th_v,
// r0 + t cos th_v) + th_v; only the beam index is iterated (it changes only
// near an elevation midpoint).  Points within 2 r0 of the axis do not
// project.  Then the range, the elevation row by the inverse table and the
// column from the azimuth minus the row's offset, rounded half up and wrapped
// (Sec. 4.1: continuous geometry at the finest level, nearest strided row and
// column).  Returns false outside the elevation field of view or at r = 0.
template <typename T>
__device__ __forceinline__ bool project(const LevelView<T> &V, T x, T y, T z, int &ul, int &vl, T &r)
{
    T r2, th;
    if (V.r0 > (T)0) {
        const SensorTab<T> &S = *V.tab;
        const T *mu0 = S.mu[0], *theta = S.theta;
        const int32_t *bins0 = S.bins[0];
        const T lo0 = S.bin_lo[0], sc0 = S.bin_scale[0];
        const int nb0 = S.nbins[0], H = S.H;
        const T r0 = V.r0, rho2 = x * x + y * y, z2 = z * z;
        if (!(rho2 > (T)4 * r0 * r0))
            return false;
        T t = sqrt(rho2 - r0 * r0);
        int v = elev_index(mu0, bins0, lo0, sc0, nb0, H, z * d_rsqrt(t * t + z2));
        T cth = (T)1, sth = (T)0;
        for (int k = 0; k < 4; ++k) {
            cth = V.row[4 * v + 2];
            sth = V.row[4 * v + 3];
            t = sqrt(rho2 - r0 * r0 * sth * sth) - r0 * cth;
            if (k == 3)
                break;
            const int vn = elev_index(mu0, bins0, lo0, sc0, nb0, H, z * d_rsqrt(t * t + z2));
            if (vn == v)
                break;
            v = vn;
        }
        r2 = t * t + z2;
        th = d_atan2(y, x) - d_atan2(t * sth, r0 + t * cth) + theta[v];
        if (th < (T)0)
            th += two_pi<T>();
        if (th < (T)0)
            th += two_pi<T>();
        if (th >= two_pi<T>())
            th -= two_pi<T>();
    } else {
        r2 = x * x + y * y + z * z;
        th = d_atan2(y, x);
        if (th < (T)0)
            th += two_pi<T>();
    }
    if (!(r2 > (T)0))
        return false;
    const T rinv = d_rsqrt(r2);
    const T sz = z * rinv;
    if (!(sz <= V.s_hi && sz >= V.s_lo))
        return false;
    const int v = elev_index(V.mu, V.bins, V.bin_lo, V.bin_scale, V.nb, V.Hl, sz);
    const int Wl = V.Wl;
    T uh = th * V.kW - V.uoff[v];
    if (uh < (T)0)
        uh += (T)Wl;
    if (uh >= (T)Wl)
        uh -= (T)Wl;
    int u = (int)floor(uh + (T)0.5);
    if (u >= Wl)
        u -= Wl;
    ul = u;
    vl = v;
    r = r2 * rinv;
    return true;
}

// Normal of level-0 pixel (u, v) from the range image (Sec. 4.1, Sec. 6.1):
// n = (P(u+1,v) - P(u-1,v)) x (P(u,v+1) - P(u,v-1)), u wrapping, oriented to
// face the sensor.  Both differences are formed without cancellation from
// the factored tables: P(+) - P(-) = (r+ - r-)(d+ + d-)/2 + (r+ + r-)(d+ - d-)/2
// (+ r0 (c+ - c-) along u), with d+ - d- in product (half-angle) form.  The
// validity predicate is evaluated in FP64 on the FP32 ranges.  Returns false
// (and leaves n untouched) for invalid pixels.
template <typename T>
struct NormalView {
    const T *row, *col, *nrow;
    T r0, cos_h, sin_h;
    int H, W;
};

template <typename T>
__device__ __forceinline__ NormalView<T> normal_view(const SensorTab<T> &S)
{
    return NormalView<T>{S.row, S.col, S.nrow, S.r0, S.cos_h, S.sin_h, S.H, S.W};
}

template <typename T>
__device__ __forceinline__ bool normal_at(const NormalView<T> &S, const float *rng, int u, int v, double edge_rel,
                                          V3<T> &n)
{
    const int H = S.H, W = S.W;
    if (v <= 0 || v >= H - 1)
        return false;
    const int ul = u == 0 ? W - 1 : u - 1;
    const int ur = u == W - 1 ? 0 : u + 1;
    const size_t row = (size_t)v * W;
    const float rc = rng[row + u], rl = rng[row + ul], rr = rng[row + ur];
    const float ru = rng[row - W + u], rd = rng[row + W + u];
    if (!(range_ok(rc) && range_ok(rl) && range_ok(rr) && range_ok(ru) && range_ok(rd)))
        return false;
    const double lim = edge_rel * (double)rc;
    const double dc = (double)rc;
    if (fabs((double)rl - dc) > lim || fabs((double)rr - dc) > lim || fabs((double)ru - dc) > lim ||
        fabs((double)rd - dc) > lim)
        return false;
    T ca, sa;
    ld2(S.col + 2 * u, ca, sa);
    // along u (same row): d+ + d- = 2 (cphi cos h cos al, cphi cos h sin al, sphi),
    // d+ - d- = 2 cphi sin h (-sin al, cos al, 0), c+ - c- = 2 sin h (-sa, ca, 0)
    V4<T> rw = ld4(S.row + 4 * v);
    T cal = ca * rw.z - sa * rw.w, sal = sa * rw.z + ca * rw.w;
    T dh = (T)rr - (T)rl, sh = (T)rr + (T)rl;
    T k1 = dh * rw.x * S.cos_h, k2 = sh * rw.x * S.sin_h, k3 = (T)2 * S.r0 * S.sin_h;
    V3<T> A = {k1 * cal - k2 * sal - k3 * sa, k1 * sal + k2 * cal + k3 * ca, dh * rw.y};
    // along v (same column)
    V4<T> rp = ld4(S.row + 4 * (v + 1)), rm = ld4(S.row + 4 * (v - 1));
    V3<T> dp = ray_dir(rp, ca, sa), dm = ray_dir(rm, ca, sa);
    V4<T> f0 = ld4(S.nrow + 8 * v), f1 = ld4(S.nrow + 8 * v + 4);
    T s_p = sa * f0.x + ca * f0.y, c_p = ca * f0.x - sa * f0.y;
    T s_m = sa * f0.z + ca * f0.w, c_m = ca * f0.z - sa * f0.w;
    V3<T> dd = {-s_m * f1.y - s_p * f1.x, c_p * f1.x + c_m * f1.y, f1.z};
    T dv = (T)rd - (T)ru, sv = (T)0.5 * ((T)rd + (T)ru);
    T hv = (T)0.5 * dv;
    V3<T> B = {hv * (dp.x + dm.x) + sv * dd.x, hv * (dp.y + dm.y) + sv * dd.y, hv * (dp.z + dm.z) + sv * dd.z};
    V3<T> c = {A.y * B.z - A.z * B.y, A.z * B.x - A.x * B.z, A.x * B.y - A.y * B.x};
    T n2 = c.x * c.x + c.y * c.y + c.z * c.z;
    if (!(n2 > (T)1e-24))
        return false;
    T inv = d_rsqrt(n2);
    c.x *= inv;
    c.y *= inv;
    c.z *= inv;
    V3<T> d = ray_dir(rw, ca, sa);
    if (c.x * d.x + c.y * d.y + c.z * d.z > (T)0) {
        c.x = -c.x;
        c.y = -c.y;
        c.z = -c.z;
    }
    n = c;
    return true;
}

}  // namespace rir
