// Device-side sensor tables and per-pixel geometry of the range-image model
// (Dong et al., Sec. 3): unprojection Eq. (1)-(2), projection Eq. (3)-(4) with
// a packed inverse elevation table, and the cross-product normal image
// (Sec. 4.1).  Everything is templated on the arithmetic type T (float or
// double).
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
//  ebin[l] [nbins[l]][4]  inverse elevation table of level l (stride 2^l) over
//               sz = sin(phi): bin b = trunc(clamp((sz - bin_lo) * bin_scale,
//               0, nbins - 1)) evaluated in T, each operation rounded.  Entry:
//               (bits c | (c + k) << 16, m, uoff(c), uoff(c + k)); the row of
//               every sz that falls in the bin is c + k [m > sz] (c midpoints
//               lie above the whole bin, k equal midpoints m inside it),
//               uoff(t) = theta_lut[s t] W / (2 pi s) is that row's column
//               offset.  The host verifies the entry against the exact bin
//               edges in T, so the lookup is exact.
template <typename T>
struct SensorTab {
    int H, W, nlev;
    int nbins[kMaxLevels];
    T r0, s_lo, s_hi, cos_h, sin_h;
    T bin_lo[kMaxLevels], bin_scale[kMaxLevels], kW[kMaxLevels];
    const T *row, *col, *nrow, *theta;
    const T *ebin[kMaxLevels];
};

template <typename T>
struct V3 {
    T x, y, z;
};

template <typename T>
struct V4 {
    T x, y, z, w;
};

// ----------------------------------------------------------------------------- memory access

// Generic-pointer loads (entry points that take caller buffers).
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

// Buffer-resource loads (raw buffers of gfx9): a 128-bit descriptor in scalar
// registers holds base and size, each lane supplies a 32-bit byte offset, and
// the hardware checks it against the size: an access beyond the buffer
// returns zero and touches no memory.  kNoLoad is beyond every buffer the
// library creates (all are below 2 GiB), so masked lanes pass it instead of
// branching.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr uint32_t kNoLoad = 0x80000000u;

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

// Only the 32-bit load builtin is used: the backend merges loads at
// consecutive offsets of one descriptor into 64- and 128-bit loads by itself
// (the vector-returning builtins do not extract their elements correctly with
// this compiler).
__device__ __forceinline__ uint32_t bld_u32(rsrc_t r, uint32_t off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

template <typename T>
__device__ __forceinline__ T bld1(rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float bld1<float>(rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, bld_u32(r, off));
}
template <>
__device__ __forceinline__ double bld1<double>(rsrc_t r, uint32_t off)
{
    const uint64_t lo = bld_u32(r, off), hi = bld_u32(r, off + 4u);
    return __builtin_bit_cast(double, lo | (hi << 32));
}

template <typename T>
__device__ __forceinline__ void bld2(rsrc_t r, uint32_t off, T &a, T &b)
{
    a = bld1<T>(r, off);
    b = bld1<T>(r, off + (uint32_t)sizeof(T));
}

template <typename T>
__device__ __forceinline__ V4<T> bld4(rsrc_t r, uint32_t off)
{
    V4<T> o;
    bld2(r, off, o.x, o.y);
    bld2(r, off + 2u * (uint32_t)sizeof(T), o.z, o.w);
    return o;
}

// Low 32 bits of a table word (the packed counts of an elevation-table entry).
__device__ __forceinline__ uint32_t low_bits(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t low_bits(double x) { return (uint32_t)__builtin_bit_cast(uint64_t, x); }

// Loads of data that no thread of the running kernel writes, at wave-uniform
// addresses: through the constant address space they become scalar loads
// (one per wave, results in scalar registers).  The scalar cache is
// invalidated at every kernel launch, so data written by earlier kernels is
// seen.
template <typename T>
__device__ __forceinline__ T cload(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)p;
}
__device__ __forceinline__ int2 cload(const int2 *p)
{
    const int *q = reinterpret_cast<const int *>(p);
    return make_int2(cload(q), cload(q + 1));
}
template <typename T>
__device__ __forceinline__ V4<T> sld4(const T *p, int idx)
{
    typedef const __attribute__((address_space(4))) T ctype;
    ctype *q = (ctype *)p + 4 * idx;
    return {q[0], q[1], q[2], q[3]};
}

// ----------------------------------------------------------------------------- math

__device__ __forceinline__ float d_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double d_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float d_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double d_rcp(double x) { return 1.0 / x; }
template <typename T>
__device__ __forceinline__ T two_pi();
template <>
__device__ __forceinline__ float two_pi<float>() { return 6.28318530717958647692f; }
template <>
__device__ __forceinline__ double two_pi<double>() { return 6.28318530717958647692; }

// atan2(|y|, x) in [0, pi].  FP32: reduction to t = min(|x|,|y|) / max(|x|,|y|)
// in [0, 1], atan(t) = t P(t^2) with P of degree 6 fitted to atan on [0, 1]
// by iteratively reweighted least squares (near-minimax: 2.6e-7 in exact
// arithmetic, 3.3e-7 evaluated in FP32), then the reflections
// atan(1/t) = pi/2 - atan(t) and atan2(y, -x) = pi - atan2(y, x).  With the
// reciprocal's 1 ulp the result is within 7e-7 rad of the true angle.
// FP64: the library atan2.
__device__ __forceinline__ float atan2_abs(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    // x = y = 0 gives NaN; such a point lies on the axis, outside every
    // elevation field of view, and never projects
    const float t = mn * d_rcp(mx);
    const float t2 = t * t;
    float p = 6.811757572e-03f;
    p = fmaf(p, t2, -3.360411525e-02f);
    p = fmaf(p, t2, 7.962355018e-02f);
    p = fmaf(p, t2, -1.323333532e-01f);
    p = fmaf(p, t2, 1.980781406e-01f);
    p = fmaf(p, t2, -3.331736922e-01f);
    p = fmaf(p, t2, 9.999961257e-01f);
    p *= t;
    p = ay > ax ? 1.57079632679489661923f - p : p;
    return x < 0.f ? 3.14159265358979323846f - p : p;
}
__device__ __forceinline__ double atan2_abs(double y, double x) { return atan2(fabs(y), x); }

// Azimuth of (x, y) in [0, 2 pi] (2 pi only by rounding just below the +x axis).
template <typename T>
__device__ __forceinline__ T azimuth(T y, T x)
{
    const T p = atan2_abs(y, x);
    return y < (T)0 ? two_pi<T>() - p : p;
}

// An angle congruent to the azimuth modulo 2 pi, in [-3 pi / 4, 5 pi / 4]
// (for callers that wrap the column afterwards).  FP32: with
// t = y / x where |y| <= |x| (angle atan(t), plus pi for x < 0) and
// t = -x / y otherwise (angle sign(y) pi / 2 + atan(t)), |t| <= 1 and the
// odd polynomial of atan2_abs gives atan(t); one fused multiply-add adds the
// offset.  FP64: from the library atan2.
__device__ __forceinline__ float azimuth_mod(float y, float x)
{
    const bool steep = fabsf(y) > fabsf(x);
    const float num = steep ? -x : y, den = steep ? y : x;
    const float t = num * d_rcp(den);  // x = y = 0: NaN (never projects)
    const float t2 = t * t;
    float p = 6.811757572e-03f;
    p = fmaf(p, t2, -3.360411525e-02f);
    p = fmaf(p, t2, 7.962355018e-02f);
    p = fmaf(p, t2, -1.323333532e-01f);
    p = fmaf(p, t2, 1.980781406e-01f);
    p = fmaf(p, t2, -3.331736922e-01f);
    p = fmaf(p, t2, 9.999961257e-01f);
    const float off = steep ? copysignf(1.57079632679489661923f, y) : (x < 0.f ? 3.14159265358979323846f : 0.f);
    return fmaf(t, p, off);
}
__device__ __forceinline__ double azimuth_mod(double y, double x) { return copysign(atan2_abs(y, x), y); }

// Half-up rounding to an integer, floor(x + 1/2).  FP32: one conversion
// instruction that rounds this way.
__device__ __forceinline__ int round_half_up(float x)
{
    int i;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(i) : "v"(x));
    return i;
}
__device__ __forceinline__ int round_half_up(double x) { return (int)floor(x + 0.5); }

// r > 0 and finite (a return).  FP32: one class test (positive normal or
// subnormal).
__device__ __forceinline__ bool range_ok(float r) { return __builtin_amdgcn_classf(r, 0x180); }

template <typename T>
__device__ __forceinline__ T quiet_nan();
template <>
__device__ __forceinline__ float quiet_nan<float>() { return __builtin_bit_cast(float, 0x7fc00000u); }
template <>
__device__ __forceinline__ double quiet_nan<double>() { return __builtin_bit_cast(double, 0x7ff8000000000000ull); }

// Ray direction of row `rw` (cos phi, sin phi, cos theta, sin theta) at encoder
// angle (ca, sa): d = (cos phi cos(a + theta), cos phi sin(a + theta), sin phi).
template <typename T>
__device__ __forceinline__ V3<T> ray_dir(V4<T> rw, T ca, T sa)
{
    T cal = ca * rw.z - sa * rw.w;
    T sal = sa * rw.z + ca * rw.w;
    return {rw.x * cal, rw.x * sal, rw.y};
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

// ----------------------------------------------------------------------------- projection

// The tables one pyramid level needs, read out of SensorTab once per tile.
template <typename T>
struct LevelView {
    rsrc_t row, col, ebin;        // full-resolution factors of Eq. (1), this level's elevation table
    const T *rowp;                // row factors for wave-uniform (scalar) reads
    const SensorTab<T> *tab;      // the rest (receiver-offset search), in device memory
    T r0, s_lo, s_hi, kW, bin_lo, bin_scale, bin_max;
    int Hl, Wl;
};

template <typename T>
__device__ __forceinline__ LevelView<T> level_view(const SensorTab<T> *tab, int l)
{
    LevelView<T> V;
    const int H = cload(&tab->H), W = cload(&tab->W), nb = cload(&tab->nbins[l]);
    V.rowp = cload(&tab->row);
    V.row = make_rsrc(V.rowp, (uint32_t)(H * 4 * sizeof(T)));
    V.col = make_rsrc(cload(&tab->col), (uint32_t)(W * 2 * sizeof(T)));
    V.ebin = make_rsrc(cload(&tab->ebin[l]), (uint32_t)(nb * 4 * sizeof(T)));
    V.tab = tab;
    V.r0 = cload(&tab->r0);
    V.s_lo = cload(&tab->s_lo);
    V.s_hi = cload(&tab->s_hi);
    V.kW = cload(&tab->kW[l]);
    V.bin_lo = cload(&tab->bin_lo[l]);
    V.bin_scale = cload(&tab->bin_scale[l]);
    V.bin_max = (T)(nb - 1);
    V.Hl = H >> l;
    V.Wl = W >> l;
    return V;
}

// Eq. (4) on sz = sin(phi): the row of the level whose elevation is nearest
// (ties to the smaller row), i.e. the number of level midpoints strictly above
// phi, from one entry of the packed table; uo receives that row's column
// offset.  The bin is (sz - bin_lo) * bin_scale with both operations rounded
// (never fused: the host builds the table for exactly this formula), clamped
// to [0, bin_max].  NaN falls in some bin (the caller has rejected it
// already).
__device__ __forceinline__ float clamp_bin(float f, float bmax) { return __builtin_amdgcn_fmed3f(f, 0.f, bmax); }
__device__ __forceinline__ double clamp_bin(double f, double bmax)
{
    f = f >= 0.0 ? f : 0.0;
    return f < bmax ? f : bmax;
}
template <typename T>
__device__ __forceinline__ int elev_row(rsrc_t ebin, T bin_lo, T bin_scale, T bin_max, T sz, T &uo)
{
#pragma clang fp contract(off)
    const T d = sz - bin_lo;
    const T f = clamp_bin(d * bin_scale, bin_max);
    const V4<T> E = bld4<T>(ebin, (uint32_t)(int)f * (uint32_t)(4 * sizeof(T)));
    const uint32_t rows = low_bits(E.x);
    const bool below = E.y > sz;
    uo = below ? E.w : E.z;
    return (int)__builtin_amdgcn_ubfe(rows, below ? 16u : 0u, 16u);
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
// column).  Returns false outside the elevation field of view or at r = 0;
// ul, vl and r are then unspecified (but in range).  No early exits: the
// per-pixel path stays free of divergent branches.  R0 = false compiles the
// receiver-offset branch out (callers that know r0 = 0); POW2 = true wraps
// the column with a mask (callers that know Wl is a power of two).
template <typename T, bool R0 = true, bool POW2 = false>
__device__ __forceinline__ bool project(const LevelView<T> &V, T x, T y, T z, int &ul, int &vl, T &r)
{
    T r2, th;
    bool ok = true;
    if (R0 && V.r0 > (T)0) {
        const SensorTab<T> *S = V.tab;
        const int nb0 = cload(&S->nbins[0]);
        const rsrc_t eb0 = make_rsrc(cload(&S->ebin[0]), (uint32_t)(nb0 * 4 * sizeof(T)));
        const rsrc_t thr = make_rsrc(cload(&S->theta), (uint32_t)(cload(&S->H) * sizeof(T)));
        const T lo0 = cload(&S->bin_lo[0]), sc0 = cload(&S->bin_scale[0]), mx0 = (T)(nb0 - 1);
        const T r0 = V.r0, rho2 = x * x + y * y, z2 = z * z;
        ok = rho2 > (T)4 * r0 * r0;
        const T rho2c = ok ? rho2 : (T)4 * r0 * r0;
        T t = sqrt(rho2c - r0 * r0), dummy;
        int v = elev_row(eb0, lo0, sc0, mx0, z * d_rsqrt(t * t + z2), dummy);
        T cth = (T)1, sth = (T)0;
        for (int k = 0; k < 4; ++k) {
            const V4<T> rw = bld4<T>(V.row, (uint32_t)v * (uint32_t)(4 * sizeof(T)));
            cth = rw.z;
            sth = rw.w;
            t = sqrt(rho2c - r0 * r0 * sth * sth) - r0 * cth;
            if (k == 3)
                break;
            const int vn = elev_row(eb0, lo0, sc0, mx0, z * d_rsqrt(t * t + z2), dummy);
            if (vn == v)
                break;
            v = vn;
        }
        r2 = t * t + z2;
        const T ys = t * sth, xs = r0 + t * cth;
        const T off = ys < (T)0 ? -atan2_abs(ys, xs) : atan2_abs(ys, xs);
        th = azimuth(y, x) - off + bld1<T>(thr, (uint32_t)v * (uint32_t)sizeof(T));
        th = th < (T)0 ? th + two_pi<T>() : th;
        th = th < (T)0 ? th + two_pi<T>() : th;
        th = th >= two_pi<T>() ? th - two_pi<T>() : th;
    } else {
        r2 = x * x + y * y + z * z;
        th = azimuth_mod(y, x);
    }
    const T rinv = d_rsqrt(r2);
    const T sz = z * rinv;
    // r2 = 0 or a non-finite point gives a NaN or infinite sz, outside the field
    ok = ok && sz <= V.s_hi && sz >= V.s_lo;
    T uo;
    const int v = elev_row(V.ebin, V.bin_lo, V.bin_scale, V.bin_max, sz, uo);
    // th * kW lies in [-3 Wl / 8, Wl] and |uo| < Wl / 2, so the rounded column
    // is within one image width of [0, Wl): wrap the integer (exact), not the
    // coordinate
    const int Wl = V.Wl;
    const int u = round_half_up(th * V.kW - uo);
    if constexpr (POW2) {
        ul = u & (Wl - 1);
    } else {
        uint32_t uu = (uint32_t)u;
        uu = min(uu, uu + (uint32_t)Wl);
        uu = min(uu, uu - (uint32_t)Wl);
        ul = (int)min(uu, (uint32_t)Wl - 1u);  // NaN inputs only
    }
    vl = v;
    r = r2 * rinv;
    return ok;
}

// ----------------------------------------------------------------------------- normals

// Normal of level-0 pixel (u, v) from the range image (Sec. 4.1, Sec. 6.1):
// n = (P(u+1,v) - P(u-1,v)) x (P(u,v+1) - P(u,v-1)), u wrapping, oriented to
// face the sensor.  Both differences are formed without cancellation from
// the factored tables: P(+) - P(-) = (r+ - r-)(d+ + d-)/2 + (r+ + r-)(d+ - d-)/2
// (+ r0 (c+ - c-) along u), with d+ - d- in product (half-angle) form.  The
// validity predicate (all five ranges valid, none differing from the centre by
// more than edge_rel times the centre range) is evaluated in FP64 on the FP32
// ranges.  Inputs: column factors (ca, sa), the rows v, v+1, v-1 of the row
// table, the two nrow words of row v, and the five ranges.  Returns false (n
// untouched) for invalid pixels; rows 0 and H-1 are the caller's to reject.
template <typename T>
__device__ __forceinline__ bool normal_core(T ca, T sa, V4<T> rw, V4<T> rp, V4<T> rm, V4<T> f0, V4<T> f1, T r0,
                                            T cos_h, T sin_h, float rc, float rl, float rr, float ru, float rd,
                                            double edge_rel, V3<T> &n)
{
    if (!(range_ok(rc) && range_ok(rl) && range_ok(rr) && range_ok(ru) && range_ok(rd)))
        return false;
    const double lim = edge_rel * (double)rc;
    const double dc = (double)rc;
    if (fabs((double)rl - dc) > lim || fabs((double)rr - dc) > lim || fabs((double)ru - dc) > lim ||
        fabs((double)rd - dc) > lim)
        return false;
    // along u (same row): d+ + d- = 2 (cphi cos h cos al, cphi cos h sin al, sphi),
    // d+ - d- = 2 cphi sin h (-sin al, cos al, 0), c+ - c- = 2 sin h (-sa, ca, 0)
    T cal = ca * rw.z - sa * rw.w, sal = sa * rw.z + ca * rw.w;
    T dh = (T)rr - (T)rl, sh = (T)rr + (T)rl;
    T k1 = dh * rw.x * cos_h, k2 = sh * rw.x * sin_h, k3 = (T)2 * r0 * sin_h;
    V3<T> A = {k1 * cal - k2 * sal - k3 * sa, k1 * sal + k2 * cal + k3 * ca, dh * rw.y};
    // along v (same column)
    V3<T> dp = ray_dir(rp, ca, sa), dm = ray_dir(rm, ca, sa);
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

// normal_core for pixel (u, v) of a range image in memory.
template <typename T>
__device__ __forceinline__ bool normal_at(const SensorTab<T> &S, const float *rng, int u, int v, double edge_rel,
                                          V3<T> &n)
{
    const int H = S.H, W = S.W;
    if (v <= 0 || v >= H - 1)
        return false;
    const int ul = u == 0 ? W - 1 : u - 1;
    const int ur = u == W - 1 ? 0 : u + 1;
    const size_t row = (size_t)v * W;
    T ca, sa;
    ld2(S.col + 2 * u, ca, sa);
    return normal_core(ca, sa, ld4(S.row + 4 * v), ld4(S.row + 4 * (v + 1)), ld4(S.row + 4 * (v - 1)),
                       ld4(S.nrow + 8 * v), ld4(S.nrow + 8 * v + 4), S.r0, S.cos_h, S.sin_h, rng[row + u],
                       rng[row + ul], rng[row + ur], rng[row - W + u], rng[row + W + u], edge_rel, n);
}

}  // namespace rir
