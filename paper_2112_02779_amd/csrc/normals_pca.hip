// Target normals by principal component analysis of a pixel window (the
// eigen-decomposition estimator that Dong et al. name in Sec. 4.1 next to the
// neighbour cross product), for batches of range images on gfx950.
//
// The window's points are unprojected (Eq. (1)) from the FP64 sensor tables
// (once per point and tile, into shared memory) and accumulated relative to
// the centre point in FP64: the covariance of a planar patch has a smallest eigenvalue many
// orders of magnitude below the largest, which FP32 sums could not resolve.
// The smallest eigenpair comes from the closed-form (trigonometric)
// eigenvalues of the symmetric 3x3 matrix and the largest cross product of
// two rows of A - lambda I.  MI355X runs FP64 vector arithmetic at half the
// FP32 rate, and the kernel is bound by that arithmetic, not by HBM.
#include "rir_ops.h"

namespace rir {

namespace {

// Smallest and middle eigenvalue of the symmetric matrix
// [[a00 a01 a02] [a01 a11 a12] [a02 a12 a22]] (and the largest), with a unit
// eigenvector of the smallest.  Returns false if no row pair of A - l0 I
// spans a plane (every eigenvalue equal).
__device__ __forceinline__ bool smallest_eigenpair(double a00, double a01, double a02, double a11, double a12,
                                                   double a22, double &l0, double &l1, double &l2, double n[3])
{
    const double q = (a00 + a11 + a22) / 3.0;
    const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
    const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
    const double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * p1;
    if (!(p2 > 0.0)) {
        l0 = l1 = l2 = q;
        return false;
    }
    const double p = sqrt(p2 / 6.0);
    // det(A - q I) / (2 p^3) = cos(3 phi)
    const double det = b00 * (b11 * b22 - a12 * a12) - a01 * (a01 * b22 - a12 * a02) + a02 * (a01 * a12 - b11 * a02);
    double r = det / (2.0 * p * p * p);
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    const double phi = acos(r) / 3.0;
    l2 = q + 2.0 * p * cos(phi);
    l0 = q + 2.0 * p * cos(phi + 2.0943951023931954923);   // + 2 pi / 3
    l1 = 3.0 * q - l0 - l2;
    // eigenvector of l0: orthogonal to every row of A - l0 I
    const double m00 = a00 - l0, m11 = a11 - l0, m22 = a22 - l0;
    const double c01[3] = {a01 * a12 - a02 * m11, a02 * a01 - m00 * a12, m00 * m11 - a01 * a01};
    const double c02[3] = {a01 * m22 - a02 * a12, a02 * a02 - m00 * m22, m00 * a12 - a01 * a02};
    const double c12[3] = {m11 * m22 - a12 * a12, a12 * a02 - a01 * m22, a01 * a12 - m11 * a02};
    const double s01 = c01[0] * c01[0] + c01[1] * c01[1] + c01[2] * c01[2];
    const double s02 = c02[0] * c02[0] + c02[1] * c02[1] + c02[2] * c02[2];
    const double s12 = c12[0] * c12[0] + c12[1] * c12[1] + c12[2] * c12[2];
    const double *c = c01;
    double s = s01;
    if (s02 > s) {
        c = c02;
        s = s02;
    }
    if (s12 > s) {
        c = c12;
        s = s12;
    }
    if (!(s > 0.0))
        return false;
    const double inv = 1.0 / sqrt(s);
    n[0] = c[0] * inv;
    n[1] = c[1] * inv;
    n[2] = c[2] * inv;
    return true;
}

}  // namespace

// The normal from the window sums about the centre point (sx.. = sums of
// q = p - pc, sxx.. of its products, cnt points): covariance about the mean,
// smallest eigenpair, the middle-eigenvalue test (a line has no normal), the
// normal turned to face the sensor.  Returns false (n untouched) if none.
template <int HALF>
__device__ __forceinline__ bool pca_from_sums(const SensorTab<double> &S, int u, int v, int cnt, double sx, double sy,
                                              double sz, double sxx, double sxy, double sxz, double syy, double syz,
                                              double szz, double n[3])
{
    constexpr int K = 2 * HALF + 1;
    constexpr int kMinPts = (K * K + 1) / 2;
    if (cnt < kMinPts)
        return false;
    const double ic = 1.0 / (double)cnt;
    const double mx = sx * ic, my = sy * ic, mz = sz * ic;
    double l0, l1, l2, m[3];
    bool ok = smallest_eigenpair(sxx * ic - mx * mx, sxy * ic - mx * my, sxz * ic - mx * mz, syy * ic - my * my,
                                 syz * ic - my * mz, szz * ic - mz * mz, l0, l1, l2, m);
    // points on a line (middle eigenvalue negligible) have no normal
    ok = ok && l1 > 1e-6 * l2;
    if (!ok)
        return false;
    V4<double> rw = ld4(S.row + 4 * v);
    double ca, sa;
    ld2(S.col + 2 * u, ca, sa);
    const V3<double> d = ray_dir(rw, ca, sa);
    const double sgn = m[0] * d.x + m[1] * d.y + m[2] * d.z > 0.0 ? -1.0 : 1.0;
    n[0] = sgn * m[0];
    n[1] = sgn * m[1];
    n[2] = sgn * m[2];
    return true;
}

// PCA normal of pixel (u, v) of one H x W range image: the covariance of the
// window points (2 HALF + 1 square, u wrapping, rows clipped) that have a
// return within edge_rel of the centre range, about their mean, in FP64;
// at least half the window must take part, the middle eigenvalue must
// exceed 1e-6 times the largest (a line has no normal); the normal faces the
// sensor.  Returns false (n untouched) otherwise.
template <int HALF>
__device__ __forceinline__ bool pca_normal(const SensorTab<double> &S, const float *rg, int H, int W, int u, int v,
                                           double edge_rel, double n[3])
{
    const float rcf = rg[(int64_t)v * W + u];
    if (!range_ok(rcf))
        return false;
    const double rc = (double)rcf, lim = edge_rel * rc;
    const V3<double> pc = unproject(S, u, v, rc);
    double sx = 0, sy = 0, sz = 0, sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
    int cnt = 0;
#pragma unroll
    for (int dv = -HALF; dv <= HALF; ++dv) {
        const int vv = v + dv;
        if (vv < 0 || vv >= H)
            continue;
#pragma unroll
        for (int du = -HALF; du <= HALF; ++du) {
            int uu = u + du;
            uu = uu < 0 ? uu + W : (uu >= W ? uu - W : uu);
            const float rf = rg[(int64_t)vv * W + uu];
            if (!range_ok(rf) || fabs((double)rf - rc) > lim)
                continue;
            const V3<double> p = unproject(S, uu, vv, (double)rf);
            const double qx = p.x - pc.x, qy = p.y - pc.y, qz = p.z - pc.z;
            sx += qx;
            sy += qy;
            sz += qz;
            sxx += qx * qx;
            sxy += qx * qy;
            sxz += qx * qz;
            syy += qy * qy;
            syz += qy * qz;
            szz += qz * qz;
            ++cnt;
        }
    }
    return pca_from_sums<HALF>(S, u, v, cnt, sx, sy, sz, sxx, sxy, sxz, syy, syz, szz, n);
}

// Tile of the PCA-normal kernel: 32 columns x 8 rows of one image per
// workgroup.  The tile's points and a HALF-pixel halo (u wrapping) are
// unprojected once into shared memory, so each point is formed once instead
// of once per window it falls in; the sums, the eigenpair and the tests are
// those of pca_normal, on the same FP64 points, in the same order.
constexpr int kPcaTileW = 32, kPcaTileH = 8;

template <int HALF>
__global__ __launch_bounds__(256) void k_normals_pca(SensorTab<double> S, const float *range, double edge_rel,
                                                     float *nrm, uint8_t *valid)
{
    constexpr int PW = kPcaTileW + 2 * HALF, PH = kPcaTileH + 2 * HALF;
    __shared__ double s_x[PH * PW], s_y[PH * PW], s_z[PH * PW];
    __shared__ float s_r[PH * PW];
    const int H = S.H, W = S.W;
    const int64_t HW = (int64_t)H * W;
    const int64_t img = blockIdx.z;
    const float *rg = range + img * HW;
    const int u0 = blockIdx.x * kPcaTileW, v0 = blockIdx.y * kPcaTileH;
    for (int k = threadIdx.x; k < PH * PW; k += blockDim.x) {
        const int r = k / PW, c = k - r * PW;
        const int vv = v0 - HALF + r;
        const int uu = ((u0 - HALF + c) % W + W) % W;
        float rf = 0.f;
        double x = 0.0, y = 0.0, z = 0.0;
        if (vv >= 0 && vv < H) {
            rf = rg[(int64_t)vv * W + uu];
            if (range_ok(rf)) {
                const V3<double> p = unproject(S, uu, vv, (double)rf);
                x = p.x;
                y = p.y;
                z = p.z;
            }
        }
        s_r[k] = rf;
        s_x[k] = x;
        s_y[k] = y;
        s_z[k] = z;
    }
    __syncthreads();
    const int tx = (int)threadIdx.x % kPcaTileW, ty = (int)threadIdx.x / kPcaTileW;
    const int u = u0 + tx, v = v0 + ty;
    if (u >= W || v >= H)
        return;
    const int64_t i = img * HW + (int64_t)v * W + u;
    const int ci = (ty + HALF) * PW + tx + HALF;
    const float rcf = s_r[ci];
    double n[3] = {0.0, 0.0, 0.0};
    bool ok = false;
    if (range_ok(rcf)) {
        const double rc = (double)rcf, lim = edge_rel * rc;
        const double pcx = s_x[ci], pcy = s_y[ci], pcz = s_z[ci];
        double sx = 0, sy = 0, sz = 0, sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
        int cnt = 0;
#pragma unroll
        for (int dv = -HALF; dv <= HALF; ++dv) {
            const int vv = v + dv;
            if (vv < 0 || vv >= H)
                continue;
#pragma unroll
            for (int du = -HALF; du <= HALF; ++du) {
                const int k = ci + dv * PW + du;
                const float rf = s_r[k];
                if (!range_ok(rf) || fabs((double)rf - rc) > lim)
                    continue;
                const double qx = s_x[k] - pcx, qy = s_y[k] - pcy, qz = s_z[k] - pcz;
                sx += qx;
                sy += qy;
                sz += qz;
                sxx += qx * qx;
                sxy += qx * qy;
                sxz += qx * qz;
                syy += qy * qy;
                syz += qy * qz;
                szz += qz * qz;
                ++cnt;
            }
        }
        ok = pca_from_sums<HALF>(S, u, v, cnt, sx, sy, sz, sxx, sxy, sxz, syy, syz, szz, n);
    }
    nrm[3 * i] = ok ? (float)n[0] : 0.f;
    nrm[3 * i + 1] = ok ? (float)n[1] : 0.f;
    nrm[3 * i + 2] = ok ? (float)n[2] : 0.f;
    valid[i] = ok ? 1 : 0;
}

// Level-0 target records of the registration from PCA normals (the
// alternative estimator of Sec. 4.1): record (n, n . q) with n the FP64 PCA
// normal rounded to T and q the target point from the T tables (as the
// cross-product prepass forms it); (0, 0, 0, NaN) where there is no normal.
// Grid: (pixel blocks, pair).
template <typename T, int HALF>
__global__ __launch_bounds__(256) void k_pca_records(PrepArgs a)
{
    const PairDesc<T> *P = reinterpret_cast<const PairDesc<T> *>(a.pairs) + a.pair_base + blockIdx.y;
    const int H = cload(&P->H), W = cload(&P->W), npx = H * W;
    const SensorTab<double> *Sd = cload(&P->tabd);
    const SensorTab<T> *S = cload(&P->tab);
    const float *rg = cload(&P->dstr[0]);
    T *d40 = cload(&P->dst4[0]);
    const T *rowt = cload(&S->row), *colt = cload(&S->col);
    const T r0 = cload(&S->r0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += gridDim.x * blockDim.x) {
        const int v = i / W, u = i - v * W;
        double n[3];
        V4<T> rec = {(T)0, (T)0, (T)0, quiet_nan<T>()};
        if (pca_normal<HALF>(*Sd, rg, H, W, u, v, a.edge_rel, n)) {
            const V4<T> rw = ld4(rowt + 4 * v);
            T ca, sa;
            ld2(colt + 2 * u, ca, sa);
            const V3<T> d = ray_dir(rw, ca, sa);
            const T rc = (T)rg[i];
            const T q0 = rc * d.x + r0 * ca, q1 = rc * d.y + r0 * sa, q2 = rc * d.z;
            const T n0 = (T)n[0], n1 = (T)n[1], n2 = (T)n[2];
            rec = V4<T>{n0, n1, n2, n0 * q0 + n1 * q1 + n2 * q2};
        }
        st4(d40 + 4 * (size_t)i, rec);
    }
}

template <typename T>
static hipError_t launch_pca_records_t(const PrepArgs &a, int half, int n_pairs, int max_px, hipStream_t stream)
{
    int64_t g = ((int64_t)max_px + 255) / 256;
    const dim3 grid((unsigned)(g > 65535 ? 65535 : (g < 1 ? 1 : g)), (unsigned)n_pairs);
    switch (half) {
    case 1:
        hipLaunchKernelGGL((k_pca_records<T, 1>), grid, dim3(256), 0, stream, a);
        break;
    case 2:
        hipLaunchKernelGGL((k_pca_records<T, 2>), grid, dim3(256), 0, stream, a);
        break;
    case 3:
        hipLaunchKernelGGL((k_pca_records<T, 3>), grid, dim3(256), 0, stream, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pca_records(bool fp64, const PrepArgs &a, int half, int n_pairs, int max_px, hipStream_t stream)
{
    return fp64 ? launch_pca_records_t<double>(a, half, n_pairs, max_px, stream)
                : launch_pca_records_t<float>(a, half, n_pairs, max_px, stream);
}

hipError_t launch_normals_pca(const SensorTab<double> &S, const float *range, int n_images, int half, double edge_rel,
                              float *nrm, uint8_t *valid, hipStream_t stream)
{
    if (half < 1 || half > 3)
        return hipErrorInvalidValue;
    const int64_t hw = (int64_t)S.H * S.W;
    const dim3 block(kPcaTileW * kPcaTileH);
    // images in launches of at most 65535 (the grid's third dimension)
    for (int k0 = 0; k0 < n_images; k0 += 65535) {
        const int nb = n_images - k0 < 65535 ? n_images - k0 : 65535;
        const dim3 grid((unsigned)((S.W + kPcaTileW - 1) / kPcaTileW),
                        (unsigned)((S.H + kPcaTileH - 1) / kPcaTileH), (unsigned)nb);
        const float *r = range + hw * k0;
        float *nm = nrm + 3 * hw * k0;
        uint8_t *vd = valid + hw * k0;
        if (half == 1)
            hipLaunchKernelGGL(k_normals_pca<1>, grid, block, 0, stream, S, r, edge_rel, nm, vd);
        else if (half == 2)
            hipLaunchKernelGGL(k_normals_pca<2>, grid, block, 0, stream, S, r, edge_rel, nm, vd);
        else
            hipLaunchKernelGGL(k_normals_pca<3>, grid, block, 0, stream, S, r, edge_rel, nm, vd);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace rir
