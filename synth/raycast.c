/*
 * Ray caster for synthetic spinning-LiDAR scans (seeded input generation).
 *
 * This file simulates how a spinning scanner forms a scan: the head turns to
 * encoder angle a = 2*pi*u/W, the receiver sits at radius r0 on the head's x
 * axis, and beam v leaves it with azimuth offset theta_v and elevation phi_v
 * relative to the head.  Each ray is intersected with a scene made of
 * infinite planes, axis-aligned boxes and vertical capped cylinders; the
 * output is the distance along the ray to the first hit.
 *
 * It is input generation only.  It contains no projection, association,
 * normal estimation, pyramid or Gauss-Newton arithmetic, and it is used by
 * the test oracle and the GPU library alike.  Noise, dropouts and spurious
 * returns are added by the Python wrapper with numpy's seeded generator.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define NO_HIT 1e300

static double hit_plane(const double o[3], const double d[3], const double *pl)
{
    double den = pl[0] * d[0] + pl[1] * d[1] + pl[2] * d[2];
    if (fabs(den) < 1e-300)
        return NO_HIT;
    double t = -(pl[0] * o[0] + pl[1] * o[1] + pl[2] * o[2] + pl[3]) / den;
    return t > 0.0 ? t : NO_HIT;
}

/* Slab test against [lo, hi]. */
static double hit_box(const double o[3], const double d[3], const double *b)
{
    double t0 = -1e300, t1 = 1e300;
    for (int i = 0; i < 3; ++i) {
        double lo = b[i], hi = b[3 + i];
        if (d[i] == 0.0) {
            if (o[i] < lo || o[i] > hi)
                return NO_HIT;
            continue;
        }
        double inv = 1.0 / d[i];
        double a = (lo - o[i]) * inv, c = (hi - o[i]) * inv;
        if (a > c) { double s = a; a = c; c = s; }
        if (a > t0) t0 = a;
        if (c < t1) t1 = c;
        if (t0 > t1)
            return NO_HIT;
    }
    if (t0 > 0.0)
        return t0;
    return NO_HIT; /* origin inside the box or box behind the ray */
}

/* Vertical cylinder: centre (cx, cy), radius rad, between heights z0 < z1,
 * with flat caps. */
static double hit_cyl(const double o[3], const double d[3], const double *c)
{
    double cx = c[0], cy = c[1], rad = c[2], z0 = c[3], z1 = c[4];
    double best = NO_HIT;
    double ox = o[0] - cx, oy = o[1] - cy;
    double A = d[0] * d[0] + d[1] * d[1];
    if (A > 1e-300) {
        double B = ox * d[0] + oy * d[1];
        double C = ox * ox + oy * oy - rad * rad;
        double disc = B * B - A * C;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double t = (-B - sq) / A;
            if (t <= 0.0)
                t = (-B + sq) / A;
            if (t > 0.0) {
                double z = o[2] + t * d[2];
                if (z >= z0 && z <= z1)
                    best = t;
            }
        }
    }
    if (d[2] != 0.0) {
        const double zc[2] = {z0, z1};
        for (int k = 0; k < 2; ++k) {
            double t = (zc[k] - o[2]) / d[2];
            if (t > 0.0 && t < best) {
                double x = ox + t * d[0], y = oy + t * d[1];
                if (x * x + y * y <= rad * rad)
                    best = t;
            }
        }
    }
    return best;
}

/*
 * Cast every ray of an H x W scan taken from sensor pose T (4x4 row-major,
 * world <- sensor).  phi[H], theta[H] in radians; theta may be NULL (all 0).
 * planes: n_pl x 4 (a, b, c, d with a x + b y + c z + d = 0)
 * boxes:  n_box x 6 (xmin, ymin, zmin, xmax, ymax, zmax)
 * cyls:   n_cyl x 5 (cx, cy, radius, zmin, zmax)
 * range_out[H*W]: distance along the ray to the nearest hit, 0 if none.
 * synth_raycast_posed with per_column = 1 takes W poses (T[16 u ...]), one per
 * column: a sensor that moves while it sweeps.
 * hit_out[H*W]: index of the primitive hit (planes first, then boxes, then
 * cylinders), -1 if none.
 */
void synth_raycast_posed(int H, int W, const double *phi, const double *theta, double r0,
                         const double *T, int per_column, int n_pl, const double *planes, int n_box,
                         const double *boxes, int n_cyl, const double *cyls,
                         double *range_out, int32_t *hit_out)
{
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(dynamic, 1)
    for (int v = 0; v < H; ++v) {
        double cph = cos(phi[v]), sph = sin(phi[v]);
        double th = theta ? theta[v] : 0.0;
        for (int u = 0; u < W; ++u) {
            const double *Tu = per_column ? T + 16 * (size_t)u : T;
            double a = two_pi * (double)u / (double)W;
            /* receiver on the head, and the beam direction: head rotation
             * a + theta_v about z applied to the elevation vector */
            double os[3] = {r0 * cos(a), r0 * sin(a), 0.0};
            double az = a + th;
            double ds[3] = {cph * cos(az), cph * sin(az), sph};
            double o[3], d[3];
            for (int i = 0; i < 3; ++i) {
                o[i] = Tu[4 * i + 0] * os[0] + Tu[4 * i + 1] * os[1] + Tu[4 * i + 2] * os[2] + Tu[4 * i + 3];
                d[i] = Tu[4 * i + 0] * ds[0] + Tu[4 * i + 1] * ds[1] + Tu[4 * i + 2] * ds[2];
            }
            double best = NO_HIT;
            int32_t id = -1;
            for (int k = 0; k < n_pl; ++k) {
                double t = hit_plane(o, d, planes + 4 * k);
                if (t < best) { best = t; id = k; }
            }
            for (int k = 0; k < n_box; ++k) {
                double t = hit_box(o, d, boxes + 6 * k);
                if (t < best) { best = t; id = n_pl + k; }
            }
            for (int k = 0; k < n_cyl; ++k) {
                double t = hit_cyl(o, d, cyls + 5 * k);
                if (t < best) { best = t; id = n_pl + n_box + k; }
            }
            size_t i = (size_t)v * W + u;
            range_out[i] = best < NO_HIT ? best : 0.0;
            hit_out[i] = best < NO_HIT ? id : -1;
        }
    }
}

void synth_raycast(int H, int W, const double *phi, const double *theta, double r0,
                   const double *T, int n_pl, const double *planes, int n_box,
                   const double *boxes, int n_cyl, const double *cyls,
                   double *range_out, int32_t *hit_out)
{
    synth_raycast_posed(H, W, phi, theta, r0, T, 0, n_pl, planes, n_box, boxes, n_cyl, cyls, range_out, hit_out);
}
