/*
 * FP64 CPU oracle for multi-scale projective point-to-plane ICP and projective
 * SDF fusion on cylindrical range images (Dong, Ryu, Kaess, Park: "Revisiting
 * LiDAR Registration and Reconstruction: A Range Image Perspective", Sec. 3,
 * Sec. 4.1 and Sec. 4.2).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or helper with the GPU library and is never called by it.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * Everything is double precision, built with -ffp-contract=off, with no
 * blocking, fusion or reordering beyond what the paper's equations state:
 *   Eq. (1)-(2)  unprojection of pixel (u, v) with range r,
 *   Eq. (3)-(4)  projection with the iterative receiver-offset compensation
 *                and the elevation argmin over the beam table,
 *   Eq. (5)-(6)  projective data association,
 *   Eq. (7)      robust point-to-plane objective solved by Gauss-Newton,
 *   Sec. 4.1     multi-scale registration on strided images with the
 *                original intrinsics,
 *   Eq. (8)-(10) projective signed distances and their running mean at
 *                query points (Sec. 4.2),
 *   Sec. 4.1     PCA normals (the eigen-decomposition alternative),
 *   Sec. 6       re-projection under per-column poses (the outlook's
 *                non-rigid model).
 * Readings of silent or ambiguous passages are listed next to the code that
 * takes them.  The learned per-pixel weight (a small MLP) is not part of the
 * paper; its forward and backward passes are written out here with the same
 * bf16 rounding points the GPU uses, so that the GPU can be checked.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846264338327950288
#define ORC_TWO_PI 6.28318530717958647692528676655900577

enum { ORC_OK = 0, ORC_DEGENERATE = 1, ORC_FALLBACK_HUBER = 2, ORC_NONFINITE = 3 };

/* Sensor intrinsics (Sec. 3): H beams, W columns, per-beam elevation phi[H]
 * (strictly decreasing, v = 0 is the top beam), per-beam azimuth offset
 * theta[H] (NULL means all zero) and receiver radius r0. */
typedef struct {
    int H, W;
    const double *phi;
    const double *theta;
    double r0;
} orc_sensor;

typedef struct {
    int levels;
    int iters[8];          /* Gauss-Newton iterations per level, index 0 = finest */
    double delta;          /* pseudo-Huber kernel size (m) */
    double edge_rel;       /* normal validity: |r_nbr - r_c| <= edge_rel * r_c */
    double max_corr_dist;  /* <= 0: no distance gate */
    int init_mode;         /* 0: given initial pose, 1: align point-set centres */
    int weight_mode;       /* 0: pseudo-Huber, 1: learned */
    const double *mlp;     /* learned-weight parameters (see orc_mlp_*) */
    double r_max;          /* range scale of the first learned feature */
    int learned_levels;    /* weight_mode 1: bit l = learned at level l, 0 = all levels */
    double stop_eps;       /* > 0: a level ends after a step with |xi| <= stop_eps */
    /* Conditioning probe (test infrastructure; all zero for the method itself):
     * with flip_band_u > 0 every association whose rounding is ambiguous --
     * column coordinate within flip_band_u pixels of a half-integer, or
     * elevation within flip_band_phi row spacings of a level midpoint or of
     * a field-of-view edge -- takes the other admissible candidate when a
     * coin drawn from (flip_seed, level, iteration, pixel) says so. */
    double flip_band_u, flip_band_phi;
    uint64_t flip_seed;
    int normal_window;     /* 0: neighbour cross product; h = 1..3: PCA normals of the
                            * (2h+1)^2 window (Sec. 4.1's eigen-decomposition estimator) */
} orc_params;

typedef struct {
    int32_t status, iters_run, n_valid, n_inlier, n_proj, pad;
    double sum_w, sum_w_e2, robust_cost, step_rot, step_trans;
    double JtJ[21], Jtr[6];
} orc_level_stats;

static double th_lut(const orc_sensor *s, int v) { return s->theta ? s->theta[v] : 0.0; }

static int range_ok(double r) { return isfinite(r) && r > 0.0; }

/* ------------------------------------------------------------------ Eq. (1)-(2) */

/* Unprojection Pi^{-1}(u, v, r): the receiver sits on a cylinder of radius r0
 * at encoder angle 2 pi u / W, and the ray leaves it at azimuth
 * theta(u, v) = 2 pi u / W + theta_lut[v] and elevation phi(v) = phi_lut[v]. */
void orc_unproject(const orc_sensor *s, int u, int v, double r, double out[3])
{
    double a = ORC_TWO_PI * (double)u / (double)s->W;
    double th = a + th_lut(s, v);
    double ph = s->phi[v];
    out[0] = r * cos(th) * cos(ph) + s->r0 * cos(a);
    out[1] = r * sin(th) * cos(ph) + s->r0 * sin(a);
    out[2] = r * sin(ph);
}

/* Unit ray direction of pixel (u, v) (the r-coefficient of Eq. (1)). */
static void ray_dir(const orc_sensor *s, int u, int v, double d[3])
{
    double th = ORC_TWO_PI * (double)u / (double)s->W + th_lut(s, v);
    double ph = s->phi[v];
    d[0] = cos(th) * cos(ph);
    d[1] = sin(th) * cos(ph);
    d[2] = sin(ph);
}

void orc_normals_pca(const orc_sensor *s, const float *range, int half, double edge_rel, double *nrm,
                     uint8_t *valid, double *lam);

/* Target normal image of the registration: the neighbour cross product, or
 * with normal_window = h > 0 the PCA normals of the (2h+1)^2 window, the
 * alternative estimator Sec. 4.1 names. */
static void target_normals(const orc_sensor *s, const float *dst, const orc_params *prm, double *nrm, uint8_t *nv);

/* ------------------------------------------------------------------ Eq. (3)-(4) */

static double atan2_wrapped(double y, double x)
{
    /* arctan2 lands in [-pi, pi]; the paper wraps it to [0, 2 pi] (Sec. 3.2 footnote) */
    double a = atan2(y, x);
    if (a < 0.0)
        a += ORC_TWO_PI;
    return a;
}

/* Eq. (4): v = argmin_t |phi_lut[t] - phi| over the rows 0, s, 2s, ... of the
 * table (s = 1 at the finest level); ties go to the smaller index.  Returns
 * the level row index t. */
static int elevation_argmin(const orc_sensor *s, int stride, double phi)
{
    int Hl = s->H / stride;
    int best = 0;
    double bd = fabs(s->phi[0] - phi);
    for (int t = 1; t < Hl; ++t) {
        double d = fabs(s->phi[t * stride] - phi);
        if (d < bd) {
            bd = d;
            best = t;
        }
    }
    return best;
}

typedef struct {
    int32_t valid, u, v, pad;
    double r, uhat, phi, theta;
} orc_proj;

/*
 * Projection Pi at pyramid level `level` (stride s = 2^level), Eq. (3)-(4).
 *
 * Readings (the paper is brief here):
 *  - Receiver-offset compensation: starting from the azimuth of (x, y), the
 *    encoder angle a is refined by rounds of: remove the receiver offset
 *    r0 (cos a, sin a, 0), re-estimate the ray azimuth and elevation, take the
 *    finest-level beam v_k by Eq. (4), and set a = theta - theta_lut[v_k],
 *    repeated until a stops changing (|change| <= 1e-15 rad, at most 100
 *    rounds).  The paper omits theta_lut while iterating; including it makes
 *    the fixed point the exact inverse of Eq. (1).  With r0 = 0 no round is
 *    needed.
 *  - Level indices (Sec. 4.1, "projective transforms at the finest level,
 *    down-sampled on coordinates at the given stride"): v_l is the Eq. (4)
 *    argmin over the strided rows s*t; u_hat_l = W/(2 pi) (theta -
 *    theta_lut[s v_l]) / s wrapped to [0, W/s) and u_l = floor(u_hat_l + 1/2)
 *    mod W/s (round half up).
 *  - Validity (the paper skips the boundary check for clarity): r > 0 and the
 *    elevation lies within half a row spacing beyond the end rows of the
 *    finest table.  With r0 > 0 the point must also lie farther than 2 r0
 *    from the sensor axis: the compensation assumes r0 << r, has no fixed
 *    point inside the receiver circle, and beyond 2 r0 contracts at least
 *    twofold per round, so it converges.
 */
void orc_project(const orc_sensor *s, int level, const double x[3], orc_proj *out)
{
    int stride = 1 << level;
    int Wl = s->W / stride;
    double xp = x[0], yp = x[1], z = x[2];
    out->valid = 0;
    out->u = out->v = -1;
    out->r = sqrt(xp * xp + yp * yp + z * z);
    out->uhat = out->phi = out->theta = 0.0;
    if (s->r0 > 0.0 && !(xp * xp + yp * yp > 4.0 * s->r0 * s->r0))
        return;
    if (s->r0 > 0.0) {
        double a = atan2_wrapped(x[1], x[0]);
        for (int k = 0; k < 100; ++k) {
            xp = x[0] - s->r0 * cos(a);
            yp = x[1] - s->r0 * sin(a);
            double thk = atan2_wrapped(yp, xp);
            double rk = sqrt(xp * xp + yp * yp + z * z);
            double sk = rk > 0.0 ? z / rk : 0.0;
            if (sk > 1.0) sk = 1.0;
            if (sk < -1.0) sk = -1.0;
            int vk = elevation_argmin(s, 1, asin(sk));
            double an = thk - th_lut(s, vk);
            double change = fabs(an - a);
            if (change > ORC_PI)
                change = ORC_TWO_PI - change;
            a = an;
            if (change <= 1e-15)
                break;
        }
        xp = x[0] - s->r0 * cos(a);
        yp = x[1] - s->r0 * sin(a);
    }
    double r = sqrt(xp * xp + yp * yp + z * z);
    out->r = r;
    out->valid = 0;
    out->u = out->v = -1;
    out->uhat = out->phi = out->theta = 0.0;
    if (!(r > 0.0))
        return;
    double sz = z / r;
    if (sz > 1.0) sz = 1.0;
    if (sz < -1.0) sz = -1.0;
    double phi = asin(sz);
    double theta = atan2_wrapped(yp, xp);
    out->phi = phi;
    out->theta = theta;
    int H = s->H;
    double phi_hi = s->phi[0] + 0.5 * (s->phi[0] - s->phi[1]);
    double phi_lo = s->phi[H - 1] - 0.5 * (s->phi[H - 2] - s->phi[H - 1]);
    int vl = elevation_argmin(s, stride, phi);
    double uh = (theta - th_lut(s, vl * stride)) * (double)s->W / ORC_TWO_PI / (double)stride;
    uh = uh - (double)Wl * floor(uh / (double)Wl);
    int ul = (int)floor(uh + 0.5);
    if (ul >= Wl)
        ul -= Wl;
    out->uhat = uh;
    out->u = ul;
    out->v = vl;
    out->valid = (phi <= phi_hi && phi >= phi_lo) ? 1 : 0;
}

/* Batch helpers used by the tests. */
void orc_unproject_image(const orc_sensor *s, const float *range, double *xyz, uint8_t *valid)
{
    for (int v = 0; v < s->H; ++v)
        for (int u = 0; u < s->W; ++u) {
            size_t i = (size_t)v * s->W + u;
            double r = range[i];
            valid[i] = (uint8_t)range_ok(r);
            if (valid[i])
                orc_unproject(s, u, v, r, xyz + 3 * i);
            else
                xyz[3 * i] = xyz[3 * i + 1] = xyz[3 * i + 2] = 0.0;
        }
}

void orc_project_points(const orc_sensor *s, int level, const double *xyz, int64_t n, int32_t *u,
                        int32_t *v, double *r, double *uhat, double *phi, uint8_t *valid)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_proj p;
        orc_project(s, level, xyz + 3 * i, &p);
        u[i] = p.u;
        v[i] = p.v;
        r[i] = p.r;
        uhat[i] = p.uhat;
        phi[i] = p.phi;
        valid[i] = (uint8_t)p.valid;
    }
}

/* ------------------------------------------------------------------ normal image */

/*
 * Target normals by the cross product of neighbour-pixel differences
 * (Sec. 4.1 forms the normal from two neighbouring pixels by a cross
 * product; Sec. 6.1 notes the normal map comes straight from the range
 * image).
 *
 * Readings: central differences n = (P(u+1,v) - P(u-1,v)) x (P(u,v+1) -
 * P(u,v-1)); u wraps around the cylinder, v does not (rows 0 and H-1 are
 * invalid); a pixel is valid iff its own and its four neighbours' ranges are
 * finite and positive and each neighbour differs from the centre by at most
 * edge_rel times the centre range; |n|^2 <= 1e-24 is invalid; n is oriented
 * towards the sensor (n . d <= 0 for the pixel's ray direction d).
 */
void orc_normals(const orc_sensor *s, const float *range, double edge_rel, double *nrm, uint8_t *valid)
{
    int H = s->H, W = s->W;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t i = (size_t)v * W + u;
            valid[i] = 0;
            nrm[3 * i] = nrm[3 * i + 1] = nrm[3 * i + 2] = 0.0;
            if (v == 0 || v == H - 1)
                continue;
            int ul = (u + W - 1) % W, ur = (u + 1) % W;
            double rc = range[i];
            double rl = range[(size_t)v * W + ul], rr = range[(size_t)v * W + ur];
            double ru = range[(size_t)(v - 1) * W + u], rd = range[(size_t)(v + 1) * W + u];
            if (!range_ok(rc) || !range_ok(rl) || !range_ok(rr) || !range_ok(ru) || !range_ok(rd))
                continue;
            double lim = edge_rel * rc;
            if (fabs(rl - rc) > lim || fabs(rr - rc) > lim || fabs(ru - rc) > lim || fabs(rd - rc) > lim)
                continue;
            double pl[3], pr[3], pu[3], pd[3];
            orc_unproject(s, ul, v, rl, pl);
            orc_unproject(s, ur, v, rr, pr);
            orc_unproject(s, u, v - 1, ru, pu);
            orc_unproject(s, u, v + 1, rd, pd);
            double a[3] = {pr[0] - pl[0], pr[1] - pl[1], pr[2] - pl[2]};
            double b[3] = {pd[0] - pu[0], pd[1] - pu[1], pd[2] - pu[2]};
            double n[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
            double n2 = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
            if (!(n2 > 1e-24))
                continue;
            double inv = 1.0 / sqrt(n2);
            n[0] *= inv;
            n[1] *= inv;
            n[2] *= inv;
            double d[3];
            ray_dir(s, u, v, d);
            if (n[0] * d[0] + n[1] * d[1] + n[2] * d[2] > 0.0) {
                n[0] = -n[0];
                n[1] = -n[1];
                n[2] = -n[2];
            }
            nrm[3 * i] = n[0];
            nrm[3 * i + 1] = n[1];
            nrm[3 * i + 2] = n[2];
            valid[i] = 1;
        }
}

/* ------------------------------------------------------------------ learned weight (not in the paper) */

/* Round a double to the nearest bfloat16 value (ties to even), via float. */
double orc_bf16(double x)
{
    float f = (float)x;
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) {
        /* inf / nan pass through (nan kept quiet) */
        if (b & 0x007fffffu)
            b |= 0x00400000u;
        b &= 0xffff0000u;
    } else {
        uint32_t lsb = (b >> 16) & 1u;
        b += 0x7fffu + lsb;
        b &= 0xffff0000u;
    }
    memcpy(&f, &b, 4);
    return (double)f;
}

/* Parameter layout (5185 doubles): W1[64][14], b1[64], W2[64][64], b2[64], W3[64], b3. */
#define MLP_IN 14
#define MLP_H 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H * MLP_IN)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_H)
#define MLP_NPARAM (OFF_B3 + 1)

int orc_mlp_nparam(void) { return MLP_NPARAM; }

/*
 * Forward pass of the 14-64-64-1 weight network for one feature vector.
 * Rounding points shared with the GPU: the inputs f, and the hidden
 * activations h1 and h2 after ReLU, are rounded to bfloat16; the weights are
 * given as their exact bfloat16 values; everything else is exact FP64 here.
 * Returns the logit z; the weight is sigmoid(z).
 */
static double mlp_forward1(const double *P, const double *f_in, double *fb, double *a1, double *h1,
                           double *a2, double *h2)
{
    for (int k = 0; k < MLP_IN; ++k)
        fb[k] = orc_bf16(f_in[k]);
    for (int j = 0; j < MLP_H; ++j) {
        double acc = P[OFF_B1 + j];
        for (int k = 0; k < MLP_IN; ++k)
            acc += P[OFF_W1 + j * MLP_IN + k] * fb[k];
        a1[j] = acc;
        h1[j] = orc_bf16(acc > 0.0 ? acc : 0.0);
    }
    for (int j = 0; j < MLP_H; ++j) {
        double acc = P[OFF_B2 + j];
        for (int k = 0; k < MLP_H; ++k)
            acc += P[OFF_W2 + j * MLP_H + k] * h1[k];
        a2[j] = acc;
        h2[j] = orc_bf16(acc > 0.0 ? acc : 0.0);
    }
    double z = P[OFF_B3];
    for (int k = 0; k < MLP_H; ++k)
        z += P[OFF_W3 + k] * h2[k];
    return z;
}

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

void orc_mlp_forward(const double *P, const float *feats, int64_t B, double *z_out, double *w_out)
{
    double f[MLP_IN], fb[MLP_IN], a1[MLP_H], h1[MLP_H], a2[MLP_H], h2[MLP_H];
    for (int64_t b = 0; b < B; ++b) {
        for (int k = 0; k < MLP_IN; ++k)
            f[k] = feats[b * MLP_IN + k];
        double z = mlp_forward1(P, f, fb, a1, h1, a2, h2);
        if (z_out)
            z_out[b] = z;
        if (w_out)
            w_out[b] = sigmoid(z);
    }
}

/*
 * The hidden pre-activations a1 = W1 bf16(f) + b1 and a2 = W2 h1 + b2 of each
 * feature vector (B x 64 each, exact FP64 sums of the exact bf16 products),
 * and the magnitude sums s1 = |W1| |bf16(f)| + |b1|, s2 = |W2| h1 + |b2| that
 * bound the rounding error of any FP32 evaluation of the same sums.  Test
 * infrastructure for deciding which rows an FP32 implementation can round to
 * another bf16 activation than the FP64 forward pass (a value within that
 * rounding of a bf16 tie).
 */
void orc_mlp_preact(const double *P, const float *feats, int64_t B, double *a1_out, double *a2_out,
                    double *s1_out, double *s2_out)
{
    double f[MLP_IN], fb[MLP_IN], a1[MLP_H], h1[MLP_H], a2[MLP_H], h2[MLP_H];
    for (int64_t b = 0; b < B; ++b) {
        for (int k = 0; k < MLP_IN; ++k)
            f[k] = feats[b * MLP_IN + k];
        mlp_forward1(P, f, fb, a1, h1, a2, h2);
        for (int j = 0; j < MLP_H; ++j) {
            double s1 = fabs(P[OFF_B1 + j]), s2 = fabs(P[OFF_B2 + j]);
            for (int k = 0; k < MLP_IN; ++k)
                s1 += fabs(P[OFF_W1 + j * MLP_IN + k] * fb[k]);
            for (int k = 0; k < MLP_H; ++k)
                s2 += fabs(P[OFF_W2 + j * MLP_H + k] * h1[k]);
            a1_out[b * MLP_H + j] = a1[j];
            a2_out[b * MLP_H + j] = a2[j];
            s1_out[b * MLP_H + j] = s1;
            s2_out[b * MLP_H + j] = s2;
        }
    }
}

/*
 * Mean binary cross-entropy of sigmoid(z) against labels y in {0, 1}, and its
 * gradient with respect to every parameter (layout as above).
 * Backward rounding points shared with the GPU: the output delta
 * dz = (sigmoid(z) - y) / B and the hidden deltas (after the ReLU mask,
 * ReLU'(0) = 0) are rounded to bfloat16 before they multiply activations or
 * weights; bias gradients are sums of those rounded deltas.
 */
double orc_mlp_loss_grad(const double *P, const float *feats, const float *labels, int64_t B, double *grad)
{
    double f[MLP_IN], fb[MLP_IN], a1[MLP_H], h1[MLP_H], a2[MLP_H], h2[MLP_H];
    double g2[MLP_H], g1[MLP_H];
    memset(grad, 0, sizeof(double) * MLP_NPARAM);
    double loss = 0.0;
    for (int64_t b = 0; b < B; ++b) {
        for (int k = 0; k < MLP_IN; ++k)
            f[k] = feats[b * MLP_IN + k];
        double z = mlp_forward1(P, f, fb, a1, h1, a2, h2);
        double y = labels[b];
        /* BCE(sigmoid(z), y) = log(1 + e^z) - y z, written stably */
        double sp = z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z));
        loss += sp - y * z;
        double dz = orc_bf16((sigmoid(z) - y) / (double)B);
        for (int k = 0; k < MLP_H; ++k)
            grad[OFF_W3 + k] += dz * h2[k];
        grad[OFF_B3] += dz;
        for (int j = 0; j < MLP_H; ++j) {
            double d = a2[j] > 0.0 ? P[OFF_W3 + j] * dz : 0.0;
            g2[j] = orc_bf16(d);
        }
        for (int j = 0; j < MLP_H; ++j) {
            for (int k = 0; k < MLP_H; ++k)
                grad[OFF_W2 + j * MLP_H + k] += g2[j] * h1[k];
            grad[OFF_B2 + j] += g2[j];
        }
        for (int k = 0; k < MLP_H; ++k) {
            double acc = 0.0;
            for (int j = 0; j < MLP_H; ++j)
                acc += P[OFF_W2 + j * MLP_H + k] * g2[j];
            g1[k] = orc_bf16(a1[k] > 0.0 ? acc : 0.0);
        }
        for (int j = 0; j < MLP_H; ++j) {
            for (int k = 0; k < MLP_IN; ++k)
                grad[OFF_W1 + j * MLP_IN + k] += g1[j] * fb[k];
            grad[OFF_B1 + j] += g1[j];
        }
    }
    return loss / (double)B;
}

/* ------------------------------------------------------------------ SE(3) */

static void skew(const double w[3], double K[9])
{
    K[0] = 0.0;   K[1] = -w[2]; K[2] = w[1];
    K[3] = w[2];  K[4] = 0.0;   K[5] = -w[0];
    K[6] = -w[1]; K[7] = w[0];  K[8] = 0.0;
}

static void mat3_mul(const double *A, const double *B, double *C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

/* Exponential map of a twist xi = (omega, tau) to a 4x4 row-major rigid
 * transform: Rodrigues' rotation and t = V tau with
 * V = I + (1 - cos a)/a^2 K + (a - sin a)/a^3 K^2, a = |omega|, K = [omega]x.
 * Taylor coefficients below a = 1e-6. */
void orc_exp_se3(const double xi[6], double T[16])
{
    const double *w = xi, *tau = xi + 3;
    double a2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double a = sqrt(a2);
    double A, Bc, C;
    if (a < 1e-6) {
        A = 1.0 - a2 / 6.0;
        Bc = 0.5 - a2 / 24.0;
        C = 1.0 / 6.0 - a2 / 120.0;
    } else {
        A = sin(a) / a;
        Bc = (1.0 - cos(a)) / a2;
        C = (a - sin(a)) / (a2 * a);
    }
    double K[9], K2[9];
    skew(w, K);
    mat3_mul(K, K, K2);
    double R[9], V[9];
    for (int i = 0; i < 9; ++i) {
        double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + A * K[i] + Bc * K2[i];
        V[i] = I + Bc * K[i] + C * K2[i];
    }
    memset(T, 0, 16 * sizeof(double));
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            T[4 * i + j] = R[3 * i + j];
        T[4 * i + 3] = V[3 * i] * tau[0] + V[3 * i + 1] * tau[1] + V[3 * i + 2] * tau[2];
    }
    T[15] = 1.0;
}

static void mat4_mul(const double *A, const double *B, double *C)
{
    double tmp[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k)
                acc += A[4 * i + k] * B[4 * k + j];
            tmp[4 * i + j] = acc;
        }
    memcpy(C, tmp, sizeof(tmp));
}

/* Registration error metrics (Sec. 6.1), read with the trace and an
 * unsquared norm: e_R = arccos((tr(R R_ref^T) - 1) / 2), e_t = |t - t_ref|. */
void orc_pose_error(const double T[16], const double Tref[16], double *e_rot, double *e_trans)
{
    double tr = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            tr += T[4 * i + k] * Tref[4 * i + k];
    double c = (tr - 1.0) / 2.0;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    *e_rot = acos(c);
    double dx = T[3] - Tref[3], dy = T[7] - Tref[7], dz = T[11] - Tref[11];
    *e_trans = sqrt(dx * dx + dy * dy + dz * dz);
}

/* ------------------------------------------------------------------ Eq. (5)-(7) */

/* Pseudo-Huber robust kernel (Barron's general kernel with alpha = 1), the
 * kernel of the paper's experiments (Sec. 6.1): rho(e) = d^2 (sqrt(1 +
 * (e/d)^2) - 1); the IRLS weight is rho'(e) / e = (1 + (e/d)^2)^(-1/2). */
static double huber_weight(double e, double d) { return 1.0 / sqrt(1.0 + (e / d) * (e / d)); }
static double huber_cost(double e, double d) { return d * d * (sqrt(1.0 + (e / d) * (e / d)) - 1.0); }

static double clamp4(double x) { return x < -4.0 ? -4.0 : (x > 4.0 ? 4.0 : x); }

/* Per-pixel output of one association pass. */
typedef struct {
    int32_t *u, *v;       /* level indices of the association (or -1) */
    uint8_t *mask;        /* 1: valid correspondence */
    uint8_t *proj_valid;  /* 1: the source pixel projected inside the image */
    double *e, *w, *J;    /* residual, weight, Jacobian row [6] */
    double *uhat, *phi;   /* continuous column and elevation (for tie analysis) */
    float *feat;          /* learned-weight features [14] or NULL */
} orc_assoc_out;

/*
 * Learned-weight features of a correspondence (not in the paper; a reading of
 * "3x3 range patch + normal + residual"): f0 = range at the associated
 * target pixel / r_max; f1..f8 = clamp((neighbour - centre) / delta, -4, 4)
 * for the 8 level-l neighbours of the associated target pixel in raster order,
 * u wrapping and rows outside the image or neighbours without a return
 * reading +4; f9..f11 = target normal; f12 = clamp(e / delta, -4, 4);
 * f13 = clamp((target range - projected range) / delta, -4, 4), the
 * projective signed distance of Eq. (8)-(9).
 */
static void features(const orc_sensor *s, int level, const float *dst, int ul, int vl, double rproj,
                     const double n[3], double e, double delta, double r_max, double f[14])
{
    int st = 1 << level, Wl = s->W / st, Hl = s->H / st;
    double rc = dst[(size_t)(st * vl) * s->W + st * ul];
    f[0] = rc / r_max;
    int k = 1;
    for (int dv = -1; dv <= 1; ++dv)
        for (int du = -1; du <= 1; ++du) {
            if (du == 0 && dv == 0)
                continue;
            int vv = vl + dv, uu = (ul + du + Wl) % Wl;
            double val = 4.0;
            if (vv >= 0 && vv < Hl) {
                double rn = dst[(size_t)(st * vv) * s->W + st * uu];
                if (range_ok(rn))
                    val = clamp4((rn - rc) / delta);
            }
            f[k++] = val;
        }
    f[9] = n[0];
    f[10] = n[1];
    f[11] = n[2];
    f[12] = clamp4(e / delta);
    f[13] = clamp4((rc - rproj) / delta);
}

/* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the output function applied to a counter. */
static uint64_t splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Conditioning probe: replaces an ambiguous rounding decision of a
 * projection by the other admissible one, each decision (column, row,
 * field-of-view edge) on its own coin.  The band is the one inside which the
 * parity bar accepts either neighbour, so a result that moves beyond its
 * tolerance under these flips is not fixed by the decisions the bar
 * prescribes. */
static void flip_ambiguous(const orc_sensor *s, int level, const orc_params *prm, uint64_t key, orc_proj *pr)
{
    int st = 1 << level, Wl = s->W / st, Hl = s->H / st, H = s->H;
    double phi = pr->phi;
    uint64_t c = splitmix64(key);
    /* elevation: the nearest level midpoint and the field-of-view edges */
    double gap_top = s->phi[0] - s->phi[1], gap_bot = s->phi[H - 2] - s->phi[H - 1];
    double edge_gap = gap_top < gap_bot ? gap_top : gap_bot;
    double phi_hi = s->phi[0] + 0.5 * gap_top, phi_lo = s->phi[H - 1] - 0.5 * gap_bot;
    if ((fabs(phi - phi_hi) < prm->flip_band_phi * edge_gap || fabs(phi - phi_lo) < prm->flip_band_phi * edge_gap) &&
        (c & 1))
        pr->valid = !pr->valid;
    int v = pr->v;
    int nb = phi > s->phi[st * v] ? v - 1 : v + 1; /* neighbour across the nearest midpoint */
    if (nb >= 0 && nb < Hl) {
        double mid = 0.5 * (s->phi[st * v] + s->phi[st * nb]);
        double gap = fabs(s->phi[st * v] - s->phi[st * nb]);
        if (fabs(phi - mid) < prm->flip_band_phi * gap && (c & 2))
            v = nb;
    }
    if (v != pr->v) {
        double uh = (pr->theta - th_lut(s, v * st)) * (double)s->W / ORC_TWO_PI / (double)st;
        uh = uh - (double)Wl * floor(uh / (double)Wl);
        pr->uhat = uh;
        pr->v = v;
        pr->u = (int)floor(uh + 0.5) % Wl;
    }
    /* column: the other side of the nearest half-integer */
    double fr = pr->uhat - floor(pr->uhat);
    if (fabs(fr - 0.5) < prm->flip_band_u && (c & 4)) {
        int alt = fr < 0.5 ? (int)floor(pr->uhat) + 1 : (int)floor(pr->uhat);
        pr->u = ((alt % Wl) + Wl) % Wl;
    }
}

/*
 * Projective data association at level l (Eq. (5)-(6)) and per-pixel
 * residual, Jacobian and weight for Eq. (7) at pose T (dst <- src).
 * Source pixel (u', v') of level l is full-resolution pixel (s u', s v').
 * A correspondence is rejected when the source has no return, the projection
 * is invalid, the target pixel has no return or no valid normal, or (if
 * enabled) |x - q| exceeds max_corr_dist.
 * e = n^T (x - q); J = [(x cross n)^T, n^T] is de/dxi for the left update
 * x <- Exp(xi) x with xi = (omega, tau).
 */
void orc_associate(const orc_sensor *s, int level, const float *src, const float *dst, const double *nrm,
                   const uint8_t *nvalid, const double T[16], const orc_params *prm, int use_learned,
                   orc_assoc_out *out)
{
    int st = 1 << level, Wl = s->W / st, Hl = s->H / st;
    for (int vp = 0; vp < Hl; ++vp)
        for (int up = 0; up < Wl; ++up) {
            size_t o = (size_t)vp * Wl + up;
            out->u[o] = out->v[o] = -1;
            out->mask[o] = 0;
            out->proj_valid[o] = 0;
            out->e[o] = out->w[o] = 0.0;
            for (int k = 0; k < 6; ++k)
                out->J[6 * o + k] = 0.0;
            out->uhat[o] = out->phi[o] = 0.0;
            if (out->feat)
                for (int k = 0; k < 14; ++k)
                    out->feat[14 * o + k] = 0.0f;
            double rs = src[(size_t)(st * vp) * s->W + st * up];
            if (!range_ok(rs))
                continue;
            double p[3], x[3];
            orc_unproject(s, st * up, st * vp, rs, p);
            for (int i = 0; i < 3; ++i)
                x[i] = T[4 * i] * p[0] + T[4 * i + 1] * p[1] + T[4 * i + 2] * p[2] + T[4 * i + 3];
            orc_proj pr;
            orc_project(s, level, x, &pr);
            out->uhat[o] = pr.uhat;
            out->phi[o] = pr.phi;
            if (prm->flip_band_u > 0.0 && pr.r > 0.0 && pr.v >= 0)
                flip_ambiguous(s, level, prm, prm->flip_seed ^ ((uint64_t)o * 0xD1B54A32D192ED03ull), &pr);
            if (!pr.valid)
                continue;
            out->proj_valid[o] = 1;
            out->u[o] = pr.u;
            out->v[o] = pr.v;
            size_t di = (size_t)(st * pr.v) * s->W + st * pr.u;
            double rd = dst[di];
            if (!range_ok(rd) || !nvalid[di])
                continue;
            const double *n = nrm + 3 * di;
            double q[3];
            orc_unproject(s, st * pr.u, st * pr.v, rd, q);
            double dx[3] = {x[0] - q[0], x[1] - q[1], x[2] - q[2]};
            if (prm->max_corr_dist > 0.0 &&
                sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]) > prm->max_corr_dist)
                continue;
            double e = n[0] * dx[0] + n[1] * dx[1] + n[2] * dx[2];
            double *J = out->J + 6 * o;
            J[0] = x[1] * n[2] - x[2] * n[1];
            J[1] = x[2] * n[0] - x[0] * n[2];
            J[2] = x[0] * n[1] - x[1] * n[0];
            J[3] = n[0];
            J[4] = n[1];
            J[5] = n[2];
            out->mask[o] = 1;
            out->e[o] = e;
            double w;
            if (use_learned) {
                double f[14];
                features(s, level, dst, pr.u, pr.v, pr.r, n, e, prm->delta, prm->r_max, f);
                float ff[14];
                for (int k = 0; k < 14; ++k)
                    ff[k] = (float)f[k];
                if (out->feat)
                    memcpy(out->feat + 14 * o, ff, sizeof(ff));
                double z;
                orc_mlp_forward(prm->mlp, ff, 1, &z, &w);
            } else {
                w = huber_weight(e, prm->delta);
                if (out->feat) {
                    double f[14];
                    features(s, level, dst, pr.u, pr.v, pr.r, n, e, prm->delta, prm->r_max, f);
                    for (int k = 0; k < 14; ++k)
                        out->feat[14 * o + k] = (float)f[k];
                }
            }
            out->w[o] = w;
        }
}

/* Weighted normal equations of Eq. (7) from per-pixel terms:
 * H = sum w J J^T (21 upper entries, row-major), g = sum w J e, plus the
 * residual statistics of the pass. */
static void accumulate(int n, const orc_assoc_out *a, double delta, double Hm[36], double g[6],
                       orc_level_stats *st)
{
    memset(Hm, 0, 36 * sizeof(double));
    memset(g, 0, 6 * sizeof(double));
    st->n_valid = st->n_inlier = st->n_proj = 0;
    st->sum_w = st->sum_w_e2 = st->robust_cost = 0.0;
    for (int o = 0; o < n; ++o) {
        st->n_proj += a->proj_valid[o];
        if (!a->mask[o])
            continue;
        const double *J = a->J + 6 * o;
        double w = a->w[o], e = a->e[o];
        for (int i = 0; i < 6; ++i) {
            for (int j = 0; j < 6; ++j)
                Hm[6 * i + j] += w * J[i] * J[j];
            g[i] += w * J[i] * e;
        }
        st->n_valid += 1;
        st->n_inlier += fabs(e) < delta ? 1 : 0;
        st->sum_w += w;
        st->sum_w_e2 += w * e * e;
        st->robust_cost += huber_cost(e, delta);
    }
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j)
            st->JtJ[k++] = Hm[6 * i + j];
    for (int i = 0; i < 6; ++i)
        st->Jtr[i] = g[i];
}

/* Cholesky solve of H xi = -g.  Fails (returns 0) when a pivot is not above
 * 1e-12 times the largest diagonal entry. */
static int cholesky_solve(const double Hm[36], const double g[6], double xi[6])
{
    double L[36] = {0};
    double dmax = 0.0;
    for (int i = 0; i < 6; ++i)
        if (Hm[7 * i] > dmax)
            dmax = Hm[7 * i];
    if (!(dmax > 0.0))
        return 0;
    for (int j = 0; j < 6; ++j) {
        double d = Hm[7 * j];
        for (int k = 0; k < j; ++k)
            d -= L[6 * j + k] * L[6 * j + k];
        if (!(d > 1e-12 * dmax))
            return 0;
        L[7 * j] = sqrt(d);
        for (int i = j + 1; i < 6; ++i) {
            double acc = Hm[6 * i + j];
            for (int k = 0; k < j; ++k)
                acc -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = acc / L[7 * j];
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double acc = -g[i];
        for (int k = 0; k < i; ++k)
            acc -= L[6 * i + k] * y[k];
        y[i] = acc / L[7 * i];
    }
    for (int i = 5; i >= 0; --i) {
        double acc = y[i];
        for (int k = i + 1; k < 6; ++k)
            acc -= L[6 * k + i] * xi[k];
        xi[i] = acc / L[7 * i];
    }
    return 1;
}

static int all_finite(const double *a, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(a[i]))
            return 0;
    return 1;
}

typedef struct {
    orc_assoc_out a;
    void *mem;
} assoc_buf;

static int assoc_alloc(assoc_buf *b, size_t n)
{
    size_t bytes = n * (10 * sizeof(double) + 2 * sizeof(int32_t) + 2);
    char *m = (char *)malloc(bytes > 0 ? bytes : 1);
    if (!m)
        return 0;
    b->mem = m;
    b->a.e = (double *)m; m += n * sizeof(double);
    b->a.w = (double *)m; m += n * sizeof(double);
    b->a.J = (double *)m; m += 6 * n * sizeof(double);
    b->a.uhat = (double *)m; m += n * sizeof(double);
    b->a.phi = (double *)m; m += n * sizeof(double);
    b->a.u = (int32_t *)m; m += n * sizeof(int32_t);
    b->a.v = (int32_t *)m; m += n * sizeof(int32_t);
    b->a.mask = (uint8_t *)m; m += n;
    b->a.proj_valid = (uint8_t *)m;
    b->a.feat = NULL;
    return 1;
}

/*
 * Multi-scale projective ICP (Sec. 4.1).  For levels l = L-1 down to 0 and
 * iters[l] Gauss-Newton iterations each: associate (Eq. (5)-(6)), build the
 * weighted normal equations of Eq. (7), solve by Cholesky, and update
 * T <- Exp(xi) T.  A level stops early (status DEGENERATE) when fewer than 6
 * correspondences remain or the Cholesky pivot test fails.  With learned
 * weights, an iteration whose weights sum below 0.1 n_valid or whose system
 * fails is redone with pseudo-Huber weights (status FALLBACK_HUBER).
 * The statistics of a level are those of its last evaluated iteration.
 *
 * Initial pose: T_init as given, or (init_mode 1) R = I and t = mean of the
 * valid target points minus mean of the valid source points (Sec. 4.1).
 * Returns 0 on success, -1 on an allocation failure.
 */
int orc_icp(const orc_sensor *s, const float *src, const float *dst, const orc_params *prm,
            const double T_init[16], double T_out[16], orc_level_stats *stats)
{
    int H = s->H, W = s->W;
    size_t N = (size_t)H * W;
    double *nrm = (double *)malloc(3 * N * sizeof(double));
    uint8_t *nv = (uint8_t *)malloc(N);
    assoc_buf ab;
    if (!nrm || !nv || !assoc_alloc(&ab, N)) {
        free(nrm);
        free(nv);
        return -1;
    }
    target_normals(s, dst, prm, nrm, nv);
    double T[16];
    memcpy(T, T_init, sizeof(T));
    if (prm->init_mode == 1) {
        double cs[3] = {0}, cd[3] = {0}, p[3];
        size_t ns = 0, nd = 0;
        for (int v = 0; v < H; ++v)
            for (int u = 0; u < W; ++u) {
                size_t i = (size_t)v * W + u;
                if (range_ok(src[i])) {
                    orc_unproject(s, u, v, src[i], p);
                    cs[0] += p[0]; cs[1] += p[1]; cs[2] += p[2];
                    ns++;
                }
                if (range_ok(dst[i])) {
                    orc_unproject(s, u, v, dst[i], p);
                    cd[0] += p[0]; cd[1] += p[1]; cd[2] += p[2];
                    nd++;
                }
            }
        memset(T, 0, sizeof(T));
        T[0] = T[5] = T[10] = T[15] = 1.0;
        if (ns > 0 && nd > 0)
            for (int i = 0; i < 3; ++i)
                T[4 * i + 3] = cd[i] / (double)nd - cs[i] / (double)ns;
    }
    for (int l = prm->levels - 1; l >= 0; --l) {
        int st = 1 << l;
        int n = (H / st) * (W / st);
        orc_level_stats *ls = &stats[l];
        memset(ls, 0, sizeof(*ls));
        for (int it = 0; it < prm->iters[l]; ++it) {
            double Hm[36], g[6], xi[6];
            int learned = prm->weight_mode == 1 && (prm->learned_levels == 0 || ((prm->learned_levels >> l) & 1));
            orc_params pit = *prm; /* the probe's coins differ per level and iteration */
            pit.flip_seed = splitmix64(prm->flip_seed + (uint64_t)(l * 4096 + it));
            orc_associate(s, l, src, dst, nrm, nv, T, &pit, learned, &ab.a);
            accumulate(n, &ab.a, prm->delta, Hm, g, ls);
            ls->iters_run = it + 1;
            ls->status = ORC_OK;
            int ok = ls->n_valid >= 6 && all_finite(Hm, 36) && all_finite(g, 6) && cholesky_solve(Hm, g, xi);
            if (learned && (!ok || ls->sum_w < 0.1 * ls->n_valid)) {
                orc_associate(s, l, src, dst, nrm, nv, T, &pit, 0, &ab.a);
                accumulate(n, &ab.a, prm->delta, Hm, g, ls);
                ok = ls->n_valid >= 6 && all_finite(Hm, 36) && all_finite(g, 6) && cholesky_solve(Hm, g, xi);
                ls->status = ORC_FALLBACK_HUBER;
            }
            if (!ok) {
                ls->status = (all_finite(Hm, 36) && all_finite(g, 6)) ? ORC_DEGENERATE : ORC_NONFINITE;
                ls->step_rot = ls->step_trans = 0.0;
                break;
            }
            double D[16];
            orc_exp_se3(xi, D);
            mat4_mul(D, T, T);
            ls->step_rot = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
            ls->step_trans = sqrt(xi[3] * xi[3] + xi[4] * xi[4] + xi[5] * xi[5]);
            /* optional small-step stop (a fixed iteration count when 0) */
            if (prm->stop_eps > 0.0 &&
                ls->step_rot * ls->step_rot + ls->step_trans * ls->step_trans <= prm->stop_eps * prm->stop_eps)
                break;
        }
    }
    memcpy(T_out, T, sizeof(T));
    free(nrm);
    free(nv);
    free(ab.mem);
    return 0;
}

/* One association + normal-equation pass at a fixed pose, for the tests:
 * writes the per-pixel terms and the level statistics (JtJ, Jtr, counts). */
int orc_system(const orc_sensor *s, int level, const float *src, const float *dst, const orc_params *prm,
               const double T[16], int use_learned, int32_t *u, int32_t *v, uint8_t *mask, uint8_t *proj_valid,
               double *e, double *w, double *J, double *uhat, double *phi, float *feat, orc_level_stats *st)
{
    size_t N = (size_t)s->H * s->W;
    int sd = 1 << level;
    int n = (s->H / sd) * (s->W / sd);
    double *nrm = (double *)malloc(3 * N * sizeof(double));
    uint8_t *nv = (uint8_t *)malloc(N);
    if (!nrm || !nv) {
        free(nrm);
        free(nv);
        return -1;
    }
    target_normals(s, dst, prm, nrm, nv);
    orc_assoc_out a = {u, v, mask, proj_valid, e, w, J, uhat, phi, feat};
    orc_associate(s, level, src, dst, nrm, nv, T, prm, use_learned, &a);
    double Hm[36], g[6];
    memset(st, 0, sizeof(*st));
    accumulate(n, &a, prm->delta, Hm, g, st);
    free(nrm);
    free(nv);
    return 0;
}

/* Association with caller-given normals (for the strided-sensor invariant). */
void orc_associate_with_normals(const orc_sensor *s, int level, const float *src, const float *dst,
                                const double *nrm, const uint8_t *nvalid, const double T[16],
                                const orc_params *prm, int32_t *u, int32_t *v, uint8_t *mask,
                                uint8_t *proj_valid, double *e, double *w, double *J, double *uhat,
                                double *phi)
{
    orc_assoc_out a = {u, v, mask, proj_valid, e, w, J, uhat, phi, NULL};
    orc_associate(s, level, src, dst, nrm, nvalid, T, prm, 0, &a);
}

/* ------------------------------------------------------------------ Sec. 4.2, Eq. (8)-(10) */

/*
 * Projective signed distance of a world point x against one range image
 * (Sec. 4.2).  T is the scan's pose as a row-major 4x4 matrix mapping world
 * points into its sensor frame (the R_j, t_j of Eq. (8)).
 *   Eq. (8): [u v r] = Pi(R x + t), at the finest level;
 *   Eq. (9): d = Omega(u, v) - r, the signed distance along the projection ray
 *            (positive in front of the observed surface).
 * Returns 1 with *d and *omega set when the projection lies in the image and
 * Omega(u, v) is a return (finite and > 0), else 0.  p (nullable) receives
 * the projection of R x + t.
 */
int orc_sdf_point(const orc_sensor *s, const float *range, const double T[16], const double x[3], double *d,
                  double *omega, orc_proj *p)
{
    double xs[3];
    for (int i = 0; i < 3; ++i)
        xs[i] = T[4 * i] * x[0] + T[4 * i + 1] * x[1] + T[4 * i + 2] * x[2] + T[4 * i + 3];
    orc_proj q;
    orc_project(s, 0, xs, &q);
    if (p)
        *p = q;
    if (!q.valid)
        return 0;
    double om = range[(size_t)q.v * s->W + q.u];
    if (!range_ok(om))
        return 0;
    *d = om - q.r;
    *omega = om;
    return 1;
}

/* orc_sdf_point over n points (for the tests): d, Omega, validity and the
 * continuous projection coordinates (column u_hat, elevation phi). */
void orc_sdf_points(const orc_sensor *s, const float *range, const double T[16], const double *pts, int64_t n,
                    double *d, double *omega, uint8_t *valid, int32_t *u, int32_t *v, double *uhat, double *phi)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_proj q;
        double di = 0.0, oi = 0.0;
        valid[i] = (uint8_t)orc_sdf_point(s, range, T, pts + 3 * i, &di, &oi, &q);
        d[i] = di;
        omega[i] = oi;
        u[i] = q.u;
        v[i] = q.v;
        uhat[i] = q.uhat;
        phi[i] = q.phi;
    }
}

/*
 * Eq. (10): the SDF at each query point is the mean of its per-scan signed
 * distances, the least-squares estimate over the scans, kept incrementally
 * as a running mean (sdf, weight = number of observations) and updated scan
 * by scan in the given order: sdf <- (sdf * weight + d) / (weight + 1).
 *
 * Readings (the section states the untruncated mean and cites classical
 * volumetric fusion, which truncates):
 *  - trunc > 0: an observation with d < -trunc is skipped (the point lies
 *    deeper behind the observed surface than the truncation band) and d is
 *    limited to at most trunc; trunc <= 0 keeps every observation (plain
 *    Eq. (10)).
 *  - r_clip > 0: observations whose range Omega(u, v) exceeds r_clip are
 *    skipped (far returns are clipped, Sec. 6); r_clip <= 0 keeps them.
 *  - Scans are those of ranges[f * H * W ...], poses[16 f ...], f = 0..F-1.
 * sdf and weight (n values each) hold the prior state and are updated in
 * place.
 */
void orc_sdf_fuse(const orc_sensor *s, int n_frames, const float *ranges, const double *poses, int64_t n,
                  const double *pts, double trunc, double r_clip, double *sdf, double *weight)
{
    size_t hw = (size_t)s->H * s->W;
    for (int f = 0; f < n_frames; ++f) {
        const float *img = ranges + (size_t)f * hw;
        const double *T = poses + 16 * (size_t)f;
        for (int64_t i = 0; i < n; ++i) {
            double d, om;
            if (!orc_sdf_point(s, img, T, pts + 3 * i, &d, &om, NULL))
                continue;
            if (r_clip > 0.0 && om > r_clip)
                continue;
            if (trunc > 0.0) {
                if (d < -trunc)
                    continue;
                if (d > trunc)
                    d = trunc;
            }
            sdf[i] = (sdf[i] * weight[i] + d) / (weight[i] + 1.0);
            weight[i] += 1.0;
        }
    }
}

/* ------------------------------------------------------------------ Sec. 4.2 block activation */

/* Voxel-block activation of Sec. 4.2 (sparse volume of 16^3-voxel blocks):
 * every return of scan f (range r, finite and > 0, and r <= r_clip when
 * r_clip > 0) is unprojected (Eq. (1)) and moved to the world frame,
 * x = R^T (x_s - t) for the scan's world -> sensor pose (R, t); it activates
 * every block whose cell o + [E b, E (b + 1)) (E = block_edge, per axis;
 * o the volume origin, where voxel (0, 0, 0) sits) meets the cube
 * [x - radius, x + radius] (reading of the paper's blocks within some radius
 * of each point: an axis-aligned cube, which is what a block grid tests
 * cheaply), i.e. b from floor((x - o - radius) / E) to
 * floor((x - o + radius) / E) on each axis.  A block's activation frame is
 * the first scan that activates it (the paper activates with each scan's
 * points before fusing that scan, so a block takes the scans from that one
 * on).
 * Output: the distinct blocks sorted by (bx, by, bz), as 4 int32 each (bx,
 * by, bz, activation frame), at most max_out of them; returns how many there
 * are (-1 if memory runs out). */
typedef struct {
    int32_t b[3];
    int32_t f;
} orc_act;

static int act_cmp(const void *pa, const void *pb)
{
    const orc_act *a = (const orc_act *)pa, *b = (const orc_act *)pb;
    for (int i = 0; i < 3; ++i)
        if (a->b[i] != b->b[i])
            return a->b[i] < b->b[i] ? -1 : 1;
    return (a->f > b->f) - (a->f < b->f);
}

int64_t orc_sdf_activate(const orc_sensor *s, int n_frames, const float *ranges, const double *poses,
                         const double origin[3], double radius, double r_clip, double block_edge, int32_t *out,
                         int64_t max_out)
{
    size_t hw = (size_t)s->H * s->W, n = 0, cap = 1024;
    orc_act *all = (orc_act *)malloc(cap * sizeof(orc_act));
    if (!all)
        return -1;
    for (int f = 0; f < n_frames; ++f) {
        const double *T = poses + 16 * (size_t)f;
        for (int v = 0; v < s->H; ++v)
            for (int u = 0; u < s->W; ++u) {
                double r = ranges[(size_t)f * hw + (size_t)v * s->W + u];
                if (!range_ok(r) || (r_clip > 0.0 && r > r_clip))
                    continue;
                double xs[3], x[3], d[3];
                orc_unproject(s, u, v, r, xs);
                for (int i = 0; i < 3; ++i)
                    d[i] = xs[i] - T[4 * i + 3];
                for (int j = 0; j < 3; ++j)  /* x = R^T d */
                    x[j] = T[j] * d[0] + T[4 + j] * d[1] + T[8 + j] * d[2];
                int64_t lo[3], hi[3];
                for (int i = 0; i < 3; ++i) {
                    const double c = x[i] - origin[i];
                    lo[i] = (int64_t)floor((c - radius) / block_edge);
                    hi[i] = (int64_t)floor((c + radius) / block_edge);
                }
                for (int64_t bz = lo[2]; bz <= hi[2]; ++bz)
                    for (int64_t by = lo[1]; by <= hi[1]; ++by)
                        for (int64_t bx = lo[0]; bx <= hi[0]; ++bx) {
                            if (n == cap) {
                                orc_act *g = (orc_act *)realloc(all, 2 * cap * sizeof(orc_act));
                                if (!g) {
                                    free(all);
                                    return -1;
                                }
                                all = g;
                                cap *= 2;
                            }
                            all[n].b[0] = (int32_t)bx;
                            all[n].b[1] = (int32_t)by;
                            all[n].b[2] = (int32_t)bz;
                            all[n].f = f;
                            ++n;
                        }
            }
    }
    qsort(all, n, sizeof(orc_act), act_cmp);
    int64_t m = 0;
    for (size_t i = 0; i < n; ++i) {
        if (i > 0 && all[i].b[0] == all[i - 1].b[0] && all[i].b[1] == all[i - 1].b[1] &&
            all[i].b[2] == all[i - 1].b[2])
            continue;  /* sorted by frame within a block: the first is the earliest */
        if (m < max_out) {
            out[4 * m] = all[i].b[0];
            out[4 * m + 1] = all[i].b[1];
            out[4 * m + 2] = all[i].b[2];
            out[4 * m + 3] = all[i].f;
        }
        ++m;
    }
    free(all);
    return m;
}

/* ------------------------------------------------------------------ PCA normals */

/* Eigenvalues (ascending) and unit eigenvectors (columns of V) of a symmetric
 * 3x3 matrix A (row-major) by the cyclic Jacobi method: plane rotations that
 * zero one off-diagonal entry at a time, swept until the off-diagonal part is
 * negligible. */
static void jacobi_eigen3(const double A[9], double lam[3], double V[9])
{
    double a[9];
    memcpy(a, A, sizeof(a));
    for (int i = 0; i < 9; ++i)
        V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        double dia = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
        if (off <= 1e-40 * dia || off == 0.0)
            break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                double apq = a[3 * p + q];
                if (apq == 0.0)
                    continue;
                /* rotation angle from tan(2 phi) = 2 a_pq / (a_qq - a_pp) */
                double th = (a[3 * q + q] - a[3 * p + p]) / (2.0 * apq);
                double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < 3; ++k) { /* A <- A G (columns p, q) */
                    double akp = a[3 * k + p], akq = a[3 * k + q];
                    a[3 * k + p] = c * akp - sn * akq;
                    a[3 * k + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) { /* A <- G^T A (rows p, q) */
                    double apk = a[3 * p + k], aqk = a[3 * q + k];
                    a[3 * p + k] = c * apk - sn * aqk;
                    a[3 * q + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) { /* V <- V G */
                    double vkp = V[3 * k + p], vkq = V[3 * k + q];
                    V[3 * k + p] = c * vkp - sn * vkq;
                    V[3 * k + q] = sn * vkp + c * vkq;
                }
            }
    }
    /* sort ascending, permuting the columns of V alongside */
    int idx[3] = {0, 1, 2};
    double d[3] = {a[0], a[4], a[8]};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2 - i; ++j)
            if (d[idx[j]] > d[idx[j + 1]]) {
                int tmp = idx[j];
                idx[j] = idx[j + 1];
                idx[j + 1] = tmp;
            }
    double W[9];
    memcpy(W, V, sizeof(W));
    for (int j = 0; j < 3; ++j) {
        lam[j] = d[idx[j]];
        for (int k = 0; k < 3; ++k)
            V[3 * k + j] = W[3 * k + idx[j]];
    }
}

/*
 * Target normals by principal component analysis of the points in a
 * (2 half + 1)^2 pixel window (the eigen-decomposition alternative that
 * Sec. 4.1 names next to the neighbour cross product).
 *
 * Readings (the paper gives no details): the window wraps around in u and is
 * cut at the first and last rows; a pixel of the window takes part iff it is
 * a return within edge_rel * r_c of the centre range r_c (the gate of the
 * cross-product normals, so no window mixes surfaces across a depth edge);
 * the centre must be a return and at least ((2 half + 1)^2 + 1) / 2 pixels
 * (more than half the window) must take part.  The normal is the eigenvector
 * of the smallest eigenvalue of the points' covariance (1/n) sum (p - mean)
 * (p - mean)^T, oriented towards the sensor (n . d <= 0 for the centre's ray
 * direction d); a window whose middle eigenvalue is at most 1e-6 times the
 * largest (points on a line) has no normal.  lam (nullable) receives the
 * three eigenvalues in ascending order per pixel (zeros where invalid).
 */
void orc_normals_pca(const orc_sensor *s, const float *range, int half, double edge_rel, double *nrm,
                     uint8_t *valid, double *lam)
{
    int H = s->H, W = s->W, k = 2 * half + 1;
    int min_pts = (k * k + 1) / 2;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t i = (size_t)v * W + u;
            valid[i] = 0;
            nrm[3 * i] = nrm[3 * i + 1] = nrm[3 * i + 2] = 0.0;
            if (lam)
                lam[3 * i] = lam[3 * i + 1] = lam[3 * i + 2] = 0.0;
            double rc = range[i];
            if (!range_ok(rc))
                continue;
            double lim = edge_rel * rc;
            double pts[121][3];
            int n = 0;
            for (int dv = -half; dv <= half; ++dv) {
                int vv = v + dv;
                if (vv < 0 || vv >= H)
                    continue;
                for (int du = -half; du <= half; ++du) {
                    int uu = ((u + du) % W + W) % W;
                    double r = range[(size_t)vv * W + uu];
                    if (!range_ok(r) || fabs(r - rc) > lim)
                        continue;
                    orc_unproject(s, uu, vv, r, pts[n]);
                    ++n;
                }
            }
            if (n < min_pts)
                continue;
            double m[3] = {0.0, 0.0, 0.0};
            for (int j = 0; j < n; ++j)
                for (int c = 0; c < 3; ++c)
                    m[c] += pts[j][c];
            for (int c = 0; c < 3; ++c)
                m[c] /= n;
            double C[9] = {0.0};
            for (int j = 0; j < n; ++j)
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        C[3 * a + b] += (pts[j][a] - m[a]) * (pts[j][b] - m[b]);
            for (int a = 0; a < 9; ++a)
                C[a] /= n;
            double ev[3], V[9];
            jacobi_eigen3(C, ev, V);
            if (lam) {
                lam[3 * i] = ev[0];
                lam[3 * i + 1] = ev[1];
                lam[3 * i + 2] = ev[2];
            }
            if (!(ev[1] > 1e-6 * ev[2]))
                continue;
            double nv[3] = {V[0], V[3], V[6]};
            double d[3];
            ray_dir(s, u, v, d);
            if (nv[0] * d[0] + nv[1] * d[1] + nv[2] * d[2] > 0.0) {
                nv[0] = -nv[0];
                nv[1] = -nv[1];
                nv[2] = -nv[2];
            }
            nrm[3 * i] = nv[0];
            nrm[3 * i + 1] = nv[1];
            nrm[3 * i + 2] = nv[2];
            valid[i] = 1;
        }
}

/* The eigen-decomposition step on its own (for the tests). */
void orc_eigen3(const double A[9], double lam[3], double V[9]) { jacobi_eigen3(A, lam, V); }

/* ------------------------------------------------------------------ per-column poses */

/*
 * Re-projection of a scan under per-column poses: the non-rigid model the
 * paper's outlook (Sec. 6, limitations) proposes, with consecutive poses
 * assigned to each column as in LOAM, for sensors whose ray centre moves
 * during the sweep.
 *
 * Readings: column u is captured at sweep time s_u = (u + 1/2) / W - 1/2
 * (in sweeps, 0 at mid-sweep, azimuth order); the motion over one sweep is
 * the constant twist xi = (omega, tau), so the column's pose relative to the
 * mid-sweep frame is Exp(s_u xi) (the interpolation between consecutive poses
 * on SE(3)).  Every return (u, v, r) is unprojected (Eq. (1)), moved into the
 * mid-sweep frame, and projected again (Eq. (3)-(4), finest level); the output
 * pixel keeps the smallest range that lands on it (the nearest surface), 0
 * where nothing lands.  For each source pixel tu, tv receive the target pixel
 * (-1 if none), rr the new range, uhat / phi the continuous projection.
 */
void orc_deskew(const orc_sensor *s, const float *range, const double xi[6], double *out, int32_t *tu, int32_t *tv,
                double *rr, double *uhat, double *phi)
{
    int H = s->H, W = s->W;
    for (size_t i = 0; i < (size_t)H * W; ++i)
        out[i] = 0.0;
    for (int u = 0; u < W; ++u) {
        double su = ((double)u + 0.5) / (double)W - 0.5;
        double xs[6], T[16];
        for (int k = 0; k < 6; ++k)
            xs[k] = su * xi[k];
        orc_exp_se3(xs, T);
        for (int v = 0; v < H; ++v) {
            size_t i = (size_t)v * W + u;
            tu[i] = tv[i] = -1;
            rr[i] = uhat[i] = phi[i] = 0.0;
            double r = range[i];
            if (!range_ok(r))
                continue;
            double p[3], x[3];
            orc_unproject(s, u, v, r, p);
            for (int a = 0; a < 3; ++a)
                x[a] = T[4 * a] * p[0] + T[4 * a + 1] * p[1] + T[4 * a + 2] * p[2] + T[4 * a + 3];
            orc_proj q;
            orc_project(s, 0, x, &q);
            uhat[i] = q.uhat;
            phi[i] = q.phi;
            if (!q.valid)
                continue;
            tu[i] = q.u;
            tv[i] = q.v;
            rr[i] = q.r;
            size_t j = (size_t)q.v * W + q.u;
            if (out[j] == 0.0 || q.r < out[j])
                out[j] = q.r;
        }
    }
}

/*
 * Level-set triangles of an SDF volume (Sec. 4.2 meshes the fused SDF with
 * marching cubes; this is its tetrahedral form, consistent without the
 * ambiguous cube cases).  Grid as in orc_sdf_extract.  Every cube of 8
 * voxels (i..i+1, j..j+1, k..k+1) is split into the six tetrahedra that
 * share its diagonal from corner (0, 0, 0) to (1, 1, 1): for each order of
 * the axes (x y z, x z y, y x z, y z x, z x y, z y x) the path 000 -> one
 * axis -> two axes -> 111.  A tetrahedron is meshed when its four voxels have
 * weight >= min_weight and every edge whose ends lie on different sides of
 * zero (s > 0 against s <= 0) has |s_a - s_b| <= max_jump.  With one vertex
 * on its own side (the other three on the other) it gives the triangle
 * through the crossings of that vertex's three edges, taken in the order of
 * the other vertices; with two on each side, positive a, b and non-positive
 * c, d (tetrahedron order), the quadrilateral ac, ad, bd, bc as the
 * triangles (ac, ad, bd) and (ac, bd, bc).  A crossing is a + t (b - a),
 * t = s_a / (s_a - s_b).  Each triangle is turned so that its normal
 * (v1 - v0) x (v2 - v0) points from the tetrahedron's non-positive vertices
 * towards its positive ones (mean against mean).  Order: cubes in index
 * order of their (0, 0, 0) voxel, then tetrahedra, then triangles.  Writes
 * at most max_tris triangles (9 doubles each) and returns how many there are.
 */
static const int orc_tet_axes[6][2] = {{0, 1}, {0, 2}, {1, 0}, {1, 2}, {2, 0}, {2, 1}};

int64_t orc_sdf_mesh(const double origin[3], double voxel, int nx, int ny, int nz, const double *sdf,
                     const double *weight, double min_weight, double max_jump, double *tris, int64_t max_tris)
{
    int64_t n = 0;
    for (int k = 0; k + 1 < nz; ++k)
        for (int j = 0; j + 1 < ny; ++j)
            for (int i = 0; i + 1 < nx; ++i)
                for (int t = 0; t < 6; ++t) {
                    int c[4][3] = {{i, j, k}, {i, j, k}, {i, j, k}, {i + 1, j + 1, k + 1}};
                    c[1][orc_tet_axes[t][0]] += 1;
                    c[2][orc_tet_axes[t][0]] += 1;
                    c[2][orc_tet_axes[t][1]] += 1;
                    double sv[4], x[4][3];
                    int pos[4], np = 0, ok = 1;
                    for (int q = 0; q < 4; ++q) {
                        size_t idx = ((size_t)c[q][2] * ny + c[q][1]) * nx + c[q][0];
                        if (!(weight[idx] >= min_weight))
                            ok = 0;
                        sv[q] = sdf[idx];
                        pos[q] = sv[q] > 0.0;
                        np += pos[q];
                        for (int a = 0; a < 3; ++a)
                            x[q][a] = origin[a] + voxel * (double)c[q][a];
                    }
                    if (!ok || np == 0 || np == 4)
                        continue;
                    for (int a = 0; a < 4; ++a)
                        for (int b = a + 1; b < 4; ++b)
                            if (pos[a] != pos[b] && fabs(sv[a] - sv[b]) > max_jump)
                                ok = 0;
                    if (!ok)
                        continue;
                    /* edges (as vertex pairs) of the triangles */
                    int e[2][3][2], ntri = 0;
                    if (np == 1 || np == 3) {
                        int lone = -1, o[3], m = 0;
                        for (int q = 0; q < 4; ++q)
                            if (pos[q] == (np == 1))
                                lone = q;
                        for (int q = 0; q < 4; ++q)
                            if (q != lone)
                                o[m++] = q;
                        for (int v = 0; v < 3; ++v) {
                            e[0][v][0] = lone;
                            e[0][v][1] = o[v];
                        }
                        ntri = 1;
                    } else {
                        int P[2], N[2], mp = 0, mn = 0;
                        for (int q = 0; q < 4; ++q) {
                            if (pos[q])
                                P[mp++] = q;
                            else
                                N[mn++] = q;
                        }
                        int quad[4][2] = {{P[0], N[0]}, {P[0], N[1]}, {P[1], N[1]}, {P[1], N[0]}};
                        int tri_of[2][3] = {{0, 1, 2}, {0, 2, 3}};
                        for (int tr = 0; tr < 2; ++tr)
                            for (int v = 0; v < 3; ++v) {
                                e[tr][v][0] = quad[tri_of[tr][v]][0];
                                e[tr][v][1] = quad[tri_of[tr][v]][1];
                            }
                        ntri = 2;
                    }
                    /* direction from the non-positive towards the positive vertices */
                    double gp[3] = {0, 0, 0}, gn[3] = {0, 0, 0}, g[3];
                    for (int q = 0; q < 4; ++q)
                        for (int a = 0; a < 3; ++a) {
                            if (pos[q])
                                gp[a] += x[q][a] / np;
                            else
                                gn[a] += x[q][a] / (4 - np);
                        }
                    for (int a = 0; a < 3; ++a)
                        g[a] = gp[a] - gn[a];
                    for (int tr = 0; tr < ntri; ++tr) {
                        double v[3][3];
                        for (int w = 0; w < 3; ++w) {
                            int a = e[tr][w][0], b = e[tr][w][1];
                            double tt = sv[a] / (sv[a] - sv[b]);
                            for (int d = 0; d < 3; ++d)
                                v[w][d] = x[a][d] + tt * (x[b][d] - x[a][d]);
                        }
                        double u1[3], u2[3], nn[3];
                        for (int d = 0; d < 3; ++d) {
                            u1[d] = v[1][d] - v[0][d];
                            u2[d] = v[2][d] - v[0][d];
                        }
                        nn[0] = u1[1] * u2[2] - u1[2] * u2[1];
                        nn[1] = u1[2] * u2[0] - u1[0] * u2[2];
                        nn[2] = u1[0] * u2[1] - u1[1] * u2[0];
                        int flip = nn[0] * g[0] + nn[1] * g[1] + nn[2] * g[2] < 0.0;
                        if (n < max_tris) {
                            double *o = tris + 9 * n;
                            int order[3] = {0, flip ? 2 : 1, flip ? 1 : 2};
                            for (int w = 0; w < 3; ++w)
                                for (int d = 0; d < 3; ++d)
                                    o[3 * w + d] = v[order[w]][d];
                        }
                        ++n;
                    }
                }
    return n;
}

/*
 * Surface points of an SDF volume: the zero crossings of the fused SDF along
 * the grid edges (the level set that Sec. 4.2 extracts with marching cubes;
 * this returns its vertices, without the triangles).  Grid of nx * ny * nz
 * voxels, index (k ny + j) nx + i, voxel (i, j, k) at origin + voxel (i, j, k).
 * For every pair of voxels a, b adjacent along x, y or z, both with weight >=
 * min_weight, whose SDF values lie on different sides of zero (s_a > 0 and
 * s_b <= 0, or the reverse) and differ by at most max_jump (a larger step is
 * the edge of the truncation band behind an occluder, not a surface), the
 * point a + t (b - a), t = s_a / (s_a - s_b), is emitted.  Order: voxel a in
 * index order, then the x, y, z edge.  Writes at most max_pts points (3
 * doubles each) and returns how many crossings there are.
 */
int64_t orc_sdf_extract(const double origin[3], double voxel, int nx, int ny, int nz, const double *sdf,
                        const double *weight, double min_weight, double max_jump, double *pts, int64_t max_pts)
{
    int64_t n = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t a = ((size_t)k * ny + j) * nx + i;
                if (!(weight[a] >= min_weight))
                    continue;
                for (int ax = 0; ax < 3; ++ax) {
                    int di = ax == 0, dj = ax == 1, dk = ax == 2;
                    if (i + di >= nx || j + dj >= ny || k + dk >= nz)
                        continue;
                    size_t b = ((size_t)(k + dk) * ny + (j + dj)) * nx + (i + di);
                    if (!(weight[b] >= min_weight))
                        continue;
                    double sa = sdf[a], sb = sdf[b];
                    if ((sa > 0.0) == (sb > 0.0) || fabs(sa - sb) > max_jump)
                        continue;
                    double t = sa / (sa - sb);
                    if (n < max_pts) {
                        pts[3 * n] = origin[0] + voxel * ((double)i + t * di);
                        pts[3 * n + 1] = origin[1] + voxel * ((double)j + t * dj);
                        pts[3 * n + 2] = origin[2] + voxel * ((double)k + t * dk);
                    }
                    ++n;
                }
            }
    return n;
}

static void target_normals(const orc_sensor *s, const float *dst, const orc_params *prm, double *nrm, uint8_t *nv)
{
    if (prm->normal_window > 0)
        orc_normals_pca(s, dst, prm->normal_window, prm->edge_rel, nrm, nv, NULL);
    else
        orc_normals(s, dst, prm->edge_rel, nrm, nv);
}
