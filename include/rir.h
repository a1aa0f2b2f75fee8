/*
 * rir.h -- C ABI of librir: multi-scale projective point-to-plane ICP and
 * projective SDF fusion on cylindrical LiDAR range images, on AMD Instinct
 * MI355X (gfx950).
 *
 * The method is that of Dong, Ryu, Kaess, Park, "Revisiting LiDAR
 * Registration and Reconstruction: A Range Image Perspective":
 *   Sec. 3.1, Eq. (1)-(2)  ray-wise unprojection with per-beam azimuth and
 *                          elevation tables and the receiver radius r0;
 *   Sec. 3.2, Eq. (3)-(4)  projection with receiver-offset compensation and
 *                          an inverse elevation table;
 *   Sec. 4.1, Eq. (5)-(7)  projective data association and robust
 *                          point-to-plane Gauss-Newton over a strided
 *                          range/normal pyramid;
 *   Sec. 4.2, Eq. (8)-(10) projective signed distances fused into a dense
 *                          voxel-block volume.
 *
 * Conventions shared by every call:
 *  - Images are row-major [v][u], v = 0 the top beam (highest elevation), u the
 *    column; azimuth grows with u counter-clockwise from +x.  Ranges are FP32
 *    metres; 0, negative, NaN and Inf mean "no return".
 *  - Poses are 4x4 row-major FP64 matrices T_dst<-src mapping source-sensor
 *    points into the target-sensor frame.  Twists are xi = (omega, tau) and
 *    updates are applied on the left: T <- Exp(xi) T.
 *  - Pointers documented as "device" must point to memory on the context's or
 *    sensor's GPU; "host" pointers to ordinary host memory.  The caller owns
 *    every data buffer; the library owns only its opaque handles (device
 *    tables, workspaces, captured graphs) and never frees caller memory.
 *  - Calls taking a `stream` (a hipStream_t passed as void*, NULL = default
 *    stream) enqueue their work asynchronously on it after validating their
 *    arguments on the host.  Validation failures return an error before
 *    anything is enqueued.  No C++ exception crosses this interface.
 *  - Errors: every call returns a rir_status; on failure rir_last_error()
 *    gives a thread-local message.  Numerical outcomes of a registration
 *    (degenerate systems, fallbacks) are not errors; they are reported per
 *    pair and per level in rir_level_stats.status.
 *  - Handles are not thread-safe; use one rir_ctx per host thread/stream.
 */
#ifndef RIR_H
#define RIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rir_status;

enum {
    RIR_OK = 0,
    RIR_E_INVALID = 1,     /* null pointer, bad enum, bad numeric argument */
    RIR_E_SHAPE = 2,       /* image shape incompatible with the pyramid or sensor */
    RIR_E_LUT = 3,         /* sensor tables rejected (not strictly decreasing, ...) */
    RIR_E_HIP = 4,         /* a HIP runtime call failed */
    RIR_E_OOM = 5,         /* device or host allocation failed */
    RIR_E_UNSUPPORTED = 6  /* valid request this build does not implement */
};

/* Per-level outcome of a registration (rir_level_stats.status). */
enum {
    RIR_LEVEL_OK = 0,
    RIR_LEVEL_DEGENERATE = 1,     /* < 6 correspondences or Cholesky pivot test failed; level stopped */
    RIR_LEVEL_FALLBACK_HUBER = 2, /* learned weights rejected; that iteration used pseudo-Huber */
    RIR_LEVEL_NONFINITE = 3       /* non-finite normal equations; level stopped */
};

enum { RIR_WEIGHT_HUBER = 0, RIR_WEIGHT_LEARNED = 1 };
enum { RIR_PREC_FP32 = 0, RIR_PREC_FP64 = 1 };
enum { RIR_MAX_LEVELS = 8 };

typedef struct rir_sensor rir_sensor;
typedef struct rir_ctx rir_ctx;
typedef struct rir_mlp rir_mlp;

/* Sensor intrinsics (Sec. 3.1): H beams, W columns, per-beam elevation
 * phi_lut[H] (radians, strictly decreasing, |phi| < pi/2), per-beam azimuth
 * offset theta_lut[H] (radians, |theta| < pi, NULL = all zero) and receiver
 * radius r0 >= 0 (metres).  Both tables are host arrays, copied at creation.
 * inv_bins: minimum bin count of the inverse elevation table per pyramid
 * level (0 = automatic: at least 2 H_l and two per smallest gap between row
 * boundaries, doubled until no bin holds two distinct boundaries; Sec. 3.2). */
typedef struct {
    int32_t H, W;
    const double *phi_lut;
    const double *theta_lut;
    double r0;
    int32_t inv_bins;
} rir_sensor_desc;

/* Registration parameters (Sec. 4.1, Sec. 6.1).
 *  levels        pyramid levels L (1..8); level l uses stride 2^l, so H and W
 *                of every pair must be divisible by 2^(L-1).
 *  iters[l]      Gauss-Newton iterations at level l (index 0 = finest); levels
 *                run coarse to fine.
 *  delta         pseudo-Huber kernel size in metres (> 0).
 *  edge_rel      target-normal validity: every 4-neighbour range within
 *                edge_rel * centre range (> 0; 0.1 by convention).
 *  max_corr_dist reject correspondences with |x - q| above this (<= 0: off).
 *  init_mode     0: start from init_poses; 1: R = I and t = difference of the
 *                centres of the valid target and source points (Sec. 4.1).
 *  weight_mode   RIR_WEIGHT_HUBER or RIR_WEIGHT_LEARNED (needs mlp).
 *  precision     RIR_PREC_FP32: per-pixel math and tile sums in FP32, FP64
 *                tile-partial sums, Cholesky and pose update;
 *                RIR_PREC_FP64: everything in FP64.
 *  use_graph     1: capture the iteration schedule once per batch shape as
 *                HIP graphs and replay them; 0: launch kernel by kernel.
 *  mlp           learned-weight network (weight_mode LEARNED), else NULL.
 *  r_max         range scale of the first learned feature (metres).
 *  learned_levels with weight_mode LEARNED: bit l set = learned weights at
 *                level l, pseudo-Huber at the others; 0 = every level.
 *  stop_eps      > 0: a level ends after the first applied step whose twist
 *                has |xi| = sqrt(|omega|^2 + |tau|^2) <= stop_eps (rad and
 *                metres mixed; the remaining iterations of that level are
 *                skipped, iters_run tells how many ran); 0: fixed iteration
 *                counts.
 *  normal_window 0: target normals by the cross product of neighbour
 *                differences (Sec. 4.1); h = 1, 2 or 3: by principal
 *                component analysis of the (2h+1)^2 window (the
 *                eigen-decomposition estimator Sec. 4.1 names; the same
 *                normals as rir_normals_pca, rounded to FP32 in FP32 plans). */
typedef struct {
    int32_t levels;
    int32_t iters[RIR_MAX_LEVELS];
    double delta;
    double edge_rel;
    double max_corr_dist;
    int32_t init_mode;
    int32_t weight_mode;
    int32_t precision;
    int32_t use_graph;
    const rir_mlp *mlp;
    double r_max;
    int32_t learned_levels;
    double stop_eps;
    int32_t normal_window;
} rir_icp_params;

/* Statistics of one pyramid level of one pair: those of the level's last
 * evaluated Gauss-Newton iteration.  JtJ holds the 21 upper-triangle entries
 * of sum w J J^T in row-major order, Jtr = sum w J e (Eq. (7) normal
 * equations, xi = (omega, tau)); n_proj counts source pixels whose projection
 * landed in the image; step_rot/step_trans are |omega|, |tau| of the last
 * applied step (0 if none); robust_cost = sum of pseudo-Huber rho(e). */
typedef struct {
    int32_t status, iters_run, n_valid, n_inlier, n_proj, pad;
    double sum_w, sum_w_e2, robust_cost, step_rot, step_trans;
    double JtJ[21], Jtr[6];
} rir_level_stats;

/* One scan pair: source and target range images (device, H x W row-major
 * FP32, H and W those of `sensor`). */
typedef struct {
    const rir_sensor *sensor;
    const float *src_range;
    const float *dst_range;
} rir_pair;

/* Tuning of the association/reduction launch (picked by rir_autotune).
 * block: threads per workgroup (64, 128 or 256); px_per_thread: pixels each
 * thread visits per tile at levels 0 and 1 (1..16; each coarser level uses
 * 4x fewer, at least 1); grid_mult: persistent workgroups per compute unit (0 =
 * one workgroup per tile); xcd_remap: 1 maps consecutive tiles to the same
 * XCD (L2) of the chip; chunk: 64-pixel row segments whose loads each
 * wavefront keeps in flight together (1, 2 or 4); solve_in_step: 1 (with
 * grid_mult 0) lets the workgroup that finishes a pair's last tile of an
 * iteration solve that pair (one launch per Gauss-Newton iteration), 0 solves
 * every pair in a launch of its own after each association/reduction launch;
 * both sum the tile records in the same order and give the same results.
 * lanes (1..4): the coarse levels (all but the finest) of a batch run as up to
 * `lanes` sub-batches of consecutive pairs (about equal pixel counts) on as
 * many streams of the context, forked from and joined back into the call's
 * stream, so that the launches of different sub-batches overlap; lane_fine: 1
 * runs the finest level in the sub-batches too, 0 as one launch per iteration
 * over the whole batch.  Neither changes any result.  Default: lanes 1 (no
 * sub-batches), lane_fine 0; lanes > 1 is switched off in this build
 * (rir_ctx_set_tuning returns RIR_E_UNSUPPORTED). */
typedef struct {
    int32_t block, px_per_thread, grid_mult, xcd_remap, chunk, solve_in_step, lanes, lane_fine;
} rir_tuning;

/* ---------------------------------------------------------------- sensors */

/* Builds the device tables of a sensor on the current HIP device (Sec. 3):
 * per-beam and per-column trigonometric factors of Eq. (1), cancellation-free
 * neighbour-difference factors for the normal image, and per-level inverse
 * elevation tables of Sec. 3.2.  Errors: RIR_E_INVALID (null), RIR_E_LUT
 * (H < 2, W < 4, non-finite or non-decreasing phi, |theta| >= pi, |phi| >=
 * pi/2, r0 < 0), RIR_E_OOM, RIR_E_HIP.  *out is owned by the caller and
 * released with rir_sensor_destroy. */
rir_status rir_sensor_create(const rir_sensor_desc *desc, rir_sensor **out);
void rir_sensor_destroy(rir_sensor *sensor);

/* Host copy of the inverse elevation table that rir_sensor_create builds for
 * pyramid level `level` (Sec. 3.2, Eq. (4)); no device is used (inspection
 * and tests).  precision (RIR_PREC_*) selects the FP32 or FP64 table.
 * Entry b is 4 values of that type at entries[4b .. 4b+3] and covers every
 * sz = sin(phi) that the kernels map to bin b = trunc(clamp((sz - bin_lo) *
 * bin_scale, 0, nbins - 1)), evaluated in that type (the subtraction and the
 * product each rounded) with bin_lo, bin_scale and nbins - 1 rounded to it:
 * the low 32 bits of the first value hold c | (c + k) << 16, then m,
 * uoff(c), uoff(c + k).  The row of sz at the level is
 * c + k [m > sz] (the nearest row, ties to the smaller index) and uoff(t) =
 * theta_lut[2^l t] W / (2 pi 2^l) its column offset.  *nbins receives the
 * entry count and bin_lo / bin_scale (nullable) the FP64 bin parameters;
 * entries may be NULL to query only, else it holds capacity values (at least
 * 4 * nbins).  Errors: as rir_sensor_create (no RIR_E_OOM / RIR_E_HIP), and
 * RIR_E_INVALID for a null desc or nbins, an unknown precision, a level
 * outside the sensor's pyramid or a capacity below 4 * nbins. */
rir_status rir_elevation_table(const rir_sensor_desc *desc, int32_t level, int32_t precision, void *entries,
                               int64_t capacity, int64_t *nbins, double *bin_lo, double *bin_scale);

/* ---------------------------------------------------------------- contexts */

/* A registration context on HIP device `device`: owns workspaces, captured
 * graphs and the tuning.  Errors: RIR_E_INVALID, RIR_E_HIP, RIR_E_OOM. */
rir_status rir_ctx_create(int device, rir_ctx **out);
void rir_ctx_destroy(rir_ctx *ctx);
rir_status rir_ctx_set_tuning(rir_ctx *ctx, const rir_tuning *tuning);
rir_status rir_ctx_get_tuning(const rir_ctx *ctx, rir_tuning *tuning);

/* Timing of rir_icp_batch with HIP events recorded in its stream order (as
 * nodes of the captured graph): on = 0 off, 1 around the normal/pyramid pass
 * and every pyramid level, 2 around the finest level only (fewer event
 * nodes, less overhead).  rir_ctx_level_times waits for the last timed call
 * and writes the elapsed milliseconds of level l to ms[l] (ms[levels]: the
 * normal/pyramid pass; 0 for parts not timed).  Host arrays.  Errors:
 * RIR_E_INVALID (null, mode outside 0..2, no timed call yet), RIR_E_HIP. */
rir_status rir_ctx_enable_timing(rir_ctx *ctx, int32_t on);
rir_status rir_ctx_level_times(rir_ctx *ctx, float *ms, int32_t n);

/* ---------------------------------------------------------------- geometry */

/* Eq. (1)-(2): unprojects every pixel of `range` (device H x W) to
 * xyz (device H*W*3 FP32, (x,y,z) per pixel) and valid (device H*W bytes,
 * 1 = return present, xyz = 0 otherwise). */
rir_status rir_unproject(const rir_sensor *sensor, const float *range, float *xyz, uint8_t *valid, void *stream);

/* Eq. (3)-(4) at pyramid level `level` (stride s = 2^level, Sec. 4.1): for n
 * points xyz (device n*3 FP32) writes the level pixel (u, v) (device int32),
 * the range r (device FP32) and valid (device bytes: inside the elevation
 * field of view and r > 0; u = v = -1 when invalid).  Level indices are the
 * nearest strided row by elevation and the nearest strided column. */
rir_status rir_project(const rir_sensor *sensor, int32_t level, const float *xyz, int64_t n, int32_t *u,
                       int32_t *v, float *r, uint8_t *valid, void *stream);

/* Target normal image by the cross product of neighbour differences
 * (Sec. 4.1, Sec. 6.1): nrm (device H*W*3 FP32) and valid (device bytes).
 * Valid iff the pixel and its 4 neighbours (u wraps, v does not) have returns
 * and every neighbour lies within edge_rel of the centre range; normals face
 * the sensor. */
rir_status rir_normals(const rir_sensor *sensor, const float *range, double edge_rel, float *nrm, uint8_t *valid,
                       void *stream);

/* Normals by principal component analysis of a (2 half + 1)^2 pixel window,
 * the eigen-decomposition estimator Sec. 4.1 names beside the neighbour cross
 * product, for n_images contiguous H x W range images (device, FP32):
 * nrm (device n_images*H*W*3 FP32) and valid (device bytes).  The window
 * wraps in u and is cut at the first and last rows; a pixel of it takes part
 * iff it is a return within edge_rel of the centre range.  Valid iff the
 * centre is a return, more than half the window takes part, and the middle
 * eigenvalue of the points' covariance exceeds 1e-6 times the largest (not
 * all on a line); the normal is the eigenvector of the smallest eigenvalue,
 * facing the sensor.  Covariance and eigen-decomposition in FP64.  half is
 * 1, 2 or 3.  Errors: RIR_E_INVALID (null, n_images < 0, half outside 1..3,
 * edge_rel <= 0), RIR_E_HIP. */
rir_status rir_normals_pca(const rir_sensor *sensor, int32_t n_images, const float *range, int32_t half,
                           double edge_rel, float *nrm, uint8_t *valid, void *stream);

/* Re-projection under per-column poses, the non-rigid model of the paper's
 * outlook (Sec. 6: each column given its own pose between consecutive poses,
 * as in LOAM) for
 * sensors that move during a sweep.  Column u of scan k is captured at sweep
 * time s_u = (u + 1/2) / W - 1/2 (0 at mid-sweep); with the constant twist
 * xi_k = (omega, tau) per sweep its pose in the mid-sweep frame is
 * Exp(s_u xi_k).  Every return (u, v, r) is unprojected (Eq. (1)), moved by its
 * column's pose and projected again (Eq. (3)-(4), finest level); each output
 * pixel keeps the smallest range landing on it, 0 where none does.  The result
 * is a rigid range image again, ready for registration or fusion.
 *   range_in   device n_images*H*W FP32 scans.
 *   twists     host n_images*6 FP64 (omega, tau) per sweep; read before the
 *              call returns.
 *   range_out  device n_images*H*W FP32, must not overlap range_in (its bits
 *              serve as the atomic minimum while the call runs).
 * FP64 pose, point and projection; output ranges rounded to FP32.  Errors:
 * RIR_E_INVALID (null, n_images < 0, overlapping buffers, non-finite
 * twist), RIR_E_HIP. */
rir_status rir_deskew(const rir_sensor *sensor, int32_t n_images, const float *range_in, const double *twists,
                      float *range_out, void *stream);

/* ---------------------------------------------------------------- registration */

/* Registers n_pairs independent scan pairs (Sec. 4.1, Eq. (5)-(7)), all with
 * the same parameters but any mix of sensors and image sizes, in one batch:
 * one association/reduction launch per Gauss-Newton iteration covers every
 * pair and writes one partial-sum record per tile; a second launch with one
 * workgroup per pair sums that pair's records in FP64 in tile order, solves
 * its 6x6 system and applies the update.  Pairs whose level image is small
 * run all iterations of that level in one launch, one workgroup per pair.
 * The whole schedule is replayed as one HIP graph per batch shape.
 *   pairs       host array of n_pairs descriptors (device images).
 *   init_poses  device n_pairs*16 FP64 (ignored with init_mode 1).
 *   poses_out   device n_pairs*16 FP64 (may alias init_poses).
 *   stats_out   device n_pairs*levels rir_level_stats, or NULL.
 * Errors: RIR_E_INVALID, RIR_E_SHAPE (H or W not divisible by 2^(L-1)),
 * RIR_E_UNSUPPORTED, RIR_E_OOM, RIR_E_HIP. */
rir_status rir_icp_batch(rir_ctx *ctx, const rir_icp_params *params, int32_t n_pairs, const rir_pair *pairs,
                         const double *init_poses, double *poses_out, rir_level_stats *stats_out, void *stream);

/* One association pass of one pair at level `level` and host pose `pose`
 * (16 FP64) without a pose update, dumping per source pixel of that level
 * (N_l = (H/s)*(W/s), row-major): u, v (int32, -1 if the projection is
 * invalid), mask (byte, 1 = correspondence used), e, w (FP32), J (FP32 N_l*6)
 * and feat (FP32 N_l*14 learned-weight features, zeros where mask = 0); each
 * output pointer is device memory or NULL.  stats_out (host, nullable)
 * receives the reduced normal equations of the pass; when given the call
 * waits for the stream. */
rir_status rir_debug_associate(rir_ctx *ctx, const rir_icp_params *params, const rir_pair *pair, int32_t level,
                               const double *pose, int32_t *u, int32_t *v, uint8_t *mask, float *e, float *w,
                               float *J, float *feat, rir_level_stats *stats_out, void *stream);

/* Times the batch for a sweep of rir_tuning candidates (each replayed a few
 * times after a warm-up, HIP events on `stream`) and installs the fastest in
 * the context; best (host, nullable) receives it and best_ms (host, nullable)
 * its time per batch.  Poses are left in poses_scratch (device n_pairs*16). */
rir_status rir_autotune(rir_ctx *ctx, const rir_icp_params *params, int32_t n_pairs, const rir_pair *pairs,
                        const double *init_poses, double *poses_scratch, rir_tuning *best, float *best_ms,
                        void *stream);

/* ---------------------------------------------------------------- reconstruction */

/* Dense SDF volume (Sec. 4.2): nbx x nby x nbz blocks of 16^3 voxels (the
 * paper's voxel-block shape, here allocated densely).  Voxel (i, j, k),
 * 0 <= i < 16 nbx etc., sits at origin + voxel * (i, j, k) in world
 * coordinates (metres).  Storage (device, caller-owned): 2 FP32 values
 * (sdf, weight) per voxel; blocks in (bz, by, bx) order, bx fastest; inside
 * a block voxels in (z, y, x) order, x fastest; block (bx, by, bz) holds
 * voxels 16 bx .. 16 bx + 15 along i, and so on.  A voxel with weight 0 has
 * not been observed; a zero-filled buffer is an empty volume. */
typedef struct {
    int32_t nbx, nby, nbz;
    double origin[3];
    double voxel;
} rir_volume_desc;

/* Fuses n_frames range scans into the volume (Sec. 4.2).  For each voxel x
 * and each scan f, in the given order: Eq. (8) [u v r] = Pi(R_f x + t_f) at the
 * finest level, Eq. (9) d = Omega_f(u, v) - r, and the running mean of Eq. (10)
 * sdf <- sdf + (d - sdf) / (weight + 1), weight <- weight + 1.  An
 * observation counts only if the projection lies in the image, Omega_f(u, v)
 * is a return, Omega_f(u, v) <= r_clip (if r_clip > 0; far returns clipped)
 * and d >= -trunc (if trunc > 0; d is then limited to at most trunc, the
 * truncated SDF of classical volumetric fusion); trunc <= 0 averages every
 * observation.
 *   sensor   the scans' intrinsics (every scan H x W of that sensor).
 *   vol      host descriptor (see rir_volume_desc).
 *   voxels   device, 2 * 4096 * nbx * nby * nbz FP32, updated in place.
 *   ranges   device, n_frames * H * W FP32 scans, contiguous.
 *   poses    host, n_frames * 16 FP64 row-major 4x4 world -> sensor poses
 *            (x_s = R x + t); read before the call returns.
 * FP32 per-voxel arithmetic; the per-block sensor-frame offsets are formed in
 * FP64.  Work is enqueued on `stream` in launches of up to 16 scans; a block
 * that no scan of a launch can reach (farther than r_clip + trunc + r0 from
 * every sensor, with both limits set) is not touched.  n_frames = 0 is a
 * no-op.  Errors: RIR_E_INVALID (null, n_frames < 0, non-finite pose,
 * origin, trunc or r_clip, voxel <= 0), RIR_E_SHAPE (block count < 1 or
 * above 2^31 - 1, 16 scans of H x W at or above 2 GiB), RIR_E_HIP. */
rir_status rir_sdf_integrate(const rir_sensor *sensor, const rir_volume_desc *vol, float *voxels, int32_t n_frames,
                             const float *ranges, const double *poses, double trunc, double r_clip, void *stream);

/* Surface points of a fused volume: the zero crossings of the SDF along the
 * grid edges (the vertices of the level set that Sec. 4.2 meshes with
 * marching cubes).  For voxels a, b adjacent along x, y or z with both
 * weights >= min_weight, SDF values on different sides of zero (s_a > 0 >= s_b
 * or the reverse) and |s_a - s_b| <= max_jump (a larger step is the edge of a
 * truncation band behind an occluder; INFINITY keeps all), the point
 * a + t (b - a), t = s_a / (s_a - s_b), in world coordinates (formed in FP64,
 * stored as FP32).
 *   voxels      device volume (rir_sdf_integrate layout), read only.
 *   points      device max_points*3 FP32 (x, y, z), order not defined.
 *   count       device uint64: number of crossings found (may exceed
 *               max_points; only the first max_points are stored).
 * Runs on the current HIP device, asynchronously on `stream`.  Errors:
 * RIR_E_INVALID (null, max_points < 0, voxel <= 0, non-finite origin or
 * min_weight, max_jump < 0 or NaN), RIR_E_SHAPE, RIR_E_HIP. */
rir_status rir_sdf_extract(const rir_volume_desc *vol, const float *voxels, double min_weight, double max_jump,
                           float *points, int64_t max_points, uint64_t *count, void *stream);

/* Level-set triangles of a fused volume (Sec. 4.2 meshes the fused SDF with
 * marching cubes; this is its tetrahedral form, which needs no resolution
 * of ambiguous cube cases).  Every cube of 8 voxels (i..i+1, j..j+1, k..k+1)
 * is split into the six tetrahedra around its diagonal from voxel (0, 0, 0)
 * to (1, 1, 1), one for each order of the axes (x y z, x z y, y x z, y z x,
 * z x y, z y x: 000 -> one axis -> two axes -> 111).  A tetrahedron whose four
 * voxels have weight >= min_weight and whose edges with values on different
 * sides of zero (s > 0 against s <= 0) step by at most max_jump gives: with
 * one vertex on its own side, the triangle through the crossings of its
 * three edges (in the order of the other vertices); with positive a, b and
 * non-positive c, d (tetrahedron order), the triangles (ac, ad, bd) and
 * (ac, bd, bc).  A crossing is a + t (b - a), t = s_a / (s_a - s_b), formed
 * in FP64 in world coordinates and stored as FP32; each triangle is turned so
 * that (v1 - v0) x (v2 - v0) points from the tetrahedron's non-positive
 * vertices towards its positive ones.
 *   voxels      device volume (rir_sdf_integrate layout), read only.
 *   triangles   device max_triangles * 9 FP32 (three vertices of x, y, z),
 *               order not defined.
 *   count       device uint64: number of triangles (may exceed
 *               max_triangles; only the first max_triangles are stored).
 * Runs asynchronously on `stream`.  Errors as rir_sdf_extract. */
rir_status rir_sdf_mesh(const rir_volume_desc *vol, const float *voxels, double min_weight, double max_jump,
                        float *triangles, int64_t max_triangles, uint64_t *count, void *stream);

/* ---------------------------------------------------------------- sparse SDF volume */

/* Sparse SDF volume of Sec. 4.2: the 16^3-voxel blocks near the returns of
 * each scan are activated in a hash table keyed by block coordinates, and
 * only activated blocks are fused.  Voxel (i, j, k) (any integers) sits at
 * origin + voxel * (i, j, k) in world coordinates (metres; origin host,
 * 3 FP64, read before the call returns); block (bx, by, bz) holds
 * voxels 16 bx .. 16 bx + 15 along i, and so on, |bx|, |by|, |bz| < 2^20.
 * The volume owns its device memory on `device`: a pool of max_blocks
 * blocks (32 KiB each: (sdf, weight) FP32 per voxel in the rir_sdf_integrate
 * block layout, voxels in (z, y, x) order, x fastest) and an open-addressing
 * table of at least 2 max_blocks entries.  Calls on one volume run in the
 * order they are made and must not overlap.  Errors: RIR_E_INVALID (null,
 * non-finite origin, voxel not finite or <= 0, max_blocks outside 1..2^26),
 * RIR_E_OOM, RIR_E_HIP.
 * *out is owned by the caller and released with rir_bvol_destroy. */
typedef struct rir_bvol rir_bvol;
rir_status rir_bvol_create(int device, const double origin[3], double voxel, int32_t max_blocks, rir_bvol **out);
void rir_bvol_destroy(rir_bvol *vol);
/* Empties the volume (no blocks, no scans); enqueued on `stream` as device
 * memsets (not for a stream under graph capture). */
rir_status rir_bvol_reset(rir_bvol *vol, void *stream);

/* Fuses n_frames scans (Sec. 4.2).  For each scan, in order: every return
 * (range finite and > 0, and <= r_clip when r_clip > 0) is unprojected
 * (Eq. (1)) and moved to the world frame, x = R^T (x_s - t); every block
 * whose cell origin + [E b, E (b + 1)) (E = 16 voxel, per axis) meets the cube
 * [x - radius, x + radius] is activated (decided in FP64); then the scan is
 * fused into every active block (the blocks this scan or an earlier one
 * activated) with the arithmetic, trunc and r_clip of rir_sdf_integrate
 * (Eq. (8)-(10); with both limits set, a block the scan cannot reach is
 * skipped).  ranges: device, n_frames * H * W FP32 scans of `sensor`; poses:
 * host, n_frames * 16 FP64 world -> sensor, read before the call returns.
 * Enqueued on `stream`; the call waits for the activation (to size the
 * fusion launches), so it cannot run on a stream under graph capture.  Errors: RIR_E_INVALID (null, n_frames < 0, radius
 * outside 0 .. 64 voxels, non-finite trunc, r_clip or pose, sensor on another
 * device),
 * RIR_E_SHAPE (16 scans of H x W at or above 2 GiB), RIR_E_OOM (more active
 * blocks than max_blocks, or a return beyond the block coordinate range: the
 * volume is then incomplete and must be reset), RIR_E_HIP. */
rir_status rir_bvol_integrate(rir_bvol *vol, const rir_sensor *sensor, int32_t n_frames, const float *ranges,
                              const double *poses, double trunc, double r_clip, double radius, void *stream);

/* Active blocks and scans fused so far (host values, no device work). */
rir_status rir_bvol_size(const rir_bvol *vol, int64_t *n_blocks, int64_t *n_frames);

/* Copies the active blocks out in pool order (not defined across runs):
 * blocks (device, n_blocks * 4 int32: bx, by, bz and the index, over the
 * volume's history, of the first scan that activated the block) and voxels
 * (device, n_blocks * 8192 FP32, block layout above); either may be NULL.
 * Enqueued on `stream`. */
rir_status rir_bvol_export(const rir_bvol *vol, int32_t *blocks, float *voxels, void *stream);

/* Zero crossings of the sparse volume, as rir_sdf_extract (edges between
 * voxels of active blocks; world coordinates).  Errors: RIR_E_INVALID (null,
 * max_points < 0, non-finite min_weight, max_jump < 0 or NaN), RIR_E_HIP. */
rir_status rir_bvol_extract(rir_bvol *vol, double min_weight, double max_jump, float *points, int64_t max_points,
                            uint64_t *count, void *stream);

/* Level-set triangles of the sparse volume, as rir_sdf_mesh (cubes whose
 * eight voxels lie in active blocks; world coordinates).  Errors as
 * rir_bvol_extract. */
rir_status rir_bvol_mesh(rir_bvol *vol, double min_weight, double max_jump, float *triangles, int64_t max_triangles,
                         uint64_t *count, void *stream);

/* ---------------------------------------------------------------- learned weight */

/* Per-pixel robust-weight network 14-64-64-1 (ReLU, ReLU, sigmoid) replacing
 * the pseudo-Huber weight of Eq. (7).  Parameters: w_bf16 = W1[64][14],
 * W2[64][64], W3[64] as bfloat16 bit patterns (host, 5056 values), b_f32 =
 * b1[64], b2[64], b3 (host, 129 values).  Training keeps FP32 master copies
 * and Adam moments on the device. */
rir_status rir_mlp_create(int device, const uint16_t *w_bf16, const float *b_f32, rir_mlp **out);
void rir_mlp_destroy(rir_mlp *mlp);
/* Host copies of the current bfloat16 weights (5056), biases (129) and, if
 * master is non-NULL, the FP32 master weights (5056). */
rir_status rir_mlp_get_params(const rir_mlp *mlp, uint16_t *w_bf16, float *b_f32, float *master);
rir_status rir_mlp_set_params(rir_mlp *mlp, const uint16_t *w_bf16, const float *b_f32);

/* Weights w = sigmoid(net(f)) for B feature rows (device B*14 FP32) into
 * w_out (device B FP32).  Inputs and hidden activations are rounded to
 * bfloat16; products accumulate in FP32 on the matrix cores. */
rir_status rir_mlp_forward(const rir_mlp *mlp, const float *feats, int64_t B, float *w_out, void *stream);

/* One Adam step (beta 0.9/0.999, eps 1e-8, learning rate lr) on the mean
 * binary cross-entropy of sigmoid(net(f)) against labels (device B FP32 in
 * {0,1}).  loss_out (device FP32, nullable) receives the batch loss;
 * grads_out (device 5185 FP32 in the layout W1, b1, W2, b2, W3, b3, nullable)
 * the gradient before the update. */
rir_status rir_mlp_train_step(rir_mlp *mlp, const float *feats, const float *labels, int64_t B, float lr,
                              float *loss_out, float *grads_out, void *stream);

/* rir_mlp_train_step without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * results as rir_mlp_train_step (bit-identical for the same inputs); the
 * per-wavefront gradient records go to a fixed device array of 512 records
 * of 5186 FP32 (10.1 MiB) that the library holds on every GPU it runs on
 * until the process ends, instead of a buffer it allocates.  B is limited to
 * 1..32768 (the records of larger batches do not fit).  Every record is
 * rewritten by each call before it is read, so nothing needs clearing
 * between calls; all calls on one GPU share that GPU's array, so calls that
 * may overlap on one GPU (different streams, threads or networks) race and
 * must be serialised by the caller.  Calls no hipMalloc or hipFree.  Errors:
 * RIR_E_INVALID (null, B outside 1..32768, lr not finite or < 0),
 * RIR_E_HIP. */
rir_status rir_mlp_train_step_noalloc(rir_mlp *mlp, const float *feats, const float *labels, int64_t B, float lr,
                                      float *loss_out, float *grads_out, void *stream);

/* ---------------------------------------------------------------- errors */

/* Message of the calling thread's last failed call ("" if none). */
const char *rir_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RIR_H */
