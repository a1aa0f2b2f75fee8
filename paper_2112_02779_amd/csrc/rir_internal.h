// Internal interface between the host runtime (api.cpp) and the kernels
// (kernels.hip, mlp.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rir.h"
#include "rir_device.h"

namespace rir {

// Per-pair view of one batch entry, in device memory.  Level images:
//  src[l]  FP32 source ranges at stride 2^l ([0] is the caller's image)
//  dstr[l] FP32 target ranges at stride 2^l ([0] is the caller's image)
//  dst4[l] 4 T per pixel: target normal n (x, y, z) and the plane offset
//          n . q of the target point q; where the normal is invalid (which
//          includes "no return") n = 0 and the offset is NaN
// Work is cut into segments: 64 consecutive pixels of one image row (one per
// lane of a wavefront), ceil(W_l / 64) per row, so every wavefront works on a
// single row.  Tiles of level l of this pair are tile0[l] .. tile0[l] +
// ntile[l] - 1 of the level's tile list.
// frames: per full-resolution row v the ray frame of Eq. (1) rotated by the
// pair's current pose R, kFrame T each: g1 = R (A, B, 0), g2 = R (-B, A, 0),
// g3 = sin(phi_v) R e_z with A = cos(phi_v) cos(theta_v), B = cos(phi_v)
// sin(theta_v), then 3 zeros; R d(u, v) = cos(a_u) g1 + sin(a_u) g2 + g3.
// Rewritten whenever the pose changes (k_frames, k_solve).
template <typename T>
struct PairDesc {
    const SensorTab<T> *tab;
    const SensorTab<double> *tabd;  // FP64 tables (PCA target normals)
    float *src[kMaxLevels];
    float *dstr[kMaxLevels];
    T *dst4[kMaxLevels];
    // levels with learned weights: per target pixel the 8 neighbour features
    // of the network (clamped range differences to the 8 level-l neighbours
    // in raster order), rounded to bf16 and packed two per word (4 words);
    // null elsewhere
    uint32_t *nbf[kMaxLevels];
    T *frames;
    int H, W;
    int tile0[kMaxLevels], ntile[kMaxLevels];
};

constexpr int kSegPx = 64;  // pixels per segment
constexpr int kFrame = 12;  // T per frame row
// Pair-resident level kernel (k_icp_level): workgroup size, and the largest
// level image (rows, pixels) it takes.
constexpr int kPairBlock = 1024;
constexpr int kPairRows = 64;
constexpr int kPairMaxPx = 8192;

// A level's target range image (learned-weight features).
struct LevelImage {
    const float *rng;
    int Hl, Wl;
};

// Per-pair flag words: flags[pair * kFlagStride + l] bit 0 = level l stopped;
// flags[pair * kFlagStride + kMaxLevels] bit 0 = learned weights rejected in
// the last iteration (a pseudo-Huber redo is pending).
constexpr int kFlagStride = kMaxLevels + 1;
// Concurrent sub-batches (streams) of the coarse levels of one batch.
constexpr int kMaxLanes = 4;
constexpr int kAccum = 32;  // float accumulators per tile (30 used)

enum StepMode { kStepNormal = 0, kStepFallback = 1, kStepDebug = 2 };

// Learned-weight network in device memory.
struct MlpDev {
    const uint16_t *w;  // bf16 W1[64][14], W2[64][64], W3[64]
    const float *b;     // b1[64], b2[64], b3
};
constexpr int kMlpW1 = 0, kMlpW2 = 64 * 14, kMlpW3 = 64 * 14 + 64 * 64, kMlpNW = 64 * 14 + 64 * 64 + 64;
constexpr int kMlpB1 = 0, kMlpB2 = 64, kMlpB3 = 128, kMlpNB = 129;

struct StepArgs {
    const void *pairs;   // PairDesc<T>[n_pairs]
    const int2 *tiles;   // (pair, first segment) of every tile of this level
    int n_tiles;         // tiles of this launch: tiles[tile_base .. tile_base + n_tiles)
    int tile_base;
    int pair_base;       // one-workgroup-per-pair launches cover pairs pair_base + blockIdx.x
    int level, iter, levels;
    int iters;           // iterations scheduled at this level
    int tile_seg;        // segments per tile at this level
    int chunk;           // pixels each thread keeps in flight (1, 2 or 4)
    int xcd_remap;
    int mode;            // StepMode
    int lean;            // 1: no receiver offset, no distance gate, no debug
                         // dumps, every row a whole number of segments and
                         // a power-of-two width (the kernel variant without
                         // those paths runs)
    int stats_pass;      // 1: also accumulate the statistics-only terms (robust
                         // cost, inlier and projection counts); set on the last
                         // scheduled iteration of a level and in debug mode
    int learned;         // the normal pass uses learned weights
    int fused;           // 1: the workgroup that finishes a pair's last tile
                         // solves that pair (no separate solve launch)
    int *tickets;        // [n_pairs] tiles finished in this launch (fused)
    void *psum;          // T[n_tiles][kAccum]
    int4 *pcnt;          // [n_tiles] (n_valid, n_inlier, n_proj, 0)
    double *poses;       // [n_pairs][16]
    rir_level_stats *stats;  // [n_pairs][levels] (debug: [1])
    int *flags;          // [n_pairs][kFlagStride]
    double delta, max_corr;
    double stop_eps;     // > 0: a level stops after a step with |xi| <= stop_eps
    float r_max;
    MlpDev mlp;
    // per-pixel dumps (debug mode; each may be null)
    int32_t *dbg_u, *dbg_v;
    uint8_t *dbg_mask;
    float *dbg_e, *dbg_w, *dbg_J, *dbg_feat;
};

// Neighbour features of the learned weight for one level (k_nbr_feats).
struct NbrArgs {
    const void *pairs;  // PairDesc<T>[n_pairs]
    int pair_base;      // the launch covers pairs pair_base + blockIdx.y
    int level;
    double delta;
};

struct PrepArgs {
    const void *pairs;  // PairDesc<T>[n_pairs]
    const int2 *tiles;  // level-0 tiles (pair, first segment)
    int n_tiles;        // tiles of this launch: tiles[tile_base .. tile_base + n_tiles)
    int tile_base;
    int pair_base;      // per-pair launches cover pairs pair_base + block index
    int tile_seg;
    int levels;
    int init_centroid;  // 1: compute t0 from the point-set centres
    int given_normals;  // 1: the level-0 records are already written (PCA
                        // target normals), the pass only copies them down
    double edge_rel;
    void *psum;         // T[n_tiles][kAccum] (centroid sums)
    double *poses;
    int xcd_remap;
};

// Launch wrappers (kernels.hip).  All enqueue on `stream` and return the
// launch status.
hipError_t launch_unproject(const SensorTab<float> &S, const float *range, float *xyz, uint8_t *valid,
                            hipStream_t stream);
hipError_t launch_project(const SensorTab<float> *tab, int level, const float *xyz, int64_t n, int32_t *u, int32_t *v,
                          float *r, uint8_t *valid, hipStream_t stream);
hipError_t launch_normals(const SensorTab<float> &S, const float *range, double edge_rel, float *nrm,
                          uint8_t *valid, hipStream_t stream);
hipError_t launch_clear(int *flags, int n_flags, rir_level_stats *stats, int n_stats, hipStream_t stream);
hipError_t launch_prepass(bool fp64, const PrepArgs &a, int grid, int block, int n_pairs, hipStream_t stream);
// Level-0 target records (n, n . q) from PCA normals of the (2 half + 1)^2
// window (normals_pca.hip) for every pair; max_px: the largest level-0 image.
hipError_t launch_pca_records(bool fp64, const PrepArgs &a, int half, int n_pairs, int max_px, hipStream_t stream);
// Neighbour features of level a.level for every pair with an nbf image there
// (FP32 instances only); max_px: the largest level image of the batch.
hipError_t launch_nbr_feats(const NbrArgs &a, int n_pairs, int max_px, hipStream_t stream);
hipError_t launch_solve(bool fp64, const StepArgs &a, int n_pairs, hipStream_t stream);
hipError_t launch_frames(bool fp64, const StepArgs &a, int n_pairs, hipStream_t stream);
hipError_t launch_step(bool fp64, int weight_mode, const StepArgs &a, int grid, int block, hipStream_t stream);
// All iterations of one level, one workgroup per pair (StepArgs::iters); FP32
// only (hipErrorInvalidValue for fp64).
hipError_t launch_level(bool fp64, const StepArgs &a, int n_pairs, hipStream_t stream);

// Learned-weight network (mlp.hip).
hipError_t launch_mlp_forward(const MlpDev &m, const float *feats, int64_t B, float *w_out, hipStream_t stream);
hipError_t launch_mlp_grad(const MlpDev &m, const float *feats, const float *labels, int64_t B, float *gpart,
                           int nblocks, hipStream_t stream);
hipError_t launch_mlp_adam(const float *gpart, int nblocks, int64_t B, float lr, int step, float *master,
                           float *bias, float *m1, float *m2, uint16_t *wbf, float *loss_out, float *grads_out,
                           hipStream_t stream);
int mlp_grad_blocks(int64_t B);
constexpr int kMlpGradRecord = 5185 + 1;  // gradient + loss per block
// Allocation-free training step: its gradient records live in a fixed device
// array of kMlpScratchRecords records per GPU, which holds the records of
// batches up to kMlpScratchMaxB samples (mlp_grad_blocks(kMlpScratchMaxB) ==
// kMlpScratchRecords).  mlp_scratch returns the array's device address on
// `device` (which must be current), looked up once per device.
constexpr int kMlpScratchRecords = 512;
constexpr int64_t kMlpScratchMaxB = 32768;
constexpr int kMlpMaxDevices = 64;
hipError_t mlp_scratch(int device, float **out);

}  // namespace rir
