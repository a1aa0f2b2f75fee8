// Device-side declarations of the entry points beside the registration path:
// projective SDF fusion into a dense block grid (Sec. 4.2, Eq. (8)-(10),
// sdf.hip), PCA normals (normals_pca.hip) and re-projection under per-column
// poses (deskew.hip).
#pragma once

#include "rir_internal.h"

namespace rir {

constexpr int kSdfEdge = 16;     // voxels per block edge
constexpr int kSdfFrames = 16;   // scans per launch (their poses travel as kernel arguments)

// World -> sensor pose of one scan (Eq. (8)): x_s = R x + t, R row-major.
struct SdfFrame {
    double R[9];
    double t[3];
};

struct SdfArgs {
    const SensorTab<float> *tab;
    const float *ranges;   // n_frames images of H x W, contiguous
    float *vox;            // (sdf, weight) per voxel, blocks in (bz, by, bx) order,
                           // voxels in (z, y, x) order inside a block
    int nbx, nby, nbz;
    int n_frames;          // 1..kSdfFrames
    int xcd_remap;
    float trunc;           // truncation band (+inf: none)
    float clip;            // largest float not above the range clip (+inf: none)
    double cull;           // > 0: blocks farther than this from a scan's sensor
                           // cannot be updated by it (< 0: no culling)
    double origin[3];      // world position of voxel (0, 0, 0)
    double voxel;          // voxel edge (m)
    SdfFrame f[kSdfFrames];
    // sparse volume (hashed launches): block b of the launch is pool slot b,
    // at block coordinates blocks[b].xyz, activated first by scan
    // act[blocks[b].w]; scan j of the launch (index frame0 + j in the
    // volume's history) updates only blocks activated by it or earlier
    const int4 *blocks;
    const int *act;
    int n_blocks;
    int frame0;
};

// One fusion launch over every block of the grid (hashed: of the pool).
hipError_t launch_sdf_fuse(const SdfArgs &a, bool r0, bool pow2, bool hashed, hipStream_t stream);

// PCA normals of n_images contiguous H x W range images; half = 1, 2 or 3
// (window 3x3, 5x5, 7x7), hipErrorInvalidValue otherwise.
hipError_t launch_normals_pca(const SensorTab<double> &S, const float *range, int n_images, int half, double edge_rel,
                              float *nrm, uint8_t *valid, hipStream_t stream);

// Re-projection of n_images contiguous H x W scans under per-column poses
// Exp(s_u xi_k) (deskew.hip); out must not overlap in.
hipError_t launch_deskew(const SensorTab<double> *tab, int H, int W, bool r0, int n_images, const float *in,
                         const double *twists, float *out, hipStream_t stream);

}  // namespace rir
