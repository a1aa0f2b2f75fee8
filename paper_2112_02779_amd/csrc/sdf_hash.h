// Sparse voxel-block volume (sdf_hash.hip): block activation in a hash table
// keyed by block coordinates, the table's neighbour and export helpers.
#pragma once

#include <algorithm>

#include "rir_ops.h"

namespace rir {

// Block coordinates are stored with this bias in 21 bits each.
constexpr int kBvolBias = 1 << 20;
constexpr unsigned long long kBvolEmpty = ~0ull;
// BvolDev::flags bits
constexpr int kBvolFull = 1;   // more blocks than the pool holds
constexpr int kBvolRange = 2;  // a return beyond the coordinate range of the table

// Device view of a block volume.  Table entry h: keys[h] (kBvolEmpty when
// free), vals[h] the entry's pool slot (-1 if none), act[h] the first scan
// that activated it (INT_MAX-like when never).  Pool slot s: blocks[s] =
// (bx, by, bz, h), voxels at s * 4096 (SdfArgs layout within a block).
struct BvolDev {
    unsigned long long *keys;
    int *vals;
    int *act;
    int4 *blocks;
    int *count;   // blocks inserted (may exceed max_blocks: then flags has kBvolFull)
    int *flags;
    uint32_t mask;  // table capacity - 1 (a power of two)
    int max_blocks;
};

struct BvolActArgs {
    const SensorTab<double> *tab;
    const float *ranges;  // n_frames images of H x W, contiguous
    int n_frames, H, W;
    int frame0;           // index of the launch's first scan in the volume's history
    double origin[3];     // world position of voxel (0, 0, 0)
    double radius;        // half edge of the activation cube (m)
    double clip;          // > 0: returns beyond it activate nothing
    double edge;          // block edge (16 voxels, m)
    SdfFrame f[kSdfFrames];
    BvolDev t;
};

hipError_t launch_bvol_activate(const BvolActArgs &a, hipStream_t stream);
hipError_t launch_bvol_neighbors(const BvolDev &t, int n_blocks, int *nbr, hipStream_t stream);
hipError_t launch_bvol_export(const BvolDev &t, int n_blocks, int4 *out, hipStream_t stream);

}  // namespace rir
