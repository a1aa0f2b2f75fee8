"""Helpers shared by the GPU parity tests: device transfer, the library
handles of a synthetic pair, and the ambiguity band of pose-dependent indices.

Indices computed in FP32 on the GPU and in FP64 by the oracle can differ only
where the continuous quantity they round lies next to a rounding boundary.
A pixel is ambiguous when its FP64 column coordinate is within BAND_U pixels
of a half-integer, or its FP64 elevation is within BAND_PHI row spacings of
a level midpoint or of a field-of-view edge.  Outside the band indices and
masks must agree bit for bit; inside it either neighbour is accepted.
"""
import numpy as np

BAND_U = 2e-3     # pixels
BAND_PHI = 1e-3   # fraction of the local row spacing


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def level_midpoints(phi_lut, level):
    s = 1 << level
    p = phi_lut[::s]
    return 0.5 * (p[:-1] + p[1:]), np.abs(np.diff(p))


def ambiguous(sensor, level, uhat, phi):
    """Boolean mask of pixels whose rounding is ambiguous (see module doc)."""
    uhat = np.asarray(uhat, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    frac = uhat - np.floor(uhat)
    amb = np.abs(frac - 0.5) < BAND_U
    mids, gaps = level_midpoints(sensor.phi, level)
    if mids.size:
        d = np.abs(phi[..., None] - mids)
        k = np.argmin(d, axis=-1)
        amb |= d.min(axis=-1) < BAND_PHI * gaps[k]
    p = sensor.phi
    hi = p[0] + 0.5 * (p[0] - p[1])
    lo = p[-1] - 0.5 * (p[-2] - p[-1])
    edge_gap = min(p[0] - p[1], p[-2] - p[-1])
    amb |= (np.abs(phi - hi) < BAND_PHI * edge_gap) | (np.abs(phi - lo) < BAND_PHI * edge_gap)
    return amb


BAND_D = 1e-4     # metres: signed distances this close to -trunc are ambiguous


def sdf_ambiguous(sensor, ranges, poses, pts, trunc, r_clip=0.0):
    """Voxels (world points pts) whose fused value FP32 and FP64 may
    legitimately disagree on: in some scan the projection falls in the
    rounding band above, or the signed distance lies within BAND_D of the
    truncation limit.  With both trunc and r_clip set, scans farther than
    r_clip + trunc + r0 from the point (plus 1 mm) cannot observe it whatever
    pixel it lands on and do not count.  Uses the oracle's projections."""
    import oracle
    amb = np.zeros(len(pts), bool)
    pts = np.asarray(pts, dtype=np.float64)
    for f in range(len(ranges)):
        o = oracle.sdf_points(sensor, ranges[f], poses[f], pts)
        a = ambiguous(sensor, 0, o["uhat"], o["phi"])
        if trunc > 0:
            a |= o["valid"] & (np.abs(o["d"] + trunc) < BAND_D)
        if trunc > 0 and r_clip > 0:
            xs = pts @ poses[f][:3, :3].T + poses[f][:3, 3]
            a &= np.linalg.norm(xs, axis=1) <= r_clip + trunc + sensor.r0 + 1e-3
        amb |= a
    return amb


def rot_trans_error(T, Tref):
    """Rotation angle (rad, via the skew part, accurate near zero) and
    translation distance between two 4x4 poses."""
    R = T[:3, :3] @ Tref[:3, :3].T
    s = np.linalg.norm([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]]) / 2
    c = (np.trace(R) - 1) / 2
    return float(np.arctan2(s, c)), float(np.linalg.norm(T[:3, 3] - Tref[:3, 3]))


# Learned weight: the products of bf16 weights and bf16 activations are exact
# in FP32, so an FP32 evaluation of a hidden pre-activation (K products plus
# the bias, summed in any order) differs from the exact sum by at most
# (K - 1) u s, and its own rounding adds u |a| <= u s (u = 2^-24, s the sum of
# the magnitudes of the terms).  A value farther than (K + 1) u s from a bf16
# tie therefore rounds to the same bf16 activation on both sides.
MLP_BAND_FACTOR = 1.0


def _bf16_tie_distance(x):
    """Distance of each value to the nearest rounding boundary of bf16
    (round-to-nearest-even ties lie halfway between neighbouring bf16
    values)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    bits = x.astype(np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    one = np.uint32(0x10000)
    # largest bf16 value <= x (float32 rounding may have stepped above x)
    bits = np.where(bits.view(np.float32).astype(np.float64) > x, bits - one, bits)
    val = lambda b: b.view(np.float32).astype(np.float64)
    lo, hi, below = val(bits), val(bits + one), val(bits - one)
    return np.minimum(np.abs(x - 0.5 * (lo + hi)), np.abs(x - 0.5 * (below + lo)))


def mlp_band(pre):
    """Rows (feature vectors) whose bf16 hidden activations an FP32
    evaluation may round to a neighbouring value: some positive hidden
    pre-activation lies within the FP32 rounding bound of a bf16 tie.
    `pre` is the oracle's mlp_preact output."""
    u = 2.0 ** -24
    band = np.zeros(pre["a1"].shape[0], bool)
    for a, s, k in ((pre["a1"], pre["s1"], 16), (pre["a2"], pre["s2"], 66)):
        tol = MLP_BAND_FACTOR * k * u * s
        band |= np.any((a > -tol) & (_bf16_tie_distance(a) <= tol), axis=1)
    return band
