"""CPU checks of the measurement helpers in bench.py that score reconstructions:
exact point-to-scene distances against dense samples of the same surfaces."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def _surface_samples(scene, n_per=4000, rng=None):
    """Dense random samples on the scene's finite surfaces (the ground plane
    only over a bounded patch)."""
    rng = rng or np.random.default_rng(0)
    pts = []
    xy = rng.uniform(-6, 6, size=(n_per * 4, 2))
    pts.append(np.column_stack([xy, np.zeros(len(xy))]))          # plane z = 0
    for b in scene.boxes:
        lo, hi = b[:3], b[3:]
        for ax in range(3):
            for side in (lo[ax], hi[ax]):
                p = rng.uniform(lo, hi, size=(n_per, 3))
                p[:, ax] = side
                pts.append(p)
    for cx, cy, r, z0, z1 in scene.cyls:
        a = rng.uniform(0, 2 * np.pi, n_per)
        pts.append(np.column_stack([cx + r * np.cos(a), cy + r * np.sin(a), rng.uniform(z0, z1, n_per)]))
        for zc in (z0, z1):
            rr = r * np.sqrt(rng.uniform(0, 1, n_per))
            pts.append(np.column_stack([cx + rr * np.cos(a), cy + rr * np.sin(a), np.full(n_per, zc)]))
    return np.concatenate(pts)


def test_scene_distance_matches_dense_samples():
    scene = synth.Scene(np.array([[0, 0, 1, 0.0]]),
                        np.array([[0.5, 0.5, 0.0, 1.5, 2.0, 1.2], [-3, -2, 0, -2, -1, 2.5]]),
                        np.array([[2.5, -2.0, 0.6, 0.0, 3.0]]))
    rng = np.random.default_rng(1)
    q = rng.uniform([-4, -4, -0.5], [4, 4, 3.5], size=(400, 3))
    d = bench._scene_distance(scene, q)
    S = _surface_samples(scene, rng=rng)
    from scipy.spatial import cKDTree
    brute = cKDTree(S).query(q)[0]
    # the samples are a subset of the surfaces: brute force is an upper bound,
    # tight to the sampling spacing
    assert np.all(d <= brute + 1e-12)
    assert np.max(brute - d) < 0.08
    # points on the surfaces are at distance 0
    assert np.max(bench._scene_distance(scene, S[::97])) < 1e-12
