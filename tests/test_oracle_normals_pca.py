"""Pins of the oracle's PCA normals (the eigen-decomposition estimator named in
Sec. 4.1) against facts other than itself (CPU only): numpy's symmetric
eigen-solver, analytic plane normals of noise-free ray-cast scans, and a
brute-force numpy evaluation of the window definition on a tiny image.
"""
import numpy as np
import pytest

import synth


def test_eigen3_matches_numpy_eigh(orc):
    rng = np.random.default_rng(1)
    cases = []
    for _ in range(200):
        M = rng.normal(size=(3, 3))
        cases.append(M @ M.T)
    cases.append(np.diag([3.0, 1.0, 2.0]))                    # already diagonal, unsorted
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    cases.append(Q @ np.diag([1e-9, 1.0, 1.0]) @ Q.T)          # repeated top pair, tiny smallest
    for A in cases:
        lam, V = orc.eigen3(A)
        l2, V2 = np.linalg.eigh(A)
        np.testing.assert_allclose(lam, l2, rtol=0, atol=1e-13 * max(1.0, abs(l2).max()))
        np.testing.assert_allclose(V.T @ V, np.eye(3), atol=1e-13)
        np.testing.assert_allclose(A @ V, V * lam, atol=1e-12 * max(1.0, abs(l2).max()))
        if l2[1] - l2[0] > 1e-6 * l2[2]:
            assert abs(abs(V[:, 0] @ V2[:, 0]) - 1) < 1e-12


@pytest.mark.parametrize("half", [1, 2])
def test_pca_normals_of_planes(orc, half):
    """Noise-free scan of a room: where every pixel of the window hits the same
    plane, the PCA normal is that plane's normal, oriented to the sensor."""
    sen = synth.uniform_sensor(64, 1024)
    rng = np.random.default_rng(4)
    scene = synth.room_scene(rng, n_boxes=10)
    pos = np.array([0.0, 0.0, 1.8])
    r, hit = synth.raycast(sen, scene, synth.make_pose(np.eye(3), pos))
    n, valid, lam = orc.normals_pca(sen, r.astype(np.float32), half=half)
    H, W = hit.shape
    same = np.ones_like(valid)
    for dv in range(-half, half + 1):
        for du in range(-half, half + 1):
            sh = np.roll(np.roll(hit, -dv, 0), -du, 1)
            same &= sh == hit
    same[:half] = False
    same[H - half:] = False
    checked = 0
    for k, pl in enumerate(scene.planes):
        m = valid & same & (hit == k)
        ref = np.asarray(pl[:3], dtype=np.float64)
        ref /= np.linalg.norm(ref)
        if pl[:3] @ pos + pl[3] < 0:
            ref = -ref
        # the scan holds FP32 ranges (relative rounding 6e-8, over a window a
        # few pixel spacings wide)
        assert np.max(np.arccos(np.clip(n[m] @ ref, -1, 1)), initial=0.0) < 5e-5
        assert np.all(lam[m][:, 0] <= 1e-8 * lam[m][:, 2])
        checked += m.sum()
    assert checked > 20000
    assert not valid[r <= 0].any()


def test_pca_window_brute_force(orc):
    """The definition evaluated directly with numpy on a tiny noisy image:
    window (u wraps, rows cut), range gate, count threshold, mean-centred
    covariance, smallest eigenvector by numpy, orientation and the line test."""
    H, W, half = 7, 12, 1
    sen = synth.staggered_sensor(H, W, r0=0.03)
    rng = np.random.default_rng(3)
    img = rng.uniform(9.0, 11.2, size=(H, W)).astype(np.float32)
    img[rng.random((H, W)) < 0.15] = 0.0
    img[3, 4] = np.nan
    n, valid, _ = orc.normals_pca(sen, img, half=half, edge_rel=0.1)
    k = 2 * half + 1
    for v in range(H):
        for u in range(W):
            c = float(img[v, u])
            ok = np.isfinite(c) and c > 0
            pts = []
            if ok:
                for dv in range(-half, half + 1):
                    if not 0 <= v + dv < H:
                        continue
                    for du in range(-half, half + 1):
                        uu = (u + du) % W
                        x = float(img[v + dv, uu])
                        if np.isfinite(x) and x > 0 and abs(x - c) <= 0.1 * c:
                            pts.append(orc.unproject(sen, uu, v + dv, x))
            ok = ok and len(pts) >= (k * k + 1) // 2
            if ok:
                P = np.array(pts)
                C = np.cov(P.T, bias=True)
                l2, V2 = np.linalg.eigh(C)
                ok = l2[1] > 1e-6 * l2[2]
            assert valid[v, u] == ok, (v, u)
            if ok:
                ref = V2[:, 0]
                d = orc.unproject(sen, u, v, 1.0) - orc.unproject(sen, u, v, 0.0)
                if ref @ d > 0:
                    ref = -ref
                np.testing.assert_allclose(n[v, u], ref, atol=1e-9)
    assert valid.sum() > 20



def test_icp_with_pca_normals_uses_exactly_the_pca_normals(orc):
    """normal_window = h: the association's Jacobian rows carry, at every
    valid correspondence, the PCA normal of the associated target pixel
    (J = [x cross n, n]); pixels whose PCA normal is invalid never associate."""
    p = synth.gen_pair(synth.CONFIGS["pair64"], 7, shape=(32, 512))
    for h in (1, 2):
        prm = orc.make_params(levels=1, iters=[1], normal_window=h)
        out = orc.system(p.sensor, 0, p.src, p.dst, prm, p.gt)
        n, valid, _ = orc.normals_pca(p.sensor, p.dst, half=h, edge_rel=0.1)
        m = out["mask"]
        assert m.sum() > 1000
        uu, vv = out["u"][m], out["v"][m]
        assert np.all(valid[vv, uu])
        np.testing.assert_array_equal(out["J"][m][:, 3:6], n[vv, uu])


@pytest.mark.parametrize("h", [1, 2])
def test_icp_with_pca_normals_converges_on_planar_scene(orc, h):
    """Sec. 4.1 with the eigen-decomposition estimator: on a noise-free room
    (ground and four walls) the multi-scale registration recovers the known
    motion from the identity."""
    sen = synth.uniform_sensor(64, 1024)
    rng = np.random.default_rng(1)
    scene = synth.room_scene(rng, n_boxes=0)
    Ta = synth.make_pose(np.eye(3), [0, 0, 1.8])
    dT = synth.random_motion(rng, 5.0, 1.0)
    nz = synth.ScanNoise(0.0, 0.5, 80.0, 0.0, 0.0)
    a = synth.scan(sen, scene, Ta, nz, rng)["range"]
    b = synth.scan(sen, scene, Ta @ dT, nz, rng)["range"]
    T, st = orc.icp(sen, b, a, orc.make_params(levels=3, iters=[10, 10, 10], normal_window=h))
    er, et = orc.pose_error(T, dT)
    assert er < 4e-4 and et < 2e-3, (er, et)
