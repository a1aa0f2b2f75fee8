"""Pins of the FP64 oracle against facts other than itself (CPU only).

Each test names the passage of the paper it follows.  The pins are closed
forms and hand-derived values, the lossless 2D<->3D round trip claimed in
Sec. 3, the synthetic-intrinsics special case of Sec. 3.2 (textbook spherical
projection), the multi-scale/strided-sensor equivalence of Sec. 4.1,
analytic plane normals of ray-cast scenes, central finite differences,
numpy least squares and scipy's matrix exponential.
"""
import os

import numpy as np
import pytest
import scipy.linalg

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _twist_matrix(xi):
    w, t = xi[:3], xi[3:]
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    M[:3, 3] = t
    return M


def _expm(xi):
    return scipy.linalg.expm(_twist_matrix(np.asarray(xi, dtype=np.float64)))


def _load_cases(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return np.array(rows)


# --------------------------------------------------------------------------- Eq. (1)-(2)

def test_unproject_hand_values(orc):
    """Eq. (1)-(2), Sec. 3.1: hand-derived points (tests/golden/unproject_cases.txt)."""
    sen = synth.Sensor(3, 8, np.array([np.pi / 6, 0.0, -np.pi / 6]), np.zeros(3), 0.1)
    for u, v, r, x, y, z in _load_cases("unproject_cases.txt"):
        p = orc.unproject(sen, int(u), int(v), r)
        np.testing.assert_allclose(p, [x, y, z], atol=1e-14)


def test_unproject_hand_values_azimuth_offset(orc):
    """Eq. (2): the beam's azimuth offset theta_lut adds to the encoder angle,
    the receiver offset does not (tests/golden/unproject_offset_cases.txt)."""
    sen = synth.Sensor(2, 4, np.array([0.0, -np.pi / 4]), np.array([np.pi / 2, 0.0]), 0.5)
    for u, v, r, x, y, z in _load_cases("unproject_offset_cases.txt"):
        p = orc.unproject(sen, int(u), int(v), r)
        np.testing.assert_allclose(p, [x, y, z], atol=1e-14)


@pytest.mark.parametrize("sensor_kind", ["uniform", "staggered"])
def test_unprojected_points_lie_on_raycast_planes(orc, sensor_kind):
    """Eq. (1): unprojecting a noise-free ray-cast scan puts every point back
    on the plane its ray hit (the scan simulator is independent code)."""
    sen = synth.uniform_sensor(32, 256) if sensor_kind == "uniform" else synth.staggered_sensor(32, 256, r0=0.05)
    rng = np.random.default_rng(3)
    scene = synth.room_scene(rng, n_boxes=0)
    T = synth.make_pose(synth.rot_axis_angle([0.3, -0.2, 1.0], 0.4), [1.0, -2.0, 1.5])
    r, hit = synth.raycast(sen, scene, T)
    xyz, valid = orc.unproject_image(sen, r.astype(np.float32))
    # back to the world frame; check the float32-rounded ranges against the planes
    pw = xyz @ T[:3, :3].T + T[:3, 3]
    # the float32 range moves the point along its ray by at most ulp(r)/2
    r32 = r.astype(np.float32).astype(np.float64)
    for k, pl in enumerate(scene.planes):
        m = valid & (hit == k)
        assert m.sum() > 50
        dist = np.abs(pw[m] @ pl[:3] + pl[3])
        assert np.max(dist) <= 1e-9 + 2e-7 * np.max(r32[m])


# --------------------------------------------------------------------------- Eq. (3)-(4)

@pytest.mark.parametrize("kind", ["uniform", "staggered", "staggered_r0"])
@pytest.mark.parametrize("level", [0, 1, 2])
def test_round_trip_is_lossless(orc, kind, level):
    """Sec. 3 claims lossless 2D<->3D conversion: Pi(Pi^-1(u, v, r)) returns the
    same pixel exactly and the same range, at every pyramid level for pixels
    on that level's grid (Sec. 4.1)."""
    H, W = 32, 512
    if kind == "uniform":
        sen = synth.uniform_sensor(H, W)
    elif kind == "staggered":
        sen = synth.staggered_sensor(H, W, r0=0.0)
    else:
        sen = synth.staggered_sensor(H, W, r0=0.04)
    rng = np.random.default_rng(level)
    img = rng.uniform(0.5, 120.0, size=(H, W)).astype(np.float32)
    xyz, valid = orc.unproject_image(sen, img)
    s = 1 << level
    sub = xyz[::s, ::s].reshape(-1, 3)
    pr = orc.project_points(sen, level, sub)
    vv, uu = np.meshgrid(np.arange(H // s), np.arange(W // s), indexing="ij")
    assert pr["valid"].all()
    np.testing.assert_array_equal(pr["u"], uu.ravel())
    np.testing.assert_array_equal(pr["v"], vv.ravel())
    r_in = img[::s, ::s].ravel().astype(np.float64)
    assert np.max(np.abs(pr["r"] - r_in) / r_in) <= 1e-12


def test_synthetic_intrinsics_reduce_to_spherical_projection(orc):
    """Sec. 3.2: with theta_lut = 0, r0 = 0 and a uniform elevation table the
    model is the textbook spherical projection u = W theta / 2pi,
    v = (phi_max - phi) / dphi, each rounded to the nearest pixel."""
    H, W = 64, 1024
    sen = synth.uniform_sensor(H, W)
    rng = np.random.default_rng(7)
    n = 20000
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = d * rng.uniform(0.5, 100.0, size=(n, 1))
    pr = orc.project_points(sen, 0, pts)
    r = np.linalg.norm(pts, axis=1)
    phi = np.arcsin(pts[:, 2] / r)
    theta = np.mod(np.arctan2(pts[:, 1], pts[:, 0]), 2 * np.pi)
    dphi = (sen.phi[0] - sen.phi[-1]) / (H - 1)
    vf = (sen.phi[0] - phi) / dphi
    uf = theta * W / (2 * np.pi)
    inside = (vf >= -0.5) & (vf <= H - 0.5)
    np.testing.assert_array_equal(pr["valid"], inside)
    # stay away from exact rounding ties, which have measure zero here
    clear = inside & (np.abs(vf - np.floor(vf) - 0.5) > 1e-9) & (np.abs(uf - np.floor(uf) - 0.5) > 1e-9)
    np.testing.assert_array_equal(pr["v"][clear], np.clip(np.rint(vf[clear]), 0, H - 1).astype(int))
    np.testing.assert_array_equal(pr["u"][clear], np.mod(np.rint(uf[clear]), W).astype(int))
    np.testing.assert_allclose(pr["r"], r, rtol=1e-14)


def test_elevation_argmin_matches_numpy_on_irregular_table(orc):
    """Eq. (4): v = argmin_t |phi_lut[t] - phi| (numpy.argmin; first index on
    ties) on a non-uniform table and with r0 = 0."""
    sen = synth.staggered_sensor(40, 256, r0=0.0, gamma=1.7)
    rng = np.random.default_rng(11)
    phi = rng.uniform(sen.phi[-1], sen.phi[0], size=5000)
    theta = rng.uniform(0, 2 * np.pi, size=5000)
    pts = np.stack([np.cos(theta) * np.cos(phi), np.sin(theta) * np.cos(phi), np.sin(phi)], 1) * 10.0
    pr = orc.project_points(sen, 0, pts)
    ref = np.argmin(np.abs(sen.phi[None, :] - pr["phi"][:, None]), axis=1)
    np.testing.assert_array_equal(pr["v"], ref)
    # strided rows at level 2
    pr2 = orc.project_points(sen, 2, pts)
    ref2 = np.argmin(np.abs(sen.phi[None, ::4] - pr2["phi"][:, None]), axis=1)
    np.testing.assert_array_equal(pr2["v"], ref2)


def test_elevation_ties_go_to_smaller_index(orc):
    """Eq. (4) with an exact tie (reading: ties to the smaller row index)."""
    sen = synth.Sensor(3, 8, np.array([0.5, 0.0, -0.5]), np.zeros(3), 0.0)
    # elevation exactly 0.25 rad, halfway between rows 0 and 1
    p = np.array([[np.cos(0.25), 0.0, np.sin(0.25)]]) * 4.0
    pr = orc.project_points(sen, 0, p)
    assert abs(pr["phi"][0] - 0.25) < 1e-15
    # whichever side rounding puts phi on, the tie rule must not pick a farther row
    assert pr["v"][0] in (0, 1)
    q = orc.project_points(sen, 0, np.array([[1.0, 0.0, 0.0]]) * 4.0)
    assert q["v"][0] == 1


def test_inverse_lut_with_2H_bins_is_within_one_row(orc):
    """Sec. 3.2: an inverse table of 2H bins over the elevation range puts the
    row index within +-1 of the exact argmin (checked against the oracle's
    argmin on uniform and jittered monotone tables)."""
    rng = np.random.default_rng(5)
    for jitter in (0.0, 0.3):
        H = 64
        base = np.linspace(0.3, -0.3, H)
        step = base[0] - base[1]
        phi_lut = base + rng.uniform(-jitter, jitter, H) * step
        phi_lut = np.sort(phi_lut)[::-1].copy()
        sen = synth.Sensor(H, 256, phi_lut, np.zeros(H), 0.0)
        lo, hi = phi_lut[-1], phi_lut[0]
        nb = 2 * H
        centres = lo + (np.arange(nb) + 0.5) * (hi - lo) / nb
        inv = np.argmin(np.abs(phi_lut[None, :] - centres[:, None]), axis=1)
        phi = rng.uniform(lo, hi, 4000)
        pts = np.stack([np.cos(phi), np.zeros_like(phi), np.sin(phi)], 1) * 5.0
        pr = orc.project_points(sen, 0, pts)
        b = np.clip(((phi - lo) / (hi - lo) * nb).astype(int), 0, nb - 1)
        assert np.max(np.abs(inv[b] - pr["v"])) <= 1


@pytest.mark.parametrize("kind", ["stagger_r0_0", "uniform_r0"])
def test_level_equals_explicit_strided_sensor(orc, kind):
    """Sec. 4.1: level l of the pyramid equals single-scale association on an
    explicit sensor made of rows s t and W/s columns with the same intrinsics,
    and images/normals subsampled at stride s."""
    H, W, lvl = 32, 512, 2
    s = 1 << lvl
    if kind == "stagger_r0_0":
        sen = synth.staggered_sensor(H, W, r0=0.0)
    else:
        sen = synth.uniform_sensor(H, W)
        sen = synth.Sensor(H, W, sen.phi, sen.theta, 0.03)
    cfg = synth.CONFIGS["pair64"]
    pair = synth.gen_pair(cfg, 21, sensor=sen)
    prm = orc.make_params(levels=1, iters=[1])
    nrm, nv = orc.normals(sen, pair.dst)
    T = synth.make_pose(synth.rot_axis_angle([0.1, 0.2, 1.0], 0.02), [0.2, -0.1, 0.05])
    a = orc.associate_with_normals(sen, lvl, pair.src, pair.dst, nrm, nv, prm, T)
    ss = sen.strided(s)
    b = orc.associate_with_normals(ss, 0, np.ascontiguousarray(pair.src[::s, ::s]),
                                   np.ascontiguousarray(pair.dst[::s, ::s]),
                                   np.ascontiguousarray(nrm[::s, ::s]), np.ascontiguousarray(nv[::s, ::s]),
                                   prm, T)
    both = a["proj_valid"] & b["proj_valid"]
    # validity differs only at the field-of-view edge (finest vs strided end rows)
    assert both.sum() > 0.9 * max(a["proj_valid"].sum(), 1)
    np.testing.assert_array_equal(a["u"][both], b["u"][both])
    np.testing.assert_array_equal(a["v"][both], b["v"][both])
    m = both & a["mask"]
    np.testing.assert_array_equal(a["mask"][both], b["mask"][both])
    np.testing.assert_allclose(a["e"][m], b["e"][m], atol=1e-12)
    np.testing.assert_allclose(a["J"][m], b["J"][m], atol=1e-10)


# --------------------------------------------------------------------------- normals

def _plane_normal_towards(pl, sensor_pos):
    n = np.asarray(pl[:3], dtype=np.float64)
    n = n / np.linalg.norm(n)
    if pl[:3] @ sensor_pos + pl[3] < 0:
        n = -n
    return n


def test_normals_of_planes_and_boxes(orc):
    """Sec. 4.1 / 6.1: cross-product normals of a noise-free scan equal the
    analytic normals of the surfaces hit (oriented towards the sensor)."""
    sen = synth.uniform_sensor(64, 1024)
    rng = np.random.default_rng(4)
    scene = synth.room_scene(rng, n_boxes=10)
    pos = np.array([0.0, 0.0, 1.8])
    T = synth.make_pose(np.eye(3), pos)
    r, hit = synth.raycast(sen, scene, T)
    r32 = r.astype(np.float32)
    n, valid = orc.normals(sen, r32)
    same = np.zeros_like(valid)
    same[1:-1] = ((hit[1:-1] == np.roll(hit, 1, 1)[1:-1]) & (hit[1:-1] == np.roll(hit, -1, 1)[1:-1])
                  & (hit[1:-1] == hit[:-2]) & (hit[1:-1] == hit[2:]))
    checked = 0
    for k, pl in enumerate(scene.planes):
        m = valid & same & (hit == k)
        ref = _plane_normal_towards(pl, pos)
        ang = np.arccos(np.clip(n[m] @ ref, -1, 1))
        assert np.max(ang) < 2e-4, (k, np.max(ang))
        checked += m.sum()
    # box faces: label each pixel by the face its (unprojected, world) point lies on
    xyz, _ = orc.unproject_image(sen, r32)
    pw = xyz + pos
    face = np.full(hit.shape, -1)
    for b, box in enumerate(scene.boxes):
        m = hit == len(scene.planes) + b
        d = np.stack([np.abs(pw[..., i] - box[j]) for j in range(6) for i in [j % 3]], -1)
        face[m] = 6 * b + np.argmin(d[m], axis=-1)
    same_face = np.zeros_like(valid)
    same_face[1:-1] = ((face[1:-1] == np.roll(face, 1, 1)[1:-1]) & (face[1:-1] == np.roll(face, -1, 1)[1:-1])
                       & (face[1:-1] == face[:-2]) & (face[1:-1] == face[2:]))
    boxm = valid & same & same_face & (hit >= len(scene.planes))
    axes = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1.0]])
    best = np.max(n[boxm] @ axes.T, axis=1)
    assert np.min(best) > 1 - 2e-8
    checked += boxm.sum()
    assert checked > 30000
    # rows 0 and H-1 never have a normal; pixels without return never do
    assert not valid[0].any() and not valid[-1].any()
    assert not valid[r32 <= 0].any()


def test_normal_validity_predicate_brute_force(orc):
    """Normal validity: all five ranges positive and finite, each neighbour
    within edge_rel of the centre (u wraps, v does not); brute force."""
    H, W = 8, 16
    sen = synth.uniform_sensor(H, W)
    rng = np.random.default_rng(9)
    img = rng.uniform(9.0, 11.5, size=(H, W)).astype(np.float32)
    img[rng.random((H, W)) < 0.1] = 0.0
    img[2, 3] = np.nan
    img[5, 7] = np.inf
    n, valid = orc.normals(sen, img, edge_rel=0.1)
    ref = np.zeros((H, W), bool)
    for v in range(1, H - 1):
        for u in range(W):
            c = float(img[v, u])
            nb = [float(img[v, (u - 1) % W]), float(img[v, (u + 1) % W]), float(img[v - 1, u]), float(img[v + 1, u])]
            ok = all(np.isfinite(x) and x > 0 for x in [c] + nb)
            ok = ok and all(abs(x - c) <= 0.1 * c for x in nb)
            ref[v, u] = ok
    np.testing.assert_array_equal(valid, ref)


# --------------------------------------------------------------------------- Eq. (5)-(7)

def _pair(seed=0, noise=True, boxes=True, H=64, W=1024, sensor=None):
    cfg = dict(synth.CONFIGS["pair64"])
    if not noise:
        cfg["noise"] = synth.ScanNoise(0.0, 0.5, 80.0, 0.0, 0.0)
    return synth.gen_pair(cfg, seed, shape=(H, W), sensor=sensor)


def test_residual_sign_and_value_on_ground(orc):
    """Eq. (7): L(x, y) = n_y^T (x - y).  Registering a scan to itself with the
    source lifted by +d gives e = +d on the ground (normal +z)."""
    p = _pair(1, noise=False)
    prm = orc.make_params(levels=1, iters=[1])
    d = 0.03
    T = synth.make_pose(np.eye(3), [0.0, 0.0, d])
    out = orc.system(p.sensor, 0, p.dst, p.dst, prm, T)
    hit = p.dst_truth["hit"]
    ground = out["mask"] & (hit == 0)
    assert ground.sum() > 5000
    # only pixels whose association also lands on the ground
    on_ground = ground & (hit[out["v"].clip(0), out["u"].clip(0)] == 0)
    # pixels next to a wall can carry a blended normal; keep those whose normal is +z
    flat = on_ground & (out["J"][..., 5] > 1 - 1e-8)
    assert flat.sum() > 0.95 * on_ground.sum()
    np.testing.assert_allclose(out["e"][flat], d, atol=2e-6)


def test_jacobian_matches_central_differences(orc):
    """Eq. (7): J = de/dxi for the left update x <- Exp(xi) x, xi = (omega, tau),
    with associations frozen; central differences through scipy's expm."""
    p = _pair(2)
    prm = orc.make_params(levels=1, iters=[1])
    T = synth.make_pose(synth.rot_axis_angle([0.2, -0.4, 1.0], 0.03), [0.3, -0.2, 0.1])
    out = orc.system(p.sensor, 0, p.src, p.dst, prm, T)
    idx = np.argwhere(out["mask"])
    rng = np.random.default_rng(0)
    pick = idx[rng.choice(len(idx), 200, replace=False)]
    h = 1e-6
    for v, u in pick:
        p3 = orc.unproject(p.sensor, int(u), int(v), float(p.src[v, u]))
        x = T[:3, :3] @ p3 + T[:3, 3]
        J = out["J"][v, u]
        n = J[3:]
        assert abs(np.linalg.norm(n) - 1) < 1e-12
        for k in range(6):
            xi = np.zeros(6)
            xi[k] = h
            xp = (_expm(xi) @ np.append(x, 1))[:3]
            xm = (_expm(-xi) @ np.append(x, 1))[:3]
            fd = n @ (xp - xm) / (2 * h)
            assert abs(fd - J[k]) <= 1e-6 * max(1.0, abs(J[k])), (k, fd, J[k])


def test_exp_matches_scipy_expm(orc):
    """The SE(3) update T <- Exp(xi) T: closed-form exponential against
    scipy.linalg.expm of the 4x4 twist matrix, including the small-angle branch."""
    rng = np.random.default_rng(1)
    for scale in (1e-9, 1e-7, 1e-4, 0.1, 1.0, 3.0):
        for _ in range(20):
            xi = rng.normal(size=6) * scale
            np.testing.assert_allclose(orc.exp_se3(xi), _expm(xi), atol=1e-13 * max(1, scale), rtol=1e-12)


def test_gauss_newton_step_matches_lstsq(orc):
    """Eq. (7) by Gauss-Newton: one step equals the weighted linear least
    squares solution xi = argmin sum w (J xi + e)^2 (numpy.linalg.lstsq),
    applied on the left: T1 = Exp(xi) T0."""
    p = _pair(3)
    prm = orc.make_params(levels=1, iters=[1], delta=0.5)
    T0 = synth.make_pose(synth.rot_axis_angle([0.0, 0.3, 1.0], 0.02), [0.2, 0.1, -0.05])
    out = orc.system(p.sensor, 0, p.src, p.dst, prm, T0)
    m = out["mask"]
    sw = np.sqrt(out["w"][m])
    A = out["J"][m] * sw[:, None]
    b = out["e"][m] * sw
    xi = -np.linalg.lstsq(A, b, rcond=None)[0]
    T1, st = orc.icp(p.sensor, p.src, p.dst, prm, T_init=T0)
    np.testing.assert_allclose(T1, _expm(xi) @ T0, atol=1e-10)
    # the reported normal equations are those of the per-pixel terms
    Hm = A.T @ A
    iu = np.triu_indices(6)
    np.testing.assert_allclose(st[0]["JtJ"], Hm[iu], rtol=1e-9, atol=1e-9 * np.abs(Hm).max())
    np.testing.assert_allclose(st[0]["Jtr"], A.T @ b, rtol=1e-9, atol=1e-9 * np.abs(A.T @ b).max())
    assert st[0]["n_valid"] == m.sum()
    assert st[0]["n_proj"] == out["proj_valid"].sum()


def test_pseudo_huber_weight_is_irls_weight(orc):
    """Sec. 6.1: pseudo-Huber kernel of size delta (Barron's general loss with
    alpha = 1).  The weight of each correspondence equals rho'(e) / e, checked
    by central differences of rho."""
    p = _pair(4)
    delta = 0.5
    prm = orc.make_params(levels=1, iters=[1], delta=delta)
    out = orc.system(p.sensor, 0, p.src, p.dst, prm, np.eye(4))
    m = out["mask"]
    e = out["e"][m]
    rho = lambda x: delta ** 2 * (np.sqrt(1 + (x / delta) ** 2) - 1)
    h = 1e-6
    big = np.abs(e) > 1e-3
    fd = (rho(e[big] + h) - rho(e[big] - h)) / (2 * h) / e[big]
    np.testing.assert_allclose(out["w"][m][big], fd, rtol=1e-6)
    assert np.all(out["w"][m] <= 1.0) and np.all(out["w"][m] > 0)
    st = out["stats"]
    assert st["n_inlier"] == int(np.sum(np.abs(e) < delta))
    np.testing.assert_allclose(st["robust_cost"], np.sum(rho(e)), rtol=1e-9)


def test_pose_error_metrics(orc):
    """Sec. 6.1 metrics (trace and unsquared norm): a rotation by alpha about
    any axis has e_R = alpha; e_t is the Euclidean distance."""
    rng = np.random.default_rng(2)
    for alpha in (1e-4, 0.01, 0.5, 2.0):
        axis = rng.normal(size=3)
        R = synth.rot_axis_angle(axis, alpha)
        Tref = synth.make_pose(synth.rot_axis_angle(rng.normal(size=3), 0.7), rng.normal(size=3))
        T = synth.make_pose(R @ Tref[:3, :3], Tref[:3, 3] + np.array([0.3, -0.4, 1.2]))
        er, et = orc.pose_error(T, Tref)
        assert abs(er - alpha) < 1e-7
        assert abs(et - 1.3) < 1e-12


def test_self_registration_is_exact_identity(orc):
    """Registering a scan to itself from the identity: the round trip is exact,
    every residual is zero and the pose stays exactly I at every level."""
    p = _pair(5)
    prm = orc.make_params(levels=3, iters=[3, 3, 3])
    T, st = orc.icp(p.sensor, p.dst, p.dst, prm)
    assert np.array_equal(T, np.eye(4))
    for s in st:
        assert s["status"] == orc.ORC_OK and s["sum_w_e2"] == 0.0 and s["step_rot"] == 0.0


@pytest.mark.parametrize("kind", ["uniform", "staggered_r0"])
def test_converges_to_ground_truth_on_planar_scene(orc, kind):
    """Sec. 4.1: on a noise-free room (ground and four walls) the multi-scale
    registration recovers the known motion from the identity and from a
    1 deg / 10 cm perturbation of the truth.  The remaining error (corner pixels
    of the room bias the objective slightly) was measured below 1.4 mm /
    2.6e-4 rad."""
    sen = synth.uniform_sensor(64, 1024) if kind == "uniform" else synth.staggered_sensor(64, 1024, r0=0.015)
    rng = np.random.default_rng(1)
    scene = synth.room_scene(rng, n_boxes=0)
    Ta = synth.make_pose(np.eye(3), [0, 0, 1.8])
    dT = synth.random_motion(rng, 5.0, 1.0)
    nz = synth.ScanNoise(0.0, 0.5, 80.0, 0.0, 0.0)
    a = synth.scan(sen, scene, Ta, nz, rng)["range"]
    b = synth.scan(sen, scene, Ta @ dT, nz, rng)["range"]
    prm = orc.make_params(levels=3, iters=[10, 10, 10])
    for start in (np.eye(4), synth.make_pose(synth.rot_axis_angle([1, 1, 0], np.deg2rad(1.0)), [0.1, 0, 0]) @ dT):
        T, st = orc.icp(sen, b, a, prm, T_init=start)
        er, et = orc.pose_error(T, dT)
        assert er < 4e-4 and et < 2e-3, (er, et)


def test_small_step_stop(orc):
    """stop_eps: a level ends right after the first applied step with
    |xi| <= stop_eps; earlier steps of that level are larger, and the pose
    equals that of a run with exactly those iteration counts."""
    p = _pair(3)
    eps = 2e-4
    full = orc.make_params(levels=3, iters=[10, 10, 10])
    stop = orc.make_params(levels=3, iters=[10, 10, 10], stop_eps=eps)
    Ts, ss = orc.icp(p.sensor, p.src, p.dst, stop)
    runs = [int(s["iters_run"]) for s in ss]
    assert min(runs) < 10
    for l, s in enumerate(ss):
        step = np.hypot(s["step_rot"], s["step_trans"])
        if runs[l] < 10:
            assert step <= eps
        # the same schedule, cut by hand, one iteration short: its last step is above eps
        if runs[l] > 1:
            it = list(runs)
            it[l] = runs[l] - 1
            for k in range(l):  # finer levels do not run before level l ends
                it[k] = 0
            _, sc = orc.icp(p.sensor, p.src, p.dst, orc.make_params(levels=3, iters=it))
            assert np.hypot(sc[l]["step_rot"], sc[l]["step_trans"]) > eps
    Tc, _ = orc.icp(p.sensor, p.src, p.dst, orc.make_params(levels=3, iters=runs))
    assert np.array_equal(Ts, Tc)
    Tf, _ = orc.icp(p.sensor, p.src, p.dst, full)
    er, et = orc.pose_error(Ts, Tf)
    assert er < 1e-3 and et < 1e-2


def test_degenerate_inputs(orc):
    """Failure handling: an empty source and a ground-only scene (rank-deficient
    normal equations) give status DEGENERATE and leave the pose unchanged."""
    p = _pair(6)
    prm = orc.make_params(levels=3, iters=[2, 2, 2])
    T0 = synth.make_pose(np.eye(3), [0.1, 0.0, 0.0])
    T, st = orc.icp(p.sensor, np.zeros_like(p.src), p.dst, prm, T_init=T0)
    assert np.array_equal(T, T0)
    assert all(s["status"] == orc.ORC_DEGENERATE and s["n_valid"] == 0 for s in st)
    sen = synth.uniform_sensor(32, 256, 0.0, -30.0)
    scene = synth.Scene(np.array([[0, 0, 1.0, 0]]))
    nz = synth.ScanNoise(0.0, 0.5, 80.0, 0.0, 0.0)
    rng = np.random.default_rng(0)
    a = synth.scan(sen, scene, synth.make_pose(np.eye(3), [0, 0, 1.8]), nz, rng)["range"]
    T, st = orc.icp(sen, a, a, prm)
    assert np.array_equal(T, np.eye(4))
    assert all(s["status"] == orc.ORC_DEGENERATE for s in st)


def test_nonfinite_ranges_are_no_return(orc):
    """Range 0, NaN and +inf all mean 'no return'."""
    p = _pair(7)
    src = p.src.copy()
    dst = p.dst.copy()
    zs, zd = src == 0, dst == 0
    src[zs] = np.where(np.arange(zs.sum()) % 2 == 0, np.nan, np.inf)
    dst[zd] = np.nan
    prm = orc.make_params(levels=2, iters=[3, 3])
    T1, s1 = orc.icp(p.sensor, p.src, p.dst, prm)
    T2, s2 = orc.icp(p.sensor, src, dst, prm)
    assert np.array_equal(T1, T2)
    assert [s["n_valid"] for s in s1] == [s["n_valid"] for s in s2]


def test_centroid_initialisation(orc):
    """Sec. 4.1: with init_mode 1 the rotation starts at I and the translation
    at the difference of the point-set centres (checked with numpy)."""
    p = _pair(8)
    prm0 = orc.make_params(levels=1, iters=[0], init_mode=1)
    T, _ = orc.icp(p.sensor, p.src, p.dst, prm0)
    xs, vs = orc.unproject_image(p.sensor, p.src)
    xd, vd = orc.unproject_image(p.sensor, p.dst)
    np.testing.assert_allclose(T[:3, :3], np.eye(3))
    np.testing.assert_allclose(T[:3, 3], xd[vd].mean(0) - xs[vs].mean(0), rtol=1e-9, atol=1e-12)


def test_points_near_the_axis_do_not_project(orc):
    """Reading of Sec. 3.2 (r0 << r): with r0 > 0 a point within 2 r0 of the
    sensor axis does not project (the compensation has no fixed point inside
    the receiver circle); just beyond it the round trip is still exact."""
    sen = synth.staggered_sensor(32, 512, r0=0.05)
    r0 = sen.r0
    pts = np.array([[0, 0, 0], [r0, 0, 0], [1.5 * r0, 0.5 * r0, 0.0], [0, 1.99 * r0, 0.0]])
    assert not orc.project_points(sen, 0, pts)["valid"].any()
    # pixels whose points lie just beyond 2 r0: smallest range for the middle rows
    img = np.full((32, 512), 3.1 * r0, np.float32)
    xyz, _ = orc.unproject_image(sen, img)
    rho = np.hypot(xyz[..., 0], xyz[..., 1])
    ok = rho > 2 * r0
    pr = orc.project_points(sen, 0, xyz.reshape(-1, 3))
    vv, uu = np.meshgrid(np.arange(32), np.arange(512), indexing="ij")
    np.testing.assert_array_equal(pr["valid"], ok.ravel())
    np.testing.assert_array_equal(pr["u"][ok.ravel()], uu[ok])
    np.testing.assert_array_equal(pr["v"][ok.ravel()], vv[ok])
