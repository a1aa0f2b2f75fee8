"""Pins of the oracle's projective SDF (Sec. 4.2, Eq. (8)-(10)) against facts
other than itself (CPU only): closed forms for a sensor inside a sphere and
above a ground plane (the synthetic-intrinsics case of Sec. 3.2, where the
projection is the textbook spherical one), exact distances along pixel rays
with a receiver offset, and the least-squares (mean) form of Eq. (10).
"""
import numpy as np

import synth


def _world_to_sensor(R, c):
    """Pose mapping world points into the frame of a sensor at c with
    orientation R (sensor axes in world coordinates): x_s = R^T (x - c)."""
    T = np.eye(4)
    T[:3, :3] = R.T
    T[:3, 3] = -R.T @ c
    return T


def _fov_edges(sm):
    p = sm.phi
    return p[0] + 0.5 * (p[0] - p[1]), p[-1] - 0.5 * (p[-2] - p[-1])


def _sphere_case(sm, seed, trunc, r_clip):
    """Frames see a constant range image (a sphere of radius rad_f centred on
    the sensor): d_f(x) = rad_f - |x_s| exactly whenever x_s projects inside the
    vertical field of view, independent of the pixel it lands on (r0 = 0)."""
    rng = np.random.default_rng(seed)
    F = 5
    rads = np.array([4.0, 6.0, 3.5, 7.5, 5.0])
    centres = rng.uniform(-0.5, 0.5, size=(F, 3))
    rots = [synth.rot_axis_angle(synth.unit_vector(rng), rng.uniform(0.0, 0.6)) for _ in range(F)]
    poses = np.stack([_world_to_sensor(R, c) for R, c in zip(rots, centres)])
    ranges = np.stack([np.full((sm.H, sm.W), r, np.float32) for r in rads])
    pts = rng.uniform(-8.0, 8.0, size=(4000, 3))
    hi, lo = _fov_edges(sm)
    exp_s, exp_w = np.zeros(len(pts)), np.zeros(len(pts))
    sums = np.zeros(len(pts))
    near = np.zeros(len(pts), bool)
    for f in range(F):
        xs = pts @ rots[f] - centres[f] @ rots[f]            # R^T (x - c) row-wise
        rr = np.linalg.norm(xs, axis=1)
        el = np.arcsin(xs[:, 2] / rr)
        inside = (el <= hi) & (el >= lo)
        near |= (np.abs(el - hi) < 1e-9) | (np.abs(el - lo) < 1e-9)
        d = rads[f] - rr
        keep = inside
        if r_clip > 0:
            keep &= rads[f] <= r_clip
        if trunc > 0:
            near |= np.abs(d + trunc) < 1e-9
            keep &= d >= -trunc
            d = np.minimum(d, trunc)
        sums += np.where(keep, d, 0.0)
        exp_w += keep
    exp_s = np.where(exp_w > 0, sums / np.maximum(exp_w, 1), 0.0)
    return ranges, poses, pts, exp_s, exp_w, near


def test_sphere_closed_form_untruncated(orc):
    """Plain Eq. (10): the mean of rad_f - |x_s| over the frames that see x;
    pins the pose convention (R and t of Eq. (8), via the tilted field of view
    and the sensor centres), the sign of Eq. (9) and the running mean."""
    import oracle
    for sm in (synth.uniform_sensor(32, 256), synth.staggered_sensor(24, 200, r0=0.0)):
        ranges, poses, pts, es, ew, near = _sphere_case(sm, 3, 0.0, 0.0)
        s, w = oracle.sdf_fuse(sm, ranges, poses, pts, 0.0, 0.0)
        ok = ~near
        np.testing.assert_array_equal(w[ok], ew[ok])
        np.testing.assert_allclose(s[ok], es[ok], rtol=0, atol=1e-12)
        assert 0 < np.mean(ew == 0) < 0.9 and np.mean(ew == 5) > 0.05


def test_sphere_closed_form_truncated_and_clipped(orc):
    """Truncation (skip d < -trunc, limit d to trunc) and the range clip
    (returns beyond r_clip are not integrated) on the same closed form."""
    import oracle
    sm = synth.uniform_sensor(32, 256)
    for trunc, r_clip in ((0.3, 0.0), (0.5, 6.5), (1.0, 3.9)):
        ranges, poses, pts, es, ew, near = _sphere_case(sm, 4, trunc, r_clip)
        s, w = oracle.sdf_fuse(sm, ranges, poses, pts, trunc, r_clip)
        ok = ~near
        np.testing.assert_array_equal(w[ok], ew[ok])
        np.testing.assert_allclose(s[ok], es[ok], rtol=0, atol=1e-12)
        assert np.all(np.abs(s) <= trunc + 1e-15)
        assert np.any(ew > 0)


def test_ground_plane_with_textbook_spherical_projection(orc):
    """A sensor at height h above the ground z = 0, synthetic intrinsics: beam
    v below the horizon returns h / (-sin phi_v).  By the textbook projection a
    point x_s lands on the beam nearest its elevation, so Eq. (9) gives
    d = h / (-sin phi_v) - |x_s| (rows that see the sky have no return)."""
    import oracle
    sm = synth.uniform_sensor(64, 512)
    h = 1.8
    img = np.zeros((sm.H, sm.W), np.float32)
    below = sm.phi < 0
    img[below, :] = (h / -np.sin(sm.phi[below]))[:, None].astype(np.float32)
    rng = np.random.default_rng(5)
    yaw = rng.uniform(0, 2 * np.pi)
    c = np.array([3.0, -2.0, h])
    T = _world_to_sensor(synth.yaw_matrix(yaw), c)
    pts = np.concatenate([c + rng.uniform(-30, 30, size=(6000, 3)) * [1, 1, 0.1]])
    out = oracle.sdf_points(sm, img, T, pts)
    xs = (pts - c) @ synth.yaw_matrix(yaw)
    rr = np.linalg.norm(xs, axis=1)
    el = np.arcsin(xs[:, 2] / rr)
    v = np.argmin(np.abs(el[:, None] - sm.phi[None, :]), axis=1)
    mids = 0.5 * (sm.phi[:-1] + sm.phi[1:])
    clear = np.min(np.abs(el[:, None] - mids[None, :]), axis=1) > 1e-9
    hi, lo = _fov_edges(sm)
    inside = (el <= hi) & (el >= lo)
    has_ret = inside & below[v]
    np.testing.assert_array_equal(out["valid"][clear], has_ret[clear])
    np.testing.assert_array_equal(out["v"][clear & inside], v[clear & inside])
    m = clear & has_ret
    exp_d = img[v[m], 0].astype(np.float64) - rr[m]          # h / -sin(phi_v) rounded to FP32
    np.testing.assert_allclose(out["d"][m], exp_d, rtol=0, atol=1e-9)
    # points between the sensor and the ground along their ray lie in front of the surface
    assert np.all((out["d"][m] > 0) == (exp_d > 0))
    assert m.sum() > 1000


def test_distance_along_pixel_rays_with_receiver_offset(orc):
    """Points placed on the ray of pixel (u, v) at range rho (Eq. (1), receiver
    offset r0 > 0, staggered azimuth table) project back to that pixel with
    r = rho, so Eq. (9) gives exactly Omega(u, v) - rho."""
    import oracle
    sm = synth.staggered_sensor(32, 512, r0=0.04)
    rng = np.random.default_rng(6)
    img = rng.uniform(2.0, 40.0, size=(sm.H, sm.W)).astype(np.float32)
    R = synth.rot_axis_angle(synth.unit_vector(rng), 0.4)
    c = np.array([1.0, 2.0, 0.5])
    T = _world_to_sensor(R, c)
    n = 3000
    us = rng.integers(0, sm.W, n)
    vs = rng.integers(0, sm.H, n)
    rho = rng.uniform(1.0, 50.0, n)
    xs = np.stack([oracle.unproject(sm, u, v, r) for u, v, r in zip(us, vs, rho)])
    pts = xs @ R.T + c                                       # sensor -> world
    out = oracle.sdf_points(sm, img, T, pts)
    assert out["valid"].all()
    np.testing.assert_array_equal(out["u"], us)
    np.testing.assert_array_equal(out["v"], vs)
    np.testing.assert_allclose(out["d"], img[vs, us].astype(np.float64) - rho, rtol=0, atol=1e-9)


def test_incremental_update_equals_least_squares_mean(orc):
    """Eq. (10): the running mean after F frames equals argmin_t sum_f (t -
    d_f)^2, i.e. the plain mean of the per-frame (truncated) distances, in any
    frame order; and fusing in two calls equals fusing in one."""
    import oracle
    seq = synth.gen_sequence(synth.CONFIGS["odometry128x2048"], 11, n_scans=6,
                             sensor=synth.uniform_sensor(32, 512))
    poses = np.stack([synth.inv_pose(P) for P in seq["poses"]])
    ranges = np.stack(seq["scans"])
    rng = np.random.default_rng(7)
    c = seq["poses"][0][:3, 3]
    pts = c + rng.uniform(-15, 15, size=(5000, 3)) * [1, 1, 0.15]
    trunc, r_clip = 0.5, 30.0
    D = np.zeros((len(ranges), len(pts)))
    K = np.zeros_like(D, dtype=bool)
    for f in range(len(ranges)):
        o = oracle.sdf_points(seq["sensor"], ranges[f], poses[f], pts)
        keep = o["valid"] & (o["omega"] <= r_clip) & (o["d"] >= -trunc)
        D[f] = np.minimum(o["d"], trunc)
        K[f] = keep
    w_ls = K.sum(0)
    t_ls = np.where(w_ls > 0, (D * K).sum(0) / np.maximum(w_ls, 1), 0.0)
    s, w = oracle.sdf_fuse(seq["sensor"], ranges, poses, pts, trunc, r_clip)
    np.testing.assert_array_equal(w, w_ls)
    np.testing.assert_allclose(s, t_ls, rtol=0, atol=1e-12)
    order = rng.permutation(len(ranges))
    s2, w2 = oracle.sdf_fuse(seq["sensor"], ranges[order], poses[order], pts, trunc, r_clip)
    np.testing.assert_array_equal(w2, w)
    np.testing.assert_allclose(s2, s, rtol=0, atol=1e-12)
    sa, wa = oracle.sdf_fuse(seq["sensor"], ranges[:2], poses[:2], pts, trunc, r_clip)
    sb, wb = oracle.sdf_fuse(seq["sensor"], ranges[2:], poses[2:], pts, trunc, r_clip, sa, wa)
    np.testing.assert_array_equal(wb, w)
    np.testing.assert_allclose(sb, s, rtol=0, atol=1e-12)
    assert (w > 0).mean() > 0.3 and (w == len(ranges)).any()


def _grid(shape, origin, voxel):
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.asarray(origin) + voxel * np.stack([i, j, k], -1).astype(np.float64)


def test_extract_plane_is_exact(orc):
    """A linear SDF (signed distance to the plane z = z0) crosses zero once
    per grid column, and linear interpolation puts every point on the plane."""
    import oracle
    origin, vx, shape = (-1.0, 2.0, -0.55), 0.1, (12, 9, 11)
    X = _grid(shape, origin, vx)
    z0 = 0.013
    sdf = X[..., 2] - z0
    pts = oracle.sdf_extract(origin, vx, sdf, np.ones(shape))
    assert len(pts) == shape[1] * shape[2]
    np.testing.assert_allclose(pts[:, 2], z0, atol=1e-12)
    # a tilted plane n . x = c: every point on it, crossings along all three axes
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    cval = float(X.reshape(-1, 3).mean(0) @ n) + 0.01234
    sdf = X @ n - cval
    pts = oracle.sdf_extract(origin, vx, sdf, np.ones(shape))
    np.testing.assert_allclose(pts @ n, cval, atol=1e-12)
    assert len(pts) > shape[1] * shape[2]


def test_extract_sphere_weights_and_jumps(orc):
    """Sphere |x - c| - R: points within voxel^2 / R of the sphere; voxels of
    weight below min_weight and steps larger than max_jump give no point."""
    import oracle
    origin, vx, shape = (-1.0, -1.0, -1.0), 0.05, (40, 40, 40)
    X = _grid(shape, origin, vx)
    c, R = np.array([0.02, -0.03, 0.01]), 0.6
    sdf = np.linalg.norm(X - c, axis=-1) - R
    w = np.ones(shape)
    pts = oracle.sdf_extract(origin, vx, sdf, w)
    d = np.linalg.norm(pts - c, axis=1) - R
    assert np.max(np.abs(d)) <= vx * vx / R
    # edge crossings per unit area average (|n_x| + |n_y| + |n_z|) / voxel^2 = 1.5 / voxel^2
    area = 4 * np.pi * R * R / (vx * vx)
    assert 1.4 * area < len(pts) < 1.6 * area
    # half the volume unobserved: no point where either end has weight 0
    w2 = w.copy()
    w2[:, :, : shape[2] // 2] = 0
    p2 = oracle.sdf_extract(origin, vx, sdf, w2)
    assert len(p2) < len(pts) and np.all(p2[:, 0] >= origin[0] + vx * (shape[2] // 2) - 1e-12)
    # clamp to a truncation band of 0.1 with a +-0.1 step planted behind it
    s3 = np.clip(sdf, -0.1, 0.1)
    s3[:, :, -1] = np.where(s3[:, :, -2] > 0, -0.1, 0.1)
    p3 = oracle.sdf_extract(origin, vx, s3, w, max_jump=0.15)
    d3 = np.linalg.norm(p3 - c, axis=1) - R
    assert np.max(np.abs(d3)) <= vx * vx / R
    p4 = oracle.sdf_extract(origin, vx, s3, w)
    assert len(p4) > len(p3)


# ----------------------------------------------------------------------------- block activation

def _activation_scans(seed, F=3, H=8, W=32):
    sm = synth.staggered_sensor(H, W, r0=0.02)
    rng = np.random.default_rng(seed)
    ranges = rng.uniform(0.5, 12.0, size=(F, H, W)).astype(np.float32)
    ranges[rng.random(ranges.shape) < 0.1] = 0.0            # no return
    ranges[0, 0, :4] = np.nan
    rots = [synth.rot_axis_angle(synth.unit_vector(rng), rng.uniform(0.0, 1.0)) for _ in range(F)]
    centres = rng.uniform(-3.0, 3.0, size=(F, 3))
    poses = np.stack([_world_to_sensor(R, c) for R, c in zip(rots, centres)])
    return sm, ranges, poses


def _brute_activation(orc, sm, ranges, poses, radius, r_clip, voxel, origin=(0.0, 0.0, 0.0)):
    """Every block whose cell o + [E b, E (b + 1)) overlaps [x - radius,
    x + radius] on all three axes, by explicit interval tests over a candidate
    range, and the first scan that does so."""
    E = 16.0 * voxel
    first = {}
    for f in range(ranges.shape[0]):
        xyz, valid = orc.unproject_image(sm, ranges[f])
        ok = valid & np.isfinite(ranges[f])
        if r_clip > 0:
            ok &= ranges[f] <= r_clip
        xs = xyz[ok]
        R, t = poses[f][:3, :3], poses[f][:3, 3]
        xw = (xs - t) @ R - np.asarray(origin)               # R^T (x_s - t) - o row-wise
        for x in xw:
            cand = [range(int(np.floor(c / E)) - 2, int(np.floor(c / E)) + 3) for c in x]
            for bx in cand[0]:
                if not (E * bx <= x[0] + radius and x[0] - radius < E * (bx + 1)):
                    continue
                for by in cand[1]:
                    if not (E * by <= x[1] + radius and x[1] - radius < E * (by + 1)):
                        continue
                    for bz in cand[2]:
                        if E * bz <= x[2] + radius and x[2] - radius < E * (bz + 1):
                            first.setdefault((bx, by, bz), f)
    return np.array(sorted((k[0], k[1], k[2], v) for k, v in first.items()), np.int64).reshape(-1, 4)


def test_activation_matches_interval_overlap_brute_force(orc):
    """Sec. 4.2 activation: the blocks whose cells meet the cube around each
    return (explicit overlap tests, not the floor formula), with the first
    activating scan, on a staggered sensor with a receiver offset, NaN and
    missing returns, rotated poses; radius above and below a block edge."""
    sm, ranges, poses = _activation_scans(5)
    for radius, r_clip, voxel, o in [(0.3, 0.0, 0.1, (0.0, 0.0, 0.0)), (0.3, 8.0, 0.05, (0.03, -1.2, 0.05)),
                                     (2.5, 0.0, 0.1, (0.0, 0.0, 0.0))]:
        got = orc.sdf_activate(sm, ranges, poses, radius, r_clip, voxel, o)
        ref = _brute_activation(orc, sm, ranges, poses, radius, r_clip, voxel, o)
        assert len(ref) > 10
        np.testing.assert_array_equal(got, ref)


def test_activation_radius_zero_and_frames(orc):
    """Radius 0 activates exactly the block holding each return; a scan seen
    again activates nothing new (every block keeps its first scan); blocks
    only the second scan reaches get that scan's index; the set grows with the
    radius."""
    sm, ranges, poses = _activation_scans(6, F=1)
    E = 1.6
    xyz, valid = orc.unproject_image(sm, ranges[0])
    ok = valid & np.isfinite(ranges[0])
    R, t = poses[0][:3, :3], poses[0][:3, 3]
    own = np.unique(np.floor(((xyz[ok] - t) @ R) / E).astype(np.int64), axis=0)
    a0 = orc.sdf_activate(sm, ranges, poses, 0.0, 0.0, 0.1)
    np.testing.assert_array_equal(a0[:, :3], own)
    assert np.all(a0[:, 3] == 0)
    twice = orc.sdf_activate(sm, np.concatenate([ranges, ranges]), np.concatenate([poses, poses]), 0.3, 0.0, 0.1)
    once = orc.sdf_activate(sm, ranges, poses, 0.3, 0.0, 0.1)
    np.testing.assert_array_equal(twice, once)
    moved = poses.copy()
    moved[0][:3, 3] += np.array([10.0, 0.0, 0.0])            # the same scan 10 m away
    both = orc.sdf_activate(sm, np.concatenate([ranges, ranges]), np.concatenate([poses, moved]), 0.3, 0.0, 0.1)
    second = orc.sdf_activate(sm, ranges, moved, 0.3, 0.0, 0.1)
    first_keys = {tuple(k) for k in once[:, :3]}
    for row in both:
        k = tuple(row[:3])
        assert row[3] == (0 if k in first_keys else 1)
    assert {tuple(k) for k in both[:, :3]} == first_keys | {tuple(k) for k in second[:, :3]}
    big = orc.sdf_activate(sm, ranges, poses, 1.0, 0.0, 0.1)
    assert {tuple(k) for k in once[:, :3]} < {tuple(k) for k in big[:, :3]}


# ----------------------------------------------------------------------------- level-set triangles

def _field(nx, ny, nz, voxel, origin, f):
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = np.asarray(origin)[0] + voxel * i
    y = np.asarray(origin)[1] + voxel * j
    z = np.asarray(origin)[2] + voxel * k
    return f(x, y, z)


def _area_normals(t):
    n = np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])
    return 0.5 * np.linalg.norm(n, axis=1), n


def test_mesh_of_a_plane_is_the_plane(orc):
    """A linear SDF (tilted plane, positive above): every vertex on the plane,
    the triangles cover exactly the plane over the grid's xy extent (area
    (nx - 1)(ny - 1) voxel^2 sqrt(1 + a^2 + b^2)), every normal points to the
    positive side."""
    a, b, c, v = 0.3, -0.2, 0.77, 0.1
    nx, ny, nz = 12, 9, 20
    s = _field(nx, ny, nz, v, (0.0, 0.0, 0.0), lambda x, y, z: (z - (a * x + b * y + c)) / np.sqrt(1 + a * a + b * b))
    w = np.ones_like(s)
    t = orc.sdf_mesh((0.0, 0.0, 0.0), v, s, w)
    assert len(t) > 100
    p = t.reshape(-1, 3)
    np.testing.assert_allclose(p[:, 2], a * p[:, 0] + b * p[:, 1] + c, atol=1e-12)
    area, nrm = _area_normals(t)
    assert abs(area.sum() - (nx - 1) * (ny - 1) * v * v * np.sqrt(1 + a * a + b * b)) < 1e-10
    up = nrm @ np.array([-a, -b, 1.0])
    assert np.all(up[area > 1e-14] > 0)


def test_mesh_of_a_sphere_is_closed_and_oriented(orc):
    """Positive outside a sphere: the mesh is closed and consistently turned
    (every directed edge once, its reverse once), its enclosed volume
    (divergence theorem) is within 1.5% of 4/3 pi R^3, and every vertex lies
    within voxel^2 / R of the sphere."""
    v, R, c = 0.1, 0.8, np.array([1.03, 0.98, 1.01])
    n = 21
    s = _field(n, n, n, v, (0.0, 0.0, 0.0), lambda x, y, z: np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) - R)
    t = orc.sdf_mesh((0.0, 0.0, 0.0), v, s, np.ones_like(s))
    key = np.round(t.reshape(-1, 3) / 1e-9).astype(np.int64).reshape(-1, 3, 3)
    ids = {}
    tri = np.array([[ids.setdefault(tuple(p), len(ids)) for p in tr] for tr in key])
    directed = {}
    for a, b, cc in tri:
        for e in ((a, b), (b, cc), (cc, a)):
            directed[e] = directed.get(e, 0) + 1
    assert all(m == 1 for m in directed.values())
    assert all((b, a) in directed for a, b in directed)
    vol = np.einsum("ij,ij->i", t[:, 0], np.cross(t[:, 1], t[:, 2])).sum() / 6.0
    assert abs(vol / (4.0 / 3.0 * np.pi * R ** 3) - 1.0) < 0.015, vol
    r = np.linalg.norm(t.reshape(-1, 3) - c, axis=1)
    assert np.max(np.abs(r - R)) < v * v / R


def test_mesh_weight_and_step_gates(orc):
    """Unobserved voxels (weight below min_weight) and steps above max_jump
    leave no triangle on a tetrahedron that holds them."""
    v = 0.1
    nx = ny = nz = 8
    s = _field(nx, ny, nz, v, (0.0, 0.0, 0.0), lambda x, y, z: z - 0.33)
    w = np.full_like(s, 2.0)
    full = orc.sdf_mesh((0.0, 0.0, 0.0), v, s, w, min_weight=2.0)
    w2 = w.copy()
    w2[:, :, 4:] = 1.0                                     # x >= 0.4 observed once
    part = orc.sdf_mesh((0.0, 0.0, 0.0), v, s, w2, min_weight=2.0)
    assert 0 < len(part) < len(full)
    assert np.all(part[:, :, 0] <= 0.3 + 1e-12)
    s2 = s.copy()
    s2[:, 4:, :] *= 10.0                                   # steep half: |s_a - s_b| up to 1 m
    cut = orc.sdf_mesh((0.0, 0.0, 0.0), v, s2, w, max_jump=0.5)
    assert 0 < len(cut) < len(full)
    assert np.all(cut[:, :, 1] <= 0.4 + 1e-12)
