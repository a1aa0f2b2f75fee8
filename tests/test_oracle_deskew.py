"""Pins of the oracle's re-projection under per-column poses (the non-rigid
model of the paper's outlook, Sec. 6) against facts other than itself (CPU
only): the zero-motion case is the lossless round trip of Sec. 3; a yaw per
sweep shifts each column by a closed-form amount; a translation per sweep
under synthetic intrinsics reduces to textbook spherical projection; the
output keeps the nearest of the ranges landing on a pixel.
"""
import numpy as np

import synth


def _scan(sm, seed=2):
    return synth.gen_pair(synth.CONFIGS["pair64"], seed, sensor=sm).dst


def test_zero_motion_is_the_identity(orc):
    for sm in (synth.uniform_sensor(32, 512), synth.staggered_sensor(32, 500, r0=0.02)):
        img = _scan(sm)
        o = orc.deskew(sm, img, np.zeros(6))
        ret = img > 0
        vv, uu = np.nonzero(ret)
        np.testing.assert_array_equal(o["u"][ret], uu)
        np.testing.assert_array_equal(o["v"][ret], vv)
        np.testing.assert_allclose(o["out"][ret], img[ret], rtol=1e-12)
        assert np.all(o["out"][~ret] == 0)


def test_yaw_per_sweep_shifts_columns(orc):
    """omega = (0, 0, a): column u turns by s_u a about the z axis, so its
    points keep their range and row and move to column u + s_u a W / (2 pi)."""
    sm = synth.uniform_sensor(32, 512)
    img = _scan(sm, 3)
    a = np.deg2rad(7.0)
    o = orc.deskew(sm, img, [0, 0, a, 0, 0, 0])
    H, W = img.shape
    vv, uu = np.nonzero(img > 0)
    s = (uu + 0.5) / W - 0.5
    cont = uu + s * a * W / (2 * np.pi)
    clear = np.abs(cont - np.floor(cont) - 0.5) > 1e-6
    exp_u = np.floor(cont + 0.5).astype(np.int64) % W
    np.testing.assert_array_equal(o["u"][vv, uu][clear], exp_u[clear])
    np.testing.assert_array_equal(o["v"][vv, uu], vv)
    np.testing.assert_allclose(o["r"][vv, uu], img[vv, uu], rtol=1e-12)
    assert clear.mean() > 0.99


def test_translation_per_sweep_textbook_projection(orc):
    """tau = (t, 0, 0) per sweep under synthetic intrinsics (r0 = 0, no azimuth
    offsets): x' = p + s_u tau, then the textbook spherical projection."""
    sm = synth.uniform_sensor(32, 512)
    img = _scan(sm, 4)
    tau = np.array([1.2, -0.4, 0.1])
    o = orc.deskew(sm, img, np.concatenate([[0, 0, 0], tau]))
    H, W = img.shape
    vv, uu = np.nonzero(img > 0)
    s = (uu + 0.5) / W - 0.5
    th = 2 * np.pi * uu / W
    r = img[vv, uu].astype(np.float64)
    ph = sm.phi[vv]
    p = np.stack([r * np.cos(th) * np.cos(ph), r * np.sin(th) * np.cos(ph), r * np.sin(ph)], 1)
    x = p + s[:, None] * tau
    rr = np.linalg.norm(x, axis=1)
    el = np.arcsin(x[:, 2] / rr)
    az = np.mod(np.arctan2(x[:, 1], x[:, 0]), 2 * np.pi) * W / (2 * np.pi)
    mids = 0.5 * (sm.phi[:-1] + sm.phi[1:])
    hi, lo = sm.phi[0] + 0.5 * (sm.phi[0] - sm.phi[1]), sm.phi[-1] - 0.5 * (sm.phi[-2] - sm.phi[-1])
    clear = (np.abs(az - np.floor(az) - 0.5) > 1e-6) & (np.min(np.abs(el[:, None] - mids), axis=1) > 1e-9)
    clear &= (np.abs(el - hi) > 1e-9) & (np.abs(el - lo) > 1e-9)
    inside = (el <= hi) & (el >= lo)
    exp_v = np.argmin(np.abs(el[:, None] - sm.phi[None, :]), axis=1)
    exp_u = np.floor(az + 0.5).astype(np.int64) % W
    m = clear & inside
    np.testing.assert_array_equal(o["u"][vv, uu][m], exp_u[m])
    np.testing.assert_array_equal(o["v"][vv, uu][m], exp_v[m])
    np.testing.assert_allclose(o["r"][vv, uu][m], rr[m], rtol=1e-12)
    assert np.all(o["u"][vv, uu][clear & ~inside] == -1)
    assert m.mean() > 0.9


def test_output_keeps_the_nearest_range(orc):
    """Each output pixel holds the minimum of the ranges landing on it."""
    sm = synth.staggered_sensor(32, 500, r0=0.02)
    img = _scan(sm, 5)
    o = orc.deskew(sm, img, [0.01, -0.02, 0.3, 2.0, 0.5, 0.05])
    ref = np.full(img.shape, np.inf)
    ok = o["u"] >= 0
    np.minimum.at(ref, (o["v"][ok], o["u"][ok]), o["r"][ok])
    ref[np.isinf(ref)] = 0.0
    np.testing.assert_array_equal(o["out"], ref)
    assert (np.bincount((o["v"][ok] * img.shape[1] + o["u"][ok])) > 1).any()   # collisions happen


def test_deskew_undoes_a_moving_sensor(orc):
    """A noise-free room scanned by a sensor moving 2 m and turning 8 degrees
    per sweep (each column cast from its own pose by the ray caster):
    re-projecting it under the same per-column poses brings it close to the
    scan a sensor resting at the mid-sweep pose takes (what remains is the
    resampling of off-centre points, largest on the grazing ground), much
    closer than the raw scan; the opposite motion makes it worse than the raw
    scan.  Pins the direction of the column poses against an independent
    ray caster."""
    sm = synth.uniform_sensor(64, 1024)
    rng = np.random.default_rng(8)
    scene = synth.room_scene(rng)
    T_mid = synth.make_pose(synth.yaw_matrix(0.3), [1.0, -2.0, 1.8])
    xi = np.array([0.0, 0.0, np.deg2rad(8.0), 2.0, 0.0, 0.0])
    static, _ = synth.raycast(sm, scene, T_mid)
    moving, _ = synth.raycast_moving(sm, scene, T_mid, xi)

    def median_err(img):
        both = (img > 0) & (static > 0)
        assert both.mean() > 0.9
        return float(np.median(np.abs(img[both] - static[both])))

    raw = median_err(moving)
    right = median_err(orc.deskew(sm, moving.astype(np.float32), xi)["out"])
    wrong = median_err(orc.deskew(sm, moving.astype(np.float32), -xi)["out"])
    assert right < 0.3 * raw and wrong > 2.0 * raw, (right, raw, wrong)
    # no motion: the moving caster is the static one
    still, _ = synth.raycast_moving(sm, scene, T_mid, np.zeros(6))
    np.testing.assert_array_equal(still, static)
