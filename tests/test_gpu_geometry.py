"""GPU parity of the geometry entry points against the FP64 oracle:
unprojection (Eq. (1)-(2)), projection (Eq. (3)-(4)) and the normal image."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import ambiguous, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rir():
    import torch
    import paper_2112_02779_amd as rir
    assert torch.cuda.is_available()
    return rir


SENSORS = {
    "uniform64x1024": lambda: synth.uniform_sensor(64, 1024),
    "uniform128x2048": lambda: synth.uniform_sensor(128, 2048),
    "staggered32x512_r0": lambda: synth.staggered_sensor(32, 512, r0=0.015),
    "staggered16x256": lambda: synth.staggered_sensor(16, 256, r0=0.0),
}


@pytest.mark.parametrize("name", list(SENSORS))
def test_unproject_matches_oracle(rir, name):
    sm = SENSORS[name]()
    sen = rir.Sensor.from_model(sm)
    rng = np.random.default_rng(1)
    img = rng.uniform(0.5, 120.0, size=(sm.H, sm.W)).astype(np.float32)
    img[rng.random(img.shape) < 0.1] = 0.0
    img[0, 0], img[1, 1], img[2, 2] = np.nan, np.inf, -3.0
    xyz, valid = rir.unproject(sen, to_dev(img))
    ref, rvalid = oracle.unproject_image(sm, img)
    valid = valid.cpu().numpy().astype(bool)
    np.testing.assert_array_equal(valid, rvalid)
    r = np.where(rvalid, img, 0).astype(np.float64)
    err = np.linalg.norm(xyz.cpu().numpy().astype(np.float64) - ref, axis=-1)
    assert np.all(err <= 4e-7 * r + 1e-7)


@pytest.mark.parametrize("name", list(SENSORS))
@pytest.mark.parametrize("level", [0, 1, 2])
def test_round_trip_on_gpu_is_lossless(rir, name, level):
    """Sec. 3's lossless claim on the GPU: unproject then project returns the
    source pixel exactly, at every level for pixels on that level's grid."""
    sm = SENSORS[name]()
    sen = rir.Sensor.from_model(sm)
    rng = np.random.default_rng(2 + level)
    img = rng.uniform(0.5, 120.0, size=(sm.H, sm.W)).astype(np.float32)
    xyz, _ = rir.unproject(sen, to_dev(img))
    s = 1 << level
    sub = xyz[::s, ::s].contiguous()
    u, v, r, valid = rir.project(sen, level, sub)
    vv, uu = np.meshgrid(np.arange(sm.H // s), np.arange(sm.W // s), indexing="ij")
    assert valid.cpu().numpy().all()
    np.testing.assert_array_equal(u.cpu().numpy(), uu.ravel())
    np.testing.assert_array_equal(v.cpu().numpy(), vv.ravel())
    r_in = img[::s, ::s].ravel()
    assert np.max(np.abs(r.cpu().numpy() - r_in) / r_in) < 2e-6


@pytest.mark.parametrize("name", list(SENSORS))
@pytest.mark.parametrize("level", [0, 2])
def test_project_matches_oracle_outside_the_band(rir, name, level):
    """Projection of arbitrary points: validity and level indices bit-exact
    outside the rounding band; inside it, one of the two neighbours."""
    sm = SENSORS[name]()
    sen = rir.Sensor.from_model(sm)
    rng = np.random.default_rng(10 + level)
    n = 200000
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = (d * rng.uniform(0.5, 120.0, size=(n, 1))).astype(np.float32)
    # the origin, straight up/down, and a close point (outside the receiver radius r0)
    pts[:5] = [[0, 0, 0], [0.6, 0, 0], [0, 0, 5.0], [0, 0, -5.0], [3.0, 0, 0]]
    u, v, r, valid = rir.project(sen, level, to_dev(pts))
    u, v, valid = u.cpu().numpy(), v.cpu().numpy(), valid.cpu().numpy().astype(bool)
    ref = oracle.project_points(sm, level, pts.astype(np.float64))
    amb = ambiguous(sm, level, ref["uhat"], ref["phi"])
    clear = ~amb
    np.testing.assert_array_equal(valid[clear], ref["valid"][clear])
    both = clear & valid
    np.testing.assert_array_equal(u[both], ref["u"][both])
    np.testing.assert_array_equal(v[both], ref["v"][both])
    Wl = sm.W >> level
    a = amb & valid & ref["valid"]
    du = np.minimum(np.abs(u[a] - ref["u"][a]), Wl - np.abs(u[a] - ref["u"][a]))
    assert np.all(du <= 1) and np.all(np.abs(v[a] - ref["v"][a]) <= 1)
    assert amb.mean() < 0.01
    rr = r.cpu().numpy()
    np.testing.assert_allclose(rr[both], ref["r"][both], rtol=2e-6)


@pytest.mark.parametrize("name", list(SENSORS))
def test_normals_match_oracle(rir, name):
    """Normal validity bit-exact everywhere; normals within FP32 rounding of
    the oracle's (the GPU forms neighbour differences cancellation-free)."""
    sm = SENSORS[name]()
    sen = rir.Sensor.from_model(sm)
    pair = synth.gen_pair(synth.CONFIGS["pair64"], 5, sensor=sm)
    n, valid = rir.normals(sen, to_dev(pair.dst), 0.1)
    rn, rvalid = oracle.normals(sm, pair.dst, 0.1)
    valid = valid.cpu().numpy().astype(bool)
    np.testing.assert_array_equal(valid, rvalid)
    a = n.cpu().numpy().astype(np.float64)[valid]
    b = rn[valid]
    ang = np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, axis=1))
    assert rvalid.sum() > 0.2 * rvalid.size
    assert np.max(ang) < 2e-5, np.max(ang)
    assert np.median(ang) < 1e-6
