"""GPU parity of PCA normals (the eigen-decomposition estimator of Sec. 4.1)
against the FP64 oracle, through the C ABI.

Both sides build the covariance and its eigen-decomposition in FP64 (the GPU
in closed form, the oracle by Jacobi rotations), so validity must agree bit
for bit and normals within the FP32 rounding of the output (2e-7 rad), except
where the
decision is ill-conditioned: the middle eigenvalue within 1e-9 of the
collinearity threshold, or the two smallest eigenvalues closer than 1e-9 of
the largest (the normal direction is then not determined).
"""
import numpy as np
import pytest

import oracle
import synth
from parity_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rir():
    import torch
    import paper_2112_02779_amd as rir
    assert torch.cuda.is_available()
    return rir


def check(sm, img, n_gpu, v_gpu, half, edge_rel=0.1):
    n_ref, v_ref, lam = oracle.normals_pca(sm, img, half=half, edge_rel=edge_rel)
    top = lam[..., 2]
    has = top > 0                       # the oracle formed a covariance
    band = has & (np.abs(lam[..., 1] - 1e-6 * top) <= 1e-9 * top)
    flat = has & ((lam[..., 1] - lam[..., 0]) <= 1e-9 * top)
    clear = ~band
    np.testing.assert_array_equal(v_gpu[clear], v_ref[clear])
    both = v_gpu & v_ref & ~flat
    a = n_gpu[both].astype(np.float64)
    b = n_ref[both]
    ang = np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, axis=1))
    assert np.max(ang, initial=0.0) < 2e-7, np.max(ang)   # FP32 rounding of a unit vector: ~1e-7
    assert np.all(n_gpu[~v_gpu] == 0)
    assert v_ref.mean() > 0.3 and band.mean() < 1e-3 and (v_ref & flat).mean() < 1e-3
    print(f"valid {v_ref.mean():.3f}, max angle {np.max(ang, initial=0.0):.2e} rad, band {band.mean():.1e}")
    return ang


SENSORS = {
    "uniform64x1024": lambda: synth.uniform_sensor(64, 1024),
    "staggered32x500_r0": lambda: synth.staggered_sensor(32, 500, r0=0.015),
}


@pytest.mark.parametrize("name", list(SENSORS))
@pytest.mark.parametrize("half", [1, 2, 3])
def test_pca_normals_match_oracle(rir, name, half):
    """A batch of three noisy room scans (dropouts included) in one call."""
    sm = SENSORS[name]()
    sen = rir.Sensor.from_model(sm)
    imgs = np.stack([synth.gen_pair(synth.CONFIGS["pair64"], 40 + k, sensor=sm).dst for k in range(3)])
    n, valid = rir.normals_pca(sen, to_dev(imgs), half=half)
    n = n.cpu().numpy()
    valid = valid.cpu().numpy().astype(bool)
    for k in range(3):
        check(sm, imgs[k], n[k], valid[k], half)


def test_pca_normals_full_size(rir):
    """One 128 x 2048 outdoor scan of the odometry workload, 5 x 5 window."""
    cfg = synth.CONFIGS["odometry128x2048"]
    seq = synth.gen_sequence(cfg, 0, n_scans=1)
    sm = seq["sensor"]
    sen = rir.Sensor.from_model(sm)
    img = seq["scans"][0]
    n, valid = rir.normals_pca(sen, to_dev(img), half=2)
    check(sm, img, n.cpu().numpy(), valid.cpu().numpy().astype(bool), 2)


def test_pca_normals_edge_cases(rir):
    """No images is a no-op; an image without returns has no normals; a bad
    window size is an error."""
    import torch
    sm = synth.uniform_sensor(16, 256)
    sen = rir.Sensor.from_model(sm)
    empty = torch.zeros((0, 16, 256), dtype=torch.float32, device="cuda:0")
    n, valid = rir.normals_pca(sen, empty)
    assert n.numel() == 0
    dead = np.zeros((16, 256), np.float32)
    dead[::2] = np.nan
    n, valid = rir.normals_pca(sen, to_dev(dead), half=1)
    assert int(valid.sum()) == 0 and float(n.abs().sum()) == 0.0
    with pytest.raises(rir.RirError):
        rir.normals_pca(sen, to_dev(dead), half=4)


@pytest.mark.parametrize("case", [("uniform", 1, 0), ("uniform", 2, 0), ("staggered_r0", 1, 0), ("uniform", 1, 1)])
def test_icp_with_pca_normals_matches_oracle(case):
    """Registration with PCA target normals (normal_window = h, Sec. 4.1's
    eigen-decomposition estimator) against the oracle with the same
    estimator: pose within 1e-4 rad / 1 mm (or ill-conditioned under the
    band flips), correspondence counts within the ambiguity band's share;
    FP32 and FP64 plans."""
    import torch
    import oracle
    import synth
    import paper_2112_02779_amd as rir
    from parity_util import BAND_PHI, BAND_U, rot_trans_error
    kind, h, prec = case
    sm = synth.uniform_sensor(64, 1024) if kind == "uniform" else synth.staggered_sensor(64, 1024, r0=0.015)
    pair = synth.gen_pair(synth.CONFIGS["pair64"], 80 + h, sensor=sm)
    sen = rir.Sensor.from_model(sm)
    dev = torch.device("cuda:0")
    prm = rir.make_params(levels=3, iters=[10, 10, 10], delta=0.5, normal_window=h, precision=prec)
    T, st = rir.icp_batch(rir.Context(0), prm,
                          [(sen, torch.from_numpy(pair.src).to(dev), torch.from_numpy(pair.dst).to(dev))])
    oprm = oracle.make_params(levels=3, iters=[10, 10, 10], delta=0.5, normal_window=h)
    To, so = oracle.icp(sm, pair.src, pair.dst, oprm)
    er, et = rot_trans_error(T.cpu().numpy()[0], To)
    if not (er < 1e-4 and et < 1e-3):
        sp = oracle.icp_flip_spread(sm, pair.src, pair.dst, oprm, T_ref=To, band_u=BAND_U, band_phi=BAND_PHI)
        assert np.any((sp[:, 0] > 1e-4) | (sp[:, 1] > 1e-3)), (er, et, sp)
    stn = rir.stats_to_numpy(st, 1, 3)
    for l in range(3):
        assert stn[0, l]["status"] == so[l]["status"] == 0
        assert abs(int(stn[0, l]["n_valid"]) - so[l]["n_valid"]) <= 0.002 * so[l]["n_valid"] + 5
