"""GPU parity of the sparse SDF volume (Sec. 4.2: 16^3-voxel blocks activated
around the returns of each scan in a hash table, only activated blocks
fused) against the FP64 oracle, through the C ABI.

Activation is decided in FP64 on both sides but from points formed in a
different order (the kernel's row/column factor tables against the oracle's
direct trigonometry), so a return within rounding of a cell boundary may
activate a block on one side only: the GPU set must contain the oracle's set
at radius - 1e-7 m and be contained in its set at radius + 1e-7 m (the set
grows with the radius), with activation scans ordered the same way.  Fusion
is checked per voxel against the oracle's Eq. (8)-(10) from the block's first
activating scan on (weights exact, SDF within the FP32 bound of the dense
volume's test, outside the same ambiguity band); extraction against the
oracle's zero crossings of the exported blocks laid out densely."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import sdf_ambiguous, to_dev
from test_gpu_sdf import sequence

pytestmark = pytest.mark.gpu

EPS = 1e-7


@pytest.fixture(scope="module")
def rir():
    import torch
    import paper_2112_02779_amd as rir
    assert torch.cuda.is_available()
    return rir


def _integrate(rir, sm, ranges, poses, trunc, r_clip, radius, voxel=0.1, max_blocks=20000, vol=None,
               origin=(0.0, 0.0, 0.0)):
    import torch
    vol = rir.BlockVolume(voxel, max_blocks, origin) if vol is None else vol
    vol.integrate(rir.Sensor.from_model(sm), to_dev(ranges), poses, trunc, r_clip, radius)
    torch.cuda.synchronize()
    return vol


def _export(vol):
    import torch
    b, v = vol.export()
    torch.cuda.synchronize()
    return b.cpu().numpy().astype(np.int64), v.cpu().numpy()


def _key_map(rows):
    return {tuple(int(x) for x in r[:3]): int(r[3]) for r in rows}


def _block_points(key, voxel, origin):
    E = 16
    k, j, i = np.meshgrid(np.arange(E), np.arange(E), np.arange(E), indexing="ij")
    idx = np.stack([i, j, k], axis=-1).reshape(-1, 3) + E * np.asarray(key)
    return np.asarray(origin) + voxel * idx.astype(np.float64)


SENSORS = {
    "uniform32x512": lambda: synth.uniform_sensor(32, 512),
    "staggered32x500_r0": lambda: synth.staggered_sensor(32, 500, r0=0.02),
}


ORIGIN = (0.03, -1.2, 0.05)


@pytest.mark.parametrize("name", list(SENSORS))
@pytest.mark.parametrize("radius,r_clip,origin", [(0.3, 30.0, ORIGIN), (0.0, 0.0, (0.0, 0.0, 0.0)),
                                                  (1.7, 20.0, ORIGIN)])
def test_activation_matches_oracle(rir, name, radius, r_clip, origin):
    """Activated blocks and first activating scans: 20 scans (two launches of
    activation), radius 0 (each return's own block), below and above one
    block edge (1.6 m), with and without an origin offset."""
    sm = SENSORS[name]()
    ranges, poses, _ = sequence(sm, 20, seed=11)
    vol = _integrate(rir, sm, ranges, poses, 0.3, r_clip, radius, origin=origin)
    rows, _ = _export(vol)
    assert vol.size() == (len(rows), 20)
    got = _key_map(rows)
    assert len(got) == len(rows)  # no block twice
    inner = _key_map(oracle.sdf_activate(sm, ranges, poses, max(radius - EPS, 0.0), r_clip, 0.1, origin))
    outer = _key_map(oracle.sdf_activate(sm, ranges, poses, radius + EPS, r_clip, 0.1, origin))
    assert len(inner) > 50
    assert set(inner) <= set(got) <= set(outer), (len(set(inner) - set(got)), len(set(got) - set(outer)))
    for k, f in got.items():
        assert outer[k] <= f <= inner.get(k, 1 << 30), (k, f)
    print(f"{len(got)} blocks (oracle {len(inner)}..{len(outer)})")


@pytest.mark.parametrize("name", list(SENSORS))
@pytest.mark.parametrize("trunc,r_clip", [(0.3, 30.0), (0.0, 0.0)])
def test_fusion_matches_oracle(rir, name, trunc, r_clip):
    """Voxels of 48 sampled active blocks against the oracle fusing the scans
    from each block's first activating scan on (20 scans: two fusion
    launches, blocks activated in either)."""
    sm = SENSORS[name]()
    ranges, poses, _ = sequence(sm, 20, seed=12)
    voxel = 0.1
    vol = _integrate(rir, sm, ranges, poses, trunc, r_clip, 0.3, voxel=voxel, origin=ORIGIN)
    rows, vox = _export(vol)
    rng = np.random.default_rng(3)
    late = np.flatnonzero(rows[:, 3] > 0)
    pick = np.concatenate([rng.choice(len(rows), 40, replace=False), late[:8]])
    assert len(late) > 0
    R = (r_clip + trunc) if r_clip > 0 else float(ranges.max())
    tol = 5e-7 * R + 1e-6
    n_obs, n_amb, amb_bound, err_max = 0, 0, 0.0, 0.0
    for b in pick:
        key, f0 = rows[b, :3], int(rows[b, 3])
        pts = _block_points(key, voxel, ORIGIN)
        g = vox[b].reshape(-1, 2).astype(np.float64)
        s_ref, w_ref = oracle.sdf_fuse(sm, ranges[f0:], poses[f0:], pts, trunc, r_clip)
        amb = sdf_ambiguous(sm, ranges[f0:], poses[f0:], pts, trunc, r_clip)
        clear = ~amb
        np.testing.assert_array_equal(g[clear, 1], w_ref[clear])
        obs = clear & (w_ref > 0)
        err = np.abs(g[obs, 0] - s_ref[obs])
        assert err.max(initial=0.0) <= tol, (err.max(), tol)
        assert np.all(g[g[:, 1] == 0, 0] == 0)
        err_max = max(err_max, err.max(initial=0.0))
        n_obs += int(obs.sum())
        n_amb += int(amb.sum())
        # the dense test's bound on the band (under 1.2% per scan), pooled
        # over the sampled blocks: one block's 4096 voxels are too coherent
        # for it alone
        amb_bound += len(pts) * (1.0 - (1.0 - 0.012) ** (len(ranges) - f0))
    assert n_obs > 10000
    assert n_amb <= amb_bound, (n_amb, amb_bound)
    print(f"max |sdf error| {err_max:.3e} (bound {tol:.3e}), band {n_amb} voxels (bound {amb_bound:.0f})")


def test_extract_matches_oracle_on_the_blocks(rir):
    """Zero crossings of the sparse volume (neighbours found through the
    table) against the oracle's crossings of the exported blocks laid out in
    a dense grid (voxels outside active blocks unobserved)."""
    import torch
    sm = synth.uniform_sensor(32, 512)
    ranges, poses, _ = sequence(sm, 12, seed=13)
    voxel = 0.1
    vol = _integrate(rir, sm, ranges, poses, 0.3, 30.0, 0.3, voxel=voxel, origin=ORIGIN)
    rows, vox = _export(vol)
    lo = rows[:, :3].min(axis=0)
    nb = rows[:, :3].max(axis=0) - lo + 1
    dense = np.zeros((nb[2] * 16, nb[1] * 16, nb[0] * 16, 2))
    for r, v in zip(rows, vox):
        x, y, z = (r[:3] - lo) * 16
        dense[z:z + 16, y:y + 16, x:x + 16] = v
    for mw, mj in [(1.0, 0.45), (3.0, np.inf)]:
        ref = oracle.sdf_extract(tuple(np.asarray(ORIGIN) + voxel * 16 * lo.astype(np.float64)), voxel,
                                 dense[..., 0], dense[..., 1],
                                 min_weight=mw, max_jump=mj)
        pts, n = vol.extract(min_weight=mw, max_jump=mj)
        torch.cuda.synchronize()
        got = pts.cpu().numpy().astype(np.float64)
        assert n == len(ref) and n > 1000
        # the same points up to the FP32 rounding of the stored coordinates
        # (matched by nearest neighbour both ways: sorting would pair points
        # differently where coordinates tie within rounding)
        from scipy.spatial import cKDTree
        assert cKDTree(ref).query(got)[0].max() < 1e-5
        assert cKDTree(got).query(ref)[0].max() < 1e-5


def test_split_calls_equal_one_call_and_reset(rir):
    """Scans fused in two calls (7 + 9) give the same blocks, activation scans
    and bit-identical voxels as one call of 16; after a reset the volume is
    empty and refills the same way."""
    import torch
    sm = synth.uniform_sensor(32, 512)
    ranges, poses, _ = sequence(sm, 16, seed=14)
    one = _integrate(rir, sm, ranges, poses, 0.3, 30.0, 0.3)
    two = _integrate(rir, sm, ranges[:7], poses[:7], 0.3, 30.0, 0.3)
    two = _integrate(rir, sm, ranges[7:], poses[7:], 0.3, 30.0, 0.3, vol=two)
    r1, v1 = _export(one)
    r2, v2 = _export(two)
    o1, o2 = np.lexsort(r1[:, :3].T[::-1]), np.lexsort(r2[:, :3].T[::-1])
    np.testing.assert_array_equal(r1[o1], r2[o2])
    assert np.array_equal(v1[o1].view(np.uint32), v2[o2].view(np.uint32))
    two.reset()
    torch.cuda.synchronize()
    assert two.size() == (0, 0)
    two = _integrate(rir, sm, ranges, poses, 0.3, 30.0, 0.3, vol=two)
    r3, v3 = _export(two)
    o3 = np.lexsort(r3[:, :3].T[::-1])
    np.testing.assert_array_equal(r1[o1], r3[o3])
    assert np.array_equal(v1[o1].view(np.uint32), v3[o3].view(np.uint32))


def test_errors_and_empty_calls(rir):
    """Too small a pool is RIR_E_OOM; no scans, scans without returns and
    bad arguments leave an empty volume or raise."""
    sm = synth.uniform_sensor(16, 256)
    ranges, poses, _ = sequence(sm, 3, seed=15)
    sen = rir.Sensor.from_model(sm)
    vol = rir.BlockVolume(0.1, 64)
    vol.integrate(sen, to_dev(ranges[:0]), poses[:0], 0.3, 30.0, 0.3)
    dead = np.zeros((2, sm.H, sm.W), np.float32)
    dead[1] = np.nan
    dead[1, ::2] = np.inf
    vol.integrate(sen, to_dev(dead), poses[:2], 0.3, 30.0, 0.3)
    assert vol.size() == (0, 2)
    pts, n = vol.extract()
    assert n == 0
    with pytest.raises(rir.RirError) as e:
        vol.integrate(sen, to_dev(ranges), poses, 0.3, 30.0, 0.3)
    assert e.value.args[0].startswith(f"librir status {rir.RIR_E_OOM}")
    bad = poses[:1].copy()
    bad[0, 0, 3] = np.nan
    with pytest.raises(rir.RirError):
        vol.integrate(sen, to_dev(ranges[:1]), bad, 0.3, 30.0, 0.3)
    with pytest.raises(rir.RirError):
        vol.integrate(sen, to_dev(ranges[:1]), poses[:1], 0.3, 30.0, -1.0)
    with pytest.raises(rir.RirError):
        rir.BlockVolume(0.0, 10)
    with pytest.raises(rir.RirError):
        rir.BlockVolume(0.1, 10, (0.0, np.nan, 0.0))
    with pytest.raises(rir.RirError):
        rir.BlockVolume(0.1, 0)
