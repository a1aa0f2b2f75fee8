"""GPU parity of projective SDF fusion (Sec. 4.2, Eq. (8)-(10)) against the
FP64 oracle, through the C ABI.

Voxel weights (observation counts) must agree exactly and SDF values within
an FP32 bound, except for voxels whose association is ambiguous in some scan:
a projection inside the rounding band of parity_util (column or elevation
next to a rounding boundary) or a signed distance within parity_util.BAND_D of
the truncation limit, where FP32 and FP64 may legitimately decide differently.

Tolerance: per observation d = Omega - r carries the FP32 error of the
sensor-frame position (block offset formed in FP64, rounded once, plus three
FMAs) and of r (a few ulps of r); the running mean adds a relative error of
about one ulp per update.  With r at most R (the clip plus the truncation
band, else the largest range in the scans) the bound used is 5e-7 R + 1e-6 m,
about 4 ulps of R.
"""
import numpy as np
import pytest

import oracle
import synth
from parity_util import sdf_ambiguous, to_dev

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def rir():
    import torch
    import paper_2112_02779_amd as rir
    assert torch.cuda.is_available()
    return rir


def grid_points(vol):
    """World coordinates of every voxel in [nz, ny, nx] order (FP64)."""
    nx, ny, nz = vol.shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    idx = np.stack([i, j, k], axis=-1).reshape(-1, 3).astype(np.float64)
    return np.asarray(vol.origin) + vol.voxel * idx


def sequence(sensor, n, seed=3):
    seq = synth.gen_sequence(synth.CONFIGS["odometry128x2048"], seed, n_scans=n, sensor=sensor)
    poses = np.stack([synth.inv_pose(P) for P in seq["poses"]])
    return np.stack(seq["scans"]), poses, seq


def run_gpu(rir, sm, vol, ranges, poses, trunc, r_clip, voxels=None):
    import torch
    sen = rir.Sensor.from_model(sm)
    vox = vol.alloc() if voxels is None else voxels
    rir.sdf_integrate(sen, vol, vox, to_dev(ranges), poses, trunc, r_clip)
    torch.cuda.synchronize()
    return vox


def compare(s_gpu, w_gpu, s_ref, w_ref, amb, tol, n_scans):
    """Exact weights and SDF within tol outside the band; the band itself
    may hold at most the share of voxels that one of n_scans projections in
    the rounding band (under 1.2% per scan) would give."""
    clear = ~amb
    np.testing.assert_array_equal(w_gpu[clear], w_ref[clear])
    obs = clear & (w_ref > 0)
    err = np.abs(s_gpu[obs] - s_ref[obs])
    assert err.max(initial=0.0) <= tol, (err.max(), tol)
    assert np.all(s_gpu[w_gpu == 0] == 0)
    max_amb = 1.0 - (1.0 - 0.012) ** n_scans
    assert amb.mean() < max_amb, (amb.mean(), max_amb)
    print(f"max |sdf error| {err.max(initial=0.0):.3e} (bound {tol:.3e}), band share {amb.mean():.4f}")
    return err


SENSORS = {
    "uniform32x512": lambda: synth.uniform_sensor(32, 512),
    "staggered32x500_r0": lambda: synth.staggered_sensor(32, 500, r0=0.02),
}


@pytest.mark.parametrize("name", list(SENSORS))
@pytest.mark.parametrize("trunc,r_clip", [(0.5, 30.0), (0.0, 0.0)])
def test_fusion_matches_oracle(rir, name, trunc, r_clip):
    """20 scans (two launches: 16 + 4) into a 4 x 4 x 2-block volume around
    the start of a sequence; truncated with a range clip (block culling on),
    and the plain mean of Eq. (10) (no truncation, no clip)."""
    sm = SENSORS[name]()
    ranges, poses, seq = sequence(sm, 20)
    c = seq["poses"][0][:3, 3]
    vol = rir.Volume((4, 4, 2), (c[0] - 6.0, c[1] - 8.0, -1.0), 0.25)
    vox = run_gpu(rir, sm, vol, ranges, poses, trunc, r_clip)
    g = vol.to_grid(vox).cpu().numpy().reshape(-1, 2).astype(np.float64)
    pts = grid_points(vol)
    s_ref, w_ref = oracle.sdf_fuse(sm, ranges, poses, pts, trunc, r_clip)
    amb = sdf_ambiguous(sm, ranges, poses, pts, trunc, r_clip)
    R = (r_clip + trunc) if r_clip > 0 else float(ranges.max())
    compare(g[:, 0], g[:, 1], s_ref, w_ref, amb, 5e-7 * R + 1e-6, len(ranges))
    assert (w_ref > 0).mean() > 0.2 and w_ref.max() == len(ranges)


def test_split_calls_equal_one_call(rir):
    """Fusing scans 0..6 and then 7..19 gives bit-identical voxels to fusing
    0..19 at once (the per-voxel update order is the scan order either way)."""
    import torch
    sm = synth.uniform_sensor(32, 512)
    ranges, poses, seq = sequence(sm, 20, seed=4)
    c = seq["poses"][0][:3, 3]
    vol = rir.Volume((3, 2, 1), (c[0] - 5.0, c[1] - 4.0, -0.5), 0.2)
    one = run_gpu(rir, sm, vol, ranges, poses, 0.4, 25.0)
    two = run_gpu(rir, sm, vol, ranges[:7], poses[:7], 0.4, 25.0)
    two = run_gpu(rir, sm, vol, ranges[7:], poses[7:], 0.4, 25.0, voxels=two)
    assert torch.equal(one, two)


def test_edge_cases(rir):
    """No scans, a scan without returns and a scan of NaN/Inf ranges leave the
    volume unchanged; a one-block volume works; bad arguments are errors."""
    import torch
    sm = synth.uniform_sensor(16, 256)
    ranges, poses, seq = sequence(sm, 3, seed=5)
    c = seq["poses"][0][:3, 3]
    vol = rir.Volume((1, 1, 1), (c[0] - 2.0, c[1] - 2.0, -0.5), 0.25)
    sen = rir.Sensor.from_model(sm)
    vox = run_gpu(rir, sm, vol, ranges, poses, 0.5, 30.0)
    before = vox.clone()
    rir.sdf_integrate(sen, vol, vox, to_dev(ranges[:0]), poses[:0], 0.5, 30.0)
    dead = np.zeros((2, sm.H, sm.W), np.float32)
    dead[1] = np.nan
    dead[1, ::2] = np.inf
    rir.sdf_integrate(sen, vol, vox, to_dev(dead), poses[:2], 0.5, 30.0)
    torch.cuda.synchronize()
    assert torch.equal(vox, before)
    g = vol.to_grid(vox).cpu().numpy().reshape(-1, 2).astype(np.float64)
    s_ref, w_ref = oracle.sdf_fuse(sm, ranges, poses, grid_points(vol), 0.5, 30.0)
    amb = sdf_ambiguous(sm, ranges, poses, grid_points(vol), 0.5, 30.0)
    compare(g[:, 0], g[:, 1], s_ref, w_ref, amb, 5e-7 * 30.5 + 1e-6, len(ranges))
    bad = poses[:1].copy()
    bad[0, 0, 3] = np.nan
    with pytest.raises(rir.RirError):
        rir.sdf_integrate(sen, vol, vox, to_dev(ranges[:1]), bad, 0.5, 30.0)
    with pytest.raises(rir.RirError):
        rir.sdf_integrate(sen, rir.Volume((1, 1, 1), (0, 0, 0), 0.0), vox, to_dev(ranges[:1]), poses[:1], 0.5, 30.0)
    # through the C ABI directly (the binding's size check would object first)
    import ctypes
    P = np.ascontiguousarray(poses[:1], dtype=np.float64)
    r1 = to_dev(ranges[:1])
    st = rir.lib().rir_sdf_integrate(sen.handle, ctypes.byref(rir.Volume((0, 1, 1), (0, 0, 0), 0.1).desc),
                                     vox.data_ptr(), 1, r1.data_ptr(),
                                     P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.5, 30.0, None)
    assert st == rir.RIR_E_SHAPE
    st = rir.lib().rir_sdf_integrate(sen.handle, ctypes.byref(vol.desc), vox.data_ptr(), -1, r1.data_ptr(),
                                     P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.5, 30.0, None)
    assert st == rir.RIR_E_INVALID
    torch.cuda.synchronize()
    assert torch.equal(vox, before)


@pytest.mark.parametrize("kind", ["uniform", "staggered_r0"])
def test_full_size_sampled(rir, kind):
    """The benchmark's fusion workload shape: 128 x 2048 scans of an outdoor
    sequence into a 0.1 m volume spanning the path plus the 30 m clip, 32
    scans (two launches); 30000 voxels sampled (half among the observed ones)
    and checked against the oracle one by one; volume-wide properties: weights
    are whole numbers no larger than the scan count, |sdf| <= trunc (in FP32).
    Also with the general sensor (staggered azimuths, receiver offset)."""
    import torch
    cfg = synth.CONFIGS["odometry128x2048"]
    if kind == "uniform":
        sm = synth.uniform_sensor(*cfg["shapes"][0])
    else:
        sm = synth.staggered_sensor(*cfg["shapes"][0], r0=0.015)
    ranges, poses, seq = sequence(sm, 32, seed=0)
    trunc, r_clip, vx = 0.3, 30.0, 0.1
    P = np.array([p[:3, 3] for p in seq["poses"]])
    lo = P.min(0) - r_clip - 1.0
    hi = P.max(0) + r_clip + 1.0
    nbx, nby = (int(np.ceil((hi[i] - lo[i]) / (16 * vx))) for i in range(2))
    vol = rir.Volume((nbx, nby, 6), (lo[0], lo[1], -1.55), vx)
    vox = run_gpu(rir, sm, vol, ranges, poses, trunc, r_clip)
    flat = vol.to_grid(vox).reshape(-1, 2)
    w_all = flat[:, 1]
    assert torch.all(w_all == torch.round(w_all)) and float(w_all.max()) <= len(ranges)
    assert float(flat[:, 0].abs().max()) <= float(np.float32(trunc)) * (1 + 2.0 ** -22)  # FP32 trunc, 2 ulps
    rng = np.random.default_rng(9)
    obs = torch.nonzero(w_all > 0).squeeze(1).cpu().numpy()
    assert obs.size > 0.02 * w_all.numel()
    pick = np.concatenate([rng.choice(obs, 15000, replace=False), rng.integers(0, w_all.numel(), 15000)])
    got = flat[torch.from_numpy(pick).to(flat.device)].cpu().numpy().astype(np.float64)
    nx, ny, nz = vol.shape
    k, rem = np.divmod(pick, nx * ny)
    j, i = np.divmod(rem, nx)
    pts = np.asarray(vol.origin) + vx * np.stack([i, j, k], axis=1).astype(np.float64)
    s_ref, w_ref = oracle.sdf_fuse(sm, ranges, poses, pts, trunc, r_clip)
    amb = sdf_ambiguous(sm, ranges, poses, pts, trunc, r_clip)
    compare(got[:, 0], got[:, 1], s_ref, w_ref, amb, 5e-7 * (r_clip + trunc) + 1e-6, len(ranges))


def to_blocks(vol, grid):
    """[nz, ny, nx, 2] grid -> the block layout of Volume.alloc (layout
    marshalling for test inputs)."""
    nbx, nby, nbz = vol.nb
    E = vol.EDGE
    g = grid.reshape(nbz, E, nby, E, nbx, E, 2)
    return np.ascontiguousarray(g.transpose(0, 2, 4, 1, 3, 5, 6))


def test_extract_matches_oracle(rir):
    """Zero crossings of a synthetic volume (a sphere and a tilted plane, a
    truncation band with planted +-0.3 steps, unobserved and light voxels)
    computed by the GPU and by the oracle from the same FP32 values: same
    count, every point matched within FP32 rounding of its coordinates."""
    from scipy.spatial import cKDTree
    vol = rir.Volume((3, 2, 2), (-1.2, -0.7, -0.9), 0.05)
    pts = grid_points(vol)
    c, R = np.array([0.0, 0.1, -0.1]), 0.5
    n = np.array([0.2, 0.1, 1.0]) / np.linalg.norm([0.2, 0.1, 1.0])
    s = np.minimum(np.linalg.norm(pts - c, axis=1) - R, pts @ n + 0.4)
    s = np.clip(s, -0.3, 0.3)
    rng = np.random.default_rng(12)
    step = rng.random(len(s)) < 0.01
    s[step] = -np.sign(s[step]) * 0.3
    w = np.where(rng.random(len(s)) < 0.05, 0.5, 3.0)
    w[pts[:, 0] > 0.9] = 0.0
    nx, ny, nz = vol.shape
    grid = np.stack([s, w], -1).astype(np.float32).reshape(nz, ny, nx, 2)
    vox = to_dev(to_blocks(vol, grid))
    for max_jump in (0.45, np.inf):
        got, n_gpu = rir.sdf_extract(vol, vox, min_weight=1.0, max_jump=max_jump)
        got = got.cpu().numpy().astype(np.float64)
        ref = oracle.sdf_extract(vol.origin, vol.voxel, grid[..., 0].astype(np.float64),
                                 grid[..., 1].astype(np.float64), 1.0, max_jump)
        assert n_gpu == len(ref) == len(got) and n_gpu > 1000
        d1, _ = cKDTree(ref).query(got)
        d2, _ = cKDTree(got).query(ref)
        assert d1.max() < 2e-6 and d2.max() < 2e-6, (d1.max(), d2.max())
    # a cap below the crossing count keeps the count and stores only the cap
    got, n_all = rir.sdf_extract(vol, vox, min_weight=1.0, max_points=100)
    assert got.shape[0] == 100 and n_all > 100
