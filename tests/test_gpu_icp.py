"""GPU parity of the registration path (Sec. 4.1, Eq. (5)-(7)) against the
FP64 oracle: per-pixel association, residuals, Jacobians and weights at a
shared pose; the reduced normal equations; full multi-scale poses; batching,
graphs, determinism and failure statuses."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import ambiguous, rot_trans_error, to_dev

pytestmark = pytest.mark.gpu

POSE_ROT_TOL = 1e-4   # rad
POSE_TRANS_TOL = 1e-3  # m
JTJ_TOL = 1e-5        # |dH_ij| <= JTJ_TOL * sqrt(H_ii H_jj)


@pytest.fixture(scope="module")
def rir():
    import torch
    import paper_2112_02779_amd as rir
    assert torch.cuda.is_available()
    return rir


@pytest.fixture(scope="module")
def ctx(rir):
    c = rir.Context(0)
    c.set_tuning(256, 8, 0, 1)
    return c


def _pair(cfg="pair64", seed=0, shape=None, sensor=None):
    return synth.gen_pair(synth.CONFIGS[cfg], seed, shape=shape, sensor=sensor)


def _jtj_matrix(upper):
    H = np.zeros((6, 6))
    iu = np.triu_indices(6)
    H[iu] = upper
    H.T[iu] = upper
    return H


def _normalised_diff(Ha, Hb):
    d = np.sqrt(np.outer(np.diag(Hb), np.diag(Hb)))
    return np.max(np.abs(Ha - Hb) / d)


@pytest.mark.parametrize("case", [("pair64", 0, (64, 1024), "uniform"), ("pair64", 1, (32, 512), "staggered"),
                                  ("dynamic64", 2, (64, 1024), "uniform")])
@pytest.mark.parametrize("level", [0, 1, 2])
def test_association_terms_match_oracle(rir, ctx, case, level):
    cfg, seed, shape, kind = case
    sm = synth.uniform_sensor(*shape) if kind == "uniform" else synth.staggered_sensor(*shape, r0=0.015)
    pair = _pair(cfg, seed, shape, sm)
    sen = rir.Sensor.from_model(sm)
    T = pair.gt @ synth.make_pose(synth.rot_axis_angle([0.3, 1.0, 0.2], 0.01), [0.05, -0.03, 0.02])
    prm = rir.make_params(levels=3, iters=[1, 1, 1], delta=0.5)
    out = rir.debug_associate(ctx, prm, sen, to_dev(pair.src), to_dev(pair.dst), level, T)
    ref = oracle.system(sm, level, pair.src, pair.dst, oracle.make_params(levels=3, iters=[1, 1, 1], delta=0.5), T)
    g = {k: out[k].cpu().numpy() for k in ("u", "v", "mask", "e", "w", "J")}
    g["mask"] = g["mask"].astype(bool)
    amb = ambiguous(sm, level, ref["uhat"], ref["phi"]) & (ref["proj_valid"] | (g["u"] >= 0))
    clear = ~amb
    # indices and masks bit-exact outside the band
    np.testing.assert_array_equal(g["u"][clear], ref["u"][clear])
    np.testing.assert_array_equal(g["v"][clear], ref["v"][clear])
    np.testing.assert_array_equal(g["mask"][clear], ref["mask"][clear])
    assert amb.mean() < 0.01
    m = clear & ref["mask"]
    assert m.sum() > 100
    # FP32 points at up to ~40 m carry ~1e-5 m of rounding, so e agrees to
    # 2e-5 m and w (|dw/de| <= 0.77 / delta) to 4e-5
    np.testing.assert_allclose(g["e"][m], ref["e"][m], atol=2e-5)
    np.testing.assert_allclose(g["w"][m], ref["w"][m], atol=4e-5)
    jscale = np.maximum(1.0, np.abs(ref["J"][m]))
    assert np.max(np.abs(g["J"][m] - ref["J"][m]) / jscale) < 2e-5
    # normal equations over the common pixels: GPU terms vs oracle terms
    def sums(J, w, e, mm):
        Jm, wm, em = J[mm].astype(np.float64), w[mm].astype(np.float64), e[mm].astype(np.float64)
        return (Jm * wm[:, None]).T @ Jm, (Jm * wm[:, None]).T @ em
    Hg, gg = sums(g["J"], g["w"], g["e"], m)
    Ho, go = sums(ref["J"], ref["w"], ref["e"], m)
    assert _normalised_diff(Hg, Ho) < JTJ_TOL
    # the kernel's own FP32 reduction against an FP64 sum of its per-pixel terms
    Hall, gall = sums(g["J"], g["w"], g["e"], g["mask"])
    Hk = _jtj_matrix(out["stats"]["JtJ"])
    assert _normalised_diff(Hk, Hall) < JTJ_TOL
    # |(J^T W e)_i| <= sqrt(H_ii * sum w e^2) bounds each entry (Cauchy-Schwarz)
    we2 = float(np.sum(g["w"][g["mask"]].astype(np.float64) * g["e"][g["mask"]].astype(np.float64) ** 2))
    jtr_scale = np.sqrt(np.diag(Hall) * we2) + 1e-12
    assert np.max(np.abs(out["stats"]["Jtr"] - gall) / jtr_scale) < JTJ_TOL
    assert out["stats"]["n_valid"] == int(g["mask"].sum())
    st = ref["stats"]
    assert abs(out["stats"]["n_valid"] - st["n_valid"]) <= amb.sum()
    # whole-image normal equations: differences come only from band pixels
    Hr = _jtj_matrix(st["JtJ"])
    assert _normalised_diff(Hk, Hr) < JTJ_TOL + 4.0 * amb.sum() / max(st["n_valid"], 1)


def _run_gpu(rir, ctx, sm, pairs, iters, levels, **kw):
    sen = rir.Sensor.from_model(sm)
    prm = rir.make_params(levels=levels, iters=iters, delta=0.5, **kw)
    batch = [(sen, to_dev(p.src), to_dev(p.dst)) for p in pairs]
    poses, stats = rir.icp_batch(ctx, prm, batch)
    return poses.cpu().numpy(), rir.stats_to_numpy(stats, len(pairs), levels)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_multiscale_pose_matches_oracle_pair64(rir, ctx, seed):
    """64x1024 pairs, 3 levels x 10 iterations (FP32 per-pixel math, FP64 solve)."""
    pair = _pair("pair64", seed)
    Tg, st = _run_gpu(rir, ctx, pair.sensor, [pair], [10, 10, 10], 3)
    To, so = oracle.icp(pair.sensor, pair.src, pair.dst, oracle.make_params(levels=3, iters=[10, 10, 10]))
    er, et = rot_trans_error(Tg[0], To)
    assert er < POSE_ROT_TOL and et < POSE_TRANS_TOL, (er, et)
    for l in range(3):
        assert st[0, l]["status"] == so[l]["status"] == 0
        assert st[0, l]["iters_run"] == so[l]["iters_run"] == 10
        assert abs(st[0, l]["n_valid"] - so[l]["n_valid"]) <= 0.002 * so[l]["n_valid"] + 5


def test_small_step_stop_matches_oracle(rir, ctx):
    """stop_eps ends a level after a small step, on the tiled and the
    pair-resident paths alike: the same iteration counts as the oracle
    (unless a step lies within 5% of the threshold) and the oracle's pose."""
    eps = 2e-4
    for seed in (3, 4):
        pair = _pair("pair64", seed)
        Tg, st = _run_gpu(rir, ctx, pair.sensor, [pair], [10, 10, 10], 3, stop_eps=eps)
        To, so = oracle.icp(pair.sensor, pair.src, pair.dst,
                            oracle.make_params(levels=3, iters=[10, 10, 10], stop_eps=eps))
        er, et = rot_trans_error(Tg[0], To)
        assert er < POSE_ROT_TOL and et < POSE_TRANS_TOL, (seed, er, et)
        assert any(so[l]["iters_run"] < 10 for l in range(3))
        for l in range(3):
            near = abs(np.hypot(so[l]["step_rot"], so[l]["step_trans"]) - eps) < 0.05 * eps
            assert near or st[0, l]["iters_run"] == so[l]["iters_run"], (seed, l)


def test_multiscale_pose_matches_oracle_general_sensor(rir, ctx):
    """Non-uniform elevation table, staggered azimuth offsets and r0 > 0."""
    sm = synth.staggered_sensor(64, 1024, r0=0.015)
    pair = _pair("pair64", 7, sensor=sm)
    Tg, st = _run_gpu(rir, ctx, sm, [pair], [10, 10, 10], 3)
    To, so = oracle.icp(sm, pair.src, pair.dst, oracle.make_params(levels=3, iters=[10, 10, 10]))
    er, et = rot_trans_error(Tg[0], To)
    assert er < POSE_ROT_TOL and et < POSE_TRANS_TOL, (er, et)


def test_fp64_mode_matches_oracle_tightly(rir, ctx):
    pair = _pair("pair64", 4)
    Tg, _ = _run_gpu(rir, ctx, pair.sensor, [pair], [10, 10, 10], 3, precision=rir.PREC_FP64)
    To, _ = oracle.icp(pair.sensor, pair.src, pair.dst, oracle.make_params(levels=3, iters=[10, 10, 10]))
    er, et = rot_trans_error(Tg[0], To)
    assert er < 1e-6 and et < 1e-5, (er, et)


def test_self_registration_is_identity(rir, ctx):
    """At the identity every source pixel projects onto itself (lossless
    round trip), so every residual vanishes up to FP32 rounding of the point
    and plane offset (|x| <= 100 m: a few ulp of 100 m) and the pose stays
    at I to the same order."""
    pair = _pair("pair64", 5)
    sen = rir.Sensor.from_model(pair.sensor)
    img = to_dev(pair.dst)
    img2 = to_dev(pair.dst)
    prm = rir.make_params(levels=3, iters=[1, 1, 1])
    for lvl in range(3):
        d = rir.debug_associate(ctx, prm, sen, img, img2, lvl, np.eye(4))
        e = d["e"].cpu().numpy()
        m = d["mask"].cpu().numpy().astype(bool)
        s = 1 << lvl
        vv, uu = np.meshgrid(np.arange(pair.sensor.H // s), np.arange(pair.sensor.W // s), indexing="ij")
        u, v = d["u"].cpu().numpy(), d["v"].cpu().numpy()
        src_ok = pair.dst[::s, ::s] > 0
        moved = src_ok & ((u != uu) | (v != vv))
        assert not moved.any(), (lvl, np.argwhere(moved)[:5], u[moved][:5], v[moved][:5])
        assert m.sum() > 0.3 * src_ok.sum()
        assert np.max(np.abs(e[m])) < 3e-5, (lvl, np.max(np.abs(e[m])))
    same = synth.Pair(pair.sensor, pair.dst, pair.dst, np.eye(4), 5)
    Tg, st = _run_gpu(rir, ctx, pair.sensor, [same], [3, 3, 3], 3)
    er, et = rot_trans_error(Tg[0], np.eye(4))
    assert er < 1e-6 and et < 1e-5, (er, et)
    assert np.all(st["sum_w_e2"] < 1e-9 * st["n_valid"])


def test_run_twice_is_bitwise_identical_and_graph_equals_eager(rir, ctx):
    pairs = [_pair("pair64", s) for s in range(3)]
    T1, s1 = _run_gpu(rir, ctx, pairs[0].sensor, pairs, [4, 4, 4], 3)
    T2, s2 = _run_gpu(rir, ctx, pairs[0].sensor, pairs, [4, 4, 4], 3)
    T3, s3 = _run_gpu(rir, ctx, pairs[0].sensor, pairs, [4, 4, 4], 3, use_graph=False)
    assert np.array_equal(T1, T2) and np.array_equal(T1, T3)
    assert s1.tobytes() == s2.tobytes() == s3.tobytes()


def test_pair_alone_equals_pair_in_mixed_batch(rir, ctx):
    """Tiles never straddle pairs, so a pair's result does not depend on the
    batch it is solved in (fixed tuning)."""
    shapes = [(16, 1024), (32, 1024), (64, 1024), (128, 2048)]
    pairs = [_pair("batch256mixed", 2000 + i, shape=shapes[i % 4]) for i in range(8)]
    sensors = {}
    batch = []
    for p in pairs:
        key = (p.sensor.H, p.sensor.W)
        if key not in sensors:
            sensors[key] = rir.Sensor.from_model(p.sensor)
        batch.append((sensors[key], to_dev(p.src), to_dev(p.dst)))
    prm = rir.make_params(levels=3, iters=[5, 5, 5], delta=0.5)
    Tb, sb = rir.icp_batch(ctx, prm, batch)
    Tb = Tb.cpu().numpy()
    for i in (0, 3, 5):
        Ti, si = rir.icp_batch(ctx, prm, [batch[i]])
        assert np.array_equal(Ti.cpu().numpy()[0], Tb[i])
    # and each pair of the batch agrees with the oracle
    for i, p in enumerate(pairs[:4]):
        To, _ = oracle.icp(p.sensor, p.src, p.dst, oracle.make_params(levels=3, iters=[5, 5, 5]))
        er, et = rot_trans_error(Tb[i], To)
        assert er < POSE_ROT_TOL and et < POSE_TRANS_TOL, (i, er, et)


@pytest.mark.skip(reason="concurrent sub-batches are switched off in this build (rir_ctx_set_tuning rejects lanes > 1): "
                         "the full benchmark with them on ended once in a host segmentation fault whose cause is not "
                         "found yet")
def test_lane_count_changes_no_result(rir):
    """The coarse levels of a batch (or all of them) run as 1-4 concurrent
    sub-batches (lanes): poses and statistics are bitwise those of one lane,
    eager and captured, with
    every timing mode (the captured schedule then carries event nodes), on a
    mixed batch whose coarse levels use the tiled and the pair-resident paths."""
    c = rir.Context(0)
    shapes = [(16, 1024), (32, 1024), (64, 1024), (128, 2048), (64, 1024)]
    pairs = [_pair("batch256mixed", 2100 + i, shape=shapes[i % 5]) for i in range(7)]
    sensors = {}
    batch = []
    for p in pairs:
        key = (p.sensor.H, p.sensor.W)
        if key not in sensors:
            sensors[key] = rir.Sensor.from_model(p.sensor)
        batch.append((sensors[key], to_dev(p.src), to_dev(p.dst)))
    ref = None
    for lanes, fine in ((1, 0), (2, 0), (3, 1), (4, 1)):
        c.set_tuning(256, 8, 0, 1, 4, 1, lanes, fine)
        for graph in (True, False):
            for timing in (0, 1, 2):
                c.enable_timing(timing > 0, finest_only=timing == 2)
                prm = rir.make_params(levels=3, iters=[4, 4, 3], delta=0.5, use_graph=graph)
                T, st = rir.icp_batch(c, prm, batch)
                got = (T.cpu().numpy(), st.cpu().numpy().tobytes())
                if timing:
                    ms = c.level_times(3)
                    assert ms[0] > 0.0, (lanes, graph, timing, ms)
                    if timing == 1:
                        assert all(x > 0.0 for x in ms), (lanes, graph, ms)
                if ref is None:
                    ref = got
                assert np.array_equal(got[0], ref[0]) and got[1] == ref[1], (lanes, fine, graph, timing)
    c.enable_timing(False)


def test_degenerate_and_empty_inputs(rir, ctx):
    """An empty source and a ground-only scene give status DEGENERATE with the
    pose unchanged, as in the oracle; a tiny ragged image still runs."""
    import torch
    pair = _pair("pair64", 6)
    sen = rir.Sensor.from_model(pair.sensor)
    prm = rir.make_params(levels=3, iters=[2, 2, 2])
    T0 = torch.tensor(synth.make_pose(np.eye(3), [0.1, 0, 0])[None], dtype=torch.float64, device="cuda:0")
    poses, stats = rir.icp_batch(ctx, prm, [(sen, to_dev(np.zeros_like(pair.src)), to_dev(pair.dst))], init_poses=T0)
    st = rir.stats_to_numpy(stats, 1, 3)
    np.testing.assert_array_equal(poses.cpu().numpy(), T0.cpu().numpy())
    assert np.all(st["status"] == rir.LEVEL_DEGENERATE) and np.all(st["n_valid"] == 0)
    sm = synth.uniform_sensor(32, 256, 0.0, -30.0)
    scene = synth.Scene(np.array([[0, 0, 1.0, 0]]))
    a = synth.scan(sm, scene, synth.make_pose(np.eye(3), [0, 0, 1.8]), synth.ScanNoise(), np.random.default_rng(0))
    sen2 = rir.Sensor.from_model(sm)
    poses, stats = rir.icp_batch(ctx, prm, [(sen2, to_dev(a["range"]), to_dev(a["range"]))])
    np.testing.assert_array_equal(poses.cpu().numpy()[0], np.eye(4))
    assert np.all(rir.stats_to_numpy(stats, 1, 3)["status"] == rir.LEVEL_DEGENERATE)
    # smallest shapes: 4 x 8 image, one level
    sm3 = synth.uniform_sensor(4, 8)
    img = np.full((4, 8), 5.0, np.float32)
    sen3 = rir.Sensor.from_model(sm3)
    poses, stats = rir.icp_batch(ctx, rir.make_params(levels=1, iters=[1]), [(sen3, to_dev(img), to_dev(img))])
    assert rir.stats_to_numpy(stats, 1, 1)["status"][0, 0] in (rir.LEVEL_OK, rir.LEVEL_DEGENERATE)


def test_host_side_errors(rir, ctx):
    pair = _pair("pair64", 0, shape=(30, 512), sensor=synth.uniform_sensor(30, 512))
    sen = rir.Sensor.from_model(pair.sensor)
    with pytest.raises(rir.RirError) as ei:
        rir.icp_batch(ctx, rir.make_params(levels=3), [(sen, to_dev(pair.src), to_dev(pair.dst))])
    assert ei.value.status == rir.RIR_E_SHAPE
    with pytest.raises(rir.RirError) as ei:
        rir.icp_batch(ctx, rir.make_params(levels=1, delta=-1.0), [(sen, to_dev(pair.src), to_dev(pair.dst))])
    assert ei.value.status == rir.RIR_E_INVALID
    # concurrent sub-batches are switched off in this build
    c = rir.Context(0)
    with pytest.raises(rir.RirError) as ei:
        c.set_tuning(256, 8, 0, 1, 4, 1, 3, 0)
    assert ei.value.status == rir.RIR_E_UNSUPPORTED
    assert c.get_tuning()["lanes"] == 1


def test_centroid_initialisation(rir, ctx):
    pair = _pair("pair64", 8)
    Tg, _ = _run_gpu(rir, ctx, pair.sensor, [pair], [0], 1, init_mode=1)
    To, _ = oracle.icp(pair.sensor, pair.src, pair.dst, oracle.make_params(levels=1, iters=[0], init_mode=1))
    np.testing.assert_allclose(Tg[0], To, atol=2e-5)


def test_full_size_odometry_pairs_match_oracle(rir, ctx):
    """The 128x2048, 4-level workload at full size: a few pairs of the
    odometry sequence (batched) against the oracle."""
    seq = synth.gen_sequence(synth.CONFIGS["odometry128x2048"], 1000, n_scans=4)
    sm = seq["sensor"]
    Tg, st = _run_gpu(rir, ctx, sm, seq["pairs"], [10, 10, 10, 10], 4)
    prm = oracle.make_params(levels=4, iters=[10, 10, 10, 10], r_max=120.0)
    for i, p in enumerate(seq["pairs"]):
        To, so = oracle.icp(sm, p.src, p.dst, prm)
        er, et = rot_trans_error(Tg[i], To)
        assert er < POSE_ROT_TOL and et < POSE_TRANS_TOL, (i, er, et)


def test_plans_never_outlive_their_sensors(rir, ctx):
    """Regression: cached plans were keyed by the sensor's address, so a new
    sensor of another shape allocated at a freed sensor's address reused a
    plan sized for the old shape.  Sensors of different shapes are now
    created and destroyed in turn through one context; every pass must write
    exactly its own image's pixels and match a fresh context."""
    import torch
    shapes = [(64, 1024), (16, 256), (32, 512), (64, 1024), (16, 256)]
    prm = rir.make_params(levels=3, iters=[1, 1, 1])
    fresh = rir.Context(0)
    fresh.set_tuning(256, 8, 0, 1)
    for k, shape in enumerate(shapes):
        sm = synth.uniform_sensor(*shape)
        pair = _pair("pair64", 40 + k, shape=shape, sensor=sm)
        sen = rir.Sensor.from_model(sm)
        src, dst = to_dev(pair.src), to_dev(pair.dst)
        guard = torch.full((1 << 16,), 7, dtype=torch.int32, device="cuda:0")
        a = rir.debug_associate(ctx, prm, sen, src, dst, 0, pair.gt)
        b = rir.debug_associate(fresh, prm, sen, src, dst, 0, pair.gt)
        assert a["u"].shape == (shape[0], shape[1])
        assert torch.equal(a["u"], b["u"]) and torch.equal(a["e"], b["e"])
        assert int((guard != 7).sum()) == 0
        P1, _ = rir.icp_batch(ctx, prm, [(sen, src, dst)])
        P2, _ = rir.icp_batch(fresh, prm, [(sen, src, dst)])
        assert torch.equal(P1, P2)
        del sen


def test_nonfinite_and_negative_ranges_count_as_no_return(rir, ctx):
    """Source and target pixels holding NaN, +-Inf or a negative range are
    'no return' on both sides (the oracle skips them): the pose and the
    statistics match the oracle and stay finite, on the tiled levels and on
    the pair-resident coarsest level alike."""
    pair = _pair("pair64", 11)
    rng = np.random.default_rng(11)
    src, dst = pair.src.copy(), pair.dst.copy()
    bad = np.array([np.nan, np.inf, -np.inf, -1.0, -0.0], np.float32)
    for img in (src, dst):
        flat = img.reshape(-1)
        hit = rng.choice(flat.size, flat.size // 50, replace=False)
        flat[hit] = bad[rng.integers(0, bad.size, hit.size)]
        # every value also on the pixels the coarser levels sample
        flat[np.arange(0, 8 * 1024, 4 * 1024 + 4)] = np.nan
        img[::4, ::4][5, 7:12] = bad
    bent = synth.Pair(pair.sensor, src, dst, pair.gt, 11)
    Tg, st = _run_gpu(rir, ctx, pair.sensor, [bent], [10, 10, 10], 3)
    To, so = oracle.icp(pair.sensor, src, dst, oracle.make_params(levels=3, iters=[10, 10, 10]))
    er, et = rot_trans_error(Tg[0], To)
    assert er < POSE_ROT_TOL and et < POSE_TRANS_TOL, (er, et)
    assert np.all(np.isfinite(st["JtJ"])) and np.all(np.isfinite(st["Jtr"]))
    for l in range(3):
        assert st[0, l]["status"] == so[l]["status"] == rir.LEVEL_OK, l
        assert abs(st[0, l]["n_valid"] - so[l]["n_valid"]) <= 0.002 * so[l]["n_valid"] + 5
    # one iteration at a shared pose: the kernel's normal equations against
    # the oracle's, and no pixel with a bad source range takes part
    T = pair.gt @ synth.make_pose(synth.rot_axis_angle([0.3, 1.0, 0.2], 0.01), [0.05, -0.03, 0.02])
    prm = rir.make_params(levels=3, iters=[1, 1, 1], delta=0.5)
    out = rir.debug_associate(ctx, prm, rir.Sensor.from_model(pair.sensor), to_dev(src), to_dev(dst), 0, T)
    ref = oracle.system(pair.sensor, 0, src, dst, oracle.make_params(levels=3, iters=[1, 1, 1], delta=0.5), T)
    mask = out["mask"].cpu().numpy().astype(bool).reshape(-1)
    assert not mask[~(src.reshape(-1) > 0) | ~np.isfinite(src.reshape(-1))].any()
    Hk = _jtj_matrix(out["stats"]["JtJ"])
    Hr = _jtj_matrix(ref["stats"]["JtJ"])
    amb = ambiguous(pair.sensor, 0, ref["uhat"], ref["phi"]) & ref["proj_valid"].astype(bool)
    assert np.all(np.isfinite(Hk))
    assert _normalised_diff(Hk, Hr) < JTJ_TOL + 4.0 * amb.sum() / max(ref["stats"]["n_valid"], 1)
