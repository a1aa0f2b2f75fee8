"""GPU parity of the learned robust weight against the FP64 oracle: the MFMA
forward, the MFMA backward (gradients), the Adam update, the fused learned
weight inside the Gauss-Newton step, features and the pseudo-Huber fallback."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import ambiguous, mlp_band, rot_trans_error, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rir():
    import torch
    import paper_2112_02779_amd as rir
    assert torch.cuda.is_available()
    return rir


def _params(seed, scale=1.0):
    import paper_2112_02779_amd as rir
    P = rir.init_mlp_params(seed)
    P[896:960] = np.random.default_rng(seed).normal(size=64) * 0.1
    P[5056:5120] = np.random.default_rng(seed + 1).normal(size=64) * 0.1
    P[5184] = 0.3
    P[0:896] *= scale
    w, b = rir.split_params(P)
    return rir.join_params(w, b)


def _feats(seed, B):
    rng = np.random.default_rng(seed)
    f = np.empty((B, 14), np.float32)
    f[:, 0] = rng.uniform(0, 1, B)
    f[:, 1:9] = np.clip(rng.normal(size=(B, 8)) * 2, -4, 4)
    n = rng.normal(size=(B, 3))
    f[:, 9:12] = n / np.linalg.norm(n, axis=1, keepdims=True)
    f[:, 12:14] = np.clip(rng.normal(size=(B, 2)), -4, 4)
    return f


@pytest.mark.parametrize("B", [1, 63, 64, 1000, 70001])
def test_forward_matches_oracle(rir, B):
    P = _params(1)
    f = _feats(2, B)
    net = rir.Mlp(P)
    w = net.forward(to_dev(f)).cpu().numpy()
    _, wo = oracle.mlp_forward(P, f)
    # FP32 accumulation vs FP64 with identical bf16 rounding points.  A row
    # whose hidden pre-activation lies within the worst-case FP32 rounding of
    # a bf16 tie may round to the neighbouring activation on one side (the
    # band, decided from the oracle's pre-activations alone; with 128 hidden
    # roundings per row it holds a large share of the rows).  Every row
    # outside it has the same bf16 activations on both sides and agrees to
    # the FP32 rounding of the logit; rows inside move by at most a few bf16
    # steps of one activation, and rarely.
    band = mlp_band(oracle.mlp_preact(P, f))
    d = np.abs(w - wo)
    assert np.all(d[~band] < 2e-4), (np.max(d[~band]), int(np.argmax(np.where(band, 0, d))))
    assert np.all(d < 5e-2)
    if B >= 1000:
        # share statistics need enough rows (a single row may lie in the band)
        assert band.mean() < 0.75
        assert np.median(d) < 1e-6
        assert np.mean(d > 2e-4) < 1e-3


@pytest.mark.parametrize("B", [64, 5000, 131072])
def test_gradient_matches_oracle(rir, B):
    import torch
    P = _params(3)
    f = _feats(4, B)
    y = (np.random.default_rng(5).random(B) < 0.7).astype(np.float32)
    net = rir.Mlp(P)
    loss, g = net.train_step(to_dev(f), to_dev(y), lr=0.0, want_grads=True)
    torch.cuda.synchronize()
    lo, go = oracle.mlp_loss_grad(P, f, y)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.cpu()) - lo) < 1e-5 * max(1.0, abs(lo))
    blocks = {"W1": (0, 896), "b1": (896, 960), "W2": (960, 5056), "b2": (5056, 5120), "W3": (5120, 5184),
              "b3": (5184, 5185)}
    for name, (a, b) in blocks.items():
        scale = np.abs(go[a:b]).max()
        err = np.abs(g[a:b] - go[a:b]).max()
        assert err <= 2e-3 * scale + 1e-9, (name, err, scale)
    # with lr = 0 the parameters do not move
    np.testing.assert_array_equal(net.get_params(), P)


def test_adam_step_matches_numpy(rir):
    """One update: Adam (0.9, 0.999, 1e-8) on FP32 masters from the gradient,
    weights re-rounded to bf16."""
    import torch
    P = _params(6)
    f = _feats(7, 4096)
    y = (np.random.default_rng(8).random(4096) < 0.5).astype(np.float32)
    net = rir.Mlp(P)
    lr = 1e-3
    _, g = net.train_step(to_dev(f), to_dev(y), lr=lr, want_grads=True)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float32)
    m = 0.1 * g
    v = 0.001 * g * g
    upd = lr * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    ref = P - upd
    got = net.get_params()
    wi = np.r_[0:896, 960:5056, 5120:5184]
    bi = np.r_[896:960, 5056:5120, 5184:5185]
    np.testing.assert_allclose(got[bi], ref[bi], rtol=1e-5, atol=1e-7)
    w_ref, _ = rir.split_params(ref)
    w_got, _ = rir.split_params(got)
    assert np.mean(w_ref == w_got) > 0.99


def test_training_reduces_loss(rir):
    """A separable toy task: the loss falls by more than half in 200 steps."""
    import torch
    rng = np.random.default_rng(9)
    f = _feats(10, 8192)
    y = (f[:, 12] ** 2 + f[:, 13] ** 2 < 0.5).astype(np.float32)
    net = rir.Mlp(rir.init_mlp_params(11))
    ft, yt = to_dev(f), to_dev(y)
    l0, _ = net.train_step(ft, yt, lr=0.0)
    for _ in range(200):
        loss, _ = net.train_step(ft, yt, lr=3e-3)
    torch.cuda.synchronize()
    assert float(loss.cpu()) < 0.5 * float(l0.cpu())
    _ = rng


@pytest.mark.parametrize("level", [0, 1])
def test_features_and_learned_weights_in_the_step_match_oracle(rir, level):
    P = _params(12, scale=0.5)
    pair = synth.gen_pair(synth.CONFIGS["dynamic64"], 13)
    sm = pair.sensor
    sen = rir.Sensor.from_model(sm)
    ctx = rir.Context(0)
    net = rir.Mlp(P)
    T = pair.gt @ synth.make_pose(synth.rot_axis_angle([0, 0, 1.0], 0.004), [0.03, 0.0, 0.0])
    prm = rir.make_params(levels=3, iters=[1, 1, 1], weight_mode=rir.WEIGHT_LEARNED, mlp=net, r_max=80.0)
    out = rir.debug_associate(ctx, prm, sen, to_dev(pair.src), to_dev(pair.dst), level, T, features=True)
    ref = oracle.system(sm, level, pair.src, pair.dst,
                        oracle.make_params(levels=3, iters=[1, 1, 1], weight_mode=1, mlp=P, r_max=80.0), T,
                        use_learned=True, with_features=True)
    amb = ambiguous(sm, level, ref["uhat"], ref["phi"])
    m = ~amb & ref["mask"]
    gm = out["mask"].cpu().numpy().astype(bool)
    np.testing.assert_array_equal(gm[~amb], ref["mask"][~amb])
    gf = out["feat"].cpu().numpy()
    np.testing.assert_allclose(gf[m], ref["feat"][m], atol=2e-5, rtol=2e-5)
    gw = out["w"].cpu().numpy()
    assert np.max(np.abs(gw[m] - ref["w"][m])) < 2e-3
    assert np.median(np.abs(gw[m] - ref["w"][m])) < 1e-5


def _huber_like_params():
    """A hand-set network whose weight falls with the residual like a robust
    kernel: w = sigmoid(2 - 3 |f12|), |f12| = relu(f12) + relu(-f12) with
    f12 = clamp(e / delta); every weight is exact in bf16.  Registration with
    it converges like pseudo-Huber, so the GPU/oracle comparison is well
    conditioned."""
    P = np.zeros(5185)
    P[0 * 14 + 12] = 1.0      # W1[0][12]
    P[1 * 14 + 12] = -1.0     # W1[1][12]
    P[960 + 0] = 1.0          # W2[0][0]
    P[960 + 1] = 1.0          # W2[0][1]
    P[5120] = -3.0            # W3[0]
    P[5184] = 2.0             # b3
    return P


def test_huber_like_network_is_what_it_claims():
    f = np.zeros((5, 14), np.float32)
    f[:, 12] = [0.0, 0.5, -0.5, 1.0, -4.0]
    _, w = oracle.mlp_forward(_huber_like_params(), f)
    a = np.abs(f[:, 12].astype(np.float64))
    np.testing.assert_allclose(w, 1.0 / (1.0 + np.exp(-(2.0 - 3.0 * a))), rtol=1e-12)


# (scene, learned_levels).  With pseudo-Huber at the finest level a dynamic
# scene need not converge (the re-association cycles at ~1e-4 rad), where no
# two precisions can agree to 1e-4; the coarse-only case uses a static scene.
@pytest.mark.parametrize("case", [("dynamic64", 0), ("dynamic64", 0b001), ("pair64", 0b110)])
def test_learned_icp_matches_oracle(rir, case):
    cfg, learned_levels = case
    P = _huber_like_params()
    pair = synth.gen_pair(synth.CONFIGS[cfg], 15)
    sm = pair.sensor
    sen = rir.Sensor.from_model(sm)
    ctx = rir.Context(0)
    net = rir.Mlp(P)
    prm = rir.make_params(levels=3, iters=[10, 10, 10], weight_mode=rir.WEIGHT_LEARNED, mlp=net, r_max=80.0,
                          learned_levels=learned_levels)
    poses, stats = rir.icp_batch(ctx, prm, [(sen, to_dev(pair.src), to_dev(pair.dst))])
    To, so = oracle.icp(sm, pair.src, pair.dst,
                        oracle.make_params(levels=3, iters=[10, 10, 10], weight_mode=1, mlp=P, r_max=80.0,
                                           learned_levels=learned_levels))
    er, et = rot_trans_error(poses.cpu().numpy()[0], To)
    assert er < 1e-4 and et < 1e-3, (er, et)
    st = rir.stats_to_numpy(stats, 1, 3)
    assert [int(s) for s in st["status"][0]] == [int(s["status"]) for s in so]


def test_rejecting_network_falls_back_to_pseudo_huber(rir):
    P = np.zeros(5185)
    P[5184] = -40.0
    pair = synth.gen_pair(synth.CONFIGS["pair64"], 16)
    sen = rir.Sensor.from_model(pair.sensor)
    ctx = rir.Context(0)
    net = rir.Mlp(P)
    src, dst = to_dev(pair.src), to_dev(pair.dst)
    prm_l = rir.make_params(levels=3, iters=[3, 3, 3], weight_mode=rir.WEIGHT_LEARNED, mlp=net)
    prm_h = rir.make_params(levels=3, iters=[3, 3, 3])
    Tl, sl = rir.icp_batch(ctx, prm_l, [(sen, src, dst)])
    Th, sh = rir.icp_batch(ctx, prm_h, [(sen, src, dst)])
    # the plain run takes the pair-resident kernel on the small coarse levels
    # (another summation order), so the poses agree to FP32 rounding
    np.testing.assert_allclose(Tl.cpu().numpy(), Th.cpu().numpy(), rtol=0, atol=1e-7)
    assert np.all(rir.stats_to_numpy(sl, 1, 3)["status"] == rir.LEVEL_FALLBACK_HUBER)
