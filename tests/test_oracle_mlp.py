"""Pins of the oracle's learned-weight network (CPU only).

The 14-64-64-1 per-pixel weight network is not part of the paper; it replaces
the pseudo-Huber weight of Eq. (7).  The oracle's forward pass and its
hand-written backward pass are pinned against torch's float64 autograd on the
same network, with the same bfloat16 rounding points expressed as
straight-through roundings (forward) and gradient roundings (backward).
"""
import numpy as np
import torch
import torch.nn.functional as F

NP = 5185


def _rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    P = np.zeros(NP)
    P[:896] = rng.normal(size=896) * scale
    P[896:960] = rng.normal(size=64) * 0.1
    P[960:5056] = rng.normal(size=4096) * scale / 2
    P[5056:5120] = rng.normal(size=64) * 0.1
    P[5120:5184] = rng.normal(size=64) * scale
    P[5184] = 0.2
    # weight matrices hold bfloat16 values
    t = torch.tensor(P)
    for a, b in ((0, 896), (960, 5056), (5120, 5184)):
        t[a:b] = t[a:b].float().bfloat16().double()
    return t.numpy()


def _rand_feats(seed, B):
    rng = np.random.default_rng(seed)
    f = np.empty((B, 14), np.float32)
    f[:, 0] = rng.uniform(0, 1, B)
    f[:, 1:9] = np.clip(rng.normal(size=(B, 8)) * 2, -4, 4)
    n = rng.normal(size=(B, 3))
    f[:, 9:12] = n / np.linalg.norm(n, axis=1, keepdims=True)
    f[:, 12:14] = np.clip(rng.normal(size=(B, 2)), -4, 4)
    return f


def _bf(x):
    return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)


class _STE(torch.autograd.Function):
    """Forward: round to bfloat16.  Backward: pass the gradient through."""

    @staticmethod
    def forward(ctx, x):
        return _bf(x)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """Forward: identity.  Backward: round the incoming gradient to bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return _bf(g)


def _torch_net(P, feats, labels=None):
    P = torch.tensor(P, dtype=torch.float64, requires_grad=True)
    W1 = P[:896].view(64, 14)
    b1 = P[896:960]
    W2 = P[960:5056].view(64, 64)
    b2 = P[5056:5120]
    W3 = P[5120:5184]
    b3 = P[5184]
    f = _bf(torch.tensor(feats, dtype=torch.float64))
    a1 = _RoundGrad.apply(f @ W1.T + b1)
    h1 = _STE.apply(torch.relu(a1))
    a2 = _RoundGrad.apply(h1 @ W2.T + b2)
    h2 = _STE.apply(torch.relu(a2))
    z = _RoundGrad.apply(h2 @ W3 + b3)
    if labels is None:
        return z.detach().numpy(), None, None
    y = torch.tensor(labels, dtype=torch.float64)
    loss = F.binary_cross_entropy_with_logits(z, y, reduction="mean")
    loss.backward()
    return z.detach().numpy(), float(loss.detach()), P.grad.numpy()


def test_bf16_rounding_is_round_to_nearest_even(orc):
    """The bfloat16 rounding point matches torch's float -> bfloat16 conversion."""
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=2000) * 10 ** rng.uniform(-6, 6, 2000),
                        [0.0, -0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0, 1e-40]])
    ref = torch.tensor(x).float().bfloat16().double().numpy()
    got = np.array([orc.bf16(v) for v in x])
    np.testing.assert_array_equal(got, ref)


def test_mlp_forward_matches_torch(orc):
    P = _rand_params(1)
    f = _rand_feats(2, 512)
    z, w = orc.mlp_forward(P, f)
    zt, _, _ = _torch_net(P, f)
    np.testing.assert_allclose(z, zt, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(w, 1 / (1 + np.exp(-zt)), rtol=1e-12)


def test_mlp_preactivations_match_torch(orc):
    """The hidden pre-activations the oracle reports (used to find the rows
    an FP32 evaluation may round differently) are those of torch's float64
    network with the same rounding points; the magnitude sums bound them."""
    P = _rand_params(11)
    f = _rand_feats(12, 300)
    pre = orc.mlp_preact(P, f)
    Pt = torch.tensor(P)
    W1, b1, W2, b2 = Pt[:896].view(64, 14), Pt[896:960], Pt[960:5056].view(64, 64), Pt[5056:5120]
    fb = _bf(torch.tensor(f, dtype=torch.float64))
    a1 = fb @ W1.T + b1
    h1 = _bf(torch.relu(a1))
    a2 = h1 @ W2.T + b2
    np.testing.assert_allclose(pre["a1"], a1.numpy(), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(pre["a2"], a2.numpy(), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(pre["s1"], (fb.abs() @ W1.abs().T + b1.abs()).numpy(), rtol=1e-13)
    np.testing.assert_allclose(pre["s2"], (h1 @ W2.abs().T + b2.abs()).numpy(), rtol=1e-13)
    assert np.all(pre["s1"] >= np.abs(pre["a1"])) and np.all(pre["s2"] >= np.abs(pre["a2"]))


def test_mlp_zero_weights_give_bias_sigmoid(orc):
    P = np.zeros(NP)
    P[5184] = -1.25
    _, w = orc.mlp_forward(P, _rand_feats(3, 16))
    np.testing.assert_allclose(w, 1 / (1 + np.exp(1.25)), rtol=1e-15)


def test_mlp_loss_and_gradient_match_torch_autograd(orc):
    P = _rand_params(4)
    f = _rand_feats(5, 256)
    y = (np.random.default_rng(6).random(256) < 0.6).astype(np.float32)
    loss, g = orc.mlp_loss_grad(P, f, y)
    _, lt, gt = _torch_net(P, f, y)
    assert abs(loss - lt) <= 1e-12 * max(1, abs(lt))
    scale = np.abs(gt).max()
    np.testing.assert_allclose(g, gt, rtol=1e-9, atol=1e-12 * scale)
    # every parameter block receives gradient
    for a, b in ((0, 896), (896, 960), (960, 5056), (5056, 5120), (5120, 5184), (5184, 5185)):
        assert np.abs(g[a:b]).max() > 0


def test_mlp_gradient_of_last_layer_matches_central_differences(orc):
    """The last layer's parameters do not pass through a rounding point, so
    central differences of the loss pin their gradient up to the bf16
    rounding of dz (relative 2^-9)."""
    P = _rand_params(7)
    f = _rand_feats(8, 64)
    y = (np.random.default_rng(9).random(64) < 0.5).astype(np.float32)
    _, g = orc.mlp_loss_grad(P, f, y)
    h = 1e-6
    for k in list(range(5120, 5185, 7)) + [5184]:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        lp, _ = orc.mlp_loss_grad(Pp, f, y)
        lm, _ = orc.mlp_loss_grad(Pm, f, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 2 ** -8 * np.abs(g[5120:5185]).max() + 1e-9, (k, fd, g[k])


def test_learned_features_indexing(orc):
    """Learned-weight features of a correspondence, recomputed with numpy
    indexing: target range / r_max, the 8 level-l neighbours of the associated
    target pixel in raster order (u wraps, missing rows or returns read +4),
    the normal, the clamped residual and the projective signed distance of
    Eq. (8)-(9)."""
    import synth
    pair = synth.gen_pair(synth.CONFIGS["dynamic64"], 31, shape=(32, 512))
    delta, r_max, lvl = 0.5, 80.0, 1
    prm = orc.make_params(levels=2, iters=[1, 1], delta=delta, r_max=r_max)
    T = synth.make_pose(synth.rot_axis_angle([0, 0, 1.0], 0.01), [0.1, 0.05, 0.0])
    out = orc.system(pair.sensor, lvl, pair.src, pair.dst, prm, T, with_features=True)
    s = 1 << lvl
    D = pair.dst[::s, ::s].astype(np.float64)
    Hl, Wl = D.shape
    idx = np.argwhere(out["mask"])
    rng = np.random.default_rng(0)
    for vp, up in idx[rng.choice(len(idx), 300, replace=False)]:
        u, v = out["u"][vp, up], out["v"][vp, up]
        f = out["feat"][vp, up]
        rc = D[v, u]
        ref = [rc / r_max]
        for dv in (-1, 0, 1):
            for du in (-1, 0, 1):
                if du == 0 and dv == 0:
                    continue
                vv, uu = v + dv, (u + du) % Wl
                val = 4.0
                if 0 <= vv < Hl and np.isfinite(D[vv, uu]) and D[vv, uu] > 0:
                    val = np.clip((D[vv, uu] - rc) / delta, -4, 4)
                ref.append(val)
        ref += list(out["J"][vp, up, 3:])
        ref.append(np.clip(out["e"][vp, up] / delta, -4, 4))
        p3 = orc.unproject(pair.sensor, s * up, s * vp, float(pair.src[s * vp, s * up]))
        x = T[:3, :3] @ p3 + T[:3, 3]
        ref.append(np.clip((rc - np.linalg.norm(x)) / delta, -4, 4))
        np.testing.assert_allclose(f, np.array(ref, np.float32), rtol=1e-6, atol=1e-6)


def test_learned_constant_weight_step_is_unweighted_least_squares(orc):
    """With a network whose output is constant (all weights zero), every
    correspondence has the same weight, so one learned Gauss-Newton step is
    the unweighted least-squares step of Eq. (7) (numpy.linalg.lstsq)."""
    import scipy.linalg
    import synth
    pair = synth.gen_pair(synth.CONFIGS["pair64"], 32, shape=(32, 512))
    P = np.zeros(NP)
    P[5184] = 0.7
    prm = orc.make_params(levels=1, iters=[1], weight_mode=1, mlp=P)
    T0 = synth.make_pose(np.eye(3), [0.05, -0.02, 0.01])
    out = orc.system(pair.sensor, 0, pair.src, pair.dst, prm, T0)
    m = out["mask"]
    xi = -np.linalg.lstsq(out["J"][m], out["e"][m], rcond=None)[0]
    T1, st = orc.icp(pair.sensor, pair.src, pair.dst, prm, T_init=T0)
    K = np.zeros((4, 4))
    K[:3, :3] = [[0, -xi[2], xi[1]], [xi[2], 0, -xi[0]], [-xi[1], xi[0], 0]]
    K[:3, 3] = xi[3:]
    np.testing.assert_allclose(T1, scipy.linalg.expm(K) @ T0, atol=1e-10)
    assert st[0]["status"] == orc.ORC_OK
    np.testing.assert_allclose(st[0]["sum_w"], m.sum() / (1 + np.exp(-0.7)), rtol=1e-12)
    # a network that rejects everything falls back to pseudo-Huber
    P[5184] = -40.0
    prm2 = orc.make_params(levels=1, iters=[1], weight_mode=1, mlp=P)
    T2, st2 = orc.icp(pair.sensor, pair.src, pair.dst, prm2, T_init=T0)
    T3, _ = orc.icp(pair.sensor, pair.src, pair.dst, orc.make_params(levels=1, iters=[1]), T_init=T0)
    assert st2[0]["status"] == orc.ORC_FALLBACK_HUBER
    np.testing.assert_array_equal(T2, T3)


def test_learned_levels_select_where_the_network_weighs(orc):
    """learned_levels = bit set of levels with learned weights: a level
    outside the set runs exactly the pseudo-Huber iteration, a level inside it
    the learned one (constant network => unweighted step, which differs)."""
    import synth
    pair = synth.gen_pair(synth.CONFIGS["pair64"], 33, shape=(32, 512))
    P = np.zeros(NP)
    P[5184] = 0.7
    T0 = synth.make_pose(synth.rot_axis_angle([0, 0, 1.0], 0.01), [0.05, -0.02, 0.01])
    huber = orc.make_params(levels=2, iters=[2, 2])
    Th, sh = orc.icp(pair.sensor, pair.src, pair.dst, huber, T_init=T0)
    # learned only at level 1: level 1 differs from Huber, so the result does
    coarse = orc.make_params(levels=2, iters=[2, 2], weight_mode=1, mlp=P, learned_levels=0b10)
    Tc, sc = orc.icp(pair.sensor, pair.src, pair.dst, coarse, T_init=T0)
    assert not np.array_equal(Tc, Th)
    np.testing.assert_allclose(sc[1]["sum_w"], sc[1]["n_valid"] / (1 + np.exp(-0.7)), rtol=1e-12)
    # learned only at level 1 with no level-0 iterations equals learned everywhere
    only1 = orc.make_params(levels=2, iters=[0, 2], weight_mode=1, mlp=P, learned_levels=0b10)
    every = orc.make_params(levels=2, iters=[0, 2], weight_mode=1, mlp=P)
    np.testing.assert_array_equal(orc.icp(pair.sensor, pair.src, pair.dst, only1, T_init=T0)[0],
                                  orc.icp(pair.sensor, pair.src, pair.dst, every, T_init=T0)[0])
    # learned only at level 0 with no level-0 iterations equals pseudo-Huber
    only0 = orc.make_params(levels=2, iters=[0, 2], weight_mode=1, mlp=P, learned_levels=0b01)
    plain = orc.make_params(levels=2, iters=[0, 2])
    T0a, s0a = orc.icp(pair.sensor, pair.src, pair.dst, only0, T_init=T0)
    np.testing.assert_array_equal(T0a, orc.icp(pair.sensor, pair.src, pair.dst, plain, T_init=T0)[0])
    assert s0a[1]["status"] == orc.ORC_OK
