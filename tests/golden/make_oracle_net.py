"""Writes tests/golden/oracle_mlp_dynamic64.npz: a learned-weight network
trained entirely by the FP64 CPU oracle (test infrastructure only).

The library's own network is trained on the GPU by the library's kernels, so
it never reaches the oracle.  Learned-mode parity (GPU registration with a
network against the oracle's registration with the same network) needs a
realistic network whose values come from the oracle side: this script makes
one with nothing but oracle/ (features, residuals, registration, the
network's forward and backward passes) and the seeded scan generator.

Labels: the oracle's residuals e* at the ground-truth pose, the exact
solution of these synthetic pairs (the library's reading): a source pixel
whose correspondence has |e*| <= 3 sigma is labelled 1 (sigma = the scans'
range noise), other associated pixels 0.  The script also registers each
pair with the oracle's pseudo-Huber Gauss-Newton started at the ground truth
and reports how often labels taken at the pose it converges to (the literal
"converged residuals") agree with these: pseudo-Huber drifts towards the
moving boxes and spurious returns, so they differ on a quarter of the
pixels.  Features are taken along the oracle's pseudo-Huber
trajectory from the identity (start, after each coarse level, end) at every
pyramid level.  Training: Adam (0.9, 0.999, 1e-8) on FP64 master weights with
the weight matrices rounded to bf16 for every forward/backward pass (the
rounding points of the oracle's network), minibatches drawn with
replacement, learning rate decayed 10x over the run, parameters selected by
the oracle's registration success on held-out pairs.

Seeds: training pairs 20000.., validation pairs 21000.. (disjoint from the
library's training 3000-12999, evaluation 13000-13999 and model selection
14000-14199 seeds).

Usage: python tests/golden/make_oracle_net.py [--pairs N] [--steps K] [--threads T]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "oracle_mlp_dynamic64.npz")
LEVELS, ITERS, DELTA, R_MAX = 3, [10, 10, 10], 0.5, 80.0
W_BLOCKS = ((0, 896), (960, 5056), (5120, 5184))  # weight matrices (bf16)


def log(msg):
    print(f"[oracle-net] {msg}", file=sys.stderr, flush=True)


def bf16_round(x):
    """Round-to-nearest-even to bfloat16 through float32 (numpy)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def device_params(master):
    """The parameters a network holds: bf16 weight matrices, FP32 biases."""
    P = master.astype(np.float32).astype(np.float64)
    for a, b in W_BLOCKS:
        P[a:b] = bf16_round(master[a:b])
    return P


def init_params(seed):
    """He-style initialisation (hidden layers), small output layer."""
    rng = np.random.default_rng(seed)
    P = np.zeros(oracle.MLP_NPARAM)
    P[0:896] = rng.normal(size=896) * np.sqrt(2.0 / 14)
    P[960:5056] = rng.normal(size=4096) * np.sqrt(2.0 / 64)
    P[5120:5184] = rng.normal(size=64) * np.sqrt(1.0 / 64)
    return P


def pair_samples(seed, per_view, sigma):
    cfg = synth.CONFIGS["dynamic64"]
    pair = synth.gen_pair(cfg, seed)
    sm = pair.sensor
    prm = oracle.make_params(levels=LEVELS, iters=ITERS, delta=DELTA, r_max=R_MAX)
    # labels: residuals at the ground-truth pose; for comparison, at the pose
    # pseudo-Huber converges to from there
    Tc, _ = oracle.icp(sm, pair.src, pair.dst, prm, T_init=pair.gt)
    ref_c = oracle.system(sm, 0, pair.src, pair.dst, prm, Tc)
    ref_g = oracle.system(sm, 0, pair.src, pair.dst, prm, pair.gt)
    y_c = (np.abs(ref_c["e"]) <= 3.0 * sigma) & ref_c["mask"]
    y_g = (np.abs(ref_g["e"]) <= 3.0 * sigma) & ref_g["mask"]
    both = ref_c["mask"] & ref_g["mask"]
    agree = (int(np.sum(y_c[both] == y_g[both])), int(both.sum()))
    # views along the plain trajectory from the identity
    views = [np.eye(4)]
    for stop in range(LEVELS - 1, 0, -1):
        sched = [0 if l < stop else ITERS[l] for l in range(LEVELS)]
        views.append(oracle.icp(sm, pair.src, pair.dst, oracle.make_params(levels=LEVELS, iters=sched,
                                                                          delta=DELTA))[0])
    views.append(oracle.icp(sm, pair.src, pair.dst, prm)[0])
    rng = np.random.default_rng(seed)
    feats, labels = [], []
    for V in views:
        for lvl in range(LEVELS):
            s = 1 << lvl
            d = oracle.system(sm, lvl, pair.src, pair.dst, prm, V, with_features=True)
            ok = d["mask"] & ref_g["mask"][::s, ::s]
            idx = np.flatnonzero(ok)
            if idx.size == 0:
                continue
            if idx.size > per_view:
                idx = rng.choice(idx, per_view, replace=False)
            feats.append(d["feat"].reshape(-1, 14)[idx])
            labels.append(y_g[::s, ::s].reshape(-1)[idx].astype(np.float32))
    drift = oracle.pose_error(Tc, pair.gt)
    return np.concatenate(feats), np.concatenate(labels), agree, drift


def loss_grad(P, F, Y, pool, n_chunks):
    """Mean loss and gradient over a minibatch, split across threads (each
    chunk's mean weighted by its size)."""
    B = len(Y)
    bounds = np.linspace(0, B, n_chunks + 1).astype(int)
    parts = [(a, b) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    res = list(pool.map(lambda ab: oracle.mlp_loss_grad(P, F[ab[0]:ab[1]], Y[ab[0]:ab[1]]), parts))
    loss = sum(r[0] * (b - a) for r, (a, b) in zip(res, parts)) / B
    grad = sum(r[1] * (b - a) for r, (a, b) in zip(res, parts)) / B
    return loss, grad


def success_rate(P, pairs, pool):
    """Oracle registration with the network at the finest level (3, 10, 10
    iterations, finest first): share within 0.25 deg and 5 cm of the truth."""
    prm = oracle.make_params(levels=LEVELS, iters=[3, 10, 10], delta=DELTA, weight_mode=1, mlp=P, r_max=R_MAX,
                             learned_levels=0b001)

    def one(p):
        T, _ = oracle.icp(p.sensor, p.src, p.dst, prm)
        er, et = oracle.pose_error(T, p.gt)
        return er <= np.deg2rad(0.25) and et <= 0.05
    return float(np.mean(list(pool.map(one, pairs))))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=300)
    ap.add_argument("--val-pairs", type=int, default=48)
    ap.add_argument("--per-view", type=int, default=160)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--val-every", type=int, default=250)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args(argv)
    sigma = synth.CONFIGS["dynamic64"]["noise"].sigma
    pool = ThreadPoolExecutor(max_workers=args.threads)
    t0 = time.perf_counter()
    res = list(pool.map(lambda s: pair_samples(s, args.per_view, sigma), range(20000, 20000 + args.pairs)))
    F = np.concatenate([r[0] for r in res]).astype(np.float32)
    Y = np.concatenate([r[1] for r in res]).astype(np.float32)
    agree = np.sum([r[2] for r in res], axis=0)
    drift = np.array([r[3] for r in res])
    log(f"{len(Y)} samples ({Y.mean():.3f} positive) from {args.pairs} pairs in {time.perf_counter() - t0:.0f}s; "
        f"labels at the pose pseudo-Huber converges to from the ground truth (median drift "
        f"{np.median(drift[:, 0]) * 1e3:.2f} mrad / {np.median(drift[:, 1]) * 100:.2f} cm) agree with "
        f"ground-truth-pose labels on {agree[0] / agree[1]:.4f} of {agree[1]} pixels")
    val = [synth.gen_pair(synth.CONFIGS["dynamic64"], 21000 + i) for i in range(args.val_pairs)]
    master = init_params(0)
    m1 = np.zeros_like(master)
    m2 = np.zeros_like(master)
    rng = np.random.default_rng(1)
    best, hist = None, []
    for k in range(args.steps):
        idx = rng.integers(0, len(Y), args.batch)
        P = device_params(master)
        loss, g = loss_grad(P, F[idx], Y[idx], pool, args.threads)
        lr = args.lr * 0.1 ** (k / args.steps)
        m1 = 0.9 * m1 + 0.1 * g
        m2 = 0.999 * m2 + 0.001 * g * g
        mh = m1 / (1 - 0.9 ** (k + 1))
        vh = m2 / (1 - 0.999 ** (k + 1))
        master = master - lr * mh / (np.sqrt(vh) + 1e-8)
        if k % 100 == 0:
            hist.append((k, float(loss)))
            log(f"step {k} loss {loss:.4f} ({time.perf_counter() - t0:.0f}s)")
        if (k + 1) % args.val_every == 0 or k == args.steps - 1:
            Pd = device_params(master)
            sc = success_rate(Pd, val, pool)
            log(f"step {k + 1} validation success {sc:.3f}")
            if best is None or sc > best[0]:
                best = (sc, k + 1, Pd.copy())
    meta = {"train_seeds": [20000, 20000 + args.pairs - 1], "val_seeds": [21000, 21000 + args.val_pairs - 1],
            "samples": int(len(Y)), "positive": float(Y.mean()), "steps": args.steps, "batch": args.batch,
            "lr": args.lr, "per_view": args.per_view, "selected_step": best[1], "val_success": best[0],
            "label_agreement_converged_vs_gt_pose": [int(agree[0]), int(agree[1])],
            "median_drift_from_gt_rad_m": [float(np.median(drift[:, 0])), float(np.median(drift[:, 1]))],
            "loss": hist}
    np.savez(args.out, params=best[2], meta=json.dumps(meta))
    log(f"kept step {best[1]} (validation success {best[0]:.3f}); wrote {args.out}")


if __name__ == "__main__":
    main()
