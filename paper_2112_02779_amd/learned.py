"""Learned per-pixel robust weight: training data, training and evaluation.

Everything here runs on the GPU through librir (the same kernels as
registration); nothing calls the test oracle.

Labels (a reading of "labels from the converged residuals"): the residuals
e* at the ground-truth pose, which for these synthetic scenes is the exact
solution (pseudo-Huber started there drifts several centimetres under moving
objects and spurious returns, i.e. towards the very outliers the labels are
meant to mark).  A source pixel whose correspondence has |e*| <= 3 sigma
(sigma = the scans' range noise) is labelled 1 (reliable), otherwise 0
(moving objects, spurious returns, occlusion edges).  Labels therefore do not
depend on the current pose.  Features are taken where the network will see
them: at the poses a plain pseudo-Huber registration from the initial pose
passes through (start, after each coarse level, end) and at every pyramid
level.

CLI:  python -m paper_2112_02779_amd.learned train  [--pairs N] [--out FILE]
      python -m paper_2112_02779_amd.learned eval   [--pairs N] [--weights FILE]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(_HERE, "weights", "robust_mlp_dynamic64.npz")


def _rir():
    import paper_2112_02779_amd as rir
    return rir


def _log(msg):
    print(f"[learned] {msg}", file=sys.stderr, flush=True)


class DeviceBatch:
    """Pairs uploaded to the GPU with one sensor handle per distinct model."""

    def __init__(self, pairs, device="cuda:0"):
        import torch
        rir = _rir()
        self.pairs = pairs
        self.sensors = {}
        self.items = []
        for p in pairs:
            key = (p.sensor.H, p.sensor.W, p.sensor.r0, p.sensor.phi.tobytes(), p.sensor.theta.tobytes())
            if key not in self.sensors:
                self.sensors[key] = rir.Sensor.from_model(p.sensor)
            self.items.append((self.sensors[key], torch.from_numpy(p.src).to(device),
                               torch.from_numpy(p.dst).to(device)))

    def __len__(self):
        return len(self.items)


def register(ctx, batch: DeviceBatch, levels, iters, init=None, mlp=None, delta=0.5, r_max=80.0, chunk=256,
             learned_levels=0):
    """Batched registration; returns host poses [n, 4, 4] and stats [n, levels]."""
    import torch
    rir = _rir()
    prm = rir.make_params(levels=levels, iters=iters, delta=delta, r_max=r_max,
                          weight_mode=rir.WEIGHT_LEARNED if mlp is not None else rir.WEIGHT_HUBER, mlp=mlp,
                          learned_levels=learned_levels)
    n = len(batch)
    poses = np.zeros((n, 4, 4))
    stats = []
    for a in range(0, n, chunk):
        items = batch.items[a:a + chunk]
        T0 = None
        if init is not None:
            T0 = torch.from_numpy(np.ascontiguousarray(init[a:a + chunk])).to("cuda:0")
        P, S = rir.icp_batch(ctx, prm, items, init_poses=T0)
        poses[a:a + len(items)] = P.cpu().numpy()
        stats.append(rir.stats_to_numpy(S, len(items), levels))
    return poses, np.concatenate(stats)


def make_samples(ctx, batch: DeviceBatch, sigma: float, levels=3, iters=(10, 10, 10), delta=0.5, r_max=80.0,
                 per_view=2048, seed=0):
    """(features [M, 14] float32, labels [M] float32) for the pairs of `batch`."""
    rir = _rir()
    rng = np.random.default_rng(seed)
    n = len(batch)
    gts = np.stack([p.gt for p in batch.pairs])
    # poses along the plain trajectory from the identity
    views = [np.tile(np.eye(4), (n, 1, 1))]
    for stop in range(levels - 1, 0, -1):
        sched = [0 if l < stop else iters[l] for l in range(levels)]
        views.append(register(ctx, batch, levels, sched, delta=delta)[0])
    views.append(register(ctx, batch, levels, list(iters), delta=delta)[0])
    prm = rir.make_params(levels=levels, iters=list(iters), delta=delta, r_max=r_max)
    feats, labels = [], []
    t0 = time.perf_counter()
    for i, (sensor, src, dst) in enumerate(batch.items):
        if i and i % 500 == 0:
            _log(f"samples from {i}/{n} pairs ({time.perf_counter() - t0:.0f}s)")
        d0 = rir.debug_associate(ctx, prm, sensor, src, dst, 0, gts[i])
        m0 = d0["mask"].cpu().numpy().astype(bool)
        y0 = (np.abs(d0["e"].cpu().numpy()) <= 3.0 * sigma) & m0
        for V in views:
            for lvl in range(levels):
                s = 1 << lvl
                d = rir.debug_associate(ctx, prm, sensor, src, dst, lvl, V[i], features=True)
                m = d["mask"].cpu().numpy().astype(bool)
                lab_ok = m & m0[::s, ::s]
                idx = np.flatnonzero(lab_ok)
                if idx.size == 0:
                    continue
                if idx.size > per_view:
                    idx = rng.choice(idx, per_view, replace=False)
                f = d["feat"].cpu().numpy().reshape(-1, 14)[idx]
                y = y0[::s, ::s].reshape(-1)[idx]
                feats.append(f)
                labels.append(y.astype(np.float32))
    return np.concatenate(feats), np.concatenate(labels)


def train(mlp, feats, labels, steps=3000, batch=8192, lr=2e-3, seed=0, log_every=500, validate=None,
          val_every=0):
    """Adam on minibatches drawn with replacement (learning rate decayed 10x
    over the run); returns the loss history.  With validate (a function of
    the network returning a score, higher is better) the parameters are
    scored every val_every steps and at the end, and the best-scoring ones are
    kept (model selection on held-out pairs by the registration quality the
    network is for, not by the classification loss)."""
    import torch
    F = torch.from_numpy(np.ascontiguousarray(feats, dtype=np.float32)).to("cuda:0")
    Y = torch.from_numpy(np.ascontiguousarray(labels, dtype=np.float32)).to("cuda:0")
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(seed)
    hist, best = [], None
    for k in range(steps):
        idx = torch.randint(0, F.shape[0], (batch,), device="cuda:0", generator=gen)
        cur_lr = lr * (0.1 ** (k / max(steps, 1)))
        loss, _ = mlp.train_step(F[idx].contiguous(), Y[idx].contiguous(), cur_lr)
        last = k == steps - 1
        if k % log_every == 0 or last:
            hist.append((k, float(loss.cpu())))
            _log(f"step {k} loss {hist[-1][1]:.4f}")
        if validate is not None and ((val_every and (k + 1) % val_every == 0) or last):
            score = float(validate(mlp))
            _log(f"step {k + 1} validation score {score:.4f}")
            if best is None or score > best[0]:
                best = (score, k + 1, mlp.get_params())
    if best is not None:
        mlp.set_params(best[2])
        _log(f"kept the parameters of step {best[1]} (validation score {best[0]:.4f})")
        hist.append(("selected_step", best[1], best[0]))
    return hist


def validation_score(ctx, batch, levels=3, iters=(3, 10, 10), learned_levels=0b001):
    """Success rate (<= 0.25 deg, <= 5 cm) of learned registration on batch."""
    gts = np.stack([p.gt for p in batch.pairs])

    def score(mlp):
        T, _ = register(ctx, batch, levels, list(iters), mlp=mlp, learned_levels=learned_levels)
        return summarize(pose_errors(T, gts))["success_rate"]
    return score


def pose_errors(poses, refs):
    out = []
    for T, R in zip(poses, refs):
        D = T[:3, :3] @ R[:3, :3].T
        s = np.linalg.norm([D[2, 1] - D[1, 2], D[0, 2] - D[2, 0], D[1, 0] - D[0, 1]]) / 2
        out.append((float(np.arctan2(s, (np.trace(D) - 1) / 2)), float(np.linalg.norm(T[:3, 3] - R[:3, 3]))))
    return np.array(out)


def summarize(err, rot_ok=np.deg2rad(0.25), trans_ok=0.05):
    return {"median_rot_rad": float(np.median(err[:, 0])), "median_trans_m": float(np.median(err[:, 1])),
            "p90_rot_rad": float(np.percentile(err[:, 0], 90)), "p90_trans_m": float(np.percentile(err[:, 1], 90)),
            "success_rate": float(np.mean((err[:, 0] <= rot_ok) & (err[:, 1] <= trans_ok)))}


# Evaluation modes: (name, iterations per level (finest first), learned?,
# learned_levels).  "learned" replaces pseudo-Huber at the finest level only
# (coarse levels start far from the solution, where per-pixel evidence cannot
# tell inliers from outliers); the "*_3" modes run 3 finest-level iterations.
MODES = (("huber", (10, 10, 10), False, 0), ("learned", (10, 10, 10), True, 0b001),
         ("learned_all_levels", (10, 10, 10), True, 0), ("huber_3", (3, 10, 10), False, 0),
         ("learned_3", (3, 10, 10), True, 0b001))


def evaluate(ctx, mlp, batch: DeviceBatch, levels=3, modes=MODES, repeats=3):
    """Learned vs plain pseudo-Huber on the same pairs: pose error against the
    ground truth, success rate (<= 0.25 deg and <= 5 cm), batched throughput
    (pairs/s on this GPU) and goodput = pairs/s x success rate."""
    import torch
    gts = np.stack([p.gt for p in batch.pairs])
    res = {}
    for name, iters, use_net, ll in modes:
        net = mlp if use_net else None
        register(ctx, batch, levels, list(iters), mlp=net, learned_levels=ll)  # warm-up (plans, graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            T, st = register(ctx, batch, levels, list(iters), mlp=net, learned_levels=ll)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / repeats
        s = summarize(pose_errors(T, gts))
        s["iters"] = list(iters)
        s["learned_levels"] = ll if use_net else None
        s["pairs_per_s"] = len(batch) / dt
        s["goodput_pairs_per_s"] = s["pairs_per_s"] * s["success_rate"]
        s["fallback_levels"] = int(np.sum(st["status"] == 2))
        res[name] = s
    return res


def save(mlp, path=WEIGHTS, meta=None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=mlp.get_params(), meta=json.dumps(meta or {}))


def load(path=WEIGHTS) -> np.ndarray:
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float64)


def main(argv=None):
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval"])
    ap.add_argument("--pairs", type=int, default=1000)
    ap.add_argument("--eval-pairs", type=int, default=1000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--per-view", type=int, default=160)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--val-pairs", type=int, default=200)
    ap.add_argument("--val-every", type=int, default=500)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--weights", default=WEIGHTS)
    args = ap.parse_args(argv)
    rir = _rir()
    cfg = synth.CONFIGS["dynamic64"]
    ctx = rir.Context(0)
    if args.cmd == "train":
        t0 = time.perf_counter()
        pairs = []
        for i in range(args.pairs):
            pairs.append(synth.gen_pair(cfg, 3000 + i))
            if (i + 1) % 1000 == 0:
                _log(f"generated {i + 1} training pairs ({time.perf_counter() - t0:.0f}s)")
        _log(f"generated {len(pairs)} training pairs in {time.perf_counter() - t0:.1f}s")
        batch = DeviceBatch(pairs)
        t0 = time.perf_counter()
        F, Y = make_samples(ctx, batch, sigma=cfg["noise"].sigma, per_view=args.per_view)
        del batch, pairs
        _log(f"{len(Y)} samples ({Y.mean():.3f} positive) in {time.perf_counter() - t0:.1f}s")
        mlp = rir.Mlp(rir.init_mlp_params(0))
        val = None
        if args.val_pairs > 0:
            val = validation_score(ctx, DeviceBatch([synth.gen_pair(cfg, 14000 + i) for i in range(args.val_pairs)]))
        hist = train(mlp, F, Y, steps=args.steps, lr=args.lr, log_every=max(1, args.steps // 10), validate=val,
                     val_every=args.val_every)
        save(mlp, args.out, {"train_pairs": args.pairs, "train_seeds": [3000, 3000 + args.pairs - 1],
                             "val_seeds": [14000, 14000 + args.val_pairs - 1], "samples": int(len(Y)),
                             "positive": float(Y.mean()), "steps": args.steps, "lr": args.lr,
                             "per_view": args.per_view, "loss": hist})
        _log(f"saved {args.out}")
    params = load(args.out if args.cmd == "train" else args.weights)
    mlp = rir.Mlp(params)
    pairs = [synth.gen_pair(cfg, 13000 + i) for i in range(args.eval_pairs)]
    _log(f"evaluating on {len(pairs)} held-out pairs")
    res = evaluate(ctx, mlp, DeviceBatch(pairs))
    res["eval_seeds"] = [13000, 13000 + args.eval_pairs - 1]
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
