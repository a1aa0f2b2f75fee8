"""Registration accuracy against frame distance (Sec. 6.1, the evaluation of
Tables 1-2 and the artifact argument of Fig. 1), on synthetic odometry
sequences registered by the library's kernels.

For frame distance d, M pairs (k + d -> k) of one sequence are registered
from the identity and compared with the ground truth (rotation and
translation error, Sec. 6.1 metrics).  Two comparisons:

* multi-scale (3 levels, 10 iterations each) against single-scale (one
  level, 30 iterations: the same iteration budget);
* the sensor's own lookup tables (non-uniform elevations, staggered azimuth
  offsets, receiver offset) against the "synthetic intrinsics" model of
  Sec. 3.2 (uniform elevations over the same field of view, no offsets),
  both registering scans of the same sensor.

    python -m paper_2112_02779_amd.frame_distance --out sweep.json
    python -m paper_2112_02779_amd.frame_distance --misalignment --out misalignment.json

A third sweep varies the initial misalignment of consecutive scans
(rotation and translation) for 1, 3 and 4 pyramid levels at the same
iteration budget (misalignment_sweep).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

#: success: within 0.25 deg and 5 cm of the ground truth
ROT_OK, TRANS_OK = np.deg2rad(0.25), 0.05


def pose_errors(T, gts):
    out = []
    for A, B in zip(T, gts):
        D = A[:3, :3] @ B[:3, :3].T
        s = np.linalg.norm([D[2, 1] - D[1, 2], D[0, 2] - D[2, 0], D[1, 0] - D[0, 1]]) / 2
        out.append((np.arctan2(s, (np.trace(D) - 1) / 2), np.linalg.norm(A[:3, 3] - B[:3, 3])))
    return np.array(out)


def summary(e):
    ok = (e[:, 0] <= ROT_OK) & (e[:, 1] <= TRANS_OK)
    return {"success": float(ok.mean()), "median_rot_rad": float(np.median(e[:, 0])),
            "median_trans_m": float(np.median(e[:, 1])), "p90_rot_rad": float(np.percentile(e[:, 0], 90)),
            "p90_trans_m": float(np.percentile(e[:, 1], 90))}


def synthetic_intrinsics(sensor):
    """The Sec. 3.2 "synthetic" model of a sensor: rows uniform between its
    first and last elevation, no azimuth offsets, no receiver offset."""
    import synth
    H = sensor.H
    phi = sensor.phi[0] - np.arange(H, dtype=np.float64) * (sensor.phi[0] - sensor.phi[-1]) / (H - 1)
    return synth.Sensor(H, sensor.W, phi, np.zeros(H), 0.0)


def run(distances=(1, 2, 4, 8, 16), n_pairs=50, seed=1000, shape=(64, 1024), log=None):
    import torch
    import synth
    import paper_2112_02779_amd as rir
    dev = torch.device("cuda:0")
    ctx = rir.Context(0)
    cfg = dict(synth.CONFIGS["odometry128x2048"])
    # walking-pace motion (0.05-0.5 m and up to 1 deg of yaw per frame), so
    # that the distances span the range where registration starts to fail
    cfg.update(shapes=[shape], step_max=0.5, yaw_max_deg=1.0)
    n_scans = n_pairs + max(distances)
    sensors = {"uniform": synth.uniform_sensor(*shape), "staggered_r0": synth.staggered_sensor(*shape, r0=0.015)}
    out = {"workload": f"odometry sequences of {n_scans} scans {shape[0]}x{shape[1]} (seed {seed}; forward "
                       f"U(0.05, 0.5) m and yaw U(0, 1) deg per frame), "
                       f"{n_pairs} pairs (k + d -> k) per frame distance d, identity start",
           "success": "within 0.25 deg and 5 cm of the ground truth", "sweeps": {}}
    for sname, sm in sensors.items():
        seq = synth.gen_sequence(cfg, seed, n_scans=n_scans, sensor=sm)
        scans = [torch.from_numpy(s).to(dev) for s in seq["scans"]]
        models = {"lut": rir.Sensor.from_model(sm)}
        if sname == "staggered_r0":
            models["synthetic_intrinsics"] = rir.Sensor.from_model(synthetic_intrinsics(sm))
        res = {}
        for d in distances:
            idx = list(range(n_pairs))
            gts = [np.linalg.inv(seq["poses"][k]) @ seq["poses"][k + d] for k in idx]
            runs = {"multi_scale": rir.make_params(levels=3, iters=[10, 10, 10], delta=cfg["delta"]),
                    "single_scale": rir.make_params(levels=1, iters=[30], delta=cfg["delta"])}
            row = {}
            for mname, model in models.items():
                batch = [(model, scans[k + d], scans[k]) for k in idx]
                for rname, prm in runs.items():
                    if mname != "lut" and rname != "multi_scale":
                        continue
                    t0 = time.perf_counter()
                    T, _ = rir.icp_batch(ctx, prm, batch)
                    torch.cuda.synchronize()
                    row[f"{mname}/{rname}"] = dict(summary(pose_errors(T.cpu().numpy(), gts)),
                                                   batch_ms=round((time.perf_counter() - t0) * 1e3, 2))
            res[str(d)] = row
            if log:
                log(f"{sname} d={d}: " + ", ".join(f"{k} {v['success']:.2f}" for k, v in row.items()))
        out["sweeps"][sname] = res
    return out


#: schedules of equal iteration budget (30 Gauss-Newton iterations in all;
#: iters[0] is the finest level)
SCHEDULES = {"levels_1": (1, (30,)), "levels_3": (3, (10, 10, 10)), "levels_4": (4, (7, 7, 8, 8))}


def perturbation(rng, rot_deg, trans_m):
    """A rigid motion of exactly rot_deg about a uniformly random axis and
    trans_m along a uniformly random direction."""
    import synth
    ax = rng.normal(size=3)
    d = rng.normal(size=3)
    return synth.make_pose(synth.rot_axis_angle(ax, np.deg2rad(rot_deg)), trans_m * d / np.linalg.norm(d))


def misalignment_sweep(rots_deg=(0, 1, 2, 5, 10, 15), trans_m=(0, 0.5, 1, 2, 3), n_pairs=50, seed=1000,
                       shape=(64, 1024), scene="outdoor", log=None):
    """Success rate against the initial misalignment (Sec. 4.1's claim that
    the multi-scale scheme widens what local ICP recovers): consecutive
    scans (k + 1 -> k) of a walking-pace sequence registered from
    T_init = T_gt Exp(perturbation), the perturbation sweeping rotation
    (translation 0) and translation (rotation 0), for 1, 3 and 4 levels at
    the same budget of 30 iterations.  The same perturbations (seeded) are
    used for every schedule.  scene "outdoor": consecutive scans of the
    walking-pace sequence; "room": the room-scene pairs of the single-pair
    workload (ground, four walls, 20 boxes; seeds seed..)."""
    import torch
    import synth
    import paper_2112_02779_amd as rir
    dev = torch.device("cuda:0")
    ctx = rir.Context(0)
    sm = synth.uniform_sensor(*shape)
    model = rir.Sensor.from_model(sm)
    if scene == "outdoor":
        cfg = dict(synth.CONFIGS["odometry128x2048"])
        cfg.update(shapes=[shape], step_max=0.5, yaw_max_deg=1.0)
        seq = synth.gen_sequence(cfg, seed, n_scans=n_pairs + 1, sensor=sm)
        scans = [torch.from_numpy(x).to(dev) for x in seq["scans"]]
        batch = [(model, scans[k + 1], scans[k]) for k in range(n_pairs)]
        gts = [np.linalg.inv(seq["poses"][k]) @ seq["poses"][k + 1] for k in range(n_pairs)]
        what = f"consecutive pairs of a walking-pace sequence {shape[0]}x{shape[1]} (seed {seed})"
    else:
        cfg = synth.CONFIGS["pair64"]
        pairs = [synth.gen_pair(cfg, seed + i, shape=shape, sensor=sm) for i in range(n_pairs)]
        batch = [(model, torch.from_numpy(p.src).to(dev), torch.from_numpy(p.dst).to(dev)) for p in pairs]
        gts = [p.gt for p in pairs]
        what = f"room-scene pairs {shape[0]}x{shape[1]} (seeds {seed}..{seed + n_pairs - 1})"
    out = {"workload": f"{n_pairs} {what}, start T_gt Exp(perturbation) of the given rotation (deg) and "
                       f"translation (m)",
           "success": "within 0.25 deg and 5 cm of the ground truth",
           "schedules": {k: {"levels": v[0], "iters_finest_first": list(v[1])} for k, v in SCHEDULES.items()},
           "rotation": {}, "translation": {}}
    axes = [("rotation", r, 0.0) for r in rots_deg] + [("translation", 0.0, t) for t in trans_m]
    for axis, r, t in axes:
        rng = np.random.default_rng(seed + int(1000 * r) + int(100 * t) + (7 if axis == "translation" else 0))
        init = np.stack([g @ perturbation(rng, r, t) for g in gts])
        T0 = torch.from_numpy(init).to(dev)
        row = {}
        for name, (L, iters) in SCHEDULES.items():
            prm = rir.make_params(levels=L, iters=list(iters), delta=cfg["delta"])
            T, _ = rir.icp_batch(ctx, prm, batch, init_poses=T0)
            torch.cuda.synchronize()
            row[name] = summary(pose_errors(T.cpu().numpy(), gts))
        out[axis][str(r if axis == "rotation" else t)] = row
        if log:
            log(f"{axis} {r if axis == 'rotation' else t}: " +
                ", ".join(f"{k} {v['success']:.2f}" for k, v in row.items()))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=None)
    ap.add_argument("--pairs", type=int, default=50)
    ap.add_argument("--distances", default="1,2,4,8,16")
    ap.add_argument("--misalignment", action="store_true",
                    help="sweep the initial misalignment instead of the frame distance")
    args = ap.parse_args(argv)
    logf = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    if args.misalignment:
        res = {sc: misalignment_sweep(n_pairs=args.pairs, scene=sc, seed=1000 if sc == "outdoor" else 0, log=logf)
               for sc in ("outdoor", "room")}
    else:
        res = run(tuple(int(x) for x in args.distances.split(",")), args.pairs, log=logf)
    text = json.dumps(res, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
    else:
        print(text)


if __name__ == "__main__":
    main()
