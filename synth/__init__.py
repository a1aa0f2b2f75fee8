"""Seeded synthetic LiDAR inputs: sensors, scenes, poses and ray-cast range images.

This module generates the inputs that both the test oracle and the GPU library
consume.  It simulates scan formation only (a spinning head casting rays into a
scene of planes, boxes and cylinders, then range noise, dropouts, spurious
returns and moving objects) and holds none of the registration method's
arithmetic: no projection, association, normals, pyramid, residuals or
Gauss-Newton.  Rotations are built from unit quaternions and plain yaw
matrices, not from the twist exponential the method uses.

The scene recipes mirror the workloads of the paper's registration
experiments (Sec. 6.1-6.3): spinning sensors with a uniform elevation table
(the "synthetic intrinsics" special case of Sec. 3.2), outdoor-scale scenes,
and a pseudo-Huber kernel size of 0.5 m.  They stand in for the paper's own
range-image dataset and KITTI, which are not available here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raycast.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the ray caster into synth/libsynth.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.synth_raycast.argtypes = [
            ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double, dp,
            ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, dp,
            dp, ctypes.POINTER(ctypes.c_int32)]
        lib.synth_raycast.restype = None
        lib.synth_raycast_posed.argtypes = [
            ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double, dp, ctypes.c_int,
            ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, dp,
            dp, ctypes.POINTER(ctypes.c_int32)]
        lib.synth_raycast_posed.restype = None
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------------------------- sensors

@dataclass
class Sensor:
    """Spinning-LiDAR intrinsics: H beams x W columns, per-beam elevation
    ``phi`` (rad, strictly decreasing, row 0 = top beam), per-beam azimuth
    offset ``theta`` (rad) and receiver radius ``r0`` (m) -- the quantities of
    the paper's Sec. 3.1."""
    H: int
    W: int
    phi: np.ndarray
    theta: np.ndarray
    r0: float = 0.0

    def strided(self, s: int) -> "Sensor":
        """Explicit sensor made of rows 0, s, 2s, ... and W/s columns."""
        return Sensor(self.H // s, self.W // s, self.phi[::s].copy(), self.theta[::s].copy(), self.r0)


def uniform_sensor(H: int, W: int, fov_up_deg: float = 16.6, fov_down_deg: float = -16.6) -> Sensor:
    """Uniform elevation over the field of view, no azimuth offsets, r0 = 0:
    row v sits at fov_up - v (fov_up - fov_down) / (H - 1), both ends included."""
    up, dn = np.deg2rad(fov_up_deg), np.deg2rad(fov_down_deg)
    v = np.arange(H, dtype=np.float64)
    phi = up - v * (up - dn) / (H - 1)
    return Sensor(H, W, phi, np.zeros(H), 0.0)


def staggered_sensor(H: int, W: int, r0: float = 0.015, fov_up_deg: float = 22.5,
                     fov_down_deg: float = -22.5, gamma: float = 1.3, stagger_px: float = 0.5) -> Sensor:
    """A sensor exercising the general model: non-uniform elevation table,
    alternating +-stagger_px azimuth offsets and a receiver offset r0."""
    up, dn = np.deg2rad(fov_up_deg), np.deg2rad(fov_down_deg)
    t = np.arange(H, dtype=np.float64) / (H - 1)
    # monotone, denser towards the horizon in the middle of the table
    s = 0.5 + 0.5 * np.sign(t - 0.5) * np.abs(2 * t - 1) ** gamma
    phi = up - s * (up - dn)
    theta = np.where(np.arange(H) % 2 == 0, -stagger_px, stagger_px) * 2 * np.pi / W
    return Sensor(H, W, phi, theta, r0)


# ----------------------------------------------------------------------------- poses

def quat_to_rot(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def rot_axis_angle(axis: np.ndarray, angle: float) -> np.ndarray:
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    q = np.concatenate([[np.cos(angle / 2)], np.sin(angle / 2) * axis])
    return quat_to_rot(q)


def yaw_matrix(psi: float) -> np.ndarray:
    c, s = np.cos(psi), np.sin(psi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def make_pose(R: np.ndarray, t) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def inv_pose(T: np.ndarray) -> np.ndarray:
    R, t = T[:3, :3], T[:3, 3]
    return make_pose(R.T, -R.T @ t)


def unit_vector(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def random_motion(rng: np.random.Generator, max_rot_deg: float, max_trans: float) -> np.ndarray:
    """Rotation about a uniform axis by U(0, max_rot) and a translation in a
    uniform direction with length U(0, max_trans)."""
    axis = unit_vector(rng)
    ang = np.deg2rad(rng.uniform(0.0, max_rot_deg))
    tdir = unit_vector(rng)
    tlen = rng.uniform(0.0, max_trans)
    return make_pose(rot_axis_angle(axis, ang), tdir * tlen)


# ----------------------------------------------------------------------------- scenes

@dataclass
class Scene:
    planes: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))
    cyls: np.ndarray = field(default_factory=lambda: np.zeros((0, 5)))

    def copy(self) -> "Scene":
        return Scene(self.planes.copy(), self.boxes.copy(), self.cyls.copy())

    @property
    def n_prims(self) -> int:
        return len(self.planes) + len(self.boxes) + len(self.cyls)


def room_scene(rng: np.random.Generator, n_boxes: int = 20, half_extent: float = 25.0,
               box_range: float = 22.0, keep_out: float = 3.0) -> Scene:
    """Ground z = 0, four walls at x, y = +-half_extent and n_boxes axis-aligned
    boxes resting on the ground (footprint 0.5-3 m, height 0.5-3 m) with
    centres uniform in +-box_range outside a keep-out radius."""
    planes = np.array([[0, 0, 1, 0],
                       [1, 0, 0, -half_extent], [1, 0, 0, half_extent],
                       [0, 1, 0, -half_extent], [0, 1, 0, half_extent]], dtype=np.float64)
    boxes = []
    while len(boxes) < n_boxes:
        c = rng.uniform(-box_range, box_range, size=2)
        if np.hypot(*c) < keep_out:
            continue
        sx, sy = rng.uniform(0.5, 3.0, size=2)
        h = rng.uniform(0.5, 3.0)
        boxes.append([c[0] - sx / 2, c[1] - sy / 2, 0.0, c[0] + sx / 2, c[1] + sy / 2, h])
    return Scene(planes, np.array(boxes, dtype=np.float64).reshape(-1, 6), np.zeros((0, 5)))


def outdoor_scene(rng: np.random.Generator, path_xy: np.ndarray, n_objects: int = 200,
                  half_size: float = 150.0, keep_out: float = 3.0) -> Scene:
    """Ground plane plus n_objects objects in a 2*half_size square centred on
    the trajectory: half axis-aligned boxes (sides 0.5-4 m), half vertical
    cylinders (radius 0.2-1.5 m, height 1-6 m), none within keep_out of the path."""
    centre = path_xy.mean(axis=0)
    planes = np.array([[0, 0, 1, 0]], dtype=np.float64)
    boxes, cyls = [], []
    n_box = n_objects // 2
    while len(boxes) + len(cyls) < n_objects:
        c = centre + rng.uniform(-half_size, half_size, size=2)
        if np.min(np.hypot(*(path_xy - c).T)) < keep_out + 4.0:
            continue
        if len(boxes) < n_box:
            sx, sy, sz = rng.uniform(0.5, 4.0, size=3)
            boxes.append([c[0] - sx / 2, c[1] - sy / 2, 0.0, c[0] + sx / 2, c[1] + sy / 2, sz])
        else:
            rad = rng.uniform(0.2, 1.5)
            h = rng.uniform(1.0, 6.0)
            cyls.append([c[0], c[1], rad, 0.0, h])
    return Scene(planes, np.array(boxes).reshape(-1, 6), np.array(cyls).reshape(-1, 5))


def displace_boxes(rng: np.random.Generator, scene: Scene, frac: float, dmin: float, dmax: float,
                   keep_out_xy=None, keep_out: float = 3.0):
    """Move a fraction of the boxes horizontally by U(dmin, dmax) in a uniform
    direction.  Returns the new scene and the indices of the moved boxes."""
    out = scene.copy()
    n = len(scene.boxes)
    k = int(round(frac * n))
    idx = rng.choice(n, size=k, replace=False) if k > 0 else np.zeros(0, dtype=np.int64)
    for i in idx:
        for _ in range(100):
            ang = rng.uniform(0, 2 * np.pi)
            d = rng.uniform(dmin, dmax)
            off = np.array([np.cos(ang), np.sin(ang)]) * d
            b = scene.boxes[i].copy()
            b[[0, 3]] += off[0]
            b[[1, 4]] += off[1]
            c = np.array([(b[0] + b[3]) / 2, (b[1] + b[4]) / 2])
            if keep_out_xy is None or np.min(np.hypot(*(np.atleast_2d(keep_out_xy) - c).T)) >= keep_out:
                out.boxes[i] = b
                break
    return out, idx


# ----------------------------------------------------------------------------- scans

def raycast(sensor: Sensor, scene: Scene, T_world_sensor: np.ndarray):
    """Exact (noise-free) ranges [H, W] float64 (0 = no hit) and hit ids (int32, -1 = none)."""
    lib = _load()
    H, W = sensor.H, sensor.W
    phi = np.ascontiguousarray(sensor.phi, dtype=np.float64)
    th = np.ascontiguousarray(sensor.theta, dtype=np.float64)
    T = np.ascontiguousarray(T_world_sensor, dtype=np.float64)
    pl = np.ascontiguousarray(scene.planes, dtype=np.float64).reshape(-1)
    bx = np.ascontiguousarray(scene.boxes, dtype=np.float64).reshape(-1)
    cy = np.ascontiguousarray(scene.cyls, dtype=np.float64).reshape(-1)
    rng_out = np.zeros((H, W), dtype=np.float64)
    hit = np.zeros((H, W), dtype=np.int32)
    lib.synth_raycast(H, W, _dptr(phi), _dptr(th), float(sensor.r0), _dptr(T),
                      len(scene.planes), _dptr(pl) if pl.size else None,
                      len(scene.boxes), _dptr(bx) if bx.size else None,
                      len(scene.cyls), _dptr(cy) if cy.size else None,
                      _dptr(rng_out), hit.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return rng_out, hit


def raycast_moving(sensor: Sensor, scene: Scene, T_mid: np.ndarray, xi):
    """Exact ranges [H, W] of a sensor that moves during its sweep: column u is
    taken at sweep time s_u = (u + 1/2)/W - 1/2 from the pose T_mid expm(s_u
    [xi]) (xi = (omega, tau) per sweep, the matrix exponential by scipy)."""
    import scipy.linalg
    lib = _load()
    H, W = sensor.H, sensor.W
    w, t = np.asarray(xi[:3], dtype=np.float64), np.asarray(xi[3:], dtype=np.float64)
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    M[:3, 3] = t
    Ts = np.stack([T_mid @ scipy.linalg.expm(((u + 0.5) / W - 0.5) * M) for u in range(W)])
    Ts = np.ascontiguousarray(Ts, dtype=np.float64)
    phi = np.ascontiguousarray(sensor.phi, dtype=np.float64)
    th = np.ascontiguousarray(sensor.theta, dtype=np.float64)
    pl = np.ascontiguousarray(scene.planes, dtype=np.float64).reshape(-1)
    bx = np.ascontiguousarray(scene.boxes, dtype=np.float64).reshape(-1)
    cy = np.ascontiguousarray(scene.cyls, dtype=np.float64).reshape(-1)
    rng_out = np.zeros((H, W), dtype=np.float64)
    hit = np.zeros((H, W), dtype=np.int32)
    lib.synth_raycast_posed(H, W, _dptr(phi), _dptr(th), float(sensor.r0), _dptr(Ts), 1,
                            len(scene.planes), _dptr(pl) if pl.size else None,
                            len(scene.boxes), _dptr(bx) if bx.size else None,
                            len(scene.cyls), _dptr(cy) if cy.size else None,
                            _dptr(rng_out), hit.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return rng_out, hit


@dataclass
class ScanNoise:
    sigma: float = 0.0        # range noise std (m)
    rmin: float = 0.5         # ranges outside [rmin, rmax] read as no return
    rmax: float = 80.0
    dropout: float = 0.0      # fraction of pixels dropped to no return
    spurious: float = 0.0     # fraction of pixels replaced by U(rmin, rmax)


def scan(sensor: Sensor, scene: Scene, T_world_sensor: np.ndarray, noise: ScanNoise,
         rng: np.random.Generator):
    """A float32 range image (metres, 0 = no return) plus truth masks."""
    r, hit = raycast(sensor, scene, T_world_sensor)
    valid = r > 0
    if noise.sigma > 0:
        r = r + rng.normal(0.0, noise.sigma, size=r.shape) * valid
    r = np.where(valid & (r >= noise.rmin) & (r <= noise.rmax), r, 0.0)
    drop = rng.random(r.shape) < noise.dropout if noise.dropout > 0 else np.zeros(r.shape, bool)
    r = np.where(drop, 0.0, r)
    spur = rng.random(r.shape) < noise.spurious if noise.spurious > 0 else np.zeros(r.shape, bool)
    if spur.any():
        r = np.where(spur, rng.uniform(noise.rmin, noise.rmax, size=r.shape), r)
    return {"range": r.astype(np.float32), "hit": hit, "dropout": drop, "spurious": spur}


# ----------------------------------------------------------------------------- workloads

#: The registration workloads (shapes, noise and schedules of the paper's experiments,
#: on synthetic scenes).  ``iters`` lists Gauss-Newton iterations per level, finest first.
CONFIGS = {
    "pair64": dict(shapes=[(64, 1024)], levels=3, iters=[10, 10, 10], delta=0.5,
                   noise=ScanNoise(0.01, 0.5, 80.0, 0.05, 0.0), max_rot_deg=5.0, max_trans=1.0,
                   dynamic=0.0, sensor_height=1.8),
    "odometry128x2048": dict(shapes=[(128, 2048)], levels=4, iters=[10, 10, 10, 10], delta=0.5,
                             noise=ScanNoise(0.02, 0.5, 120.0, 0.08, 0.0), n_scans=100,
                             step_min=0.05, step_max=1.5, yaw_max_deg=3.0, n_objects=200,
                             sensor_height=1.8),
    "batch256mixed": dict(shapes=[(16, 1024), (32, 1024), (64, 1024), (128, 2048)], levels=3,
                          iters=[10, 10, 10], delta=0.5, noise=ScanNoise(0.01, 0.5, 80.0, 0.05, 0.0),
                          max_rot_deg=5.0, max_trans=1.0, dynamic=0.0, n_pairs=256,
                          sensor_height=1.8),
    "dynamic64": dict(shapes=[(64, 1024)], levels=3, iters=[10, 10, 10], delta=0.5,
                      noise=ScanNoise(0.01, 0.5, 80.0, 0.05, 0.10), max_rot_deg=5.0, max_trans=1.0,
                      dynamic=0.2, dyn_min=0.5, dyn_max=3.0, sensor_height=1.8),
    "combined64mixed": dict(shapes=[(16, 1024), (32, 1024), (64, 1024), (128, 2048), (128, 4096)],
                            levels=3, iters=[10, 10, 10], delta=0.5,
                            noise=ScanNoise(0.01, 0.5, 80.0, 0.05, 0.10), max_rot_deg=5.0,
                            max_trans=1.0, dynamic=0.2, dyn_min=0.5, dyn_max=3.0, n_pairs=64,
                            sensor_height=1.8),
}


@dataclass
class Pair:
    sensor: Sensor
    src: np.ndarray            # float32 [H, W] source scan (registered into dst)
    dst: np.ndarray            # float32 [H, W] target scan
    gt: np.ndarray             # 4x4 float64 ground truth T_dst<-src
    seed: int
    src_truth: dict = field(default_factory=dict)
    dst_truth: dict = field(default_factory=dict)


def gen_pair(cfg: dict, seed: int, shape=None, sensor: Sensor | None = None) -> Pair:
    """One scan pair in a room scene: dst is taken at (0, 0, h) with identity
    orientation, src from dst * dT with a random motion dT; the registration
    ground truth T_dst<-src equals dT.  With cfg['dynamic'] > 0, that fraction
    of the boxes moves between the two scans."""
    rng = np.random.default_rng(seed)
    if shape is None:
        shape = cfg["shapes"][int(rng.integers(len(cfg["shapes"])))] if len(cfg["shapes"]) > 1 else cfg["shapes"][0]
    if sensor is None:
        sensor = uniform_sensor(*shape)
    scene = room_scene(rng)
    T_a = make_pose(np.eye(3), [0.0, 0.0, cfg["sensor_height"]])
    dT = random_motion(rng, cfg["max_rot_deg"], cfg["max_trans"])
    T_b = T_a @ dT
    scene_b, moved = scene, np.zeros(0, dtype=np.int64)
    if cfg.get("dynamic", 0.0) > 0:
        scene_b, moved = displace_boxes(rng, scene, cfg["dynamic"], cfg["dyn_min"], cfg["dyn_max"],
                                        keep_out_xy=np.stack([T_a[:2, 3], T_b[:2, 3]]))
    a = scan(sensor, scene, T_a, cfg["noise"], rng)
    b = scan(sensor, scene_b, T_b, cfg["noise"], rng)
    n_pl = len(scene.planes)
    moved_ids = set((n_pl + moved).tolist())
    for s in (a, b):
        s["dynamic"] = np.isin(s["hit"], list(moved_ids)) if moved_ids else np.zeros(s["hit"].shape, bool)
    return Pair(sensor, b["range"], a["range"], dT, seed, src_truth=b, dst_truth=a)


def gen_batch(cfg: dict, seed0: int, n_pairs: int | None = None) -> list:
    n = cfg.get("n_pairs", 1) if n_pairs is None else n_pairs
    return [gen_pair(cfg, seed0 + i) for i in range(n)]


def gen_sequence(cfg: dict, seed: int, n_scans: int | None = None, sensor: Sensor | None = None) -> dict:
    """An odometry sequence: the sensor moves forward U(step_min, step_max) and
    turns by a yaw of U(0, yaw_max) per frame through an outdoor scene.
    Returns the scans and the pairs (k+1 -> k) with their ground truth."""
    rng = np.random.default_rng(seed)
    n = cfg["n_scans"] if n_scans is None else n_scans
    H, W = cfg["shapes"][0]
    if sensor is None:
        sensor = uniform_sensor(H, W)
    poses = []
    T = make_pose(np.eye(3), [0.0, 0.0, cfg["sensor_height"]])
    for k in range(n):
        poses.append(T.copy())
        step = rng.uniform(cfg["step_min"], cfg["step_max"])
        yaw = np.deg2rad(rng.uniform(0.0, cfg["yaw_max_deg"]))
        T = T @ make_pose(yaw_matrix(yaw), [step, 0.0, 0.0])
    path_xy = np.array([p[:2, 3] for p in poses])
    scene = outdoor_scene(rng, path_xy, n_objects=cfg["n_objects"])
    scans = [scan(sensor, scene, P, cfg["noise"], rng)["range"] for P in poses]
    pairs = []
    for k in range(n - 1):
        gt = inv_pose(poses[k]) @ poses[k + 1]
        pairs.append(Pair(sensor, scans[k + 1], scans[k], gt, seed))
    return {"sensor": sensor, "poses": poses, "scans": scans, "pairs": pairs, "scene": scene}
