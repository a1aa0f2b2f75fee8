"""Python binding of librir (include/rir.h): multi-scale projective
point-to-plane ICP on cylindrical LiDAR range images for MI355X (gfx950).

Argument marshalling only: every step of the registration runs in the HIP
kernels of librir.so.  Torch tensors provide device memory and the current
HIP stream.  Importing this module does not need a GPU; creating a sensor,
context or network does, and fails loudly if librir.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librir.so")
_lib = None

RIR_OK, RIR_E_INVALID, RIR_E_SHAPE, RIR_E_LUT, RIR_E_HIP, RIR_E_OOM, RIR_E_UNSUPPORTED = range(7)
LEVEL_OK, LEVEL_DEGENERATE, LEVEL_FALLBACK_HUBER, LEVEL_NONFINITE = range(4)
WEIGHT_HUBER, WEIGHT_LEARNED = 0, 1
PREC_FP32, PREC_FP64 = 0, 1
MAX_LEVELS = 8
MLP_NW, MLP_NB, MLP_NPARAM = 5056, 129, 5185

#: Symbols the C ABI exports (every function declared in include/rir.h).
EXPORTS = [
    "rir_sensor_create", "rir_sensor_destroy", "rir_ctx_create", "rir_ctx_destroy", "rir_ctx_set_tuning",
    "rir_ctx_get_tuning", "rir_ctx_enable_timing", "rir_ctx_level_times", "rir_unproject", "rir_project",
    "rir_normals", "rir_icp_batch", "rir_debug_associate", "rir_autotune", "rir_mlp_create", "rir_mlp_destroy",
    "rir_mlp_get_params", "rir_mlp_set_params", "rir_mlp_forward", "rir_mlp_train_step", "rir_last_error",
    "rir_elevation_table", "rir_sdf_integrate", "rir_normals_pca", "rir_deskew",
    "rir_sdf_extract", "rir_mlp_train_step_noalloc", "rir_bvol_create", "rir_bvol_destroy", "rir_bvol_reset",
    "rir_bvol_integrate", "rir_bvol_size", "rir_bvol_export", "rir_bvol_extract", "rir_sdf_mesh", "rir_bvol_mesh",
]


class RirError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"librir status {status}: {msg}")
        self.status = status


class SensorDesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("phi_lut", ctypes.POINTER(ctypes.c_double)),
                ("theta_lut", ctypes.POINTER(ctypes.c_double)), ("r0", ctypes.c_double),
                ("inv_bins", ctypes.c_int32)]


class IcpParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("iters", ctypes.c_int32 * MAX_LEVELS), ("delta", ctypes.c_double),
                ("edge_rel", ctypes.c_double), ("max_corr_dist", ctypes.c_double), ("init_mode", ctypes.c_int32),
                ("weight_mode", ctypes.c_int32), ("precision", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("mlp", ctypes.c_void_p), ("r_max", ctypes.c_double), ("learned_levels", ctypes.c_int32),
                ("stop_eps", ctypes.c_double), ("normal_window", ctypes.c_int32)]


class Pair(ctypes.Structure):
    _fields_ = [("sensor", ctypes.c_void_p), ("src_range", ctypes.c_void_p), ("dst_range", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("px_per_thread", ctypes.c_int32), ("grid_mult", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("chunk", ctypes.c_int32), ("solve_in_step", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("lane_fine", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LevelStatsC(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters_run", ctypes.c_int32), ("n_valid", ctypes.c_int32),
                ("n_inlier", ctypes.c_int32), ("n_proj", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("sum_w", ctypes.c_double), ("sum_w_e2", ctypes.c_double), ("robust_cost", ctypes.c_double),
                ("step_rot", ctypes.c_double), ("step_trans", ctypes.c_double),
                ("JtJ", ctypes.c_double * 21), ("Jtr", ctypes.c_double * 6)]


#: numpy layout of rir_level_stats (for device arrays copied to the host)
STATS_DTYPE = np.dtype([("status", "<i4"), ("iters_run", "<i4"), ("n_valid", "<i4"), ("n_inlier", "<i4"),
                        ("n_proj", "<i4"), ("pad", "<i4"), ("sum_w", "<f8"), ("sum_w_e2", "<f8"),
                        ("robust_cost", "<f8"), ("step_rot", "<f8"), ("step_trans", "<f8"),
                        ("JtJ", "<f8", (21,)), ("Jtr", "<f8", (6,))])
assert STATS_DTYPE.itemsize == ctypes.sizeof(LevelStatsC) == 280


class VolumeDesc(ctypes.Structure):
    _fields_ = [("nbx", ctypes.c_int32), ("nby", ctypes.c_int32), ("nbz", ctypes.c_int32),
                ("origin", ctypes.c_double * 3), ("voxel", ctypes.c_double)]


def lib():
    """The loaded librir.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -m paper_2112_02779_amd.build); there is no fallback path")
    # torch ships its own HIP runtime under the same soname as the system one;
    # loading torch first makes librir bind to that single runtime (loaded the
    # other way round, torch would find the system runtime and no device)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    pvp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "rir_sensor_create": [ctypes.POINTER(SensorDesc), pvp],
        "rir_sensor_destroy": [vp],
        "rir_ctx_create": [ctypes.c_int, pvp],
        "rir_ctx_destroy": [vp],
        "rir_ctx_set_tuning": [vp, ctypes.POINTER(Tuning)],
        "rir_ctx_get_tuning": [vp, ctypes.POINTER(Tuning)],
        "rir_ctx_enable_timing": [vp, i32],
        "rir_ctx_level_times": [vp, ctypes.POINTER(f32), i32],
        "rir_unproject": [vp, vp, vp, vp, vp],
        "rir_project": [vp, i32, vp, i64, vp, vp, vp, vp, vp],
        "rir_normals": [vp, vp, f64, vp, vp, vp],
        "rir_icp_batch": [vp, ctypes.POINTER(IcpParams), i32, ctypes.POINTER(Pair), vp, vp, vp, vp],
        "rir_debug_associate": [vp, ctypes.POINTER(IcpParams), ctypes.POINTER(Pair), i32,
                                ctypes.POINTER(f64), vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(LevelStatsC), vp],
        "rir_autotune": [vp, ctypes.POINTER(IcpParams), i32, ctypes.POINTER(Pair), vp, vp, ctypes.POINTER(Tuning),
                         ctypes.POINTER(f32), vp],
        "rir_mlp_create": [ctypes.c_int, ctypes.POINTER(ctypes.c_uint16), ctypes.POINTER(f32), pvp],
        "rir_mlp_destroy": [vp],
        "rir_mlp_get_params": [vp, ctypes.POINTER(ctypes.c_uint16), ctypes.POINTER(f32), ctypes.POINTER(f32)],
        "rir_mlp_set_params": [vp, ctypes.POINTER(ctypes.c_uint16), ctypes.POINTER(f32)],
        "rir_mlp_forward": [vp, vp, i64, vp, vp],
        "rir_mlp_train_step": [vp, vp, vp, i64, f32, vp, vp, vp],
        "rir_mlp_train_step_noalloc": [vp, vp, vp, i64, f32, vp, vp, vp],
        "rir_sdf_extract": [ctypes.POINTER(VolumeDesc), vp, f64, f64, vp, i64, vp, vp],
        "rir_deskew": [vp, i32, vp, ctypes.POINTER(f64), vp, vp],
        "rir_normals_pca": [vp, i32, vp, i32, f64, vp, vp, vp],
        "rir_sdf_integrate": [vp, ctypes.POINTER(VolumeDesc), vp, i32, vp, ctypes.POINTER(f64), f64, f64, vp],
        "rir_bvol_create": [ctypes.c_int, ctypes.POINTER(f64), f64, i32, pvp],
        "rir_bvol_destroy": [vp],
        "rir_bvol_reset": [vp, vp],
        "rir_bvol_integrate": [vp, vp, i32, vp, ctypes.POINTER(f64), f64, f64, f64, vp],
        "rir_bvol_size": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "rir_bvol_export": [vp, vp, vp, vp],
        "rir_bvol_extract": [vp, f64, f64, vp, i64, vp, vp],
        "rir_bvol_mesh": [vp, f64, f64, vp, i64, vp, vp],
        "rir_sdf_mesh": [ctypes.POINTER(VolumeDesc), vp, f64, f64, vp, i64, vp, vp],
        "rir_last_error": [],
        "rir_elevation_table": [ctypes.POINTER(SensorDesc), i32, i32, vp, i64, ctypes.POINTER(i64),
                                ctypes.POINTER(f64), ctypes.POINTER(f64)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    L.rir_sensor_destroy.restype = None
    L.rir_ctx_destroy.restype = None
    L.rir_mlp_destroy.restype = None
    L.rir_bvol_destroy.restype = None
    L.rir_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int):
    if status != RIR_OK:
        raise RirError(status, lib().rir_last_error().decode(errors="replace"))


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _require(t, dtype, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


# ----------------------------------------------------------------------------- handles

class Sensor:
    """Device tables of a spinning-LiDAR model (H, W, phi_lut, theta_lut, r0)."""

    def __init__(self, H, W, phi, theta=None, r0=0.0, inv_bins=0):
        self._phi = np.ascontiguousarray(phi, dtype=np.float64)
        self._theta = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
        self.H, self.W, self.r0 = int(H), int(W), float(r0)
        d = SensorDesc(self.H, self.W, self._phi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       None if self._theta is None else self._theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       self.r0, int(inv_bins))
        h = ctypes.c_void_p()
        _check(lib().rir_sensor_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    @classmethod
    def from_model(cls, m, inv_bins=0):
        """From any object with H, W, phi, theta, r0 attributes."""
        return cls(m.H, m.W, m.phi, m.theta, m.r0, inv_bins)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rir_sensor_destroy(self.handle)
            self.handle = None


def elevation_table(m, level: int, fp64: bool = False, inv_bins: int = 0):
    """Host copy of the packed inverse elevation table of pyramid level
    `level` for the sensor model m (H, W, phi, theta, r0): (entries
    [nbins, 4] of float32 or float64, bin_lo, bin_scale).  No device is used."""
    phi = np.ascontiguousarray(m.phi, dtype=np.float64)
    theta = None if m.theta is None else np.ascontiguousarray(m.theta, dtype=np.float64)
    d = SensorDesc(int(m.H), int(m.W), phi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   None if theta is None else theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   float(m.r0), int(inv_bins))
    nb, lo, sc = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    prec = PREC_FP64 if fp64 else PREC_FP32
    _check(lib().rir_elevation_table(ctypes.byref(d), int(level), prec, None, 0, ctypes.byref(nb), ctypes.byref(lo),
                                     ctypes.byref(sc)))
    out = np.zeros((nb.value, 4), dtype=np.float64 if fp64 else np.float32)
    _check(lib().rir_elevation_table(ctypes.byref(d), int(level), prec, out.ctypes.data, out.size, ctypes.byref(nb),
                                     None, None))
    return out, lo.value, sc.value


class Context:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().rir_ctx_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rir_ctx_destroy(self.handle)
            self.handle = None

    def set_tuning(self, block=256, px_per_thread=8, grid_mult=0, xcd_remap=1, chunk=4, solve_in_step=1, lanes=1,
                   lane_fine=0):
        t = Tuning(block, px_per_thread, grid_mult, xcd_remap, chunk, solve_in_step, lanes, lane_fine)
        _check(lib().rir_ctx_set_tuning(self.handle, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().rir_ctx_get_tuning(self.handle, ctypes.byref(t)))
        return t.as_dict()

    def enable_timing(self, on=True, finest_only=False):
        """Event timing of later icp_batch calls: every level and the
        normal/pyramid pass, or only the finest level (less overhead)."""
        _check(lib().rir_ctx_enable_timing(self.handle, 0 if not on else (2 if finest_only else 1)))

    def level_times(self, levels: int):
        """ms per pyramid level (index l) of the last timed call, plus the
        normal/pyramid pass at index `levels`."""
        out = (ctypes.c_float * (levels + 1))()
        _check(lib().rir_ctx_level_times(self.handle, out, levels + 1))
        return list(out)


def make_params(levels=3, iters=(10, 10, 10), delta=0.5, edge_rel=0.1, max_corr_dist=0.0, init_mode=0,
                weight_mode=WEIGHT_HUBER, precision=PREC_FP32, use_graph=True, mlp=None, r_max=80.0,
                learned_levels=0, stop_eps=0.0, normal_window=0) -> IcpParams:
    p = IcpParams()
    p.levels = int(levels)
    for i in range(MAX_LEVELS):
        p.iters[i] = int(iters[i]) if i < len(iters) else 0
    p.delta, p.edge_rel, p.max_corr_dist = float(delta), float(edge_rel), float(max_corr_dist)
    p.init_mode, p.weight_mode, p.precision = int(init_mode), int(weight_mode), int(precision)
    p.use_graph = int(bool(use_graph))
    p.mlp = None if mlp is None else mlp.handle
    p.r_max = float(r_max)
    p.learned_levels = int(learned_levels)
    p.stop_eps = float(stop_eps)
    p.normal_window = int(normal_window)
    p._mlp_ref = mlp
    return p


# ----------------------------------------------------------------------------- geometry

def unproject(sensor: Sensor, rng, stream=None):
    import torch
    _require(rng, torch.float32, "range", sensor.H * sensor.W)
    xyz = torch.empty((sensor.H, sensor.W, 3), dtype=torch.float32, device=rng.device)
    valid = torch.empty((sensor.H, sensor.W), dtype=torch.uint8, device=rng.device)
    _check(lib().rir_unproject(sensor.handle, _ptr(rng), _ptr(xyz), _ptr(valid), _stream(stream)))
    return xyz, valid


def project(sensor: Sensor, level: int, xyz, stream=None):
    import torch
    _require(xyz, torch.float32, "xyz")
    n = xyz.numel() // 3
    dev = xyz.device
    u = torch.empty(n, dtype=torch.int32, device=dev)
    v = torch.empty(n, dtype=torch.int32, device=dev)
    r = torch.empty(n, dtype=torch.float32, device=dev)
    valid = torch.empty(n, dtype=torch.uint8, device=dev)
    _check(lib().rir_project(sensor.handle, int(level), _ptr(xyz), n, _ptr(u), _ptr(v), _ptr(r), _ptr(valid),
                             _stream(stream)))
    return u, v, r, valid


def normals(sensor: Sensor, rng, edge_rel=0.1, stream=None):
    import torch
    _require(rng, torch.float32, "range", sensor.H * sensor.W)
    n = torch.empty((sensor.H, sensor.W, 3), dtype=torch.float32, device=rng.device)
    valid = torch.empty((sensor.H, sensor.W), dtype=torch.uint8, device=rng.device)
    _check(lib().rir_normals(sensor.handle, _ptr(rng), float(edge_rel), _ptr(n), _ptr(valid), _stream(stream)))
    return n, valid


# ----------------------------------------------------------------------------- registration

class Volume:
    """Dense SDF volume of nb = (nbx, nby, nbz) blocks of 16^3 voxels; voxel
    (i, j, k) sits at origin + voxel * (i, j, k) (world, metres)."""

    EDGE = 16

    def __init__(self, nb, origin, voxel: float):
        self.nb = tuple(int(n) for n in nb)
        self.origin = tuple(float(o) for o in origin)
        self.voxel = float(voxel)
        self.desc = VolumeDesc(self.nb[0], self.nb[1], self.nb[2], (ctypes.c_double * 3)(*self.origin),
                               self.voxel)

    @property
    def shape(self):
        """Voxel counts (nx, ny, nz)."""
        return tuple(self.EDGE * n for n in self.nb)

    def alloc(self, device="cuda:0"):
        """An empty volume: (sdf, weight) = 0 for every voxel, stored as
        [nbz, nby, nbx, 16 (z), 16 (y), 16 (x), 2] FP32."""
        import torch
        nbx, nby, nbz = self.nb
        E = self.EDGE
        return torch.zeros((nbz, nby, nbx, E, E, E, 2), dtype=torch.float32, device=device)

    def to_grid(self, voxels):
        """View of the block layout as [nz, ny, nx, 2] (a permuted copy)."""
        nbx, nby, nbz = self.nb
        E = self.EDGE
        return voxels.permute(0, 3, 1, 4, 2, 5, 6).reshape(nbz * E, nby * E, nbx * E, 2)


def sdf_integrate(sensor: Sensor, vol: Volume, voxels, ranges, poses, trunc: float, r_clip: float, stream=None):
    """Fuses scans ranges [F, H, W] (device FP32) taken at poses [F, 4, 4]
    (host FP64, world -> sensor) into voxels (Volume.alloc layout) in place."""
    import torch
    _require(voxels, torch.float32, "voxels", 2 * 4096 * vol.nb[0] * vol.nb[1] * vol.nb[2])
    P = np.ascontiguousarray(poses, dtype=np.float64).reshape(-1, 16)
    F = P.shape[0]
    if F > 0:
        _require(ranges, torch.float32, "ranges", F * sensor.H * sensor.W)
    _check(lib().rir_sdf_integrate(sensor.handle, ctypes.byref(vol.desc), _ptr(voxels), F,
                                   _ptr(ranges) if F > 0 else None,
                                   P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(trunc), float(r_clip),
                                   _stream(stream)))
    return voxels


def normals_pca(sensor: Sensor, rng, half: int = 1, edge_rel=0.1, stream=None):
    """PCA normals of one [H, W] or a batch [n, H, W] of range images."""
    import torch
    _require(rng, torch.float32, "range")
    if rng.numel() % (sensor.H * sensor.W) != 0:
        raise ValueError("range must hold whole H x W images")
    n_img = rng.numel() // (sensor.H * sensor.W)
    shape = tuple(rng.shape)
    n = torch.empty(shape + (3,), dtype=torch.float32, device=rng.device)
    valid = torch.empty(shape, dtype=torch.uint8, device=rng.device)
    _check(lib().rir_normals_pca(sensor.handle, n_img, _ptr(rng), int(half), float(edge_rel), _ptr(n), _ptr(valid),
                                 _stream(stream)))
    return n, valid


def sdf_extract(vol: Volume, voxels, min_weight=1.0, max_jump=float("inf"), max_points=None, stream=None):
    """Zero-crossing surface points of a fused volume: (points [n, 3] FP32
    device tensor, total crossings).  Synchronises the stream to read the
    count; with max_points None a counting pass sizes the result exactly,
    else at most max_points points are stored."""
    import torch
    _require(voxels, torch.float32, "voxels", 2 * 4096 * vol.nb[0] * vol.nb[1] * vol.nb[2])
    s = torch.cuda.current_stream() if stream is None else stream
    cnt = torch.zeros(1, dtype=torch.int64, device=voxels.device)

    def run(pts, cap):
        _check(lib().rir_sdf_extract(ctypes.byref(vol.desc), _ptr(voxels), float(min_weight), float(max_jump),
                                     _ptr(pts), cap, _ptr(cnt), _stream(s)))
        s.synchronize()
        return int(cnt.item())

    cap = run(None, 0) if max_points is None else int(max_points)
    pts = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=voxels.device)
    n = run(pts, cap)
    return pts[:min(n, cap)], n


class BlockVolume:
    """Sparse SDF volume of 16^3-voxel blocks activated around the returns of
    each scan (hash table keyed by block coordinates); voxel (i, j, k) sits at
    origin + voxel * (i, j, k) (world, metres)."""

    EDGE = 16

    def __init__(self, voxel: float, max_blocks: int, origin=(0.0, 0.0, 0.0), device: int = 0):
        h = ctypes.c_void_p()
        o = (ctypes.c_double * 3)(*(float(x) for x in origin))
        _check(lib().rir_bvol_create(int(device), o, float(voxel), int(max_blocks), ctypes.byref(h)))
        self.handle = h
        self.origin = tuple(float(x) for x in origin)
        self.voxel = float(voxel)
        self.max_blocks = int(max_blocks)
        self.device = device

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rir_bvol_destroy(self.handle)
            self.handle = None

    def reset(self, stream=None):
        _check(lib().rir_bvol_reset(self.handle, _stream(stream)))

    def integrate(self, sensor: Sensor, ranges, poses, trunc: float, r_clip: float, radius: float, stream=None):
        """Activates and fuses scans ranges [F, H, W] (device FP32) taken at
        poses [F, 4, 4] (host FP64, world -> sensor)."""
        import torch
        P = np.ascontiguousarray(poses, dtype=np.float64).reshape(-1, 16)
        F = P.shape[0]
        if F > 0:
            _require(ranges, torch.float32, "ranges", F * sensor.H * sensor.W)
        _check(lib().rir_bvol_integrate(self.handle, sensor.handle, F, _ptr(ranges) if F > 0 else None,
                                        P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(trunc),
                                        float(r_clip), float(radius), _stream(stream)))

    def size(self):
        """(active blocks, scans fused)."""
        nb, nf = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().rir_bvol_size(self.handle, ctypes.byref(nb), ctypes.byref(nf)))
        return nb.value, nf.value

    def export(self, stream=None):
        """(blocks int32 [n, 4]: bx, by, bz, first activating scan; voxels
        FP32 [n, 16 (z), 16 (y), 16 (x), 2]) as device tensors, pool order."""
        import torch
        n = self.size()[0]
        dev = torch.device("cuda", self.device)
        blocks = torch.empty((max(n, 1), 4), dtype=torch.int32, device=dev)
        vox = torch.empty((max(n, 1), 16, 16, 16, 2), dtype=torch.float32, device=dev)
        _check(lib().rir_bvol_export(self.handle, _ptr(blocks), _ptr(vox), _stream(stream)))
        return blocks[:n], vox[:n]

    def extract(self, min_weight=1.0, max_jump=float("inf"), max_points=None, stream=None):
        """Zero-crossing surface points: (points [n, 3] FP32 device tensor,
        total crossings), as sdf_extract."""
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        dev = torch.device("cuda", self.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)

        def run(pts, cap):
            _check(lib().rir_bvol_extract(self.handle, float(min_weight), float(max_jump), _ptr(pts), cap,
                                          _ptr(cnt), _stream(s)))
            s.synchronize()
            return int(cnt.item())

        cap = run(None, 0) if max_points is None else int(max_points)
        pts = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
        n = run(pts, cap)
        return pts[:min(n, cap)], n

    def mesh(self, min_weight=1.0, max_jump=float("inf"), max_triangles=None, stream=None):
        """Level-set triangles: (triangles [n, 3, 3] FP32 device tensor, total
        triangles), as sdf_mesh."""
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        dev = torch.device("cuda", self.device)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)

        def run(tri, cap):
            _check(lib().rir_bvol_mesh(self.handle, float(min_weight), float(max_jump), _ptr(tri), cap, _ptr(cnt),
                                       _stream(s)))
            s.synchronize()
            return int(cnt.item())

        cap = run(None, 0) if max_triangles is None else int(max_triangles)
        tri = torch.empty((max(cap, 1), 3, 3), dtype=torch.float32, device=dev)
        n = run(tri, cap)
        return tri[:min(n, cap)], n


def sdf_mesh(vol: Volume, voxels, min_weight=1.0, max_jump=float("inf"), max_triangles=None, stream=None):
    """Level-set triangles of a fused volume (the tetrahedral form of marching
    cubes): (triangles [n, 3, 3] FP32 device tensor, total triangles).
    Synchronises the stream to read the count; with max_triangles None a
    counting pass sizes the result exactly."""
    import torch
    _require(voxels, torch.float32, "voxels", 2 * 4096 * vol.nb[0] * vol.nb[1] * vol.nb[2])
    s = torch.cuda.current_stream() if stream is None else stream
    cnt = torch.zeros(1, dtype=torch.int64, device=voxels.device)

    def run(tri, cap):
        _check(lib().rir_sdf_mesh(ctypes.byref(vol.desc), _ptr(voxels), float(min_weight), float(max_jump),
                                  _ptr(tri), cap, _ptr(cnt), _stream(s)))
        s.synchronize()
        return int(cnt.item())

    cap = run(None, 0) if max_triangles is None else int(max_triangles)
    tri = torch.empty((max(cap, 1), 3, 3), dtype=torch.float32, device=voxels.device)
    n = run(tri, cap)
    return tri[:min(n, cap)], n


def deskew(sensor: Sensor, rng, twists, stream=None):
    """Re-projects one [H, W] or a batch [n, H, W] of scans under per-column
    poses Exp(s_u xi) with one twist xi = (omega, tau) per scan (host [n, 6])."""
    import torch
    _require(rng, torch.float32, "range")
    if rng.numel() % (sensor.H * sensor.W) != 0:
        raise ValueError("range must hold whole H x W images")
    n_img = rng.numel() // (sensor.H * sensor.W)
    tw = np.ascontiguousarray(twists, dtype=np.float64).reshape(-1)
    if tw.size != 6 * n_img:
        raise ValueError(f"need {n_img} twists of 6 values")
    out = torch.empty_like(rng)
    _check(lib().rir_deskew(sensor.handle, n_img, _ptr(rng), tw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            _ptr(out), _stream(stream)))
    return out


def _pairs_array(pairs):
    arr = (Pair * len(pairs))()
    import torch
    for i, (sensor, src, dst) in enumerate(pairs):
        _require(src, torch.float32, f"pairs[{i}].src", sensor.H * sensor.W)
        _require(dst, torch.float32, f"pairs[{i}].dst", sensor.H * sensor.W)
        arr[i].sensor = sensor.handle
        arr[i].src_range = src.data_ptr()
        arr[i].dst_range = dst.data_ptr()
    return arr


def icp_batch(ctx: Context, params: IcpParams, pairs, init_poses=None, poses_out=None, stats_out=None,
              stream=None):
    """Registers pairs [(sensor, src, dst)] (device FP32 images).  init_poses:
    device float64 [n, 4, 4] (identity if None).  Returns (poses [n, 4, 4]
    float64 device tensor, stats uint8 device tensor of n * levels records)."""
    import torch
    n = len(pairs)
    dev = pairs[0][1].device
    if init_poses is None:
        init_poses = torch.eye(4, dtype=torch.float64, device=dev).repeat(n, 1, 1)
    _require(init_poses, torch.float64, "init_poses", 16 * n)
    if poses_out is None:
        poses_out = torch.empty((n, 4, 4), dtype=torch.float64, device=dev)
    _require(poses_out, torch.float64, "poses_out", 16 * n)
    if stats_out is None:
        stats_out = torch.empty(n * params.levels * STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    arr = _pairs_array(pairs)
    _check(lib().rir_icp_batch(ctx.handle, ctypes.byref(params), n, arr, _ptr(init_poses), _ptr(poses_out),
                               _ptr(stats_out), _stream(stream)))
    return poses_out, stats_out


def stats_to_numpy(stats_dev, n_pairs: int, levels: int) -> np.ndarray:
    """[n_pairs, levels] structured array of per-level statistics."""
    raw = stats_dev.cpu().numpy()
    return raw.view(STATS_DTYPE).reshape(n_pairs, levels)


def debug_associate(ctx: Context, params: IcpParams, sensor: Sensor, src, dst, level: int, pose, features=False,
                    stream=None) -> dict:
    """One association pass at a fixed host pose (4x4) without update; returns
    per-pixel device tensors and the reduced statistics (dict)."""
    import torch
    s = 1 << level
    Hl, Wl = sensor.H // s, sensor.W // s
    n = Hl * Wl
    dev = src.device
    out = {"u": torch.empty(n, dtype=torch.int32, device=dev), "v": torch.empty(n, dtype=torch.int32, device=dev),
           "mask": torch.empty(n, dtype=torch.uint8, device=dev), "e": torch.empty(n, dtype=torch.float32, device=dev),
           "w": torch.empty(n, dtype=torch.float32, device=dev),
           "J": torch.empty((n, 6), dtype=torch.float32, device=dev)}
    feat = torch.zeros((n, 14), dtype=torch.float32, device=dev) if features else None
    arr = _pairs_array([(sensor, src, dst)])
    P = np.ascontiguousarray(pose, dtype=np.float64).reshape(16)
    st = LevelStatsC()
    _check(lib().rir_debug_associate(ctx.handle, ctypes.byref(params), arr, int(level),
                                     P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(out["u"]),
                                     _ptr(out["v"]), _ptr(out["mask"]), _ptr(out["e"]), _ptr(out["w"]),
                                     _ptr(out["J"]), _ptr(feat), ctypes.byref(st), _stream(stream)))
    for k in ("u", "v", "mask", "e", "w"):
        out[k] = out[k].view(Hl, Wl)
    out["J"] = out["J"].view(Hl, Wl, 6)
    if feat is not None:
        out["feat"] = feat.view(Hl, Wl, 14)
    d = {k: getattr(st, k) for k, _ in LevelStatsC._fields_ if k not in ("JtJ", "Jtr", "pad")}
    d["JtJ"] = np.array(st.JtJ[:])
    d["Jtr"] = np.array(st.Jtr[:])
    out["stats"] = d
    return out


def autotune(ctx: Context, params: IcpParams, pairs, init_poses=None, stream=None):
    """Times the tuning candidates on this batch and installs the fastest;
    returns (tuning dict, ms per batch)."""
    import torch
    n = len(pairs)
    dev = pairs[0][1].device
    if init_poses is None:
        init_poses = torch.eye(4, dtype=torch.float64, device=dev).repeat(n, 1, 1)
    scratch = torch.empty((n, 4, 4), dtype=torch.float64, device=dev)
    best = Tuning()
    ms = ctypes.c_float()
    _check(lib().rir_autotune(ctx.handle, ctypes.byref(params), n, _pairs_array(pairs), _ptr(init_poses),
                              _ptr(scratch), ctypes.byref(best), ctypes.byref(ms), _stream(stream)))
    return best.as_dict(), ms.value


# ----------------------------------------------------------------------------- learned weight

class Mlp:
    """The 14-64-64-1 per-pixel weight network on the device."""

    def __init__(self, params: np.ndarray | None = None, device: int = 0, seed: int = 0):
        if params is None:
            params = init_mlp_params(seed)
        w, b = split_params(params)
        h = ctypes.c_void_p()
        _check(lib().rir_mlp_create(int(device), w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                    b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rir_mlp_destroy(self.handle)
            self.handle = None

    def get_params(self) -> np.ndarray:
        """Current parameters as float64 in the layout W1, b1, W2, b2, W3, b3."""
        w = np.zeros(MLP_NW, np.uint16)
        b = np.zeros(MLP_NB, np.float32)
        _check(lib().rir_mlp_get_params(self.handle, w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                        b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), None))
        return join_params(w, b)

    def set_params(self, params: np.ndarray):
        w, b = split_params(params)
        _check(lib().rir_mlp_set_params(self.handle, w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                        b.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def forward(self, feats, stream=None):
        import torch
        _require(feats, torch.float32, "feats")
        B = feats.numel() // 14
        w = torch.empty(B, dtype=torch.float32, device=feats.device)
        _check(lib().rir_mlp_forward(self.handle, _ptr(feats), B, _ptr(w), _stream(stream)))
        return w

    def train_step(self, feats, labels, lr, want_grads=False, stream=None):
        import torch
        _require(feats, torch.float32, "feats")
        B = feats.numel() // 14
        _require(labels, torch.float32, "labels", B)
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        grads = torch.empty(MLP_NPARAM, dtype=torch.float32, device=feats.device) if want_grads else None
        _check(lib().rir_mlp_train_step(self.handle, _ptr(feats), _ptr(labels), B, float(lr), _ptr(loss),
                                        _ptr(grads), _stream(stream)))
        return loss, grads


def _bf16_bits(x: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def split_params(params: np.ndarray):
    """Layout W1[64*14], b1[64], W2[64*64], b2[64], W3[64], b3 -> (bf16 bits of
    W1, W2, W3; float32 b1, b2, b3)."""
    P = np.asarray(params, dtype=np.float64).reshape(-1)
    assert P.size == MLP_NPARAM
    w = np.concatenate([P[0:896], P[960:5056], P[5120:5184]])
    b = np.concatenate([P[896:960], P[5056:5120], P[5184:5185]])
    return _bf16_bits(w), np.ascontiguousarray(b, dtype=np.float32)


def join_params(w_bits: np.ndarray, b: np.ndarray) -> np.ndarray:
    w = (w_bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    b = b.astype(np.float64)
    return np.concatenate([w[0:896], b[0:64], w[896:4992], b[64:128], w[4992:5056], b[128:129]])


def init_mlp_params(seed: int = 0) -> np.ndarray:
    """He-initialised weights (bf16-exact), zero hidden biases, output bias 0."""
    rng = np.random.default_rng(seed)
    P = np.zeros(MLP_NPARAM)
    P[0:896] = rng.normal(size=896) * np.sqrt(2.0 / 14)
    P[960:5056] = rng.normal(size=4096) * np.sqrt(2.0 / 64)
    P[5120:5184] = rng.normal(size=64) * np.sqrt(1.0 / 64)
    w, b = split_params(P)
    return join_params(w, b)
