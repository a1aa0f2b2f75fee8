"""Python access to the FP64 CPU oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this module; the GPU library never does.  It shares no
code with the GPU path.  Functions return numpy arrays; every computation
happens in the single-threaded double-precision C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ORC_OK, ORC_DEGENERATE, ORC_FALLBACK_HUBER, ORC_NONFINITE = 0, 1, 2, 3
MLP_NPARAM = 5185


def build(force: bool = True) -> str:
    """Compile oracle.c: plain C, -O2, no FP contraction, no vector intrinsics."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OrcSensor(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("phi", ctypes.POINTER(ctypes.c_double)),
                ("theta", ctypes.POINTER(ctypes.c_double)), ("r0", ctypes.c_double)]


class OrcParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("iters", ctypes.c_int * 8), ("delta", ctypes.c_double),
                ("edge_rel", ctypes.c_double), ("max_corr_dist", ctypes.c_double),
                ("init_mode", ctypes.c_int), ("weight_mode", ctypes.c_int),
                ("mlp", ctypes.POINTER(ctypes.c_double)), ("r_max", ctypes.c_double),
                ("learned_levels", ctypes.c_int), ("stop_eps", ctypes.c_double),
                ("flip_band_u", ctypes.c_double), ("flip_band_phi", ctypes.c_double),
                ("flip_seed", ctypes.c_uint64), ("normal_window", ctypes.c_int)]


class OrcLevelStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters_run", ctypes.c_int32), ("n_valid", ctypes.c_int32),
                ("n_inlier", ctypes.c_int32), ("n_proj", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("sum_w", ctypes.c_double), ("sum_w_e2", ctypes.c_double), ("robust_cost", ctypes.c_double),
                ("step_rot", ctypes.c_double), ("step_trans", ctypes.c_double),
                ("JtJ", ctypes.c_double * 21), ("Jtr", ctypes.c_double * 6)]

    def to_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("JtJ", "Jtr", "pad")}
        d["JtJ"] = np.array(self.JtJ[:])
        d["Jtr"] = np.array(self.Jtr[:])
        return d


class OrcProj(ctypes.Structure):
    _fields_ = [("valid", ctypes.c_int32), ("u", ctypes.c_int32), ("v", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("r", ctypes.c_double), ("uhat", ctypes.c_double),
                ("phi", ctypes.c_double), ("theta", ctypes.c_double)]


_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U8 = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        S = ctypes.POINTER(OrcSensor)
        P = ctypes.POINTER(OrcParams)
        ST = ctypes.POINTER(OrcLevelStats)
        L.orc_unproject.argtypes = [S, ctypes.c_int, ctypes.c_int, ctypes.c_double, _D]
        L.orc_project.argtypes = [S, ctypes.c_int, _D, ctypes.POINTER(OrcProj)]
        L.orc_unproject_image.argtypes = [S, _F, _D, _U8]
        L.orc_project_points.argtypes = [S, ctypes.c_int, _D, ctypes.c_int64, _I32, _I32, _D, _D, _D, _U8]
        L.orc_normals.argtypes = [S, _F, ctypes.c_double, _D, _U8]
        L.orc_bf16.argtypes = [ctypes.c_double]
        L.orc_bf16.restype = ctypes.c_double
        L.orc_mlp_nparam.restype = ctypes.c_int
        L.orc_mlp_forward.argtypes = [_D, _F, ctypes.c_int64, _D, _D]
        L.orc_mlp_preact.argtypes = [_D, _F, ctypes.c_int64, _D, _D, _D, _D]
        L.orc_mlp_loss_grad.argtypes = [_D, _F, _F, ctypes.c_int64, _D]
        L.orc_mlp_loss_grad.restype = ctypes.c_double
        L.orc_exp_se3.argtypes = [_D, _D]
        L.orc_pose_error.argtypes = [_D, _D, _D, _D]
        L.orc_icp.argtypes = [S, _F, _F, P, _D, _D, ST]
        L.orc_icp.restype = ctypes.c_int
        L.orc_system.argtypes = [S, ctypes.c_int, _F, _F, P, _D, ctypes.c_int, _I32, _I32, _U8, _U8,
                                 _D, _D, _D, _D, _D, _F, ST]
        L.orc_system.restype = ctypes.c_int
        L.orc_associate_with_normals.argtypes = [S, ctypes.c_int, _F, _F, _D, _U8, _D, P, _I32, _I32, _U8,
                                                 _U8, _D, _D, _D, _D, _D]
        L.orc_sdf_points.argtypes = [S, _F, _D, _D, ctypes.c_int64, _D, _D, _U8, _I32, _I32, _D, _D]
        L.orc_sdf_fuse.argtypes = [S, ctypes.c_int, _F, _D, ctypes.c_int64, _D, ctypes.c_double,
                                   ctypes.c_double, _D, _D]
        L.orc_normals_pca.argtypes = [S, _F, ctypes.c_int, ctypes.c_double, _D, _U8, _D]
        L.orc_eigen3.argtypes = [_D, _D, _D]
        L.orc_deskew.argtypes = [S, _F, _D, _D, _I32, _I32, _D, _D, _D]
        L.orc_sdf_extract.argtypes = [_D, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D,
                                      ctypes.c_double, ctypes.c_double, _D, ctypes.c_int64]
        L.orc_sdf_extract.restype = ctypes.c_int64
        L.orc_sdf_mesh.argtypes = [_D, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D,
                                   ctypes.c_double, ctypes.c_double, _D, ctypes.c_int64]
        L.orc_sdf_mesh.restype = ctypes.c_int64
        L.orc_sdf_activate.argtypes = [S, ctypes.c_int, _F, _D, _D, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _I32, ctypes.c_int64]
        L.orc_sdf_activate.restype = ctypes.c_int64
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


class _SensorHolder:
    """Keeps the numpy tables alive while the C struct points at them."""

    def __init__(self, sensor):
        self.phi = np.ascontiguousarray(sensor.phi, dtype=np.float64)
        self.theta = np.ascontiguousarray(sensor.theta, dtype=np.float64)
        self.s = OrcSensor(int(sensor.H), int(sensor.W), _p(self.phi, _D), _p(self.theta, _D), float(sensor.r0))
        self.H, self.W = int(sensor.H), int(sensor.W)


def make_params(levels=3, iters=(10, 10, 10), delta=0.5, edge_rel=0.1, max_corr_dist=0.0, init_mode=0,
                weight_mode=0, mlp=None, r_max=80.0, learned_levels=0, stop_eps=0.0, normal_window=0):
    prm = OrcParams()
    prm.levels = levels
    for i in range(8):
        prm.iters[i] = int(iters[i]) if i < len(iters) else 0
    prm.delta, prm.edge_rel, prm.max_corr_dist = delta, edge_rel, max_corr_dist
    prm.init_mode, prm.weight_mode, prm.r_max = init_mode, weight_mode, r_max
    prm.learned_levels = int(learned_levels)
    prm.stop_eps = float(stop_eps)
    prm.normal_window = int(normal_window)
    holder = None
    if mlp is not None:
        holder = np.ascontiguousarray(mlp, dtype=np.float64)
        assert holder.size == MLP_NPARAM
        prm.mlp = _p(holder, _D)
    prm._keep = holder  # keep alive
    return prm


def unproject(sensor, u: int, v: int, r: float) -> np.ndarray:
    h = _SensorHolder(sensor)
    out = np.zeros(3)
    lib().orc_unproject(ctypes.byref(h.s), int(u), int(v), float(r), _p(out, _D))
    return out


def unproject_image(sensor, rng_img: np.ndarray):
    h = _SensorHolder(sensor)
    r = np.ascontiguousarray(rng_img, dtype=np.float32)
    xyz = np.zeros((h.H, h.W, 3))
    valid = np.zeros((h.H, h.W), np.uint8)
    lib().orc_unproject_image(ctypes.byref(h.s), _p(r, _F), _p(xyz, _D), _p(valid, _U8))
    return xyz, valid.astype(bool)


def project_points(sensor, level: int, xyz: np.ndarray) -> dict:
    h = _SensorHolder(sensor)
    pts = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    n = pts.shape[0]
    u = np.zeros(n, np.int32)
    v = np.zeros(n, np.int32)
    r = np.zeros(n)
    uh = np.zeros(n)
    ph = np.zeros(n)
    valid = np.zeros(n, np.uint8)
    lib().orc_project_points(ctypes.byref(h.s), int(level), _p(pts, _D), n, _p(u, _I32), _p(v, _I32),
                             _p(r, _D), _p(uh, _D), _p(ph, _D), _p(valid, _U8))
    return {"u": u, "v": v, "r": r, "uhat": uh, "phi": ph, "valid": valid.astype(bool)}


def normals(sensor, rng_img: np.ndarray, edge_rel: float = 0.1):
    h = _SensorHolder(sensor)
    r = np.ascontiguousarray(rng_img, dtype=np.float32)
    n = np.zeros((h.H, h.W, 3))
    valid = np.zeros((h.H, h.W), np.uint8)
    lib().orc_normals(ctypes.byref(h.s), _p(r, _F), float(edge_rel), _p(n, _D), _p(valid, _U8))
    return n, valid.astype(bool)


def sdf_points(sensor, rng_img: np.ndarray, pose: np.ndarray, pts: np.ndarray) -> dict:
    """Eq. (8)-(9) for world points pts [n, 3] against one range image taken at
    pose (4x4, world -> sensor): d = Omega(u, v) - r where valid."""
    h = _SensorHolder(sensor)
    r = np.ascontiguousarray(rng_img, dtype=np.float32)
    T = np.ascontiguousarray(pose, dtype=np.float64)
    p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    n = p.shape[0]
    out = {k: np.zeros(n) for k in ("d", "omega", "uhat", "phi")}
    u = np.zeros(n, np.int32)
    v = np.zeros(n, np.int32)
    valid = np.zeros(n, np.uint8)
    lib().orc_sdf_points(ctypes.byref(h.s), _p(r, _F), _p(T, _D), _p(p, _D), n, _p(out["d"], _D),
                         _p(out["omega"], _D), _p(valid, _U8), _p(u, _I32), _p(v, _I32),
                         _p(out["uhat"], _D), _p(out["phi"], _D))
    out.update(u=u, v=v, valid=valid.astype(bool))
    return out


def sdf_fuse(sensor, ranges: np.ndarray, poses: np.ndarray, pts: np.ndarray, trunc: float, r_clip: float,
             sdf: np.ndarray | None = None, weight: np.ndarray | None = None):
    """Eq. (10): running mean of the truncated projective SDF of points pts
    [n, 3] over the scans ranges [F, H, W] with poses [F, 4, 4] (world ->
    sensor), in order, starting from (sdf, weight) (zeros if None).  Returns
    new (sdf, weight) arrays."""
    h = _SensorHolder(sensor)
    r = np.ascontiguousarray(ranges, dtype=np.float32).reshape(-1, h.H, h.W)
    T = np.ascontiguousarray(poses, dtype=np.float64).reshape(-1, 4, 4)
    assert T.shape[0] == r.shape[0]
    p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    n = p.shape[0]
    s = np.zeros(n) if sdf is None else np.array(sdf, dtype=np.float64).reshape(n)
    w = np.zeros(n) if weight is None else np.array(weight, dtype=np.float64).reshape(n)
    lib().orc_sdf_fuse(ctypes.byref(h.s), int(r.shape[0]), _p(r, _F), _p(T, _D), n, _p(p, _D),
                       float(trunc), float(r_clip), _p(s, _D), _p(w, _D))
    return s, w


def sdf_activate(sensor, ranges: np.ndarray, poses: np.ndarray, radius: float, r_clip: float, voxel: float,
                 origin=(0.0, 0.0, 0.0)):
    """Sec. 4.2 block activation (orc_sdf_activate): the distinct 16^3-voxel
    blocks (edge 16 voxel, voxel (0, 0, 0) at `origin`) that the returns of
    the scans ranges [F, H, W] (poses [F, 4, 4], world -> sensor) activate
    within `radius`, sorted, as int [n, 4] rows (bx, by, bz, first activating
    scan)."""
    h = _SensorHolder(sensor)
    r = np.ascontiguousarray(ranges, dtype=np.float32).reshape(-1, h.H, h.W)
    T = np.ascontiguousarray(poses, dtype=np.float64).reshape(-1, 4, 4)
    assert T.shape[0] == r.shape[0]
    o = np.ascontiguousarray(origin, dtype=np.float64)
    args = (ctypes.byref(h.s), int(r.shape[0]), _p(r, _F), _p(T, _D), _p(o, _D), float(radius), float(r_clip),
            16.0 * float(voxel))
    n = lib().orc_sdf_activate(*args, None, 0)
    if n < 0:
        raise MemoryError("oracle allocation failed")
    out = np.zeros((max(n, 1), 4), np.int32)
    lib().orc_sdf_activate(*args, _p(out, _I32), n)
    return out[:n]


def normals_pca(sensor, rng_img: np.ndarray, half: int = 1, edge_rel: float = 0.1):
    """PCA normals in a (2 half + 1)^2 window: (normals [H, W, 3], valid [H, W],
    eigenvalues [H, W, 3] ascending)."""
    assert 1 <= half <= 5
    h = _SensorHolder(sensor)
    r = np.ascontiguousarray(rng_img, dtype=np.float32)
    n = np.zeros((h.H, h.W, 3))
    lam = np.zeros((h.H, h.W, 3))
    valid = np.zeros((h.H, h.W), np.uint8)
    lib().orc_normals_pca(ctypes.byref(h.s), _p(r, _F), int(half), float(edge_rel), _p(n, _D), _p(valid, _U8),
                          _p(lam, _D))
    return n, valid.astype(bool), lam


def eigen3(A: np.ndarray):
    """Ascending eigenvalues and eigenvector columns of a symmetric 3x3."""
    a = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
    lam = np.zeros(3)
    V = np.zeros(9)
    lib().orc_eigen3(_p(a, _D), _p(lam, _D), _p(V, _D))
    return lam, V.reshape(3, 3)


def deskew(sensor, rng_img: np.ndarray, xi) -> dict:
    """Re-projection of a scan under per-column poses Exp(s_u xi), s_u =
    (u + 1/2)/W - 1/2: the output image (nearest range per pixel, 0 = none)
    and per source pixel the target pixel, new range and continuous
    projection coordinates."""
    h = _SensorHolder(sensor)
    r = np.ascontiguousarray(rng_img, dtype=np.float32)
    x = np.ascontiguousarray(xi, dtype=np.float64).reshape(6)
    out = np.zeros((h.H, h.W))
    tu = np.zeros((h.H, h.W), np.int32)
    tv = np.zeros((h.H, h.W), np.int32)
    rr, uh, ph = np.zeros((h.H, h.W)), np.zeros((h.H, h.W)), np.zeros((h.H, h.W))
    lib().orc_deskew(ctypes.byref(h.s), _p(r, _F), _p(x, _D), _p(out, _D), _p(tu, _I32), _p(tv, _I32), _p(rr, _D),
                     _p(uh, _D), _p(ph, _D))
    return {"out": out, "u": tu, "v": tv, "r": rr, "uhat": uh, "phi": ph}


def sdf_extract(origin, voxel: float, sdf: np.ndarray, weight: np.ndarray, min_weight: float = 1.0,
                max_jump: float = np.inf) -> np.ndarray:
    """Zero crossings of an SDF grid sdf/weight [nz, ny, nx] along grid edges:
    points [n, 3] (see orc_sdf_extract)."""
    s = np.ascontiguousarray(sdf, dtype=np.float64)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    nz, ny, nx = s.shape
    o = np.ascontiguousarray(origin, dtype=np.float64)
    n = lib().orc_sdf_extract(_p(o, _D), float(voxel), nx, ny, nz, _p(s, _D), _p(w, _D), float(min_weight),
                              float(max_jump), None, 0)
    pts = np.zeros((max(n, 1), 3))
    lib().orc_sdf_extract(_p(o, _D), float(voxel), nx, ny, nz, _p(s, _D), _p(w, _D), float(min_weight),
                          float(max_jump), _p(pts, _D), n)
    return pts[:n]


def sdf_mesh(origin, voxel: float, sdf: np.ndarray, weight: np.ndarray, min_weight: float = 1.0,
             max_jump: float = np.inf) -> np.ndarray:
    """Level-set triangles of an SDF grid sdf/weight [nz, ny, nx] by the
    tetrahedral split of every cube: triangles [n, 3, 3] (see orc_sdf_mesh)."""
    s = np.ascontiguousarray(sdf, dtype=np.float64)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    nz, ny, nx = s.shape
    o = np.ascontiguousarray(origin, dtype=np.float64)
    args = (_p(o, _D), float(voxel), nx, ny, nz, _p(s, _D), _p(w, _D), float(min_weight), float(max_jump))
    n = lib().orc_sdf_mesh(*args, None, 0)
    t = np.zeros((max(n, 1), 3, 3))
    lib().orc_sdf_mesh(*args, _p(t, _D), n)
    return t[:n]


def bf16(x: float) -> float:
    return lib().orc_bf16(float(x))


def exp_se3(xi) -> np.ndarray:
    x = np.ascontiguousarray(xi, dtype=np.float64)
    T = np.zeros((4, 4))
    lib().orc_exp_se3(_p(x, _D), _p(T, _D))
    return T


def pose_error(T: np.ndarray, Tref: np.ndarray):
    a = np.ascontiguousarray(T, dtype=np.float64)
    b = np.ascontiguousarray(Tref, dtype=np.float64)
    er, et = ctypes.c_double(), ctypes.c_double()
    lib().orc_pose_error(_p(a, _D), _p(b, _D), ctypes.byref(er), ctypes.byref(et))
    return er.value, et.value


def icp(sensor, src: np.ndarray, dst: np.ndarray, params: OrcParams, T_init=None):
    """Run the full multi-scale ICP; returns (pose 4x4, list of per-level stats dicts)."""
    h = _SensorHolder(sensor)
    s = np.ascontiguousarray(src, dtype=np.float32)
    d = np.ascontiguousarray(dst, dtype=np.float32)
    Ti = np.eye(4) if T_init is None else np.ascontiguousarray(T_init, dtype=np.float64)
    To = np.zeros((4, 4))
    stats = (OrcLevelStats * 8)()
    rc = lib().orc_icp(ctypes.byref(h.s), _p(s, _F), _p(d, _F), ctypes.byref(params), _p(Ti, _D), _p(To, _D),
                       stats)
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return To, [stats[i].to_dict() for i in range(params.levels)]


def icp_spread(sensor, src: np.ndarray, dst: np.ndarray, params: OrcParams, T_ref=None, n_draws=3, rel=1e-7,
               seed=0):
    """Conditioning of the registration result itself: the oracle's pose
    error (rad, m) against T_ref (default: its own result on the given
    images) after each of n_draws perturbations of both range images by one
    relative FP32 rounding (range * (1 + rel * N(0, 1)), rounded to FP32).
    A result that moves by more than a tolerance under such a perturbation
    cannot be reproduced to that tolerance by any FP32 implementation."""
    if T_ref is None:
        T_ref, _ = icp(sensor, src, dst, params)
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_draws):
        s = (src * (1 + rel * rng.standard_normal(src.shape))).astype(np.float32)
        d = (dst * (1 + rel * rng.standard_normal(dst.shape))).astype(np.float32)
        T1, _ = icp(sensor, s, d, params)
        out.append(pose_error(T1, T_ref))
    return np.array(out)


def icp_flip_spread(sensor, src: np.ndarray, dst: np.ndarray, params: OrcParams, T_ref=None, n_draws=3,
                    band_u=2e-3, band_phi=1e-3, seed=0):
    """Conditioning of the registration result against the rounding
    decisions the parity bar leaves open: the oracle's pose error (rad, m)
    against T_ref (default: its own result) after each of n_draws runs in
    which every association whose column coordinate lies within band_u
    pixels of a half-integer, or whose elevation lies within band_phi row
    spacings of a level midpoint or a field-of-view edge, takes the other
    admissible candidate on a coin (seeded SplitMix64 draws, per level,
    iteration and pixel).  A pair whose result moves beyond a tolerance under
    these flips cannot be held to that tolerance by an implementation whose
    rounding differs from FP64 inside the band."""
    if T_ref is None:
        T_ref, _ = icp(sensor, src, dst, params)
    saved = (params.flip_band_u, params.flip_band_phi, params.flip_seed)
    out = []
    try:
        for k in range(n_draws):
            params.flip_band_u, params.flip_band_phi = float(band_u), float(band_phi)
            params.flip_seed = (int(seed) * 1000003 + k + 1) & 0xFFFFFFFFFFFFFFFF
            T1, _ = icp(sensor, src, dst, params)
            out.append(pose_error(T1, T_ref))
    finally:
        params.flip_band_u, params.flip_band_phi, params.flip_seed = saved
    return np.array(out)


def system(sensor, level: int, src, dst, params: OrcParams, T, use_learned=False, with_features=False) -> dict:
    """Per-pixel association terms and the normal equations at a fixed pose."""
    h = _SensorHolder(sensor)
    s = np.ascontiguousarray(src, dtype=np.float32)
    d = np.ascontiguousarray(dst, dtype=np.float32)
    Tm = np.ascontiguousarray(T, dtype=np.float64)
    st = 1 << level
    Hl, Wl = h.H // st, h.W // st
    n = Hl * Wl
    out = {"u": np.zeros(n, np.int32), "v": np.zeros(n, np.int32), "mask": np.zeros(n, np.uint8),
           "proj_valid": np.zeros(n, np.uint8), "e": np.zeros(n), "w": np.zeros(n), "J": np.zeros((n, 6)),
           "uhat": np.zeros(n), "phi": np.zeros(n)}
    feat = np.zeros((n, 14), np.float32) if with_features else None
    ls = OrcLevelStats()
    rc = lib().orc_system(ctypes.byref(h.s), int(level), _p(s, _F), _p(d, _F), ctypes.byref(params), _p(Tm, _D),
                          int(bool(use_learned)), _p(out["u"], _I32), _p(out["v"], _I32), _p(out["mask"], _U8),
                          _p(out["proj_valid"], _U8), _p(out["e"], _D), _p(out["w"], _D), _p(out["J"], _D),
                          _p(out["uhat"], _D), _p(out["phi"], _D), _p(feat, _F) if feat is not None else None,
                          ctypes.byref(ls))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    for k in ("mask", "proj_valid"):
        out[k] = out[k].astype(bool)
    for k in ("u", "v", "mask", "proj_valid", "e", "w", "uhat", "phi"):
        out[k] = out[k].reshape(Hl, Wl)
    out["J"] = out["J"].reshape(Hl, Wl, 6)
    if feat is not None:
        out["feat"] = feat.reshape(Hl, Wl, 14)
    out["stats"] = ls.to_dict()
    return out


def associate_with_normals(sensor, level, src, dst, nrm, nvalid, params, T) -> dict:
    h = _SensorHolder(sensor)
    s = np.ascontiguousarray(src, dtype=np.float32)
    d = np.ascontiguousarray(dst, dtype=np.float32)
    nr = np.ascontiguousarray(nrm, dtype=np.float64)
    nv = np.ascontiguousarray(nvalid, dtype=np.uint8)
    Tm = np.ascontiguousarray(T, dtype=np.float64)
    st = 1 << level
    Hl, Wl = h.H // st, h.W // st
    n = Hl * Wl
    out = {"u": np.zeros(n, np.int32), "v": np.zeros(n, np.int32), "mask": np.zeros(n, np.uint8),
           "proj_valid": np.zeros(n, np.uint8), "e": np.zeros(n), "w": np.zeros(n), "J": np.zeros((n, 6)),
           "uhat": np.zeros(n), "phi": np.zeros(n)}
    lib().orc_associate_with_normals(ctypes.byref(h.s), int(level), _p(s, _F), _p(d, _F), _p(nr, _D), _p(nv, _U8),
                                     _p(Tm, _D), ctypes.byref(params), _p(out["u"], _I32), _p(out["v"], _I32),
                                     _p(out["mask"], _U8), _p(out["proj_valid"], _U8), _p(out["e"], _D),
                                     _p(out["w"], _D), _p(out["J"], _D), _p(out["uhat"], _D), _p(out["phi"], _D))
    out["mask"] = out["mask"].astype(bool)
    out["proj_valid"] = out["proj_valid"].astype(bool)
    return out


def mlp_forward(params: np.ndarray, feats: np.ndarray):
    P = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, 14)
    B = f.shape[0]
    z = np.zeros(B)
    w = np.zeros(B)
    lib().orc_mlp_forward(_p(P, _D), _p(f, _F), B, _p(z, _D), _p(w, _D))
    return z, w


def mlp_preact(params: np.ndarray, feats: np.ndarray) -> dict:
    """Hidden pre-activations a1, a2 [B, 64] of the FP64 forward pass and the
    magnitude sums s1, s2 [B, 64] that bound FP32 rounding of the same sums."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, 14)
    B = f.shape[0]
    out = {k: np.zeros((B, 64)) for k in ("a1", "a2", "s1", "s2")}
    lib().orc_mlp_preact(_p(P, _D), _p(f, _F), B, _p(out["a1"], _D), _p(out["a2"], _D), _p(out["s1"], _D),
                         _p(out["s2"], _D))
    return out


def mlp_loss_grad(params: np.ndarray, feats: np.ndarray, labels: np.ndarray):
    P = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feats, dtype=np.float32).reshape(-1, 14)
    y = np.ascontiguousarray(labels, dtype=np.float32).reshape(-1)
    g = np.zeros(MLP_NPARAM)
    loss = lib().orc_mlp_loss_grad(_p(P, _D), _p(f, _F), _p(y, _F), f.shape[0], _p(g, _D))
    return loss, g
