"""The C ABI library loads, exports every function include/rir.h declares,
and rejects invalid arguments on the host before touching a GPU (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2112_02779_amd as rir

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "rir.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rir_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(rir.LIB_PATH):
        pytest.fail("librir.so is not built (run __graft_entry__.build())")
    return rir.lib()


def test_library_exports_every_declared_symbol(L):
    declared = _declared()
    assert len(declared) >= 20
    assert sorted(rir.EXPORTS) == declared
    for name in declared:
        assert hasattr(L, name), name


def test_struct_sizes_match_header(L):
    assert ctypes.sizeof(rir.LevelStatsC) == 280
    assert rir.STATS_DTYPE.itemsize == 280
    assert ctypes.sizeof(rir.Tuning) == 32
    assert ctypes.sizeof(rir.VolumeDesc) == 48


def test_sensor_validation_errors(L):
    h = ctypes.c_void_p()
    assert L.rir_sensor_create(None, ctypes.byref(h)) == rir.RIR_E_INVALID
    assert b"null" in L.rir_last_error()

    def make(H, W, phi, theta=None, r0=0.0):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
        d = rir.SensorDesc(H, W, phi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           None if th is None else th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), r0, 0)
        return L.rir_sensor_create(ctypes.byref(d), ctypes.byref(h)), (phi, th)

    assert make(1, 64, [0.1])[0] == rir.RIR_E_LUT                       # H < 2
    assert make(4, 2, [0.3, 0.1, 0.0, -0.2])[0] == rir.RIR_E_LUT        # W < 4
    assert make(4, 64, [0.3, 0.1, 0.2, -0.2])[0] == rir.RIR_E_LUT       # not decreasing
    assert make(4, 64, [0.3, 0.1, 0.1, -0.2])[0] == rir.RIR_E_LUT       # repeated entry
    assert make(4, 64, [2.0, 0.1, 0.0, -0.2])[0] == rir.RIR_E_LUT       # |phi| >= pi/2
    assert make(4, 64, [0.3, 0.1, np.nan, -0.2])[0] == rir.RIR_E_LUT    # NaN
    assert make(4, 64, [0.3, 0.1, 0.0, -0.2], [0, 0, 4.0, 0])[0] == rir.RIR_E_LUT  # |theta| >= pi
    assert make(4, 64, [0.3, 0.1, 0.0, -0.2], r0=-1.0)[0] == rir.RIR_E_LUT
    assert b"phi_lut" in L.rir_last_error() or b"r0" in L.rir_last_error()


def test_null_handles_are_rejected(L):
    p = rir.make_params()
    assert L.rir_icp_batch(None, ctypes.byref(p), 1, None, None, None, None, None) == rir.RIR_E_INVALID
    assert L.rir_ctx_create(0, None) == rir.RIR_E_INVALID
    assert L.rir_unproject(None, None, None, None, None) == rir.RIR_E_INVALID
    assert L.rir_project(None, 0, None, 0, None, None, None, None, None) == rir.RIR_E_INVALID
    assert L.rir_normals(None, None, 0.1, None, None, None) == rir.RIR_E_INVALID
    assert L.rir_mlp_create(0, None, None, None) == rir.RIR_E_INVALID
    assert L.rir_mlp_forward(None, None, 0, None, None) == rir.RIR_E_INVALID
    assert L.rir_ctx_level_times(None, None, 0) == rir.RIR_E_INVALID
    assert L.rir_normals_pca(None, 1, None, 1, 0.1, None, None, None) == rir.RIR_E_INVALID
    assert L.rir_deskew(None, 1, None, None, None, None) == rir.RIR_E_INVALID
    assert L.rir_sdf_extract(None, None, 1.0, 1.0, None, 0, None, None) == rir.RIR_E_INVALID
    vol = rir.Volume((1, 1, 1), (0.0, 0.0, 0.0), 0.1)
    assert L.rir_sdf_integrate(None, ctypes.byref(vol.desc), None, 0, None, None, 0.3, 30.0,
                               None) == rir.RIR_E_INVALID


def test_mlp_parameter_packing_round_trips():
    P = rir.init_mlp_params(3)
    w, b = rir.split_params(P)
    np.testing.assert_array_equal(rir.join_params(w, b), P)
    assert w.dtype == np.uint16 and w.size == rir.MLP_NW and b.size == rir.MLP_NB
