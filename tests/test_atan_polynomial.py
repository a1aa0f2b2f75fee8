"""The FP32 arctangent of the projection kernels (rir_device.h, atan2_abs and
azimuth_mod; Eq. (3)'s azimuth) against its stated error bounds, on the CPU.

The coefficients are read from the header itself, so the test follows the
code.  atan(t) = t P(t^2) on [0, 1] with P of degree 6 (a near-minimax fit by
iteratively reweighted least squares): within 2.6e-7 rad in exact
arithmetic (2.53e-7 measured), within 3.3e-7 rad evaluated as the kernels do (Horner with FP32
fused multiply-adds, then one FP32 product), and atan2 built from it by the
reflections atan(1/t) = pi/2 - atan(t), atan2(y, -x) = pi - atan2(y, x) within
7e-7 rad for any (x, y) (the kernels' reciprocal adds at most 1 ulp to t;
here t is formed exactly and rounded once)."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2112_02779_amd", "csrc", "rir_device.h")


def _coefficients(fn):
    text = open(HEADER).read()
    body = text[text.index(fn):]
    body = body[:body.index("\n}\n")]
    first = re.search(r"float p = ([-0-9.e+]+)f;", body).group(1)
    rest = re.findall(r"p = fmaf\(p, t2, ([-0-9.e+]+)f\);", body)
    return np.array([float(first)] + [float(c) for c in rest], dtype=np.float32)


def _fma32(a, b, c):
    """FP32 fused multiply-add: the product of two FP32 values is exact in
    the 64-bit extended type, the sum is rounded there once and then to
    FP32 (exact for the magnitudes involved except in ties, far below the
    bounds tested)."""
    ld = np.longdouble
    return (a.astype(ld) * b.astype(ld) + c.astype(ld)).astype(np.float32)


def _poly32(C, t):
    t = t.astype(np.float32)
    t2 = (t * t).astype(np.float32)
    p = np.full_like(t, C[0])
    for c in C[1:]:
        p = _fma32(p, t2, np.float32(c))
    return (p * t).astype(np.float32)


def test_coefficients_are_shared():
    C = _coefficients("float atan2_abs(float y, float x)")
    assert C.size == 7
    np.testing.assert_array_equal(C, _coefficients("float azimuth_mod(float y, float x)"))


def test_exact_arithmetic_bound():
    C = _coefficients("float atan2_abs(float y, float x)").astype(np.float64)
    t = np.linspace(0.0, 1.0, 2_000_001)
    p = np.zeros_like(t)
    for c in C:
        p = p * t * t + c
    err = np.abs(t * p - np.arctan(t))
    assert err.max() < 2.6e-7, err.max()


def test_fp32_evaluation_bound():
    C = _coefficients("float atan2_abs(float y, float x)")
    # every FP32 value of t in [2^-12, 1] at a stride, plus the small ones
    bits = np.arange(np.float32(2.0 ** -12).view(np.int32), np.float32(1.0).view(np.int32) + 1, 97,
                     dtype=np.int32)
    t = np.concatenate([bits.view(np.float32), np.float32([0.0, 1e-30, 1e-10, 1e-6, 1.0])])
    err = np.abs(_poly32(C, t).astype(np.float64) - np.arctan(t.astype(np.float64)))
    assert err.max() < 3.3e-7, err.max()


def test_atan2_reflections_bound():
    C = _coefficients("float atan2_abs(float y, float x)")
    rng = np.random.default_rng(3)
    n = 400_000
    ang = rng.uniform(-np.pi, np.pi, n)
    rad = np.exp(rng.uniform(np.log(0.5), np.log(120.0), n))
    x = (rad * np.cos(ang)).astype(np.float32)
    y = (rad * np.sin(ang)).astype(np.float32)
    ax, ay = np.abs(x), np.abs(y)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    t = (mn.astype(np.float64) / mx.astype(np.float64)).astype(np.float32)
    p = _poly32(C, t)
    p = np.where(ay > ax, (np.float32(np.pi / 2) - p).astype(np.float32), p)
    p = np.where(x < 0, (np.float32(np.pi) - p).astype(np.float32), p)
    ref = np.arctan2(np.abs(y.astype(np.float64)), x.astype(np.float64))
    err = np.abs(p.astype(np.float64) - ref)
    assert err.max() < 7e-7, err.max()
