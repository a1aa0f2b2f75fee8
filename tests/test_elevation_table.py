"""The packed inverse elevation table (Sec. 3.2, Eq. (4)) on the host, no GPU:
its lookup, evaluated in the table's own precision exactly as the kernels
evaluate it, gives the nearest row of every elevation.  Pinned two ways:
against a brute-force count of the level's row boundaries (all rounding
cases, including values one ulp around every boundary and every bin edge)
and against the oracle's projection outside the rounding band."""
import numpy as np
import pytest

import oracle
import paper_2112_02779_amd as rir
import synth
from parity_util import ambiguous

SENSORS = {
    "uniform64x1024": lambda: synth.uniform_sensor(64, 1024),
    "uniform128x2048": lambda: synth.uniform_sensor(128, 2048),
    "staggered32x512_r0": lambda: synth.staggered_sensor(32, 512, r0=0.015),
    "staggered16x256": lambda: synth.staggered_sensor(16, 256, r0=0.0),
}


def _lookup(tab, lo, sc, sz, T):
    """The kernels' lookup (elev_row) in precision T: (row, column offset)."""
    sz = np.asarray(sz, dtype=T)
    f = (sz - T(lo)) * T(sc)
    f = np.where(f >= 0, f, T(0))
    bmax = T(tab.shape[0] - 1)
    f = np.where(f < bmax, f, bmax)
    b = f.astype(np.int64)
    E = tab[b]
    rows = E[:, 0].view(np.uint32 if T is np.float32 else np.uint64).astype(np.uint64) & 0xFFFFFFFF
    below = E[:, 1] > sz
    c, ck = (rows & 0xFFFF).astype(np.int64), (rows >> 16).astype(np.int64)
    return np.where(below, ck, c), np.where(below, E[:, 3], E[:, 2])


def _midpoints(m, level):
    s = 1 << level
    p = np.asarray(m.phi, dtype=np.float64)[::s]
    return np.sin(0.5 * (p[:-1] + p[1:]))


def _probe_values(mids_t, lo, hi, T, seed):
    rng = np.random.default_rng(seed)
    vals = [rng.uniform(lo - 0.05, hi + 0.05, 200000).astype(T)]
    for m in mids_t:
        x = T(m)
        vals.append(np.array([x, np.nextafter(x, T(-2)), np.nextafter(x, T(2)),
                              np.nextafter(np.nextafter(x, T(-2)), T(-2)),
                              np.nextafter(np.nextafter(x, T(2)), T(2))], dtype=T))
    vals.append(np.array([lo, hi, -1.0, 1.0, 0.0, -0.0], dtype=T))
    return np.concatenate(vals)


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("level", [0, 1, 2])
@pytest.mark.parametrize("name", list(SENSORS))
def test_lookup_equals_brute_force_count(name, level, fp64):
    m = SENSORS[name]()
    T = np.float64 if fp64 else np.float32
    tab, lo, sc = rir.elevation_table(m, level, fp64=fp64)
    assert tab.dtype == T and tab.shape[0] >= 2 * (m.H >> level)
    mids = _midpoints(m, level).astype(T)
    sz = _probe_values(mids, lo, lo + tab.shape[0] / sc, T, level)
    # bin edges: the values just around each b / sc + lo
    edges = (T(lo) + np.arange(tab.shape[0] + 1, dtype=np.float64) / sc).astype(T)
    sz = np.concatenate([sz, edges, np.nextafter(edges, T(-2)), np.nextafter(edges, T(2))])
    v, uo = _lookup(tab, lo, sc, sz, T)
    # nearest row, ties to the smaller index = number of boundaries strictly above
    want = (mids[None, :] > sz[:, None]).sum(axis=1)
    np.testing.assert_array_equal(v, want)
    s = 1 << level
    theta = np.zeros(m.H) if m.theta is None else np.asarray(m.theta)
    uoff = (theta[::s] * m.W / (2 * np.pi * s)).astype(T)
    np.testing.assert_array_equal(uo, uoff[v])


@pytest.mark.parametrize("level", [0, 2])
@pytest.mark.parametrize("name", list(SENSORS))
def test_lookup_gives_the_oracles_row(name, level):
    """Random points: the table's row (FP32) for the elevation the oracle
    computes is the oracle's nearest row wherever that elevation is outside
    the rounding band."""
    m = SENSORS[name]()
    tab, lo, sc = rir.elevation_table(m, level)
    rng = np.random.default_rng(7 + level)
    d = rng.normal(size=(50000, 3))
    d[:, 2] *= 0.3
    pts = d / np.linalg.norm(d, axis=1, keepdims=True) * rng.uniform(1.0, 80.0, size=(50000, 1))
    ref = oracle.project_points(m, level, pts)
    ok = ref["valid"]
    assert ok.mean() > 0.3
    v, _ = _lookup(tab, lo, sc, np.sin(ref["phi"]).astype(np.float32), np.float32)
    clear = ~ambiguous(m, level, np.full(len(pts), 0.25), ref["phi"]) & ok
    assert clear.sum() > 0.98 * ok.sum()
    np.testing.assert_array_equal(v[clear], ref["v"][clear])


def test_bad_arguments_are_rejected():
    m = synth.uniform_sensor(64, 1024)
    with pytest.raises(rir.RirError):
        rir.elevation_table(m, 11)
    bad = synth.uniform_sensor(64, 1024)
    bad.phi = bad.phi[::-1].copy()
    with pytest.raises(rir.RirError):
        rir.elevation_table(bad, 0)
