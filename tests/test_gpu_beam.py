"""GPU parity of the Eq. (S3) decorrelation factor (bs_decorrelation, C ABI) against the oracle's
enumeration over closed grid triangles and baseline triplets (oracle/beam.py).

The library computes D by a Gauss rule in the characteristic-function form and the FP64 MABS of
per-cell phase averages; the oracle writes the definition out.  Agreement to 1e-12 (the rule is
exact to 4e-14 at 12 nodes per axis for offsets within a cell; FP64 estimator sums add 1e-15).
"""
import math

import numpy as np
import pytest

from oracle import beam as obm
from oracle import bins as ob
from paper_2506_10526_amd import bs, synth

from gpu_common import Ctx, cuda, torch

pytestmark = pytest.mark.gpu

THETA0 = 0.6 * math.radians(24.68)
DU = math.sqrt(math.log(2.0)) / (math.pi * THETA0)
EDGES = np.array([1.0, 2.0, 3.2, 5.0])


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def _points(n, per_cell):
    pts = [(u, v) for u in range(-n // 2 + 1, n // 2) for v in range(0, n // 2)]
    return np.repeat(np.array(pts, dtype=np.float64), per_cell, axis=0)


def _run(ctx, n, uv, theta0=THETA0, nodes=12):
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, n, 1, EDGES)
    try:
        return bs.bs_decorrelation(ctx, h, ncand, cuda(np.ascontiguousarray(uv, dtype=np.float64)), DU, theta0, nodes)
    finally:
        bs.bs_free_bins(h)


def _compare(got, ref):
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = np.isfinite(ref)
    assert ok.sum() >= 5
    assert np.max(np.abs(got[ok] - ref[ok])) <= 1e-12, float(np.max(np.abs(got[ok] - ref[ok])))


@pytest.mark.parametrize("case", ["uniform3", "tracks", "theta2"])
def test_decorrelation_matches_oracle(ctx, case):
    n = 16
    rng = np.random.default_rng({"uniform3": 1, "tracks": 2, "theta2": 3}[case])
    if case == "tracks":
        # baselines of a compact-array-like distribution (log-uniform radius), both half planes
        uv = synth.uv_tracks(400, seed=5, umin=0.6 * DU, umax=6.5 * DU)
    else:
        pts = _points(n, 3)
        uv = (pts + rng.uniform(-0.5, 0.5, size=pts.shape)) * DU
        # a few baselines reversed (v < 0): they grid to the mirror point
        flip = rng.random(len(uv)) < 0.3
        uv[flip] = -uv[flip]
    theta0 = 2 * THETA0 if case == "theta2" else THETA0
    nodes = 16 if case == "theta2" else 12
    print(f"[beam] {case}: n_vis={len(uv)} theta0={theta0:.4f} nodes={nodes}", flush=True)
    b = ob.make_bins(ob.RING_U, n, 1, EDGES)
    ref = obm.decorrelation_factor(b, uv, DU, theta0)
    got = _run(ctx, n, uv, theta0, nodes)
    _compare(got, ref)
    assert np.all(got[np.isfinite(got)] < 1.0)


def test_on_grid_baselines_give_one(ctx):
    uv = _points(16, 2) * DU
    got = _run(ctx, 16, uv)
    ok = np.isfinite(got)
    assert ok.sum() >= 5 and np.max(np.abs(got[ok] - 1.0)) <= 1e-13


def test_rejects_bad_arguments(ctx):
    uv = _points(16, 1) * DU
    for kw in ({"nodes": 7}, {"nodes": 40}, {"theta0": -1.0}):
        with pytest.raises(bs.BsError):
            _run(ctx, 16, uv, **kw)
