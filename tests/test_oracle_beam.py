"""Pins of the Eq. (S3) decorrelation factor of the gridded estimator (oracle/beam.py).

* The printed number: Sec. 4 quotes exp(-pi^2 theta_0^2 dU^2 / 3) = 0.89 for dU^2 = dU_g^2 / 2 with
  dU_g = sqrt(ln 2) / (pi theta_0) (Sec. 3.2), i.e. 2^(-1/6) (tests/golden/paper_constants.json).
* Baselines on grid points close exactly: D = 1 for every valid triangle.
* Many baselines spread uniformly over every cell: the offsets of the three cells of a closed
  triangle are independent and uniform, so D tends to the closed form
  [int exp(-a s^2) p3(s) ds]^2, p3 the density of a sum of three uniforms on [-dU_g/2, dU_g/2]
  (Irwin-Hall), evaluated here by quadrature; a planted mistake (offsets of mirrored cells not
  reversed) breaks the symmetry of the construction below and is caught.
* D decreases with theta_0 and tends to 1 as theta_0 -> 0.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import beam as ob_
from oracle import bins as ob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")
THETA0 = 0.6 * math.radians(24.68)
DU = math.sqrt(math.log(2.0)) / (math.pi * THETA0)


def test_rate_reproduces_printed_factor():
    g = json.load(open(GOLDEN))["decorrelation_at_half_cell"]
    f = math.exp(-ob_.decorrelation_rate(THETA0) * DU * DU / 2.0)
    assert abs(f - g["value"]) <= g["tol"]
    assert f == pytest.approx(2.0 ** (-1.0 / 6.0), rel=1e-12)


def _bins(n=16):
    return ob.make_bins(ob.RING_U, n, 1, np.array([1.0, 2.0, 3.2, 5.0]))


def _grid_points(n, rng, per_cell):
    """per_cell baselines at every grid point with |q| < n/2 of the upper half plane (q_v >= 0)."""
    pts = [(u, v) for u in range(-n // 2 + 1, n // 2) for v in range(0, n // 2)]
    return np.repeat(np.array(pts, dtype=np.float64), per_cell, axis=0)


def test_on_grid_baselines_close_exactly():
    b = _bins()
    uv = _grid_points(b.n, None, 1) * DU
    D = ob_.decorrelation_factor(b, uv, DU, THETA0)
    ok = np.isfinite(D)
    assert ok.sum() >= 5
    assert np.all(D[ok] == 1.0)


def _uniform_closed_form(a, h):
    def p3(s):
        y = (s + 3 * h) / (2 * h)
        if y < 0 or y > 3:
            return 0.0
        f = y * y / 2 if y < 1 else ((-2 * y * y + 6 * y - 3) / 2 if y < 2 else (3 - y) ** 2 / 2)
        return f / (2 * h)
    ex, _ = integrate.quad(lambda s: math.exp(-a * s * s) * p3(s), -3 * h, 3 * h, points=[-h, h], epsabs=1e-13)
    return ex * ex


def test_uniform_offsets_match_closed_form():
    rng = np.random.default_rng(7)
    b = _bins()
    pts = _grid_points(b.n, rng, 8)
    uv = (pts + rng.uniform(-0.5, 0.5, size=pts.shape)) * DU
    # keep the grid point of every baseline (no baseline may cross to v < 0 or to another point)
    uv[:, 1] = np.where(pts[:, 1] == 0, np.abs(uv[:, 1]), uv[:, 1])
    D = ob_.decorrelation_factor(b, uv, DU, THETA0)
    ref = _uniform_closed_form(ob_.decorrelation_rate(THETA0), DU / 2)
    ok = np.isfinite(D)
    assert ok.sum() >= 5
    # each bin averages its closed triangles' 512 triplets: a Monte Carlo spread of about 0.01 for
    # the smallest rings (few triangles), well below that over all bins together
    assert np.all(np.abs(D[ok] - ref) < 0.025), (D[ok], ref)
    assert abs(float(np.mean(D[ok])) - ref) < 0.004
    assert 0.88 < ref < 0.91


def test_reversed_offsets_matter(monkeypatch):
    """Every baseline at the same offset (0.4 dU_g, 0): a triangle's non-closure is the sum of
    +-offsets, reversed for mirrored cells.  Leaving the reversal out makes every triangle's
    non-closure 3 x 0.4 dU_g, which the correct oracle never gives for all triangles at once."""
    b = _bins()
    pts = _grid_points(b.n, None, 1)
    uv = (pts + np.array([0.4, 0.0])) * DU
    a = ob_.decorrelation_rate(THETA0)
    D = ob_.decorrelation_factor(b, uv, DU, THETA0)
    ok = np.isfinite(D)
    allsame = math.exp(-a * (1.2 * DU) ** 2)
    # every triangle mixes reversed and direct cells: the non-closures are +-0.4 or +-1.2 dU_g
    lo, hi = math.exp(-a * (1.2 * DU) ** 2), math.exp(-a * (0.4 * DU) ** 2)
    assert np.all((D[ok] >= lo - 1e-12) & (D[ok] <= hi + 1e-12))
    assert not np.allclose(D[ok], allsame)
    orig = ob_.cell_offsets

    def no_reversal(n, uv_, du):
        out = orig(n, uv_, du)
        return {k: np.abs(v) * np.sign(0.4) for k, v in out.items()}

    monkeypatch.setattr(ob_, "cell_offsets", no_reversal)
    D2 = ob_.decorrelation_factor(b, uv, DU, THETA0)
    assert np.allclose(D2[ok], allsame)


def test_monotone_in_theta0():
    rng = np.random.default_rng(3)
    b = _bins()
    pts = _grid_points(b.n, rng, 2)
    uv = (pts + rng.uniform(-0.45, 0.45, size=pts.shape) * np.array([1.0, 1.0])) * DU
    uv[:, 1] = np.where(pts[:, 1] == 0, np.abs(uv[:, 1]), uv[:, 1])
    Ds = [ob_.decorrelation_factor(b, uv, DU, th) for th in (1e-6 * THETA0, 0.5 * THETA0, THETA0, 2 * THETA0)]
    ok = np.isfinite(Ds[0])
    assert np.allclose(Ds[0][ok], 1.0, atol=1e-10)
    for x, y in zip(Ds, Ds[1:]):
        assert np.all(y[ok] < x[ok])


def test_enumeration_equals_gauss_rule_over_estimator_runs():
    """exp(-a |dU|^2) = E[exp(i sqrt(2a) z . dU)] (2D standard normal z): the decorrelation factor is
    the Gauss-rule sum of the estimator's triangle averages of per-cell phase means (gridded with
    estimator.grid_visibilities, weighted by 1/N_g, estimated with estimator.estimate_mabs).  Two
    independent computations of the same quantity."""
    from oracle import estimator as oe
    n = 16
    b = _bins(n)
    rng = np.random.default_rng(1)
    pts = _grid_points(n, None, 3)
    uv = (pts + rng.uniform(-0.5, 0.5, size=pts.shape)) * DU
    flip = rng.random(len(uv)) < 0.3
    uv[flip] = -uv[flip]
    ref = ob_.decorrelation_factor(b, uv, DU, THETA0)
    t = math.sqrt(2.0 * ob_.decorrelation_rate(THETA0))
    z, w = np.polynomial.hermite_e.hermegauss(12)
    w = w / w.sum()
    d = uv - DU * np.rint(uv / DU)
    D = np.zeros(len(b.triangles))
    for i in range(12):
        for j in range(12):
            vis = np.exp(1j * (d @ np.array([t * z[i], t * z[j]])))[None, :]
            Vg, Ng = oe.grid_visibilities(uv, vis, None, n, DU)
            B, _, _, _ = oe.estimate_mabs(b, Vg, oe.Weights(ng=Ng), norm=float(n * n))
            D += w[i] * w[j] * B[:, 0, 0, 0]
    ok = np.isfinite(ref)
    assert np.array_equal(np.isfinite(D), ok) and ok.sum() >= 5
    assert np.max(np.abs(D[ok] - ref[ok])) < 1e-13
