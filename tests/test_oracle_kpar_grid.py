"""Pins of the (k_par1, k_par2) binning of the cylindrical 3D BS (oracle.estimator.bs_kpar_grid;
Sec. 5, Fig. 4: a 20 x 20 grid over the k_par plane).

* Brute force: plain loops over the cells with explicit edge comparisons (no searchsorted) give the
  same counts and means on small odd and even nc, edges that cut through cells, edges that fall on
  cells exactly and edges wider than the k_par range.
* A constant B gives that constant in every filled bin; the counts are the outer product of the
  one-axis histograms and add up to the cells inside the edges.
* Hermitian symmetry B(-k_par1, -k_par2) = B*(k_par1, k_par2) with edges symmetric about 0 makes
  the binned means symmetric under (i, j) -> (ne - 1 - i, ne - 1 - j) wherever no cell sits on an
  edge (planted mistakes: the unsigned index a for a', a dropped last closed bin, the imaginary part,
  each fail one of these).
"""
import numpy as np
import pytest

from oracle import estimator as oe


def brute(B, unit, edges):
    nt, nc = B.shape[0], B.shape[1]
    ne = len(edges) - 1

    def bin_of(k):
        for i in range(ne):
            lo, hi = edges[i], edges[i + 1]
            if lo <= k < hi or (i == ne - 1 and k == hi):
                return i
        return -1

    sums = np.zeros((nt, ne, ne))
    cnt = np.zeros((ne, ne), dtype=np.int64)
    for a in range(nc):
        ka = unit * (a if 2 * a < nc else a - nc)
        ia = bin_of(ka)
        if ia < 0:
            continue
        for b in range(nc):
            kb = unit * (b if 2 * b < nc else b - nc)
            jb = bin_of(kb)
            if jb < 0:
                continue
            cnt[ia, jb] += 1
            for t in range(nt):
                sums[t, ia, jb] += B[t, a, b].real
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.where(cnt > 0, sums / np.maximum(cnt, 1), np.nan)
    return mean, cnt


@pytest.mark.parametrize("nc,edges", [
    (7, [-0.31, -0.1, 0.05, 0.2, 0.31]),
    (8, [-0.4, -0.2, 0.0, 0.2, 0.3]),        # edges on cells (unit 0.1): half-open, last closed
    (12, list(np.linspace(-0.6, 0.5, 12))),   # the full range, k = +-0.5 / -0.6 on edges
    (9, [-2.0, -0.05, 0.05, 2.0]),             # wider than the k_par range
])
def test_matches_brute_force(nc, edges):
    rng = np.random.default_rng(nc)
    B = rng.normal(size=(3, nc, nc)) + 1j * rng.normal(size=(3, nc, nc))
    m, c = oe.bs_kpar_grid(B, 0.1, np.array(edges))
    bm, bc = brute(B, 0.1, np.array(edges))
    assert np.array_equal(c, bc)
    assert np.array_equal(np.isnan(m), np.isnan(bm))
    ok = ~np.isnan(bm)
    assert np.allclose(m[ok], bm[ok], rtol=1e-13, atol=1e-15)


def test_constant_and_count_structure():
    nc, unit = 16, 0.0124
    edges = np.linspace(-0.09, 0.09, 7)
    B = np.full((2, nc, nc), 2.5 - 1.0j)
    m, c = oe.bs_kpar_grid(B, unit, edges)
    assert np.all(m[:, c > 0] == 2.5) and np.all(np.isnan(m[:, c == 0]))
    kp = unit * np.where(2 * np.arange(nc) < nc, np.arange(nc), np.arange(nc) - nc)
    h = np.array([np.sum(oe.kpar_bins(kp, edges) == i) for i in range(6)])
    assert np.array_equal(c, np.outer(h, h))
    inside = np.sum((kp >= edges[0]) & (kp <= edges[-1]))
    assert c.sum() == inside * inside


@pytest.mark.parametrize("nc", [10, 11])
def test_hermitian_symmetry(nc):
    rng = np.random.default_rng(3 + nc)
    X = rng.normal(size=(2, nc, nc)) + 1j * rng.normal(size=(2, nc, nc))
    idx = (-np.arange(nc)) % nc
    B = X + np.conj(X[:, idx][:, :, idx])        # B(-a, -b) = conj B(a, b)
    edges = np.array([-0.37, -0.23, -0.11, 0.11, 0.23, 0.37])   # symmetric, no cell on an edge
    m, c = oe.bs_kpar_grid(B, 0.1, edges)
    assert np.array_equal(c, c[::-1, ::-1])
    ok = c > 0
    assert np.allclose(m[:, ok], m[:, ::-1, ::-1][:, ok], rtol=1e-12, atol=1e-14)
