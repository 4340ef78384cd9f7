"""Pins of the multipole moments B_l^m(k1, mu, t) (oracle.estimator.triangle_orientation and
bs_multipoles; Eqs. orient and bs_lm).

* The line-of-sight direction in the triangle frame from the formulas of Eq. orient equals the one
  found by building the frame from explicit 3D wave vectors (k_1 along z, k_2 in the x-z plane) and
  projecting the line of sight on it.
* Cell by cell with explicit vectors: every cylindrical cell of ring triples whose k_perp close in
  the plane of the sky is rebuilt as three 3D vectors, its frame and the spherical angles of the
  line of sight found by explicit projections, Y_l^m(theta, phi) and Y_l^m(theta, -phi) averaged;
  the moments agree with bs_multipoles.
* l = 0 is the monopole.
"""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

from oracle import estimator as oe


def frame_projection(v1, v2, los):
    """Line of sight projected on the frame of sides v1 (largest, along z) and v2 (x-z plane)."""
    ez = v1 / np.linalg.norm(v1)
    u2 = v2 / np.linalg.norm(v2)
    mu = -np.dot(ez, u2)
    ex = (u2 + mu * ez) / math.sqrt(1.0 - mu * mu)
    ey = np.cross(ez, ex)
    return np.dot(los, ex), np.dot(los, ey), np.dot(los, ez)


def test_orientation_matches_explicit_frames():
    rng = np.random.default_rng(7)
    los = np.array([0.0, 0.0, 1.0])
    checked = 0
    for _ in range(2000):
        k1, k2 = rng.normal(size=3), rng.normal(size=3)
        vs = [k1, k2, -(k1 + k2)]
        kperp = np.array([[np.hypot(v[0], v[1]) for v in vs]])
        kpar1, kpar2 = np.array([vs[0][2]]), np.array([vs[1][2]])
        px, py, pz = oe.triangle_orientation(kperp, kpar1, kpar2)
        order = np.argsort([-np.dot(v, v) for v in vs], kind="stable")
        ex, ey, ez = frame_projection(vs[order[0]], vs[order[1]], los)
        mu = -np.dot(vs[order[0]], vs[order[1]]) / (np.linalg.norm(vs[order[0]]) * np.linalg.norm(vs[order[1]]))
        if mu > 1 - 1e-9:
            continue
        assert pz[0] == pytest.approx(ez, abs=1e-12)
        assert px[0] == pytest.approx(ex, abs=1e-9)
        assert py[0] == pytest.approx(abs(ey), abs=1e-7)
        checked += 1
    assert checked > 1900


def closing_kperp(rng, n):
    """n ring triples whose k_perp close in the plane of the sky (|a - b| < c < a + b)."""
    out = []
    while len(out) < n:
        a, b = rng.uniform(0.01, 0.06, 2)
        c = rng.uniform(abs(a - b) + 1e-3, a + b - 1e-3)
        out.append((a, b, c))
    return np.array(out)


@pytest.mark.parametrize("case", ["closing", "collinear"])
def test_moments_match_explicit_vectors(case):
    rng = np.random.default_rng(3)
    if case == "closing":
        nt, nc, lmax = 3, 24, 4
        kperp = closing_kperp(rng, nt)
        kunit = 0.02
        edges = np.geomspace(0.02, 0.4, 5)
    else:
        # k_perp collinear in the sky plane (c = a - b): the cells with kpar_2 = -kpar_1 / 2 have
        # k_2 = k_3 = -k_1 / 2, mu = 1 up to rounding and no defined azimuth
        nt, nc, lmax = 1, 16, 3
        kperp = np.array([[0.25, 0.125, 0.125]])
        kunit = 0.125
        edges = np.array([0.1, 0.3, 0.6, 1.2])
    B = rng.normal(size=(nt, nc, nc)) + 1j * rng.normal(size=(nt, nc, nc))
    mom, cnt = oe.bs_multipoles(B, kperp, kunit, edges, lmax)
    pairs = oe.lm_pairs(lmax)
    sums = np.zeros((len(pairs), len(edges) - 1, 5, 5))
    counts = np.zeros((len(edges) - 1, 5, 5), dtype=np.int64)
    los = np.array([0.0, 0.0, 1.0])
    for t in range(nt):
        a, b, c = kperp[t]
        # k_perp vectors: p1 along x, p2 at the angle that closes p1 + p2 + p3 = 0 with |p3| = c
        cphi = (c * c - a * a - b * b) / (2 * a * b)
        p1 = np.array([a, 0.0])
        p2 = b * np.array([cphi, math.sqrt(max(0.0, 1 - cphi * cphi))])
        for ia in range(nc):
            for ib in range(nc):
                q1 = kunit * (ia if 2 * ia < nc else ia - nc)
                q2 = kunit * (ib if 2 * ib < nc else ib - nc)
                v1 = np.array([p1[0], p1[1], q1])
                v2 = np.array([p2[0], p2[1], q2])
                vs = [v1, v2, -(v1 + v2)]
                norms = np.array([np.linalg.norm(v) for v in vs])
                order = np.argsort(-norms ** 2, kind="stable")
                K1, K2 = norms[order[0]], norms[order[1]]
                j = np.searchsorted(edges, K1, side="right") - 1
                if j < 0 or j >= len(edges) - 1:
                    continue
                mu = -np.dot(vs[order[0]], vs[order[1]]) / (K1 * K2)
                tt = K2 / K1
                ib_mu, ib_t = oe.shape_bin(np.clip(mu, 0.5, 1.0)), oe.shape_bin(np.clip(tt, 0.5, 1.0))
                counts[j, ib_mu, ib_t] += 1
                if mu <= 1 - oe.COLLINEAR_TOL:
                    ex, ey, ez = frame_projection(vs[order[0]], vs[order[1]], los)
                    theta, phi = math.acos(max(-1.0, min(1.0, ez))), math.atan2(ey, ex)
                else:
                    theta, phi = math.acos(max(-1.0, min(1.0, vs[order[0]][2] / K1))), None
                for i, (l, m) in enumerate(pairs):
                    if phi is None:
                        y = 0.0 if m > 0 else float(np.real(sph_harm_y(l, 0, theta, 0.0)))
                    else:   # mean over the two mirror orientations
                        y = 0.5 * float(np.real(np.conj(sph_harm_y(l, m, theta, phi)) + np.conj(sph_harm_y(l, m, theta, -phi))))
                    sums[i, j, ib_mu, ib_t] += math.sqrt(4 * math.pi * (2 * l + 1)) * y * B[t, ia, ib].real
    assert np.array_equal(cnt, counts)
    ok = counts > 0
    if case == "collinear":
        kp = kunit * np.where(2 * np.arange(nc) < nc, np.arange(nc), np.arange(nc) - nc)
        _, mu, _ = oe.triangle_shape(np.broadcast_to(kperp[0], (nc, nc, 3)), kp[:, None], kp[None, :])
        assert np.sum(mu > 1 - oe.COLLINEAR_TOL) >= 6   # the collinear cells are there
    ref = sums[:, ok] / counts[ok]
    assert np.allclose(mom[:, ok], ref, rtol=1e-9, atol=1e-11 * np.abs(B.real).max())
    assert ok.sum() >= 10


def test_l0_is_the_monopole():
    rng = np.random.default_rng(5)
    B = rng.normal(size=(4, 32, 32)) + 1j * rng.normal(size=(4, 32, 32))
    kperp = np.abs(rng.normal(size=(4, 3))) * 0.05 + 0.005
    edges = np.geomspace(0.01, 1.0, 6)
    mom, cnt = oe.bs_multipoles(B, kperp, 0.03, edges, 2)
    mono, mcnt = oe.bs_monopole(B, kperp, 0.03, edges)
    assert np.array_equal(cnt, mcnt)
    ok = mcnt > 0
    assert np.allclose(mom[0][ok], mono[ok], rtol=1e-13, atol=1e-15)
    assert np.all(np.isnan(mom[:, ~ok]))
