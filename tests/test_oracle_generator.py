"""Pins for the oracle's counter-based cube generator (oracle/generator.py).

* Philox4x64-10 against NumPy's independent implementation (numpy.random.Philox, which
  advances the 256-bit counter before producing each block);
* the Box-Muller white noise is standard normal and independent across realizations;
* the Gaussian field has the normalised power spectrum it is defined with;
* the quadratic field's 3D estimator mean matches the exact bispectrum (Eq. mb1 / Eq. bsana
  plus the one-loop term), as for the host generator.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import bins as ob
from oracle import estimator as oe
from oracle import generator as og
from oracle import theory as th


@pytest.mark.parametrize("key,start", [((0, 0), 0), ((123, 456), 7), ((2**64 - 1, 2**63 + 5), 2**40 + 3)])
def test_philox_matches_numpy(key, start):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array([start, 0, 0, 0], dtype=np.uint64))
    raw = bg.random_raw(4 * 64).reshape(64, 4)
    c = np.arange(start + 1, start + 65, dtype=np.uint64)
    z = np.zeros_like(c)
    out = np.stack(og.philox4x64_10((c, z, z, z), key), axis=1)
    assert np.array_equal(out, raw)


def test_uniforms_are_open_interval_24_bit():
    x = np.array([0, 2**64 - 1, 1 << 40, (1 << 40) - 1], dtype=np.uint64)
    u = og.uniforms24(x)
    assert u[0] == 2.0 ** -25 and u[1] == 1 - 2.0 ** -25
    assert u[2] == 1.5 * 2.0 ** -24 and u[3] == u[0]


def test_white_noise_is_standard_normal_and_independent():
    w = og.white_noise(1 << 20, seed=7, realization=0)
    assert abs(w.mean()) < 5 / math.sqrt(w.size)
    assert abs(w.var() - 1.0) < 5 * math.sqrt(2.0 / w.size)
    assert stats.kstest(w, "norm").pvalue > 1e-3
    # the four values of a block are uncorrelated with each other
    q = w.reshape(-1, 4)
    cc = np.corrcoef(q.T)
    assert np.max(np.abs(cc - np.eye(4))) < 5 / math.sqrt(q.shape[0])
    w2 = og.white_noise(1 << 20, seed=7, realization=1)
    assert abs(np.corrcoef(w, w2)[0, 1]) < 5 / math.sqrt(w.size)
    w3 = og.white_noise(1 << 20, seed=8, realization=0)
    assert abs(np.corrcoef(w, w3)[0, 1]) < 5 / math.sqrt(w.size)


def test_physical_wave_vectors():
    """k_par of the first delay mode is 2 pi / (r' B_bw); k_perp of one cell is 2 pi dU_g / r."""
    du, r, rp, dnu = 1.0253902, 711.0 / 0.077, 17.0, 0.04
    k2 = og.k_squared(256, 768, "physical", du=du, r_mpc=r, rprime=rp, dnu=dnu, full=False)
    assert math.isclose(math.sqrt(k2[1, 0, 0]), 2 * math.pi / (17.0 * 30.72), rel_tol=1e-12)
    assert math.isclose(math.sqrt(k2[0, 0, 1]), 2 * math.pi * du / r, rel_tol=1e-12)
    assert math.isclose(math.sqrt(k2[0, 255, 0]), 2 * math.pi * du / r, rel_tol=1e-12)  # q_x = -1
    assert math.sqrt(k2[1, 0, 0]) == pytest.approx(0.01203, abs=5e-6)


def test_field_power_matches_normalised_spectrum():
    n, nc = 16, 8
    P = th.power_spectrum_full(th.kmag_full_cubic(nc, n), -2.0, 0.5)
    acc = np.zeros((nc, n, n))
    R = 300
    for r in range(R):
        V = og.generate_cube(n, nc, "cubic", seed=3, realization=r, f=0.0)
        g = np.fft.irfft2(V, s=(n, n), axes=(1, 2))
        acc += np.abs(np.fft.fftn(g)) ** 2
    est = acc / R / (nc * n * n)
    sel = P > 0
    assert abs((est[sel] / P[sel]).mean() - 1.0) < 0.015
    assert np.all(est[~sel] < 1e-20)


def test_quadratic_field_3d_mean_matches_closed_form():
    n, nc = 16, 8
    edges = 2 * np.pi * np.geomspace(1 / 16, 5.5 / 16, 6)
    b = ob.make_bins(ob.SHELL_K, n, nc, edges, du=1.0, r_mpc=float(n), rprime=1.0, dnu=1.0)
    P = th.power_spectrum_full(th.kmag_full_cubic(nc, n), -2.0, 0.5)
    qb = th.QuadraticBispectrum(P, 0.5)
    E = np.array([th.expected_3d(b, qb, t) for t in b.triangles])
    R = 2500
    acc = np.array([oe.estimate_3d(b, og.generate_cube(n, nc, "cubic", 11, r))[0] for r in range(R)])
    ok = np.isfinite(E)
    m, s = acc.mean(0)[ok], acc.std(0, ddof=1)[ok] / np.sqrt(R)
    z = (m - E[ok]) / s
    assert np.max(np.abs(z)) < 4.0
    assert np.mean(z * z) < 2.0
