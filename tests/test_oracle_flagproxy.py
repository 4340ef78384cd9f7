"""Pins of the surrogate's flag-aware inputs (oracle/mlp.py: window_power_weights, windowed_power,
flag_proxy, features_flag, baseline_flag) and the library's host-side bs_var_features_flag.

Flags multiply the cube by w(nu); the delay transform turns that into a circular convolution along
eta, so a Gaussian field of power P is seen with P_w(eta) = sum_q |w~(q)|^2 / nc^2 P(eta - q), and
the Gaussian variance of a triangle average follows the mean over its closed triangles of
P_w P_w P_w.  Pins: brute-force enumeration of closed triangles with P_w evaluated at every vertex,
the unflagged identity P_w = P, Parseval (sum of c_q = mean w^2), shift invariance of the mask, and
the closed form of a one-harmonic window.
"""
import math
import os

import numpy as np
import pytest

from oracle import bins as ob
from oracle import brute as obr
from oracle import mlp as om
from paper_2506_10526_amd import bs

needs_lib = pytest.mark.skipif(not os.path.exists(bs.LIBPATH), reason="libbs.so not built")


def small_case(n=8, nc=8):
    # cubic-like physical constants: k_perp = 2 pi |U| / n, k_par = 2 pi eta / n
    kw = dict(du=1.0, r_mpc=float(n), rprime=1.0, dnu=float(n) / nc)
    edges = 2 * np.pi * np.geomspace(1.0 / n, 4.5 / n, 5)
    b = ob.make_bins(ob.SHELL_K, n, nc, edges, umax=2.0, **kw)
    return b, kw, edges


def test_unflagged_window_is_the_identity():
    b, kw, _ = small_case()
    c = om.window_power_weights(np.ones(8))
    assert c[0] == pytest.approx(1.0, abs=1e-15) and np.all(np.abs(c[1:]) < 1e-30)
    Pw = om.windowed_power(b.n, b.nc, kw["du"], kw["r_mpc"], kw["rprime"], kw["dnu"], None, -2.0)
    k = ob.shell_kmag(b.n, b.nc, **{"du": kw["du"], "r_mpc": kw["r_mpc"], "rprime": kw["rprime"], "dnu": kw["dnu"]})
    with np.errstate(divide="ignore"):
        P = np.where(k > 0, k ** -2.0, 0.0)
    assert np.allclose(Pw, P, rtol=1e-14, atol=0)


def test_parseval_and_shift_invariance():
    rng = np.random.default_rng(1)
    w = (rng.random(24) > 0.3).astype(float) * rng.random(24)
    c = om.window_power_weights(w)
    assert np.sum(c) == pytest.approx(np.mean(w ** 2), rel=1e-13)
    assert np.allclose(om.window_power_weights(np.roll(w, 5)), c, rtol=1e-12, atol=1e-16)


def test_one_harmonic_window_closed_form():
    # w = 1 + alpha cos(2 pi m nu / nc): c_0 = 1, c_{+-m} = alpha^2 / 4, so
    # P_w(eta) = P(eta) + alpha^2 / 4 (P(eta - m) + P(eta + m))
    nc, n, m, alpha = 16, 8, 3, 0.6
    w = 1.0 + alpha * np.cos(2 * np.pi * m * np.arange(nc) / nc)
    c = om.window_power_weights(w)
    ref = np.zeros(nc)
    ref[0], ref[m], ref[nc - m] = 1.0, alpha ** 2 / 4, alpha ** 2 / 4
    assert np.allclose(c, ref, rtol=0, atol=1e-15)
    kw = dict(du=1.0, r_mpc=float(n), rprime=1.0, dnu=float(n) / nc)
    Pw = om.windowed_power(n, nc, kw["du"], kw["r_mpc"], kw["rprime"], kw["dnu"], w, -2.0)
    k = ob.shell_kmag(n, nc, **kw)
    with np.errstate(divide="ignore"):
        P = np.where(k > 0, k ** -2.0, 0.0)
    e = ob.signed_index(nc)
    for i in range(nc):
        im, ip = (i - m) % nc, (i + m) % nc
        assert np.allclose(Pw[i], P[i] + alpha ** 2 / 4 * (P[im] + P[ip]), rtol=1e-13, atol=0), e[i]


@pytest.mark.parametrize("kind", ["periodic", "random", "fractional"])
def test_flag_proxy_matches_brute_force(kind):
    b, kw, edges = small_case()
    rng = np.random.default_rng({"periodic": 2, "random": 3, "fractional": 4}[kind])
    if kind == "periodic":
        w = np.ones(8); w[[0, 4]] = 0.0
    elif kind == "random":
        w = (rng.random(8) > 0.35).astype(float); w[1] = 1.0
    else:
        w = rng.random(8) * 0.8 + 0.2
    G = om.flag_proxy(b, kw["du"], kw["r_mpc"], kw["rprime"], kw["dnu"], w, -2.0)
    Pw = om.windowed_power(b.n, b.nc, kw["du"], kw["r_mpc"], kw["rprime"], kw["dnu"], w, -2.0)
    Pf = obr.full_volume(Pw.astype(np.complex128), b.n).real.ravel()
    lut = obr._lut_full_shell(b)
    checked = 0
    for t, (b1, b2, b3) in enumerate(b.triangles):
        f1, f2, f3 = obr._enumerate(lut, int(b1), int(b2), int(b3))
        if len(f1) == 0:
            assert np.isnan(G[t])
            continue
        ref = np.mean(Pf[f1] * Pf[f2] * Pf[f3])
        assert G[t] == pytest.approx(ref, rel=1e-10), (t, kind)
        checked += 1
    assert checked >= 5


def test_features_and_baseline_hand_worked():
    edges = np.array([1.0, 4.0, 16.0, 64.0])
    tri = np.array([[2, 1, 0], [1, 1, 0], [2, 2, 2]])
    G = np.array([8.0, 2.0, 0.0])
    G1 = np.array([2.0, 2.0, 1.0])
    X = om.features_flag(edges, tri, G, G1, 0.5)
    # log(8 / 2) - 2 log 0.5 = log 4 + log 4 = log 16
    assert np.allclose(X[0], [math.log(32.0), math.log(8.0), math.log(2.0), math.log(16.0)], rtol=0, atol=1e-15)
    assert X[1, 3] == pytest.approx(2 * math.log(2.0), abs=1e-15)
    assert np.isnan(X[2, 3])
    base = om.baseline_flag(np.array([10, 0, 5]), 1000, G, 0.5)
    assert base[0] == pytest.approx(math.log(100.0) + math.log(8.0) + 2 * math.log(2.0), abs=1e-13)
    assert base[1] == -math.inf and base[2] == -math.inf


@needs_lib
def test_library_flag_features_match_oracle():
    b, kw, edges = small_case(16, 16)
    h, ncand = bs.bs_make_bins(None, bs.BS_SHELL_K, 16, 16, edges, umax=2.0, du_lambda=kw["du"], r_mpc=kw["r_mpc"],
                               rprime_mpc_per_mhz=kw["rprime"], dnu_mhz=kw["dnu"])
    try:
        tri, _ = bs.bs_bins_triangles(h, ncand, 4)
        rng = np.random.default_rng(5)
        G = rng.random(ncand) * 10.0 ** rng.integers(-3, 4, ncand)
        G1 = rng.random(ncand) + 0.1
        G[0] = 0.0
        T = rng.integers(1, 10 ** 6, ncand)
        T[1] = 0
        X, base = bs.bs_var_features_flag(h, ncand, T, G, G1, 0.75)
    finally:
        bs.bs_free_bins(h)
    Xr = om.features_flag(edges, tri, G, G1, 0.75)
    assert np.array_equal(np.isnan(X), np.isnan(Xr))
    ok = ~np.isnan(Xr)
    assert np.array_equal(X[ok], Xr[ok].astype(np.float32))
    br = om.baseline_flag(T, 16 * 16 * 16, G, 0.75)
    fin = np.isfinite(br)
    assert np.array_equal(np.isfinite(base), fin)
    assert np.allclose(base[fin], br[fin], rtol=1e-14, atol=1e-12)
