"""The surrogate's inputs: the library's bs_var_features (host code, no GPU needed) against the
oracle's features / baseline_log_var, and a pin of baseline_log_var on a hand-worked triangle.

The network sees X = (log k1, log k2, log k3, rho) with k_i the geometric centre of each shell
(Mpc^-1) and rho the flag summary, and its output is added to the Gaussian-shaped baseline
log(N_vox / T3D) + n_s sum_i log k_i (the variance of a triangle average of a Gaussian field
scales as P1 P2 P3 N_vox / T3D with P ~ k^n_s).  Every number the network sees is checked here.
"""
import math
import os

import numpy as np
import pytest

from oracle import bins as ob
from oracle import mlp as om
from paper_2506_10526_amd import bs, synth

needs_lib = pytest.mark.skipif(not os.path.exists(bs.LIBPATH), reason="libbs.so not built")


def test_baseline_log_var_hand_worked():
    # shells with edges 1, 4, 16, 64: geometric centres 2, 8, 32; triangle (2, 1, 0) has
    # k = (32, 8, 2), sum log k = log 512; N_vox = 1000, T3D = 10, n_s = -2:
    # log(1000 / 10) - 2 log 512 = 4.605170185988092 - 12.476649250079015
    edges = np.array([1.0, 4.0, 16.0, 64.0])
    tri = np.array([[2, 1, 0], [1, 1, 0], [2, 2, 2]])
    got = om.baseline_log_var(edges, tri, np.array([10, 0, 1]), 1000, -2.0)
    assert got[0] == pytest.approx(4.605170185988092 - 12.476649250079015, rel=0, abs=1e-13)
    assert got[1] == -math.inf                      # no closed triangle: no variance defined
    assert got[2] == pytest.approx(math.log(1000.0) - 6.0 * math.log(32.0), abs=1e-13)
    X = om.features(edges, tri, 0.75)
    assert np.allclose(X[0], [math.log(32.0), math.log(8.0), math.log(2.0), 0.75], rtol=0, atol=1e-15)


@needs_lib
@pytest.mark.parametrize("flagged", [False, True])
def test_library_features_match_oracle(flagged):
    w = synth.config3() if flagged else synth.config2()
    edges = w.shell_edges(20)
    h, ncand = bs.bs_make_bins(None, bs.BS_SHELL_K, w.n, w.nc, edges, du_lambda=w.du, r_mpc=w.r_mpc,
                               rprime_mpc_per_mhz=w.rprime, dnu_mhz=w.dnu)
    try:
        tri, _ = bs.bs_bins_triangles(h, ncand, 20)
        rng = np.random.default_rng(3)
        T = rng.integers(0, 10 ** 11, size=ncand)
        T[rng.random(ncand) < 0.1] = 0
        rho = float(np.mean(w.chan_w()))
        X, base = bs.bs_var_features(h, ncand, T, pk_index=-2.0, rho=rho)
    finally:
        bs.bs_free_bins(h)
    ref_b = ob.make_bins(ob.SHELL_K, w.n, w.nc, edges, du=w.du, r_mpc=w.r_mpc, rprime=w.rprime, dnu=w.dnu)
    assert np.array_equal(tri, ref_b.triangles)
    Xr = om.features(edges, tri, rho)
    assert np.array_equal(X, Xr.astype(np.float32))
    br = om.baseline_log_var(edges, tri, T, w.nc * w.n * w.n, -2.0)
    ok = T > 0
    assert np.all(base[~ok] == -np.inf)
    assert np.allclose(base[ok], br[ok], rtol=1e-14, atol=1e-12)
