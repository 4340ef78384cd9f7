"""GPU parity of the surrogate's Gaussian flag proxy (bs_var_flag_proxy, C ABI) against the oracle.

The library builds a cube whose delay transform is the window-convolved power P_w (its channel form
a(nu) xi(nu): the window's autocorrelation times the inverse DFT of P along eta, one cosine
transform per |U|^2) and runs the FP64 3D estimator on it; the oracle writes the convolution out
over q and runs its own FFT route.  Both are FP64; agreement to 1e-9 relative.
"""
import numpy as np
import pytest

from oracle import bins as ob
from oracle import mlp as om
from paper_2506_10526_amd import bs, synth

from gpu_common import Ctx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def run(ctx, n, nc, edges, kw, w, pk=-2.0, umax=0.0):
    h, ncand = bs.bs_make_bins(ctx, bs.BS_SHELL_K, n, nc, edges, umax=umax, du_lambda=kw["du"], r_mpc=kw["r_mpc"],
                               rprime_mpc_per_mhz=kw["rprime"], dnu_mhz=kw["dnu"])
    try:
        return bs.bs_var_flag_proxy(ctx, h, ncand, pk, w)
    finally:
        bs.bs_free_bins(h)


@pytest.mark.parametrize("kind", ["none", "periodic", "random", "fractional"])
def test_small_cube_matches_oracle(ctx, kind):
    n, nc = 16, 32
    kw = dict(du=1.0, r_mpc=float(n), rprime=1.0, dnu=float(n) / nc)
    edges = 2 * np.pi * np.geomspace(1.0 / n, 5.0 / n, 7)
    rng = np.random.default_rng(11)
    w = {"none": None, "periodic": synth.mwa_flags(nc, (0, 16, 31)),
         "random": (rng.random(nc) > 0.2).astype(np.float64),
         "fractional": (0.3 + 0.7 * rng.random(nc)).astype(np.float32).astype(np.float64)}[kind]   # the ABI takes float32 weights
    G = run(ctx, n, nc, edges, kw, w)
    b = ob.make_bins(ob.SHELL_K, n, nc, edges, **kw)
    ref = om.flag_proxy(b, kw["du"], kw["r_mpc"], kw["rprime"], kw["dnu"], w, -2.0)
    assert np.array_equal(np.isnan(G), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert ok.sum() >= 10
    assert np.all(G[ok] > 0)
    assert np.allclose(G[ok], ref[ok], rtol=1e-9, atol=0), float(np.max(np.abs(G[ok] / ref[ok] - 1)))


@pytest.mark.parametrize("flags", [(), (0, 16, 31), (0, 1, 2, 16, 29, 30, 31)])
def test_mwa_shaped_cube_matches_oracle(ctx, flags):
    # 48^2 x 768 channels at the MWA constants, the 20 shells of the full cube (eta up to 104, the
    # window harmonics at multiples of 24 fold power from low to high k_par)
    w2 = synth.config2()
    n, nc = 48, w2.nc
    kw = dict(du=w2.du, r_mpc=w2.r_mpc, rprime=w2.rprime, dnu=w2.dnu)
    edges = w2.shell_edges(20)
    w = synth.mwa_flags(nc, flags) if flags else None
    G = run(ctx, n, nc, edges, kw, w)
    b = ob.make_bins(ob.SHELL_K, n, nc, edges, **kw)
    ref = om.flag_proxy(b, kw["du"], kw["r_mpc"], kw["rprime"], kw["dnu"], w, -2.0)
    assert np.array_equal(np.isnan(G), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert ok.sum() >= 50
    assert np.allclose(G[ok], ref[ok], rtol=1e-9, atol=0), float(np.max(np.abs(G[ok] / ref[ok] - 1)))


def test_errors(ctx):
    n, nc = 16, 16
    kw = dict(du=1.0, r_mpc=float(n), rprime=1.0, dnu=1.0)
    edges = 2 * np.pi * np.geomspace(1.0 / n, 5.0 / n, 5)
    with pytest.raises(bs.BsError):
        run(ctx, n, nc, edges, kw, np.zeros(nc))                       # every channel flagged
    with pytest.raises(bs.BsError):
        run(ctx, n, nc, edges, kw, -np.ones(nc))                       # negative weights
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, n, nc, np.geomspace(1, 5, 4))
    try:
        with pytest.raises(bs.BsError):
            bs.bs_var_flag_proxy(ctx, h, ncand, -2.0, None)            # ring bins
    finally:
        bs.bs_free_bins(h)
