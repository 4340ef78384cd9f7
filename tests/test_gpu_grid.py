"""GPU parity of Eq. (vg) gridding (C ABI) against the oracle.

Counts are compared bit for bit: the grid point of a visibility is rint of the same float64
quotient on both sides.  Sums: the GPU adds the visibilities of a cell in another order (float64
atomics), so every cell must lie within 1e-12 (complex128 output) or 1.2e-7 (complex64 output:
the float64 sum rounded once to float32, 2^-24 relative, plus the float64 spread) of the cell's
sum of |Re V| + |Im V|.
"""
import numpy as np
import pytest

from oracle import bins as ob
from oracle import estimator as oe
from paper_2506_10526_amd import bs, synth

from gpu_common import Ctx, compare_B, cuda, host, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def run(ctx, n, du, uv, vis, flags, chan_avg, precision):
    nc = vis.shape[0]
    shp = (nc // chan_avg, n, n // 2 + 1)
    Vg = torch.empty(shp, dtype=torch.complex128 if precision == bs.BS_FP64 else torch.complex64, device="cuda")
    Ng = torch.empty(shp, dtype=torch.int32, device="cuda")
    bs.bs_grid_visibilities(ctx, n, du, cuda(uv), cuda(vis.astype(np.complex64)), Vg, Ng,
                            flags=None if flags is None else cuda(flags), chan_avg=chan_avg, precision=precision)
    return host(Vg), host(Ng)


def check(got, uv, vis, flags, n, du, chan_avg, precision, label):
    Vg, Ng = got
    v64 = vis.astype(np.complex64).astype(np.complex128)
    rV, rN = oe.grid_visibilities(uv, v64, flags, n, du, chan_avg)
    assert np.array_equal(Ng, rN), f"{label}: counts differ in {int((Ng != rN).sum())} cells"
    mag, _ = oe.grid_visibilities(uv, np.abs(v64.real) + np.abs(v64.imag), flags, n, du, chan_avg)
    tol = 1e-12 if precision == bs.BS_FP64 else 1.2e-7
    err = np.abs(Vg.astype(np.complex128) - rV)
    assert np.all(err <= tol * np.abs(mag) + 1e-300), f"{label}: worst {float((err / np.maximum(np.abs(mag), 1e-300)).max()):.3e}"


@pytest.mark.parametrize("n,nc,nvis,avg", [(8, 4, 1, 1), (16, 4, 0, 2), (16, 8, 100, 2), (64, 8, 5000, 4),
                                            (256, 12, 200000, 4), (32, 6, 3000, 3)])
@pytest.mark.parametrize("precision", [bs.BS_FP64, bs.BS_FP32])
@pytest.mark.parametrize("flagged", [False, True])
def test_grid_matches_oracle(ctx, n, nc, nvis, avg, precision, flagged):
    du = synth.DU_G
    rng = np.random.default_rng(n + nc + nvis)
    # baselines over and beyond the grid (the ones beyond are dropped)
    uv = synth.uv_tracks(nvis, n + nvis, 0.3 * du, 0.7 * n * du) if nvis else np.zeros((0, 2))
    vis = (rng.normal(size=(nc, nvis)) + 1j * rng.normal(size=(nc, nvis))).astype(np.complex64)
    chan_w = np.ones(nc)
    chan_w[::5] = 0
    flags = synth.rfi_flags(nc, nvis, 3, 0.05, chan_w) if flagged else None
    print(f"[grid] n={n} nc={nc} nvis={nvis} avg={avg} prec={precision} flagged={flagged}", flush=True)
    got = run(ctx, n, du, uv, vis, flags, avg, precision)
    check(got, uv, vis, flags, n, du, avg, precision, f"n={n} nvis={nvis}")


def test_grid_rejects_bad_arguments(ctx):
    uv = np.zeros((4, 2))
    vis = np.zeros((6, 4), dtype=np.complex64)
    for n, du, avg in ((7, 1.0, 1), (8, 0.0, 1), (8, 1.0, 4)):
        with pytest.raises((RuntimeError, ValueError)):
            run(ctx, n, du, uv, vis, None, avg, bs.BS_FP32)


def test_gridded_cube_feeds_the_mabs_estimator(ctx):
    """Eq. (vg) then Eq. (estimator_t) with the cell-average weights W_g = 1/N_g: the gridded cube and
    counts from the GPU enter bs_estimate_mabs, against the oracle's gridding and estimator."""
    n, nc, du = 32, 8, synth.DU_G
    uv = synth.uv_tracks(4000, 11, 0.8 * du, 11 * du)
    rng = np.random.default_rng(12)
    vis = (rng.normal(size=(nc, 4000)) + 1j * rng.normal(size=(nc, 4000))).astype(np.complex64)
    flags = synth.rfi_flags(nc, 4000, 13, 0.1)
    Vg, Ng = run(ctx, n, du, uv, vis, flags, 1, bs.BS_FP64)
    rV, rN = oe.grid_visibilities(uv, vis.astype(np.complex128), flags, n, du)
    assert np.array_equal(Ng, rN) and Ng.max() < 65536
    b = ob.make_bins(ob.RING_U, n, nc, np.array([1.0, 2.5, 4.0, 6.0, 9.0]))
    w = oe.Weights(ng=rN)
    Bref, Nref, _, _ = oe.estimate_mabs(b, rV, w)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, n, nc, [1.0, 2.5, 4.0, 6.0, 9.0])
    Bd = torch.empty((ncand, nc, nc, nc), dtype=torch.float64, device="cuda")
    Nd = torch.empty((ncand, nc, nc, nc), dtype=torch.int64, device="cuda")
    bs.bs_estimate_mabs(ctx, h, cuda(Vg), bs.BS_FP64, Bd, Nd, ng=cuda(Ng.astype(np.uint16)))
    bs.bs_free_bins(h)
    Nh = host(Nd)
    assert np.array_equal(Nh, Nref)
    ok = Nref > 0
    Bh = host(Bd)
    assert np.all(np.abs(Bh[ok] - Bref[ok]) <= 1e-9 * np.abs(Bref[ok]) + 1e-9 * np.max(np.abs(Bref[ok])))


def test_grid_full_size(ctx):
    """256 x 256 grid, 768 channels of which the periodic flags remove 72, 1 % random RFI flags,
    131,072 baselines, collapsed 4:1 to 192 channels (Sec. 4), complex64 output."""
    n, nc, nvis, du = 256, 768, 131072, synth.DU_G
    uv = synth.uv_tracks(nvis, 21, 0.5 * du, 120 * du)
    g = torch.Generator(device="cuda")
    g.manual_seed(22)
    vd = torch.randn((nc, nvis), dtype=torch.complex64, device="cuda", generator=g)
    flags = synth.rfi_flags(nc, nvis, 23, 0.01, synth.mwa_flags(nc))
    shp = (nc // 4, n, n // 2 + 1)
    Vg = torch.empty(shp, dtype=torch.complex64, device="cuda")
    Ng = torch.empty(shp, dtype=torch.int32, device="cuda")
    print("[grid] full size", flush=True)
    bs.bs_grid_visibilities(ctx, n, du, cuda(uv), vd, Vg, Ng, flags=cuda(flags), chan_avg=4)
    check((host(Vg), host(Ng)), uv, vd.cpu().numpy(), flags, n, du, 4, bs.BS_FP32, "full")
