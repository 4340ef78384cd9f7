"""The paper's whole route on the GPU, from baselines and visibilities to the monopole, against the
same route in the oracle: Eq. (vg) gridding -> Eq. (estimator_t) MABS with W_g = 1/N_g (FP64) ->
ergodic collapse (non-circular, or circular over the channels) -> Eq. (dft) -> monopole B(k1, mu, t).

Monopole counts depend only on the geometry and must be equal; each mean must lie within 1e-9 of
the bin's mean |Re B| (the FP64 MABS agrees with the oracle to about 1e-12 relative per entry,
and the later stages are FP64 transforms and averages).
"""
import numpy as np
import pytest

from oracle import bins as ob
from oracle import estimator as oe
from paper_2506_10526_amd import bs, synth

from gpu_common import Ctx, cuda, host, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


@pytest.mark.parametrize("circular", [False, True])
def test_baselines_to_monopole(ctx, circular):
    n, nc, nvis, du = 32, 12, 3000, synth.DU_G
    redges = np.array([1.0, 2.5, 4.0, 6.0, 9.0])
    uv = synth.uv_tracks(nvis, 51, 0.8 * du, 12 * du)
    rng = np.random.default_rng(52)
    vis = (rng.normal(size=(nc, nvis)) + 1j * rng.normal(size=(nc, nvis))).astype(np.complex64)
    flags = synth.rfi_flags(nc, nvis, 53, 0.05)
    # oracle route
    rV, rN = oe.grid_visibilities(uv, vis.astype(np.complex128), flags, n, du)
    b = ob.make_bins(ob.RING_U, n, nc, redges)
    B, N, _, _ = oe.estimate_mabs(b, rV, oe.Weights(ng=rN))
    Bbar, Nnu, _ = oe.collapse_mabs(B, N, circular=circular)
    Bc = oe.mabs_dft(Bbar, circular=circular)
    cen = np.sqrt(redges[:-1] * redges[1:]) * 2 * np.pi / n
    kperp = np.array([[cen[i] for i in tri] for tri in b.triangles])
    unit = 2 * np.pi / nc
    edges = np.geomspace(0.2, 8.0, 9)
    rm, rc = oe.bs_monopole(Bc, kperp, unit, edges)
    mag, _ = oe.bs_monopole(np.abs(np.real(Bc)), kperp, unit, edges)
    # GPU route
    shp = (nc, n, n // 2 + 1)
    Vg = torch.empty(shp, dtype=torch.complex128, device="cuda")
    Ng = torch.empty(shp, dtype=torch.int32, device="cuda")
    bs.bs_grid_visibilities(ctx, n, du, cuda(uv), cuda(vis), Vg, Ng, flags=cuda(flags), precision=bs.BS_FP64)
    ng16 = Ng.to(torch.int16)
    assert int(Ng.max().item()) < 32768
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, n, nc, redges)
    size = nc if circular else 2 * nc - 1
    Bd = torch.empty((ncand, size, size), dtype=torch.float64, device="cuda")
    Nd = torch.empty((ncand, size, size), dtype=torch.int64, device="cuda")
    Nn = torch.empty((ncand, size, size), dtype=torch.int32, device="cuda")
    bs.bs_estimate_mabs(ctx, h, Vg, bs.BS_FP64, Bd, Nd, N_nu=Nn, collapse=2 if circular else 1, ng=ng16)
    bs.bs_free_bins(h)
    assert ncand == len(b.triangles)
    assert np.array_equal(host(Nn), Nnu)
    out = torch.empty((ncand, nc, nc), dtype=torch.complex128, device="cuda")
    bs.bs_mabs_dft(ctx, nc, Bd, out, circular=circular)
    mean = torch.empty((8, 5, 5), dtype=torch.float64, device="cuda")
    cnt = torch.empty((8, 5, 5), dtype=torch.int64, device="cuda")
    bs.bs_monopole(ctx, out, kperp, unit, edges, mean, cnt)
    gm, gc = host(mean), host(cnt)
    assert np.array_equal(gc, rc) and gc.sum() > 100
    ok = rc > 0
    err = np.abs(gm[ok] - rm[ok])
    assert np.all(err <= 1e-9 * mag[ok]), f"worst {float((err / mag[ok]).max()):.3e}"
