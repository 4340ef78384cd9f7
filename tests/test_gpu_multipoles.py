"""GPU parity of the multipole moments B_l^m(k1, mu, t) (bs_multipoles, C ABI) against the oracle.

Counts are compared bit for bit (the monopole's FP64 bin decision).  Moments: the GPU evaluates
P_l^m(p_z) cos(m phi) by a recurrence times Re((p_x + i p_y)^m) and adds the cells of a bin in
another order than the oracle, which takes Y_l^m from scipy; each moment must lie within 1e-11
(2l + 1) of the bin's mean |Re B| (|(2l+1) sqrt((l-m)!/(l+m)!) P_l^m cos(m phi)| <= 2l + 1).
"""
import numpy as np
import pytest

from oracle import estimator as oe
from paper_2506_10526_amd import bs, synth

from gpu_common import Ctx, cuda, host, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def run(ctx, Bcyl_dev, kperp, unit, edges, lmax):
    nk = len(edges) - 1
    nlm = (lmax + 1) * (lmax + 2) // 2
    mom = torch.empty((nlm, nk, 5, 5), dtype=torch.float64, device="cuda")
    cnt = torch.empty((nk, 5, 5), dtype=torch.int64, device="cuda")
    bs.bs_multipoles(ctx, Bcyl_dev, kperp, unit, edges, lmax, mom, cnt)
    return host(mom), host(cnt)


def check(got, Bcyl, kperp, unit, edges, lmax, label):
    gm, gc = got
    rm, rc = oe.bs_multipoles(Bcyl, kperp, unit, edges, lmax)
    assert np.array_equal(gc, rc), f"{label}: counts differ in {int((gc != rc).sum())} bins"
    mag, _ = oe.bs_monopole(np.abs(np.real(Bcyl)), kperp, unit, edges)
    ok = rc > 0
    assert np.all(np.isnan(gm[:, ~ok])), f"{label}: empty bins must be NaN"
    for i, (l, m) in enumerate(oe.lm_pairs(lmax)):
        err = np.abs(gm[i][ok] - rm[i][ok])
        bound = 1e-11 * (2 * l + 1) * mag[ok] + 1e-300
        assert np.all(err <= bound), f"{label} (l, m) = ({l}, {m}): worst {float((err / bound).max()):.3e}"


def random_triangles(rng, nt, scale):
    v1, v2 = rng.normal(size=(nt, 2)) * scale, rng.normal(size=(nt, 2)) * scale
    return np.stack([np.hypot(*v1.T), np.hypot(*v2.T), np.hypot(*(v1 + v2).T)], axis=1)


@pytest.mark.parametrize("nc,nt,lmax", [(1, 2, 4), (3, 5, 2), (12, 7, 4), (48, 5, 3), (96, 3, 4), (301, 2, 1)])
def test_multipoles_match_oracle(ctx, nc, nt, lmax):
    rng = np.random.default_rng(nc * 13 + nt)
    kperp = random_triangles(rng, nt, 0.05)
    unit = 0.02
    B = rng.normal(size=(nt, nc, nc)) + 1j * rng.normal(size=(nt, nc, nc))
    edges = np.geomspace(0.01, 0.3 + unit * nc, 7)
    print(f"[multi] nc={nc} nt={nt} lmax={lmax}", flush=True)
    got = run(ctx, cuda(B), kperp, unit, edges, lmax)
    check(got, B, kperp, unit, edges, lmax, f"nc={nc}")
    assert got[1].sum() > 0


def test_collinear_cells_and_the_monopole(ctx):
    # sky-plane-collinear rings: some cells have collinear sides (no azimuth: m > 0 gets nothing);
    # the (0, 0) moment equals bs_monopole
    kperp = np.array([[0.25, 0.125, 0.125], [0.2, 0.15, 0.1]])
    nc, unit, lmax = 16, 0.125, 4
    rng = np.random.default_rng(9)
    B = rng.normal(size=(2, nc, nc)) + 1j * rng.normal(size=(2, nc, nc))
    edges = np.array([0.1, 0.3, 0.6, 1.2])
    got = run(ctx, cuda(B), kperp, unit, edges, lmax)
    check(got, B, kperp, unit, edges, lmax, "collinear")
    mean = torch.empty((3, 5, 5), dtype=torch.float64, device="cuda")
    cnt = torch.empty((3, 5, 5), dtype=torch.int64, device="cuda")
    bs.bs_monopole(ctx, cuda(B), kperp, unit, edges, mean, cnt)
    ok = host(cnt) > 0
    assert np.array_equal(host(cnt), got[1])
    assert np.allclose(got[0][0][ok], host(mean)[ok], rtol=1e-12, atol=1e-14)


def test_errors(ctx):
    kperp = np.array([[0.1, 0.1, 0.1]])
    B = cuda(np.full((1, 4, 4), 1.0 + 0j))
    with pytest.raises(RuntimeError):
        run(ctx, B, kperp, 0.1, [0.05, 0.2], 5)                                  # lmax > 4
    with pytest.raises(RuntimeError):
        run(ctx, B, kperp, 0.1, list(np.geomspace(0.05, 1.0, 20)), 4)            # 25 x 19 x 15 > 6400
    with pytest.raises(RuntimeError):
        run(ctx, B, kperp, -0.1, [0.05, 0.2], 2)                                 # kpar unit <= 0


def test_multipoles_full_size_sample(ctx):
    """Eight of the 133 ring triples of the 256^2 x 768 cube at full nc = 768 (ring k_perp at the
    geometric centres of the ring edges), seeded cylindrical BS, 12 log k1 bins, lmax = 4."""
    w = synth.config2()
    redges = w.shell_edges(20)
    h, ncand = bs.bs_make_bins(0, bs.BS_RING_U, w.n, w.nc, redges / (2 * np.pi * w.du / w.r_mpc))
    tri, _ = bs.bs_bins_triangles(h, ncand, 20)
    bs.bs_free_bins(h)
    cen = np.sqrt(redges[:-1] * redges[1:])
    kperp = cen[np.asarray(tri).reshape(-1, 3)][::17][:8]
    unit = 2 * np.pi / (w.rprime * w.dnu * w.nc)
    edges = np.geomspace(0.003, 1.258, 13)
    g = torch.Generator(device="cuda")
    g.manual_seed(23)
    Bd = torch.randn((kperp.shape[0], w.nc, w.nc), dtype=torch.complex128, device="cuda", generator=g)
    print(f"[multi] full nc sample nt={kperp.shape[0]}", flush=True)
    got = run(ctx, Bd, kperp, unit, edges, 4)
    check(got, Bd.cpu().numpy(), kperp, unit, edges, 4, "full")


def test_multipoles_of_the_dft_chain(ctx):
    """The paper's chain on a small periodic cube: the oracle's MABS collapse, then Eq. (dft) and the
    moments on the GPU, against Eq. (dft) and the moments in the oracle (ring k_perp at the
    geometric centres of the ring edges, in grid units)."""
    from oracle import bins as ob
    n, nc = 16, 12
    redges = np.array([1.0, 2.5, 4.0, 5.5])
    rb = ob.make_bins(ob.RING_U, n, nc, redges)
    V = synth.make_cube(synth.small_workload(n, nc), 53)
    B, N, _, _ = oe.estimate_mabs(rb, V)
    Bbar, _, _ = oe.collapse_mabs(B, N)
    cen = np.sqrt(redges[:-1] * redges[1:]) * 2 * np.pi / n
    kperp = np.array([[cen[i] for i in tri] for tri in rb.triangles])
    out = torch.empty((len(rb.triangles), nc, nc), dtype=torch.complex128, device="cuda")
    bs.bs_mabs_dft(ctx, nc, cuda(Bbar), out)
    unit = 2 * np.pi / nc
    edges = np.geomspace(0.2, 8.0, 9)
    got = run(ctx, out, kperp, unit, edges, 4)
    check(got, oe.mabs_dft(Bbar), kperp, unit, edges, 4, "chain")
