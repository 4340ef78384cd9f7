"""GPU parity of the monopole B(k1, mu, t) of the cylindrical 3D BS (C ABI) against the oracle.

Counts are compared bit for bit: the bin of every cell is decided in FP64 by the same formula,
each operation rounded separately, on both sides.  Means: the GPU adds the cells of a bin in a
different order than the oracle, so each mean must lie within 1e-12 of the mean of |Re B| over
the bin (the rounding of a sum of n terms is bounded by about n eps times the sum of magnitudes;
n eps is below 1e-9 at a million cells a bin, and far below at these sizes, so 1e-12 of the
magnitude mean is a bound with margin for the sizes tested).
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


def run(ctx, Bcyl_dev, kperp, unit, edges):
    nk = len(edges) - 1
    mean = torch.empty((nk, 5, 5), dtype=torch.float64, device="cuda")
    cnt = torch.empty((nk, 5, 5), dtype=torch.int64, device="cuda")
    bs.bs_monopole(ctx, Bcyl_dev, kperp, unit, edges, mean, cnt)
    return host(mean), host(cnt)


def check(got, ref, Bcyl, kperp, unit, edges, label):
    gm, gc = got
    rm, rc = ref
    assert np.array_equal(gc, rc), f"{label}: counts differ in {int((gc != rc).sum())} bins"
    mag, _ = oe.bs_monopole(np.abs(np.real(Bcyl)), kperp, unit, edges)
    ok = rc > 0
    assert np.all(np.isnan(gm[~ok])), f"{label}: empty bins must be NaN"
    err = np.abs(gm[ok] - rm[ok])
    assert np.all(err <= 1e-12 * mag[ok] + 1e-300), f"{label}: worst {float((err / mag[ok]).max()):.3e}"


def random_triangles(rng, nt, scale):
    v1, v2 = rng.normal(size=(nt, 2)) * scale, rng.normal(size=(nt, 2)) * scale
    return np.stack([np.hypot(*v1.T), np.hypot(*v2.T), np.hypot(*(v1 + v2).T)], axis=1)


@pytest.mark.parametrize("nc,nt", [(1, 2), (2, 3), (3, 5), (6, 4), (9, 3), (12, 7), (48, 5), (96, 3), (300, 2)])
def test_monopole_matches_oracle(ctx, nc, nt):
    rng = np.random.default_rng(nc * 7 + nt)
    kperp = random_triangles(rng, nt, 0.05)
    unit = 0.02
    B = rng.normal(size=(nt, nc, nc)) + 1j * rng.normal(size=(nt, nc, nc))
    edges = np.geomspace(0.01, 0.3 + unit * nc, 7)
    print(f"[mono] nc={nc} nt={nt}", flush=True)
    got = run(ctx, cuda(B), kperp, unit, edges)
    check(got, oe.bs_monopole(B, kperp, unit, edges), B, kperp, unit, edges, f"nc={nc}")
    assert got[1].sum() > 0


def test_monopole_special_and_edge_cases(ctx):
    # equilateral rings with k_par = 0 land in (mu, t) = (0.5, 1): bins (0, 4); every other cell too
    # falls somewhere, and cells beyond the last edge are dropped
    kperp = np.array([[0.1, 0.1, 0.1]])
    B = np.full((1, 4, 4), 3.0 + 0.5j)
    edges = [0.05, 0.2]
    gm, gc = run(ctx, cuda(B), kperp, 1e-6, edges)
    assert gc[0, 0, 4] == 16 and gc.sum() == 16 and gm[0, 0, 4] == 3.0
    # nothing in range: all counts zero, all means NaN
    gm, gc = run(ctx, cuda(B), kperp, 1e-6, [1.0, 2.0, 3.0])
    assert gc.sum() == 0 and np.all(np.isnan(gm))
    # no triangles at all
    gm, gc = run(ctx, torch.empty((0, 4, 4), dtype=torch.complex128, device="cuda"), np.zeros((0, 3)), 0.1, [0.1, 1.0])
    assert gc.sum() == 0
    # invalid arguments are refused
    for args in ((kperp, 0.1, [0.2, 0.1]), (kperp, -1.0, [0.1, 0.2]), (np.array([[0.1, 0.0, 0.1]]), 0.1, [0.1, 0.2]),
                 (kperp, 0.1, list(np.geomspace(0.1, 1, 66)))):
        with pytest.raises(RuntimeError):
            run(ctx, cuda(B), *args)


def test_monopole_of_the_dft_chain(ctx):
    """The paper's chain on a small periodic cube: the oracle's MABS collapse, then Eq. (dft) and the
    monopole on the GPU, against Eq. (dft) and the monopole in the oracle."""
    n, nc = 16, 12
    redges = np.array([1.0, 2.5, 4.0, 5.5])
    rb = ob.make_bins(ob.RING_U, n, nc, redges)
    V = synth.make_cube(synth.small_workload(n, nc), 43)
    B, N, _, _ = oe.estimate_mabs(rb, V)
    Bbar, _, _ = oe.collapse_mabs(B, N)
    cen = np.sqrt(redges[:-1] * redges[1:]) * 2 * np.pi / n       # ring k_perp (grid units)
    kperp = np.array([[cen[i] for i in tri] for tri in rb.triangles])
    unit = 2 * np.pi / nc
    edges = np.geomspace(0.2, 8.0, 9)
    out = torch.empty((len(rb.triangles), nc, nc), dtype=torch.complex128, device="cuda")
    bs.bs_mabs_dft(ctx, nc, cuda(Bbar), out)
    got = run(ctx, out, kperp, unit, edges)
    Bc = oe.mabs_dft(Bbar)
    check(got, oe.bs_monopole(Bc, kperp, unit, edges), Bc, kperp, unit, edges, "chain")


def test_monopole_full_size(ctx):
    """133 ring triples of the 256^2 x 768 cube (ring k_perp at the geometric centres of the ring
    edges, k_par unit 2 pi / (r' B_bw)), seeded cylindrical BS, 12 log k1 bins over 0.003-1.258."""
    w = synth.config2()
    redges = w.shell_edges(20)
    h, ncand = bs.bs_make_bins(0, bs.BS_RING_U, w.n, w.nc, redges / (2 * np.pi * w.du / w.r_mpc))
    tri, _ = bs.bs_bins_triangles(h, ncand, 20)
    bs.bs_free_bins(h)
    cen = np.sqrt(redges[:-1] * redges[1:])
    kperp = cen[np.asarray(tri).reshape(-1, 3)]
    unit = 2 * np.pi / (w.rprime * w.dnu * w.nc)
    edges = np.geomspace(0.003, 1.258, 13)
    nt = kperp.shape[0]
    g = torch.Generator(device="cuda")
    g.manual_seed(17)
    Bd = torch.randn((nt, w.nc, w.nc), dtype=torch.complex128, device="cuda", generator=g)
    print(f"[mono] full size nt={nt} nc={w.nc}", flush=True)
    got = run(ctx, Bd, kperp, unit, edges)
    Bh = Bd.cpu().numpy()
    check(got, oe.bs_monopole(Bh, kperp, unit, edges), Bh, kperp, unit, edges, "full")
