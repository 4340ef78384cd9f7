"""GPU parity of the (k_par1, k_par2) binning of the cylindrical 3D BS (bs_kpar_grid, C ABI; Sec. 5,
Fig. 4) against oracle.estimator.bs_kpar_grid.

Counts are compared bit for bit (the bin of every index is decided in float64 from the same
product kpar_unit a' on both sides); the means differ only by summation order and must lie within
1e-12 of the bin's mean |Re B|.
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


def run(ctx, Bd, unit, edges):
    nt, ne = int(Bd.shape[0]), len(edges) - 1
    mean = torch.empty((nt, ne, ne), dtype=torch.float64, device="cuda")
    cnt = torch.empty((ne, ne), dtype=torch.int64, device="cuda")
    bs.bs_kpar_grid(ctx, Bd, unit, edges, mean, cnt)
    return host(mean), host(cnt)


def check(got, Bh, unit, edges, label):
    gm, gc = got
    rm, rc = oe.bs_kpar_grid(Bh, unit, np.asarray(edges))
    assert np.array_equal(gc, rc), f"{label}: counts differ in {int((gc != rc).sum())} bins"
    mag, _ = oe.bs_kpar_grid(np.abs(np.real(Bh)), unit, np.asarray(edges))
    ok = np.broadcast_to(rc > 0, rm.shape)
    assert np.all(np.isnan(gm[~ok])), f"{label}: empty bins must be NaN"
    err = np.abs(gm[ok] - rm[ok])
    assert np.all(err <= 1e-12 * mag[ok] + 1e-300), f"{label}: worst {float((err / mag[ok]).max()):.3e}"


@pytest.mark.parametrize("nc,nt,ne", [(1, 2, 1), (7, 3, 4), (12, 5, 6), (96, 4, 20), (301, 2, 7), (768, 3, 20)])
def test_matches_oracle(ctx, nc, nt, ne):
    rng = np.random.default_rng(nc + ne)
    unit = 0.0124
    kmax = unit * (nc // 2)
    edges = list(np.linspace(-kmax * 0.93, kmax * 0.97, ne + 1)) if nc > 1 else [-1.0, 1.0]
    B = rng.normal(size=(nt, nc, nc)) + 1j * rng.normal(size=(nt, nc, nc))
    print(f"[kpar] nc={nc} nt={nt} ne={ne}", flush=True)
    check(run(ctx, cuda(B), unit, edges), B, unit, edges, f"nc={nc}")


def test_edges_on_cells_and_outside(ctx):
    """Edges that fall exactly on cells (half-open bins, the last one closed at its top edge), a
    range wider than the k_par axis, and one that misses it entirely (every bin empty: NaN, 0)."""
    nc, unit = 16, 0.125
    B = np.random.default_rng(5).normal(size=(2, nc, nc)) + 0j
    for edges in ([-0.5, -0.25, 0.0, 0.25, 0.5], [-9.0, -1.0, 1.0, 9.0], [5.0, 6.0, 7.0]):
        check(run(ctx, cuda(B), unit, edges), B, unit, edges, f"edges={edges}")
    gm, gc = run(ctx, cuda(B), unit, [5.0, 6.0, 7.0])
    assert gc.sum() == 0 and np.all(np.isnan(gm))


def test_errors(ctx):
    B = torch.zeros((1, 4, 4), dtype=torch.complex128, device="cuda")
    mean = torch.empty((1, 2, 2), dtype=torch.float64, device="cuda")
    cnt = torch.empty((2, 2), dtype=torch.int64, device="cuda")
    for edges, unit in (([0.0, 0.0, 1.0], 0.1), ([0.0, 0.5, float("nan")], 0.1), ([0.0, 0.5, 1.0], 0.0)):
        with pytest.raises(bs.BsError):
            bs.bs_kpar_grid(ctx, B, unit, edges, mean, cnt)


def test_kpar_grid_of_the_dft_chain(ctx):
    """The paper's chain on a small periodic cube: the oracle's MABS collapse, then Eq. (dft) and the
    (k_par1, k_par2) grid on the GPU, against Eq. (dft) and the grid in the oracle."""
    n, nc = 16, 12
    rb = ob.make_bins(ob.RING_U, n, nc, np.array([1.0, 2.5, 4.0, 5.5]))
    V = synth.make_cube(synth.small_workload(n, nc), 47)
    B, N, _, _ = oe.estimate_mabs(rb, V)
    Bbar, _, _ = oe.collapse_mabs(B, N)
    out = torch.empty((len(rb.triangles), nc, nc), dtype=torch.complex128, device="cuda")
    bs.bs_mabs_dft(ctx, nc, cuda(Bbar), out)
    unit = 2 * np.pi / nc
    edges = list(np.linspace(-3.2, 3.2, 6))
    check(run(ctx, out, unit, edges), oe.mabs_dft(Bbar), unit, edges, "chain")
