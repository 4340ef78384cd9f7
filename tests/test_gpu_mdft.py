"""GPU parity of Eq. (dft), collapsed MABS -> cylindrical 3D BS (C ABI), against the FP64 oracle.

The path is FP64 throughout: two radix-2/3/4/8 FFT passes of length nc.  Their rounding error is
of order eps log2(nc) times the output's largest magnitude (each output is a sum of (nc + 1)^2
terms whose magnitudes the FFT's orthogonal butterflies preserve up to that factor), so every
entry must lie within TOL = 1e-12 of max |out| (about 40 eps log2 nc at nc = 768, with margin).
"""
import numpy as np
import pytest

from oracle import bins as ob
from oracle import estimator as oe
from paper_2506_10526_amd import bs, synth

from gpu_common import Ctx, cuda, host, torch

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def run(ctx, Bbar: np.ndarray, nc: int, scale=1.0, circular=False):
    out = torch.empty((Bbar.shape[0], nc, nc), dtype=torch.complex128, device="cuda")
    bs.bs_mabs_dft(ctx, nc, cuda(Bbar), out, scale=scale, circular=circular)
    return host(out)


def check(got, ref, label):
    err = float(np.max(np.abs(got - ref)))
    top = float(np.max(np.abs(ref)))
    assert np.all(np.isfinite(got)), f"{label}: non-finite output"
    assert err <= TOL * top, f"{label}: max |gpu - oracle| = {err:.3e} vs max |out| {top:.3e}"
    return err / top


# lengths: every radix (2, 3, 4, 8), odd and even, and blocks with ragged row / column tails
@pytest.mark.parametrize("nc", [2, 3, 4, 6, 9, 12, 18, 24, 48, 54, 96, 162, 256])
@pytest.mark.parametrize("circular", [False, True])
def test_mdft_matches_oracle(ctx, nc, circular):
    nt = 3 if nc <= 96 else 2
    Bbar = synth.collapsed_mabs(nt, nc, 100 + nc, circular=circular)
    print(f"[mdft] nc={nc} circular={circular} nt={nt}", flush=True)
    got = run(ctx, Bbar, nc, scale=0.75, circular=circular)
    check(got, oe.mabs_dft(Bbar, 0.75, circular=circular), f"nc={nc} circ={circular}")


def test_mdft_of_the_oracle_collapse_of_a_cube(ctx):
    """The paper's route end to end on a small periodic cube: the oracle's MABS, collapsed both
    ways, then Eq. (dft) on the GPU and in the oracle."""
    n, nc = 16, 12
    rb = ob.make_bins(ob.RING_U, n, nc, np.array([1.0, 2.5, 4.0, 5.5]))
    V = synth.make_cube(synth.small_workload(n, nc), 41)
    B, N, _, _ = oe.estimate_mabs(rb, V, norm=2.0)
    for circular in (False, True):
        Bbar, _, _ = oe.collapse_mabs(B, N, circular=circular)
        got = run(ctx, Bbar, nc, scale=1.5, circular=circular)
        check(got, oe.mabs_dft(Bbar, 1.5, circular=circular), f"cube circ={circular}")


@pytest.mark.parametrize("ncols,mrows,nth,mth", [(1, 1, 256, 256), (2, 4, 512, 512), (4, 1, 256, 512),
                                                  (8, 2, 256, 256)])
def test_mdft_block_shapes(ctx, monkeypatch, ncols, mrows, nth, mth):
    """Lines per group and block sizes other than the defaults give the same result."""
    monkeypatch.setenv("BS_MDFT_NCOLS", str(ncols))
    monkeypatch.setenv("BS_MDFT_MROWS", str(mrows))
    monkeypatch.setenv("BS_MDFT_NCOLS_THREADS", str(nth))
    monkeypatch.setenv("BS_MDFT_MROWS_THREADS", str(mth))
    monkeypatch.setenv("BS_MDFT_GRID", "37")
    for nc in (72, 81):
        Bbar = synth.collapsed_mabs(3, nc, 7)
        check(run(ctx, Bbar, nc), oe.mabs_dft(Bbar), f"nc={nc} ncols={ncols} mrows={mrows}")


def test_mdft_full_size_sampled(ctx):
    """nc = 768 (the 768-channel cube), 133 triangles as in the bench; three triangles checked
    against the oracle, and the Hermitian mirror of every output."""
    nc, nt = 768, 133
    size = 2 * nc - 1
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    Bd = torch.randn((nt, size, size), dtype=torch.float64, device="cuda", generator=g)
    d = torch.arange(size, device="cuda") - (nc - 1)
    Bd[:, (d[None, :] - d[:, None]).abs() >= nc] = float("nan")
    out = torch.empty((nt, nc, nc), dtype=torch.complex128, device="cuda")
    print("[mdft] full size nc=768 nt=133", flush=True)
    bs.bs_mabs_dft(ctx, nc, Bd, out, scale=1.0)
    torch.cuda.synchronize()
    for t in (0, 66, nt - 1):
        Bt = Bd[t:t + 1].cpu().numpy()
        check(out[t:t + 1].cpu().numpy(), oe.mabs_dft(Bt), f"full t={t}")
    neg = (-torch.arange(nc, device="cuda")) % nc
    mirror = out[:, neg][:, :, neg].conj()
    herm = float((out - mirror).abs().max() / out.abs().max())
    assert herm <= TOL


def test_mdft_edge_cases(ctx):
    # no triangles: nothing is read or written
    bs.bs_mabs_dft(ctx, 8, torch.empty((0, 15, 15), dtype=torch.float64, device="cuda"),
                   torch.empty((0, 8, 8), dtype=torch.complex128, device="cuda"))
    # all separations unsampled: zero output
    Bbar = np.full((2, 11, 11), np.nan)
    assert np.max(np.abs(run(ctx, Bbar, 6))) == 0.0
    # lengths outside 2^a 3^b or beyond 4096 are refused
    for nc in (5, 10, 6144):
        with pytest.raises(RuntimeError):
            bs.bs_mabs_dft(ctx, nc, torch.zeros((1, 2 * nc - 1, 2 * nc - 1), dtype=torch.float64, device="cuda"),
                           torch.empty((1, nc, nc), dtype=torch.complex128, device="cuda"))
