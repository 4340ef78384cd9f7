"""The allocation-free monopole (bs_monopole_noalloc, scratch in a fixed device array) against the
allocating entry point bs_monopole and the oracle, on two calls in a row, the second smaller.

Counts bit for bit; means within 1e-12 of the bin's mean |Re B| (the two entry points may add a
bin's cells in another order: the allocation-free one uses fewer blocks when the scratch is full).
"""
import numpy as np
import pytest

from oracle import estimator as oe
from paper_2506_10526_amd import bs, synth

from gpu_common import Ctx, cuda, host, torch

pytestmark = pytest.mark.gpu


def _both(ctx, Bd, kperp, unit, edges):
    nk = len(edges) - 1
    m1 = torch.empty((nk, 5, 5), dtype=torch.float64, device="cuda")
    c1 = torch.empty((nk, 5, 5), dtype=torch.int64, device="cuda")
    bs.bs_monopole(ctx, Bd, kperp, unit, edges, m1, c1)
    m2 = torch.full((nk, 5, 5), -7.0, dtype=torch.float64, device="cuda")
    c2 = torch.full((nk, 5, 5), -7, dtype=torch.int64, device="cuda")
    bs.bs_monopole_noalloc(ctx, Bd, cuda(np.asarray(kperp, dtype=np.float64)), unit,
                           cuda(np.asarray(edges, dtype=np.float64)), m2, c2)
    return (host(m1), host(c1)), (host(m2), host(c2))


def _check(a, b, Bh, kperp, unit, edges, label):
    (m1, c1), (m2, c2) = a, b
    assert np.array_equal(c1, c2), f"{label}: counts differ"
    mag, _ = oe.bs_monopole(np.abs(np.real(Bh)), kperp, unit, edges)
    ok = c1 > 0
    assert np.all(np.isnan(m2[~ok]))
    assert np.all(np.abs(m2[ok] - m1[ok]) <= 1e-12 * mag[ok] + 1e-300), label


def test_noalloc_monopole_matches_allocating_entry_point():
    c = Ctx()
    try:
        # call 1: the 133 ring triples of the 256^2 x 768 cube, 12 k1 bins (scratch-limited blocks)
        w = synth.config2()
        redges = w.shell_edges(20)
        h, ncand = bs.bs_make_bins(0, bs.BS_RING_U, w.n, w.nc, redges / (2 * np.pi * w.du / w.r_mpc))
        tri, _ = bs.bs_bins_triangles(h, ncand, 20)
        bs.bs_free_bins(h)
        cen = np.sqrt(redges[:-1] * redges[1:])
        kperp = cen[np.asarray(tri).reshape(-1, 3)]
        unit = 2 * np.pi / (w.rprime * w.dnu * w.nc)
        edges = np.geomspace(0.003, 1.258, 13)
        g = torch.Generator(device="cuda")
        g.manual_seed(23)
        Bd = torch.randn((kperp.shape[0], w.nc, w.nc), dtype=torch.complex128, device="cuda", generator=g)
        print(f"[noalloc] call 1: nt={kperp.shape[0]} nc={w.nc} n_k1=12", flush=True)
        a, b = _both(c.h, Bd, kperp, unit, edges)
        Bh = Bd.cpu().numpy()
        _check(a, b, Bh, kperp, unit, edges, "call 1")
        assert a[1].sum() > 0
        # call 2: smaller (5 triangles, nc = 48, 6 k1 bins) on the same scratch, also against the oracle
        rng = np.random.default_rng(5)
        v1, v2 = rng.normal(size=(5, 2)) * 0.05, rng.normal(size=(5, 2)) * 0.05
        kp2 = np.stack([np.hypot(*v1.T), np.hypot(*v2.T), np.hypot(*(v1 + v2).T)], axis=1)
        B2 = rng.normal(size=(5, 48, 48)) + 1j * rng.normal(size=(5, 48, 48))
        e2 = np.geomspace(0.01, 1.3, 7)
        print("[noalloc] call 2: nt=5 nc=48 n_k1=6", flush=True)
        a, b = _both(c.h, cuda(B2), kp2, 0.02, e2)
        _check(a, b, B2, kp2, 0.02, e2, "call 2")
        rm, rc = oe.bs_monopole(B2, kp2, 0.02, e2)
        assert np.array_equal(b[1], rc)
        mag, _ = oe.bs_monopole(np.abs(np.real(B2)), kp2, 0.02, e2)
        ok = rc > 0
        assert np.all(np.abs(b[0][ok] - rm[ok]) <= 1e-12 * mag[ok] + 1e-300)
        # sizes beyond the limits are refused with a clear error
        with pytest.raises(RuntimeError, match="n_k1"):
            _both(c.h, cuda(B2), kp2, 0.02, np.geomspace(0.01, 1.3, 66))
    finally:
        c.close()
