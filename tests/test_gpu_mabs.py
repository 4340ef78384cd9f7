"""GPU parity of the MABS estimator (C ABI) against the FP64 oracle.

Counts must be bit-exact.  B: relative error <= 1e-10 (FP64 path), 1e-5 (FP32 MFMA) and 1e-4 (split-BF16
MFMA) where cond = sum |F1 F2 F3| / |sum F1 F2 F3| <= 1e3, or within the precision's normwise
floor there, and error <= tol of the |F1 F2 F3| estimate beyond (see gpu_common.compare_B).
"""
import numpy as np
import pytest

from oracle import bins as ob
from oracle import estimator as oe
from paper_2506_10526_amd import bs, synth

from gpu_common import Ctx, compare_B, cuda, host, need_gpu, torch, vis_tensor

pytestmark = pytest.mark.gpu

TOL = {bs.BS_FP64: 1e-10, bs.BS_FP32: 1e-5, bs.BS_SPLIT_BF16: 1e-4}
PREC = [bs.BS_FP64, bs.BS_FP32, bs.BS_SPLIT_BF16]


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def oracle_full(b, V, w, tri=None, nu1=None):
    f = oe.MabsFields(b, V, w)
    B, N, S, dev = oe.estimate_mabs(b, V, w, tri=tri, nu1=nu1, fields=f)
    tri = b.triangles if tri is None else np.asarray(tri)
    nu1 = np.arange(b.nc) if nu1 is None else np.asarray(nu1)
    npix = b.n * b.n
    A = np.empty_like(S)
    for t, (b1, b2, b3) in enumerate(tri):
        d1 = np.abs(f.data(b1).reshape(b.nc, -1))[nu1]
        d2 = np.abs(f.data(b2).reshape(b.nc, -1))
        d3 = np.abs(f.data(b3).reshape(b.nc, -1))
        A[t] = oe.triple_sum(d1, d2, d3)
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.where(N > 0, npix * A / np.maximum(N, 1), 0.0)
    return B, N, scale


def run_gpu(ctx, b_h, V, prec, nt, nnu1, nc, tri=None, nu1=None, collapse=0, **wk):
    shape = (nt, nnu1, nc, nc) if not collapse else (nt,) + ((2 * nc - 1,) * 2 if collapse == 1 else (nc, nc))
    B = torch.empty(shape, dtype=torch.float64, device="cuda")
    N = torch.empty(shape, dtype=torch.int64, device="cuda")
    Nnu = torch.empty(shape, dtype=torch.int32, device="cuda") if collapse else None
    bs.bs_estimate_mabs(ctx, b_h, vis_tensor(V, prec), prec, B, N, Nnu, tri3=tri, nu1=nu1, collapse=collapse, **wk)
    out = (host(B), host(N))
    return out + ((host(Nnu),) if collapse else ())


@pytest.mark.parametrize("prec", PREC)
def test_config1_full_mabs(ctx, prec):
    """64x64 uv x 16 channels, 8 log rings, every channel triple (workload of the first config)."""
    w = synth.config1()
    edges = w.ring_edges(8)
    V = synth.make_cube(w, seed=1)
    b = ob.make_bins(ob.RING_U, w.n, w.nc, edges)
    Bref, Nref, scale = oracle_full(b, V, None)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, w.n, w.nc, edges)
    try:
        Bg, Ng = run_gpu(ctx, h, V, prec, ncand, w.nc, w.nc)
    finally:
        bs.bs_free_bins(h)
    assert np.array_equal(Ng, Nref)
    assert (Nref[:, 0, 0, 0] > 0).sum() == 72
    compare_B(Bg, Bref, Nref, scale, TOL[prec], f"config1 prec={prec}")


@pytest.mark.parametrize("prec", PREC)
def test_ragged_subset_flags_permuted(ctx, prec):
    """Ragged tiles (n=48, nc=12), a nu1 subset, permuted triangles and flagged channels."""
    n, nc = 48, 12
    w = synth.small_workload(n, nc, flags_mod32=(1, 7))
    edges = np.geomspace(1.0, synth.default_umax(n) + 1.0, 6)
    V = synth.make_cube(w, seed=5)
    cw = w.chan_w()
    uvm = synth.disk_mask(n)
    b = ob.make_bins(ob.RING_U, n, nc, edges)
    tri = b.triangles[::2][:, [2, 0, 1]]
    nu1 = [0, 5, 11]
    ow = oe.Weights(uv_mask=uvm, chan_w=cw)
    Bref, Nref, scale = oracle_full(b, V, ow, tri=tri, nu1=nu1)
    h, _ = bs.bs_make_bins(ctx, bs.BS_RING_U, n, nc, edges)
    try:
        Bg, Ng = run_gpu(ctx, h, V, prec, len(tri), len(nu1), nc, tri=tri, nu1=nu1,
                         uv_mask=cuda(uvm), chan_w=cuda(cw, np.float32))
    finally:
        bs.bs_free_bins(h)
    assert np.array_equal(Ng, Nref)
    assert (Nref == 0).any() and (Nref > 0).any()
    compare_B(Bg, Bref, Nref, scale, TOL[prec], f"ragged prec={prec}")


@pytest.mark.parametrize("prec", [bs.BS_FP64, bs.BS_SPLIT_BF16])
def test_cell_count_weights(ctx, prec):
    """Per-cell N_g weights (W_g = 1/N_g, counts from [N_g > 0]) with empty cells."""
    n, nc = 32, 6
    rng = np.random.default_rng(3)
    ng = rng.integers(0, 4, size=(nc, n, n // 2 + 1)).astype(np.uint16)
    neg = (-np.arange(n)) % n
    ng[:, :, 0] = np.maximum(ng[:, :, 0], ng[:, neg, 0])
    edges = np.geomspace(1.0, 11.0, 5)
    V = synth.make_cube(synth.small_workload(n, nc), seed=9)
    b = ob.make_bins(ob.RING_U, n, nc, edges)
    Bref, Nref, scale = oracle_full(b, V, oe.Weights(ng=ng))
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, n, nc, edges)
    try:
        Bg, Ng = run_gpu(ctx, h, V, prec, ncand, nc, nc, ng=cuda(ng))
    finally:
        bs.bs_free_bins(h)
    assert np.array_equal(Ng, Nref)
    compare_B(Bg, Bref, Nref, scale, TOL[prec], f"ng prec={prec}")


@pytest.mark.parametrize("nc,weighted", [(1, False), (1, True), (2, True), (3, False), (4, True)])
def test_fp64_few_channels(ctx, nc, weighted):
    """FP64 MABS with few channels (n_nu1 nc^2 <= 64 entries a triangle, the per-entry pixel sums
    instead of the tiled GEMM), unweighted and with per-cell N_g weights (whose counts also take
    that path); counts bit-exact."""
    n = 32
    rng = np.random.default_rng(11 + nc)
    edges = np.geomspace(1.0, 11.0, 5)
    V = synth.make_cube(synth.small_workload(n, nc), seed=13 + nc)
    b = ob.make_bins(ob.RING_U, n, nc, edges)
    wk, ow = {}, None
    if weighted:
        ng = rng.integers(0, 4, size=(nc, n, n // 2 + 1)).astype(np.uint16)
        neg = (-np.arange(n)) % n
        ng[:, :, 0] = np.maximum(ng[:, :, 0], ng[:, neg, 0])
        wk, ow = {"ng": cuda(ng)}, oe.Weights(ng=ng)
    Bref, Nref, scale = oracle_full(b, V, ow)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, n, nc, edges)
    try:
        Bg, Ng = run_gpu(ctx, h, V, bs.BS_FP64, ncand, nc, nc, **wk)
    finally:
        bs.bs_free_bins(h)
    assert np.array_equal(Ng, Nref)
    compare_B(Bg, Bref, Nref, scale, TOL[bs.BS_FP64], f"few channels nc={nc}")


@pytest.mark.parametrize("collapse", [1, 2])
def test_collapse(ctx, collapse):
    n, nc = 32, 8
    w = synth.small_workload(n, nc, flags_mod32=(3,))
    edges = np.geomspace(1.0, 11.0, 5)
    V = synth.make_cube(w, seed=13)
    cw = w.chan_w()
    b = ob.make_bins(ob.RING_U, n, nc, edges)
    ow = oe.Weights(chan_w=cw)
    B, N, _, _ = oe.estimate_mabs(b, V, ow)
    Bbar, Nnu, Ntot = oe.collapse_mabs(B, N, circular=(collapse == 2))
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, n, nc, edges)
    try:
        Bg, Ng, Nnug = run_gpu(ctx, h, V, bs.BS_FP64, ncand, nc, nc, collapse=collapse, chan_w=cuda(cw, np.float32))
    finally:
        bs.bs_free_bins(h)
    assert np.array_equal(Nnug, Nnu)
    assert np.array_equal(Ng, Ntot)
    ok = Nnu > 0
    assert np.all(np.isnan(Bg[~ok]))
    assert np.allclose(Bg[ok], Bbar[ok], rtol=1e-9, atol=1e-12 * np.nanmax(np.abs(Bbar)))


@pytest.mark.parametrize("prec", [bs.BS_FP32, bs.BS_SPLIT_BF16])
def test_sign_flip_and_scaling_are_exact(ctx, prec):
    w = synth.config1()
    edges = w.ring_edges(8)
    V = synth.make_cube(w, seed=2)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, w.n, w.nc, edges)
    try:
        B1, N1 = run_gpu(ctx, h, V, prec, ncand, w.nc, w.nc)
        B2, N2 = run_gpu(ctx, h, -V, prec, ncand, w.nc, w.nc)
        B3, N3 = run_gpu(ctx, h, 2 * V, prec, ncand, w.nc, w.nc)
    finally:
        bs.bs_free_bins(h)
    ok = N1 > 0
    assert np.array_equal(N1, N2) and np.array_equal(N1, N3)
    if prec == bs.BS_FP32:
        # negation and scaling by 2 commute with every FP32 rounding step
        assert np.array_equal(B2[ok], -B1[ok])
        assert np.array_equal(B3[ok], 8 * B1[ok])
    else:
        # the bf16 MFMAs do not round their internal sum symmetrically: on the MI355X one
        # v_mfma_f32_*_bf16 whose products span many binades is off by -0.7 ulp on average
        # (toward -inf), and D(-A, B, -C) differs from -D(A, B, C) by one ulp in about 30 % of
        # outputs (measured with ones as B and known exact sums); the split hi/lo of -x is exactly
        # -(hi, lo), so this is the one asymmetric step, and the split path is checked to a few
        # FP32 ulps of the entry
        assert np.all(np.abs(B2[ok] + B1[ok]) <= 1e-6 * (np.abs(B1[ok]) + np.nanmax(np.abs(B1))))
        assert np.array_equal(B3[ok], 8 * B1[ok]) or np.allclose(B3[ok], 8 * B1[ok], rtol=1e-6)


def test_mabs_fields_match_oracle(ctx):
    w = synth.config1()
    edges = w.ring_edges(8)
    V = synth.make_cube(w, seed=4)
    b = ob.make_bins(ob.RING_U, w.n, w.nc, edges)
    f = oe.MabsFields(b, V)
    h, _ = bs.bs_make_bins(ctx, bs.BS_RING_U, w.n, w.nc, edges)
    try:
        F = torch.empty((8, w.nc, w.n, w.n), dtype=torch.float64, device="cuda")
        I = torch.empty((8, w.nc, w.n, w.n), dtype=torch.float64, device="cuda")
        bs.bs_filter_fields(ctx, h, vis_tensor(V, bs.BS_FP64), 0, bs.BS_FP64, F, I)
        F32 = torch.empty((8, w.nc, w.n, w.n), dtype=torch.float32, device="cuda")
        bs.bs_filter_fields(ctx, h, vis_tensor(V, bs.BS_FP32), 0, bs.BS_FP32, F32)
        Fh, Ih, F32h = host(F), host(I), host(F32)
    finally:
        bs.bs_free_bins(h)
    for j in range(8):
        ref = f.data(j)
        scale = np.abs(ref).max()
        assert np.abs(Fh[j] - ref).max() <= 1e-12 * scale
        assert np.abs(F32h[j] - ref).max() <= 3e-6 * scale
        assert np.abs(Ih[j] - f.count(j)).max() <= 1e-12 * max(np.abs(f.count(j)).max(), 1e-300)


def test_error_paths(ctx):
    w = synth.config1()
    edges = w.ring_edges(8)
    V = vis_tensor(synth.make_cube(w, seed=1), bs.BS_FP32)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, w.n, w.nc, edges)
    B = torch.empty((1, 1, w.nc, w.nc), dtype=torch.float64, device="cuda")
    N = torch.empty((1, 1, w.nc, w.nc), dtype=torch.int64, device="cuda")
    try:
        with pytest.raises(bs.BsError):
            bs.bs_estimate_mabs(ctx, h, V, 7, B, N)
        with pytest.raises(bs.BsError):
            bs.bs_estimate_mabs(ctx, h, V, bs.BS_FP32, B, N, tri3=[(0, 0, 9)])
        with pytest.raises(bs.BsError):
            bs.bs_estimate_mabs(ctx, h, V, bs.BS_FP32, B, N, nu1=[99])
        with pytest.raises(bs.BsError):
            bs.bs_estimate_mabs(ctx, h, V, bs.BS_FP32, B, N, collapse=1)       # no N_nu
    finally:
        bs.bs_free_bins(h)


def test_full_row_tiles(ctx):
    """nc = 256 (a multiple of the 128-row tile, so every row tile lies within one nu1 and no tile
    row is padding); the pixel count 48^2 = 2304 is not a multiple of the 4096-pixel FP64 flush,
    and its 72 stages exercise both LDS buffer parities and the final partial flush."""
    n, nc = 48, 256
    w = synth.small_workload(n, nc)
    edges = np.geomspace(1.0, synth.default_umax(n) + 1.0, 5)
    V = synth.make_cube(w, seed=31)
    b = ob.make_bins(ob.RING_U, n, nc, edges)
    nu1 = [0, 77, 255]
    Bref, Nref, scale = oracle_full(b, V, None, nu1=nu1)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, n, nc, edges)
    try:
        Bg, Ng = run_gpu(ctx, h, V, bs.BS_SPLIT_BF16, ncand, len(nu1), nc, nu1=nu1)
    finally:
        bs.bs_free_bins(h)
    assert np.array_equal(Ng, Nref)
    compare_B(Bg, Bref, Nref, scale, TOL[bs.BS_SPLIT_BF16], "full row tiles")


@pytest.mark.parametrize("prec", [bs.BS_SPLIT_BF16, bs.BS_FP32])
def test_multi_flush(ctx, prec, monkeypatch):
    """128^2 pixels in one pixel chunk (BS_MABS_KCHUNKS=1): every split-BF16 block adds two FP32 runs
    of 8192 pixels into its FP64 sums (the read-modify-write of the flush), and the FP32 kernel 64
    runs of 256; checked against the oracle for two nu1 rows."""
    monkeypatch.setenv("BS_MABS_KCHUNKS", "1")
    n, nc = 128, 8
    w = synth.small_workload(n, nc)
    edges = np.geomspace(1.0, synth.default_umax(n) + 1.0, 5)
    V = synth.make_cube(w, seed=41)
    b = ob.make_bins(ob.RING_U, n, nc, edges)
    nu1 = [1, 6]
    Bref, Nref, scale = oracle_full(b, V, None, nu1=nu1)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, n, nc, edges)
    try:
        Bg, Ng = run_gpu(ctx, h, V, prec, ncand, len(nu1), nc, nu1=nu1)
    finally:
        bs.bs_free_bins(h)
    assert np.array_equal(Ng, Nref)
    compare_B(Bg, Bref, Nref, scale, TOL[prec], f"multi flush prec={prec}")


@pytest.mark.parametrize("m1", [4, 8, 16, 32])
def test_row_blockings(ctx, m1, monkeypatch):
    """Every row blocking of the 256 x 192 split-BF16 tiles (m1 nu1 rows x 256 / m1 nu2 rows, set by
    BS_MABS_M1): 33 nu1 rows and nc = 40 leave partial nu1, nu2 and column blocks, and the raw-row
    copies of the F_b1 and F_b2 rows start at different copy instructions for each m1."""
    monkeypatch.setenv("BS_MABS_M1", str(m1))
    n, nc = 32, 40
    w = synth.small_workload(n, nc)
    edges = np.geomspace(1.0, synth.default_umax(n) + 1.0, 5)
    V = synth.make_cube(w, seed=53 + m1)
    b = ob.make_bins(ob.RING_U, n, nc, edges)
    nu1 = list(range(0, 40, 3)) + list(range(1, 40, 2))[:20]
    Bref, Nref, scale = oracle_full(b, V, None, nu1=nu1)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, n, nc, edges)
    try:
        Bg, Ng = run_gpu(ctx, h, V, bs.BS_SPLIT_BF16, ncand, len(nu1), nc, nu1=nu1)
    finally:
        bs.bs_free_bins(h)
    assert np.array_equal(Ng, Nref)
    compare_B(Bg, Bref, Nref, scale, TOL[bs.BS_SPLIT_BF16], f"row blocking m1={m1}")
