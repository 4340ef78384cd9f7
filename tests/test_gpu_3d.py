"""GPU parity of the 3D bispectrum (C ABI) against the FP64 oracle.

Counts (T3D) bit-exact; B within 1e-10 (FP64), 1e-5 (FP32 MFMA), 1e-4 (split-BF16)
relative where cond <= 1e3 (or within the precision's normwise floor), normwise beyond
(tests/gpu_common.compare_B).
"""
import numpy as np
import pytest

from oracle import bins as ob
from oracle import estimator as oe
from paper_2506_10526_amd import bs, synth

from gpu_common import Ctx, compare_B, cuda, host, torch, vis_tensor

pytestmark = pytest.mark.gpu

TOL = {bs.BS_FP64: 1e-10, bs.BS_FP32: 1e-5, bs.BS_SPLIT_BF16: 1e-4}
PREC = [bs.BS_FP64, bs.BS_FP32, bs.BS_SPLIT_BF16]


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def cubic_case(n, nc, nb, kmax_cells):
    edges = 2 * np.pi * np.geomspace(1.0 / n, kmax_cells / n, nb + 1)
    kw = dict(du_lambda=1.0, r_mpc=float(n), rprime_mpc_per_mhz=1.0, dnu_mhz=float(n) / nc)
    okw = dict(du=1.0, r_mpc=float(n), rprime=1.0, dnu=float(n) / nc)
    return edges, kw, okw


def oracle_3d(b, V, w):
    f = oe.ShellFields(b, V, w)
    B, T, neff, S, dev = oe.estimate_3d(b, V, w, fields=f)
    nvox = b.nc * b.n * b.n
    A = np.array([np.sum(np.abs(f.data(a) * f.data(bb) * f.data(c))) for a, bb, c in b.triangles])
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.where(T > 0, nvox * A / np.maximum(neff, 1e-300), 0.0)
    return B, T, neff, scale, dev


def run3(ctx, h, V, prec, ncand, **wk):
    B = torch.empty(ncand, dtype=torch.float64, device="cuda")
    N = torch.empty(ncand, dtype=torch.int64, device="cuda")
    E = torch.empty(ncand, dtype=torch.float64, device="cuda")
    bs.bs_estimate_3d(ctx, h, vis_tensor(V, prec), prec, B, N, E, **wk)
    return host(B), host(N), host(E)


@pytest.mark.parametrize("prec", PREC)
@pytest.mark.parametrize("case", ["cubic16x8", "cubic32x24_flags", "cubic32x128_fused", "cubic32x128_unfused",
                                  "cubic32x256_coarse", "cubic32x256_fullgrid", "cubic32x128_wide",
                                  "cubic32x128_wide_fft", "cubic32x128_wide_groups", "cubic32x128_wide_twobuf",
                                  "cubic32x128_wide_table", "cubic32x128_many"])
def test_3d_matches_oracle(ctx, prec, case, monkeypatch):
    """Small cubes: radix-2/3 delay axes, flags, and (nc = 128) the fused eta-C2R + contraction
    kernels (split-BF16: synthesis on MFMA, or the FFT form with BS_3D_FFT=1) next to the path that
    materialises the fields (BS_3D_UNFUSED=1)."""
    if case.endswith("_unfused"):
        monkeypatch.setenv("BS_3D_UNFUSED", "1")
    if case.endswith("_fullgrid"):
        monkeypatch.setenv("BS_3D_FULLGRID", "1")
    if case.endswith("_fft"):
        monkeypatch.setenv("BS_3D_FFT", "1")
    if case.endswith("_table"):
        # v pass reading the shell table per cell instead of each item's range of s
        monkeypatch.setenv("BS_3D_SHELL_TABLE", "1")
    if case.endswith("_twobuf"):
        # delay, v and u passes with the two-buffer LDS FFT instead of the in-place one
        monkeypatch.setenv("BS_3D_FFT_TWO_BUFFERS", "1")
    if case.endswith("_groups"):
        # four blocks: 16 line groups and 16 tiles per wave, flushes every 512 voxels (split-BF16
        # path: the next group's fragment copy and the FP64 read-modify-write both run)
        monkeypatch.setenv("BS_3D_DFT_BLOCKS", "4")
        monkeypatch.setenv("BS_3D_DFT_FLUSH", "512")
    if case.startswith("cubic32x128_wide"):
        # delay modes up to |eta| = 40: three 16-mode steps of the MFMA synthesis for the outer shells
        n, nc, nb, kmax = 32, 128, 6, 40.0
        wl = synth.small_workload(n, nc)
        cw = None
    elif case == "cubic32x128_many":
        # 18 shells: fields 16 and 17 are contraction columns of the second column tile, which the
        # MFMA kernel contracts only for the leading pair row tiles
        n, nc, nb, kmax = 32, 128, 18, 40.0
        wl = synth.small_workload(n, nc)
        cw = None
    elif case.startswith("cubic32x256"):
        # delay modes |eta| <= 9: the fused path contracts on a 128-point delay grid
        n, nc, nb, kmax = 32, 256, 6, 10.0
        wl = synth.small_workload(n, nc)
        cw = None
    elif case.startswith("cubic32x128"):
        n, nc, nb, kmax = 32, 128, 6, 10.0
        wl = synth.small_workload(n, nc, flags_mod32=(0, 16, 31))
        cw = wl.chan_w()
    elif case == "cubic16x8":
        n, nc, nb, kmax = 16, 8, 5, 5.5
        wl = synth.small_workload(n, nc)
        cw = None
    else:
        n, nc, nb, kmax = 32, 24, 7, 10.0
        wl = synth.small_workload(n, nc, flags_mod32=(0, 11, 23))
        cw = wl.chan_w()
    edges, kw, okw = cubic_case(n, nc, nb, kmax)
    V = synth.make_cube(wl, seed=17)
    uvm = synth.disk_mask(n)
    b = ob.make_bins(ob.SHELL_K, n, nc, edges, **okw)
    ow = oe.Weights(uv_mask=uvm, chan_w=cw)
    Bref, Tref, Nref, scale, dev = oracle_3d(b, V, ow)
    assert dev < 1e-6
    h, ncand = bs.bs_make_bins(ctx, bs.BS_SHELL_K, n, nc, edges, **kw)
    try:
        assert ncand == len(b.triangles)
        wk = dict(uv_mask=cuda(uvm))
        if cw is not None:
            wk["chan_w"] = cuda(cw, np.float32)
        Bg, Tg, Eg = run3(ctx, h, V, prec, ncand, **wk)
    finally:
        bs.bs_free_bins(h)
    assert np.array_equal(Tg, Tref)
    assert (Tref > 0).sum() > 10
    assert np.allclose(Eg, Nref, rtol=1e-15, atol=0)
    compare_B(Bg, Bref, Tref, scale, TOL[prec], f"3d {case} prec={prec}")


def test_3d_fields_match_oracle(ctx):
    n, nc = 16, 12
    edges, kw, okw = cubic_case(n, nc, 5, 5.5)
    V = synth.make_cube(synth.small_workload(n, nc), seed=21)
    b = ob.make_bins(ob.SHELL_K, n, nc, edges, **okw)
    f = oe.ShellFields(b, V)
    h, _ = bs.bs_make_bins(ctx, bs.BS_SHELL_K, n, nc, edges, **kw)
    try:
        F = torch.empty((5, nc, n, n), dtype=torch.float64, device="cuda")
        I = torch.empty((5, nc, n, n), dtype=torch.float64, device="cuda")
        bs.bs_filter_fields(ctx, h, vis_tensor(V, bs.BS_FP64), 1, bs.BS_FP64, F, I)
        F32 = torch.empty((5, nc, n, n), dtype=torch.float32, device="cuda")
        bs.bs_filter_fields(ctx, h, vis_tensor(V, bs.BS_FP32), 1, bs.BS_FP32, F32)
        Fh, Ih, F32h = host(F), host(I), host(F32)
    finally:
        bs.bs_free_bins(h)
    for j in range(5):
        ref = f.data(j)
        sc = max(np.abs(ref).max(), 1e-300)
        assert np.abs(Fh[j] - ref).max() <= 1e-12 * sc, j
        assert np.abs(F32h[j] - ref).max() <= 3e-6 * sc, j
        ic = f.count(j)
        assert np.abs(Ih[j] - ic).max() <= 1e-12 * max(np.abs(ic).max(), 1e-300), j


@pytest.mark.parametrize("prec", [bs.BS_FP32, bs.BS_SPLIT_BF16])
def test_3d_sign_flip(ctx, prec):
    n, nc = 16, 8
    edges, kw, _ = cubic_case(n, nc, 5, 5.5)
    V = synth.make_cube(synth.small_workload(n, nc), seed=23)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_SHELL_K, n, nc, edges, **kw)
    try:
        B1, T1, _ = run3(ctx, h, V, prec, ncand)
        B2, T2, _ = run3(ctx, h, -V, prec, ncand)
    finally:
        bs.bs_free_bins(h)
    ok = T1 > 0
    assert np.array_equal(T1, T2)
    if prec == bs.BS_FP32:
        assert np.array_equal(B2[ok], -B1[ok])
    else:  # bf16 MFMA sums round toward -inf (not symmetric in sign), see test_gpu_mabs.py
        assert np.all(np.abs(B2[ok] + B1[ok]) <= 1e-6 * (np.abs(B1[ok]) + np.nanmax(np.abs(B1))))


def test_3d_rejects_cell_weights(ctx):
    n, nc = 16, 8
    edges, kw, _ = cubic_case(n, nc, 5, 5.5)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_SHELL_K, n, nc, edges, **kw)
    try:
        V = vis_tensor(synth.make_cube(synth.small_workload(n, nc), seed=1), bs.BS_FP32)
        ng = cuda(np.ones((nc, n, n // 2 + 1), np.uint16))
        B = torch.empty(ncand, dtype=torch.float64, device="cuda")
        N = torch.empty(ncand, dtype=torch.int64, device="cuda")
        with pytest.raises(bs.BsError) as e:
            bs.bs_estimate_3d(ctx, h, V, bs.BS_FP32, B, N, ng=ng)
        assert e.value.code == bs.BS_EUNSUPPORTED
    finally:
        bs.bs_free_bins(h)


@pytest.mark.parametrize("prec", [bs.BS_FP32, bs.BS_SPLIT_BF16])
def test_3d_plan_reuse_across_bins(prec):
    """Unweighted estimates reuse their prepared plan while bins, precision and workspaces stay the
    same.  Alternating two bin sets (and a weighted call in between) on one context must give, for
    every call, the bits a fresh context gives for that call alone."""
    n, nc = 32, 128
    wl = synth.small_workload(n, nc)
    V = synth.make_cube(wl, seed=29)
    ea, kwa, _ = cubic_case(n, nc, 6, 40.0)
    eb, kwb, _ = cubic_case(n, nc, 5, 10.0)

    def fresh(edges, kw, **wk):
        c = Ctx()
        try:
            h, ncand = bs.bs_make_bins(c.h, bs.BS_SHELL_K, n, nc, edges, **kw)
            try:
                return run3(c.h, h, V, prec, ncand, **wk)
            finally:
                bs.bs_free_bins(h)
        finally:
            c.close()

    ref_a, ref_b = fresh(ea, kwa), fresh(eb, kwb)
    uvm = synth.disk_mask(n)
    ref_aw = fresh(ea, kwa, uv_mask=cuda(uvm))
    c = Ctx()
    try:
        ha, na = bs.bs_make_bins(c.h, bs.BS_SHELL_K, n, nc, ea, **kwa)
        hb, nb = bs.bs_make_bins(c.h, bs.BS_SHELL_K, n, nc, eb, **kwb)
        try:
            seq = [("a", ha, na, {}), ("a", ha, na, {}), ("b", hb, nb, {}), ("a", ha, na, {}),
                   ("aw", ha, na, {"uv_mask": cuda(uvm)}), ("a", ha, na, {}), ("b", hb, nb, {})]
            refs = {"a": ref_a, "b": ref_b, "aw": ref_aw}
            for name, h, ncand, wk in seq:
                got = run3(c.h, h, V, prec, ncand, **wk)
                for g, r in zip(got, refs[name]):
                    assert np.array_equal(np.nan_to_num(g, nan=-1.0), np.nan_to_num(r, nan=-1.0)), name
        finally:
            bs.bs_free_bins(ha)
            bs.bs_free_bins(hb)
    finally:
        c.close()
