"""GPU seeded cube generator and Monte Carlo runs (C ABI) against the oracle.

* bs_generate_cube vs oracle.generator.generate_cube (same Philox stream, FP32 vs FP64 transforms);
* bs_mc_run: per-triangle mean and variance over realizations vs the oracle estimator applied to
  the oracle's cubes of the same realizations; graph replays vs direct launches (bitwise).
"""
import numpy as np
import pytest

from oracle import bins as ob
from oracle import estimator as oe
from oracle import generator as og
from paper_2506_10526_amd import bs, synth

from gpu_common import Ctx, compare_B, cuda, host, torch

pytestmark = pytest.mark.gpu

MWA = dict(du_lambda=synth.DU_G, r_mpc=synth.R_MPC, rprime_mpc_per_mhz=synth.RPRIME_MPC_PER_MHZ,
           dnu_mhz=synth.DNU_MHZ)
MWA_O = dict(du=synth.DU_G, r_mpc=synth.R_MPC, rprime=synth.RPRIME_MPC_PER_MHZ, dnu=synth.DNU_MHZ)


@pytest.fixture(scope="module")
def ctx():
    c = Ctx()
    yield c.h
    c.close()


def gen_gpu(ctx, n, nc, kind, seed, real, cw=None, **kw):
    desc = bs.field_desc(n, nc, kind, **kw)
    V = torch.empty((nc, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    bs.bs_generate_cube(ctx, desc, seed, real, V, chan_w=None if cw is None else cuda(cw, np.float32))
    return host(V)


def check_cube(Vg, Vr, label):
    err = np.abs(Vg.astype(np.complex128) - Vr)
    big = np.abs(Vr).max()
    rms = np.sqrt(np.mean(np.abs(Vr) ** 2))
    print(f"{label}: max err / max|V| {err.max() / big:.2e}, rms err / rms V {np.sqrt(np.mean(err ** 2)) / rms:.2e}")
    assert err.max() <= 3e-6 * big, label
    assert np.sqrt(np.mean(err ** 2)) <= 1.5e-6 * rms, label


@pytest.mark.parametrize("case", ["cubic16x8", "cubic48x12_flags", "physical64x96_flags", "cubic32x32"])
def test_generate_cube_matches_oracle(ctx, case):
    if case == "cubic16x8":
        n, nc, kind, flags, kw, okw = 16, 8, "cubic", None, {}, {}
    elif case == "cubic48x12_flags":
        n, nc, kind, flags, kw, okw = 48, 12, "cubic", (1, 7), {}, {}
    elif case == "cubic32x32":
        n, nc, kind, flags, kw, okw = 32, 32, "cubic", None, dict(pk_index=-1.5, f_ng=0.3, sigma=1.0), \
            dict(index=-1.5, f=0.3, sigma=1.0)
    else:
        n, nc, kind, flags, kw, okw = 64, 96, "physical", (0, 16, 31), MWA, MWA_O
    cw = synth.mwa_flags(nc, flags) if flags else None
    k = bs.BS_K_CUBIC if kind == "cubic" else bs.BS_K_PHYSICAL
    Vg = gen_gpu(ctx, n, nc, k, 5, 3, cw, **kw)
    Vr = og.generate_cube(n, nc, kind, 5, 3, chan_w=cw, **okw)
    check_cube(Vg, Vr, case)
    if flags:
        assert np.all(Vg[cw == 0] == 0)


def test_generate_full_size_mwa_cube(ctx):
    """256 x 256 uv x 768 channels, MWA constants: the cube the benchmark and the labels use."""
    Vg = gen_gpu(ctx, 256, 768, bs.BS_K_PHYSICAL, 1, 0, None, **MWA)
    Vr = og.generate_cube(256, 768, "physical", 1, 0, **MWA_O)
    check_cube(Vg, Vr, "mwa256x768")


def tiny_bins(ctx, n, nc, nb, kmax):
    edges = 2 * np.pi * np.geomspace(1.0 / n, kmax / n, nb + 1)
    kw = dict(du_lambda=1.0, r_mpc=float(n), rprime_mpc_per_mhz=1.0, dnu_mhz=float(n) / nc)
    okw = dict(du=1.0, r_mpc=float(n), rprime=1.0, dnu=float(n) / nc)
    b = ob.make_bins(ob.SHELL_K, n, nc, edges, **okw)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_SHELL_K, n, nc, edges, **kw)
    return b, h, ncand


def oracle_mc(b, n, nc, seed, R, w=None, cw=None):
    Bs, last = [], None
    for r in range(R):
        V = og.generate_cube(n, nc, "cubic", seed, r, chan_w=cw)
        f = oe.ShellFields(b, V, w)
        B, T, neff, S, _ = oe.estimate_3d(b, V, w, fields=f)
        Bs.append(B)
        last = (B, T, neff, f)
    return np.array(Bs), last


def last_scale(b, last):
    B, T, neff, f = last
    nvox = b.nc * b.n * b.n
    A = np.array([np.sum(np.abs(f.data(x) * f.data(y) * f.data(z))) for x, y, z in b.triangles])
    return np.where(T > 0, nvox * A / np.maximum(neff, 1e-300), 0.0)


def check_stats(cnt, mean, var, Bs, R, label):
    ok = np.all(np.isfinite(Bs), axis=0)
    assert np.all(cnt[ok] == R) and np.all(cnt[~ok] == 0), label
    mr, vr = Bs[:, ok].mean(0), Bs[:, ok].var(0, ddof=1)
    dm = np.abs(mean[ok] - mr)
    dv = np.abs(var[ok] - vr)
    print(f"{label}: max |dmean|/(|mean|+sd) {np.max(dm / (np.abs(mr) + np.sqrt(vr))):.2e}, "
          f"max |dvar|/var {np.max(dv / vr):.2e}")
    assert np.all(dm <= 1e-4 * (np.abs(mr) + np.sqrt(vr))), label
    assert np.all(dv <= 1e-3 * vr), label


def test_mc_matches_oracle_and_graph_replays(ctx):
    n, nc, R, seed = 16, 8, 12, 9
    b, h, ncand = tiny_bins(ctx, n, nc, 5, 5.5)
    desc = bs.field_desc(n, nc, bs.BS_K_CUBIC)
    mg = me = None
    try:
        mg = bs.bs_mc_create(ctx, h, desc, bs.BS_FP32)
        bs.bs_mc_run(mg, seed, 0, 5, use_graph=True)
        bs.bs_mc_run(mg, seed, 5, 7, use_graph=True)       # replays of the same captured graph
        cg, mug, vg = bs.bs_mc_stats(mg, ncand)
        Bl, Nl = bs.bs_mc_last(mg, ncand)
        me = bs.bs_mc_create(ctx, h, desc, bs.BS_FP32)
        bs.bs_mc_run(me, seed, 0, R, use_graph=False)
        ce, mue, ve = bs.bs_mc_stats(me, ncand)
    finally:
        for m in (mg, me):
            if m:
                bs.bs_mc_destroy(m)
        bs.bs_free_bins(h)
    # graph replays and direct launches run the same deterministic kernels
    assert np.array_equal(cg, ce)
    assert np.array_equal(mug, mue, equal_nan=True) and np.array_equal(vg, ve, equal_nan=True)
    Bs, last = oracle_mc(b, n, nc, seed, R)
    assert np.array_equal(Nl, last[1])
    compare_B(Bl, last[0], last[1], last_scale(b, last), 1e-5, "mc last realization")
    check_stats(cg, mug, vg, Bs, R, "mc fp32")


def test_mc_flagged_split_and_reset(ctx):
    n, nc, R, seed = 32, 24, 6, 21
    b, h, ncand = tiny_bins(ctx, n, nc, 6, 10.0)
    cw = synth.mwa_flags(nc, (0, 11, 23))
    uvm = synth.disk_mask(n)
    desc = bs.field_desc(n, nc, bs.BS_K_CUBIC)
    m = None
    try:
        m = bs.bs_mc_create(ctx, h, desc, bs.BS_SPLIT_BF16, uv_mask=cuda(uvm), chan_w=cuda(cw, np.float32))
        bs.bs_mc_run(m, 77, 0, 3)                          # discarded by the reset
        bs.bs_mc_reset(m)
        bs.bs_mc_run(m, seed, 0, R)
        c, mu, v = bs.bs_mc_stats(m, ncand)
    finally:
        if m:
            bs.bs_mc_destroy(m)
        bs.bs_free_bins(h)
    w = oe.Weights(uv_mask=uvm, chan_w=cw)
    Bs, _ = oracle_mc(b, n, nc, seed, R, w=w, cw=cw)
    check_stats(c, mu, v, Bs, R, "mc split flagged")


def test_mc_rejects_mismatched_sizes(ctx):
    _, h, _ = tiny_bins(ctx, 16, 8, 5, 5.5)
    try:
        with pytest.raises(bs.BsError):
            bs.bs_mc_create(ctx, h, bs.field_desc(32, 8, bs.BS_K_CUBIC), bs.BS_FP32)
        with pytest.raises(bs.BsError):
            bs.bs_mc_create(ctx, h, bs.field_desc(16, 8, bs.BS_K_CUBIC), bs.BS_FP64)
    finally:
        bs.bs_free_bins(h)
    V = torch.empty((8, 18, 10), dtype=torch.complex64, device="cuda")
    with pytest.raises(bs.BsError):
        bs.bs_generate_cube(ctx, bs.field_desc(18, 8, bs.BS_K_CUBIC), 1, 0, V)   # n % 4 != 0


def test_mc_fused_path_flagged(ctx):
    """nc = 128: the estimate inside the Monte Carlo graph uses the fused eta-C2R contraction."""
    n, nc, R, seed = 32, 128, 4, 3
    b, h, ncand = tiny_bins(ctx, n, nc, 6, 10.0)
    cw = synth.mwa_flags(nc, (0, 16, 31))
    desc = bs.field_desc(n, nc, bs.BS_K_CUBIC)
    m = None
    try:
        m = bs.bs_mc_create(ctx, h, desc, bs.BS_FP32, chan_w=cuda(cw, np.float32))
        bs.bs_mc_run(m, seed, 0, R)
        c, mu, v = bs.bs_mc_stats(m, ncand)
    finally:
        if m:
            bs.bs_mc_destroy(m)
        bs.bs_free_bins(h)
    Bs, _ = oracle_mc(b, n, nc, seed, R, w=oe.Weights(chan_w=cw), cw=cw)
    check_stats(c, mu, v, Bs, R, "mc fused flagged")
