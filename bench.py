#!/usr/bin/env python3
"""Benchmark: 3D bispectrum of an MWA-shaped cube on one MI355X.

Workload (the metric's configuration): 256 x 256 uv x 768 channels of 40 kHz (30.72 MHz
band), quadratic non-Gaussian field delta = g + 0.5 (g^2 - <g^2>) with P(k) ~ k^-2,
20 log |k| shells over 0.003 - 1.258 Mpc^-1 and every candidate triangle k1 >= k2 >= k3
(483).  One step = one bs_estimate_3d call on a cube already resident in HBM: delay
transform, shell-filtered 3D inverse transforms, the triple-product contraction and the
normalisation (triangle counts depend only on the geometry and are cached after the
first call).  The metric counts one product per valid triangle per voxel of the cube
(`value`); the contraction itself runs on the exact 384-point delay grid, and the products it
forms there are reported as `value_formed`.  `cpu_baseline` is the FP64 oracle on the whole step
on up to 16 host threads (its single-thread figure on a bounded sample beside it).

Also reported on the same cube: the plain FP32 path of the same step, and the MABS
contraction on MFMA for 133 ring triples x 8 nu1 rows (768 x 768 x 65536 GEMMs); the 2D DFT of
Eq. (dft) on a collapsed MABS of 133 triples and its monopole; Eq. (vg) gridding of 262,144
baselines x 768 channels; Monte Carlo, batch and surrogate blocks.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-mabs] [--no-mabs-dft] [--no-grid]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_MFMA_PEAK_TFLOPS = 157.3
# HBM bytes per launch of the dominant kernel from the rocprofv3 FETCH_SIZE / WRITE_SIZE passes
# (calibrated by a 1 GiB copy: FETCH_SIZE x 2, WRITE_SIZE x 1), kept with the kernel version they
# were taken on; None once that kernel changes until the counters are taken again.
TRAFFIC_BYTES = {"k3_dft": (269.0 + 71.3) * 1e6,   # profiles/k3_dft_split_3d_256x256x768.md
                 "mdft": (1805.9 + 629.2 + 630.1 + 1255.2) * 1e6,   # profiles/mdft_fp64_133x1535x1535_nc768.md
                 "mono": (73.0 + 7.4) * 1e6,   # profiles/mono_multi_bin_133x768x768_k1x12.md
                 "multi": (73.1 + 19.1) * 1e6,   # the same
                 "kpar": (78.1 + 3.4) * 1e6,   # the same
                 "grid": (0.0 + 126.8 + 1675.0 + 1213.4 + 123.9 + 8.3 + 126.8 + 76.1) * 1e6}   # profiles/grid_262144x768_to_192x256x129.md


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-mabs", action="store_true")
    p.add_argument("--no-fp32", action="store_true")
    p.add_argument("--no-mabs-dft", action="store_true")
    p.add_argument("--no-mabs-fp32", action="store_true", help="MABS block in split-BF16 only")
    p.add_argument("--no-grid", action="store_true")
    p.add_argument("--no-mc", action="store_true")
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--no-surrogate", action="store_true")
    p.add_argument("--full-mabs", action="store_true",
                   help="only time the full MABS of the cube (all 133 ring triples x all 768^3 channel triples, "
                        "ergodic collapse), unflagged and flagged, once each, and print that JSON line")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device-to-device copy (counter calibration) and exit")
    return p.parse_args()


def copy_calibration(torch):
    """A copy kernel of known size: 1 GiB read + 1 GiB written per launch, three launches."""
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": 2 * a.numel() * 4, "launches": 3}))


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def host_cpu_info():
    """Cores this process may use and the CPU model (lscpu / /proc/cpuinfo)."""
    info = {"nproc_affinity": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return info


def cpu_baseline_allcore(w, V, edges, gpu_B, gpu_T, threads):
    """The FP64 oracle on the whole step of the same workload, its independent pieces run on
    `threads` host threads (NumPy's FFTs and elementwise products release the GIL): the delay
    transform, the 20 shell fields (one task per shell) and the triple sums of every candidate
    triangle (one task per triangle).  Counts are excluded as on the GPU (cached per geometry):
    B = N_vox S_D / T3D with the GPU's T3D, checked against the GPU's B."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import bins as ob
    from oracle import estimator as oe
    b = ob.make_bins(ob.SHELL_K, w.n, w.nc, edges, du=w.du, r_mpc=w.r_mpc, rprime=w.rprime, dnu=w.dnu)
    Vh = V.astype(np.complex128)
    t0 = time.perf_counter()
    sf = oe.ShellFields(b, Vh)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(sf.data, range(b.nbins)))
        S = np.array(list(ex.map(lambda t: float(np.sum(sf.data(t[0]) * sf.data(t[1]) * sf.data(t[2]))), b.triangles)))
    dt = time.perf_counter() - t0
    nvox = w.nc * w.n * w.n
    ok = gpu_T > 0
    Bref = np.where(ok, nvox * S / np.maximum(gpu_T, 1), np.nan)
    err = np.abs(gpu_B[ok] - Bref[ok]) / np.abs(Bref[ok])
    del sf
    return {"value": int(ok.sum()) * nvox / dt, "unit": "products/s", "cores": threads, "kind": "oracle",
            "seconds": dt,
            "sample": (f"the whole step: float64 NumPy oracle, delay transform, 20 shell fields and all {len(b.triangles)} "
                       f"candidate triangle sums on {threads} threads, counts excluded as on the GPU"),
            "median_rel_err_vs_gpu": float(np.median(err)), "host": host_cpu_info()}


def cpu_baseline(w, V, edges, gpu_B, tri_all):
    """The FP64 oracle on a bounded sample of the same workload: the delay transform, the
    fields of the six largest shells and every candidate triangle among them.  The full-
    workload time is extrapolated from the per-field and per-triangle times."""
    import threading
    from oracle import bins as ob
    from oracle import estimator as oe
    b = ob.make_bins(ob.SHELL_K, w.n, w.nc, edges, du=w.du, r_mpc=w.r_mpc, rprime=w.rprime, dnu=w.dnu)
    t0 = time.perf_counter()
    sf = oe.ShellFields(b, V.astype(np.complex128))
    t_delay = time.perf_counter() - t0
    shells = [14, 15, 16, 17, 18, 19]
    t0 = time.perf_counter()
    for j in shells:
        sf.data(j)
    t_field = (time.perf_counter() - t0) / len(shells)
    sel = [i for i, t in enumerate(b.triangles) if all(x in shells for x in t)]
    t0 = time.perf_counter()
    S = np.array([np.sum(sf.data(b.triangles[i][0]) * sf.data(b.triangles[i][1]) * sf.data(b.triangles[i][2]))
                  for i in sel])
    t_tri = (time.perf_counter() - t0) / max(len(sel), 1)
    for j in shells:
        sf.count(j)
    SI = np.array([np.sum(sf.count(b.triangles[i][0]) * sf.count(b.triangles[i][1]) * sf.count(b.triangles[i][2]))
                   for i in sel])
    nvox = w.nc * w.n * w.n
    T = np.rint(float(nvox) ** 2 * SI)
    Bref = np.where(T > 0, nvox * S / np.maximum(T, 1), np.nan)
    err = np.abs(gpu_B[sel] - Bref) / np.abs(Bref)
    n_valid = int(np.count_nonzero(T)) if len(sel) else 0
    t_full = t_delay + 20 * t_field + len(tri_all) * t_tri
    products_full = len(tri_all) * nvox
    return {
        "value": products_full / t_full,
        "unit": "products/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"float64 NumPy oracle (single thread) on the same cube: delay transform ({t_delay:.1f} s), "
                   f"{len(shells)} of 20 shell fields ({t_field:.1f} s each), {len(sel)} of {len(tri_all)} triangles "
                   f"({t_tri:.2f} s each); full step extrapolated as delay + 20 fields + all triangles "
                   f"= {t_full:.0f} s, counts excluded as on the GPU"),
        "max_rel_err_vs_gpu_on_sample": float(np.nanmax(err)) if len(sel) else None,
        "sample_valid_triangles": n_valid,
    }


def mabs_dft_block(bs, ctx, w, torch, nt=133):
    """Eq. (dft) on a collapsed MABS of the cube's shape: nt = 133 ring triples (as in the MABS
    block), nc = 768, the non-circular collapse [133][1535][1535] in HBM (seeded standard normal
    values, NaN where no channel triplet exists, |d2 - d1| >= nc), scaled by (r^2 r' dnu_c)^2.
    HBM-bound: the algorithmic bytes per launch are the window read once (nc^2 float64 per
    triangle: one period of separations) and the output written once (nc^2 complex128 per
    triangle); the half spectra the two
    passes exchange (nc (nc/2 + 1) complex128 per triangle, written and read once) are counted
    apart.  The oracle's time for the same transform on two triangles is reported beside it."""
    from oracle import estimator as oe
    nc = w.nc
    size = 2 * nc - 1
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    Bd = torch.randn((nt, size, size), dtype=torch.float64, device="cuda", generator=g)
    d = torch.arange(size, device="cuda") - (nc - 1)
    Bd[:, (d[None, :] - d[:, None]).abs() >= nc] = float("nan")
    out = torch.empty((nt, nc, nc), dtype=torch.complex128, device="cuda")
    scale = (w.r_mpc ** 2 * w.rprime * w.dnu) ** 2
    f = lambda: bs.bs_mabs_dft(ctx, nc, Bd, out, scale=scale)
    f()
    torch.cuda.synchronize()
    pn, pm, tot = [], [], []
    for _ in range(5):
        f()
        tm = bs.bs_last_timing(ctx)
        tot.append(tm[0])
        pm.append(tm[1])
        pn.append(tm[2])
    t_wall = time_steps(f, 5, 0, torch)
    ms_n, ms_m, ms = float(np.median(pn)), float(np.median(pm)), float(np.median(tot))
    win = nt * nc * nc * 8
    outb = nt * nc * nc * 16
    half = nt * nc * (nc // 2 + 1) * 16
    alg = win + outb
    ach = alg / ((ms_n + ms_m) * 1e-3) / 1e9
    # the oracle on two triangles, checked against the GPU output
    t0 = time.perf_counter()
    errs = []
    for t in (0, nt - 1):
        ref = oe.mabs_dft(Bd[t:t + 1].cpu().numpy(), scale)
        got = out[t:t + 1].cpu().numpy()
        errs.append(float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    t_cpu = (time.perf_counter() - t0) / 2
    mono = monopole_block(bs, ctx, w, torch, out)
    return {
        "value": nt / t_wall, "unit": "triangles/s", "ms_per_call": t_wall * 1e3, "kernels_ms": ms,
        "pass_n_ms": ms_n, "pass_m_ms": ms_m,
        "pass_n_GBps_moved": (win + half) / (ms_n * 1e-3) / 1e9,
        "pass_m_GBps_moved": (half + outb) / (ms_m * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "kernel": "k_mdft_n + k_mdft_m (Eq. dft, FP64)", "achieved": ach,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": alg, "half_spectrum_bytes_exchanged": 2 * half,
                     "traffic": TRAFFIC_BYTES.get("mdft")},
        "max_rel_err_vs_oracle_2_triangles": max(errs),
        "cpu_oracle": {"value": 1.0 / t_cpu, "unit": "triangles/s", "cores": 1, "kind": "oracle",
                       "sample": "2 of 133 triangles, float64 NumPy, the literal sum as two matrix products"},
        "workload": f"{nt} triangles x collapsed MABS [{size}][{size}] (nc = {nc}) -> [{nc}][{nc}] complex128",
        "monopole": mono,
    }


def monopole_block(bs, ctx, w, torch, Bcyl):
    """Monopole B(k1, mu, t) of the cylindrical BS just computed: the 133 ring triples of the
    cube's rings (k_perp at the geometric centres of the ring edges), k_par unit 2 pi / (r' B_bw),
    12 log k1 bins over 0.003-1.258 Mpc^-1 x 5 mu x 5 t.  Only the cells inside the k1 edges are
    read: the algorithmic bytes are 16 B (one complex128 entry) per binned cell, and the rate over
    the whole cube (what a kernel that reads every cell must move) is reported beside it.  The
    oracle on two triangles beside it."""
    from oracle import estimator as oe
    redges = w.shell_edges(20)
    h, ncand = bs.bs_make_bins(None, bs.BS_RING_U, w.n, w.nc, redges / (2 * np.pi * w.du / w.r_mpc))
    tri, _ = bs.bs_bins_triangles(h, ncand, 20)
    bs.bs_free_bins(h)
    kperp = np.sqrt(redges[:-1] * redges[1:])[np.asarray(tri).reshape(-1, 3)]
    nt, nc = int(Bcyl.shape[0]), int(Bcyl.shape[1])
    assert kperp.shape[0] == nt
    unit = 2 * np.pi / (w.rprime * w.dnu * w.nc)
    edges = np.geomspace(0.003, 1.258, 13)
    mean = torch.empty((12, 5, 5), dtype=torch.float64, device="cuda")
    cnt = torch.empty((12, 5, 5), dtype=torch.int64, device="cuda")
    f = lambda: bs.bs_monopole(ctx, Bcyl, kperp, unit, edges, mean, cnt)
    f()
    kb, kr = [], []
    for _ in range(5):
        f()
        tm = bs.bs_last_timing(ctx)
        kb.append(tm[1])
        kr.append(tm[2])
    t_wall = time_steps(f, 5, 0, torch)
    ms_b = float(np.median(kb))
    gc = cnt.cpu().numpy()
    cube = nt * nc * nc * 16
    byt = int(gc.sum()) * 16
    ach = byt / (ms_b * 1e-3) / 1e9
    t0 = time.perf_counter()
    Bh = Bcyl[:2].cpu().numpy()
    ref_m, ref_c = oe.bs_monopole(Bh, kperp[:2], unit, edges)
    t_cpu = (time.perf_counter() - t0) / 2
    # multipole moments l <= 4 (15 moments) of the same cells and bins
    mom = torch.empty((15, 12, 5, 5), dtype=torch.float64, device="cuda")
    cnt2 = torch.empty((12, 5, 5), dtype=torch.int64, device="cuda")
    g = lambda: bs.bs_multipoles(ctx, Bcyl, kperp, unit, edges, 4, mom, cnt2)
    g()
    mb = []
    for _ in range(5):
        g()
        mb.append(bs.bs_last_timing(ctx)[1])
    tm_wall = time_steps(g, 5, 0, torch)
    ms_m = float(np.median(mb))
    ach_m = byt / (ms_m * 1e-3) / 1e9
    t0 = time.perf_counter()
    oe.bs_multipoles(Bh[:1], kperp[:1], unit, edges, 4)
    t_cpu_m = time.perf_counter() - t0
    multipoles = {
        "value": nt / tm_wall, "unit": "triangles/s", "ms_per_call": tm_wall * 1e3, "bin_kernel_ms": ms_m,
        "moments": "l = 0..4, m = 0..l (15)", "counts_equal_monopole": bool(np.array_equal(cnt2.cpu().numpy(), gc)),
        "roofline": {"bound": "hbm", "kernel": "k_multi_bin", "achieved": ach_m, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach_m / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": byt,
                     "traffic": TRAFFIC_BYTES.get("multi")},
        "whole_cube_rate_GBps": cube / (ms_m * 1e-3) / 1e9,
        "cpu_oracle": {"value": 1.0 / t_cpu_m, "unit": "triangles/s", "cores": 1, "kind": "oracle",
                       "sample": "1 of 133 triangles, float64 NumPy with scipy Y_l^m"},
    }
    # the (k_par1, k_par2) grid of Fig. 4: 20 x 20 linear bins over +-1.149 Mpc^-1 per ring triple
    kedges = np.linspace(-1.149, 1.149, 21)
    kmean = torch.empty((nt, 20, 20), dtype=torch.float64, device="cuda")
    kcnt = torch.empty((20, 20), dtype=torch.int64, device="cuda")
    q = lambda: bs.bs_kpar_grid(ctx, Bcyl, unit, kedges, kmean, kcnt)
    q()
    kb2 = []
    for _ in range(5):
        q()
        kb2.append(bs.bs_last_timing(ctx)[1])
    tk_wall = time_steps(q, 5, 0, torch)
    ms_k = float(np.median(kb2))
    kc = kcnt.cpu().numpy()
    byt_k = nt * int(kc.sum()) * 16
    t0 = time.perf_counter()
    rk_m, rk_c = oe.bs_kpar_grid(Bh, unit, kedges)
    t_cpu_k = (time.perf_counter() - t0) / 2
    kpar_grid = {
        "value": nt / tk_wall, "unit": "triangles/s", "ms_per_call": tk_wall * 1e3, "bin_kernel_ms": ms_k,
        "grid": "20 x 20 linear k_par bins over +-1.149 Mpc^-1", "counts_equal_oracle": bool(np.array_equal(kc, rk_c)),
        "max_rel_err_vs_oracle_2_triangles": float(np.nanmax(np.abs(kmean[:2].cpu().numpy() - rk_m) /
                                                             np.maximum(np.abs(rk_m), 1e-300))),
        "roofline": {"bound": "hbm", "kernel": "k_kpar_bin", "achieved": byt_k / (ms_k * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": byt_k / (ms_k * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": byt_k, "traffic": TRAFFIC_BYTES.get("kpar")},
        "cpu_oracle": {"value": 1.0 / t_cpu_k, "unit": "triangles/s", "cores": 1, "kind": "oracle",
                       "sample": "2 of 133 triangles, float64 NumPy"},
    }
    return {
        "multipoles": multipoles,
        "kpar_grid": kpar_grid,
        "value": nt / t_wall, "unit": "triangles/s", "ms_per_call": t_wall * 1e3, "bin_kernel_ms": ms_b,
        "reduce_kernel_ms": float(np.median(kr)), "cells_binned": int(gc.sum()), "bins_filled": int((gc > 0).sum()),
        "roofline": {"bound": "hbm", "kernel": "k_mono_bin", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": byt,
                     "traffic": TRAFFIC_BYTES.get("mono")},
        "whole_cube_bytes": cube, "whole_cube_rate_GBps": cube / (ms_b * 1e-3) / 1e9,
        "cpu_oracle": {"value": 1.0 / t_cpu, "unit": "triangles/s", "cores": 1, "kind": "oracle",
                       "sample": "2 of 133 triangles, float64 NumPy"},
        "workload": f"{nt} triangles x [{nc}][{nc}] cells -> 12 k1 x 5 mu x 5 t bins",
    }


def decorrelation_block(bs, ctx, w, torch, nvis=262144, nodes=12):
    """Eq. (S3): the primary-beam decorrelation factor D of every candidate ring triangle of the
    cube's 20 log rings, for 262,144 seeded baselines (log-uniform radius over 0.5-120 cells, as the
    grid block) gridded with the cube's spacing, theta_0 = 0.6 x 24.68 deg, a 12-point Gauss rule
    per axis (72 nodes after the z -> -z symmetry): per node one phase-mode gridding and one FP64
    MABS of the per-cell phase averages.  The oracle's enumeration over closed grid triangles and
    baseline triplets on a 16^2 grid with 400 baselines and 3 rings (a bounded sample) beside it."""
    import math as _m
    from oracle import beam as obm
    from oracle import bins as ob
    from paper_2506_10526_amd import synth
    theta0 = 0.6 * _m.radians(24.68)
    redges = w.shell_edges(20) / (2 * np.pi * w.du / w.r_mpc)
    h, ncand = bs.bs_make_bins(ctx, bs.BS_RING_U, w.n, 1, redges)
    try:
        uv = synth.uv_tracks(nvis, 31, 0.5 * w.du, 120 * w.du)
        uvd = torch.from_numpy(np.ascontiguousarray(uv, dtype=np.float64)).cuda()
        f = lambda: bs.bs_decorrelation(ctx, h, ncand, uvd, w.du, theta0, nodes)
        D = f()
        t_wall = time_steps(f, 3, 0, torch)
    finally:
        bs.bs_free_bins(h)
    fin = D[np.isfinite(D)]
    # the oracle's enumeration on a small case, as in the parity tests
    small_edges = np.array([1.0, 2.0, 3.2, 5.0])
    sb = ob.make_bins(ob.RING_U, 16, 1, small_edges)
    suv = synth.uv_tracks(400, 5, 0.6 * w.du, 6.5 * w.du)
    t0 = time.perf_counter()
    Dref = obm.decorrelation_factor(sb, suv, w.du, theta0)
    t_cpu = time.perf_counter() - t0
    return {
        "value": ncand / t_wall, "unit": "ring triangles/s", "ms_per_call": t_wall * 1e3, "triangles": int(ncand),
        "baselines": int(nvis), "gauss_nodes": f"{nodes} per axis, {nodes * nodes // 2} after the z -> -z symmetry",
        "D_finite": int(fin.size), "D_min": float(fin.min()) if fin.size else None,
        "D_median": float(np.median(fin)) if fin.size else None,
        "cpu_oracle": {"value": int(np.isfinite(Dref).sum()) / t_cpu, "unit": "ring triangles/s", "cores": 1,
                       "kind": "oracle", "sample": "16^2 grid, 400 baselines, 3 rings: enumeration over closed grid "
                                                   "triangles and baseline triplets"},
        "workload": f"{ncand} ring triangles of the {w.n}^2 grid, {nvis} baselines",
    }


def grid_block(bs, ctx, w, torch, nvis=262144):
    """Eq. (vg) gridding of the cube's shape: 262,144 seeded baselines (log-uniform radius over
    0.5-120 cells, uniform angle) x 768 channels of complex64 visibilities in HBM, the periodic
    channel flags plus 1 % random RFI flags, onto the 256 x 256 half-plane grid, four channels
    collapsed into one (Sec. 4), complex64 output.  HBM-bound: the algorithmic bytes are the
    visibilities (8 B) and flags (1 B) read once and the gridded cube and counts (12 B a cell)
    written once.  The oracle on 24 of the 768 channels beside it."""
    from oracle import estimator as oe
    from paper_2506_10526_amd import synth
    n, nc, avg = w.n, w.nc, 4
    uv = synth.uv_tracks(nvis, 31, 0.5 * w.du, 120 * w.du)
    flags = synth.rfi_flags(nc, nvis, 32, 0.01, synth.mwa_flags(nc))
    g = torch.Generator(device="cuda")
    g.manual_seed(33)
    vd = torch.randn((nc, nvis), dtype=torch.complex64, device="cuda", generator=g)
    uvd = torch.from_numpy(uv).cuda()
    fd = torch.from_numpy(flags).cuda()
    shp = (nc // avg, n, n // 2 + 1)
    Vg = torch.empty(shp, dtype=torch.complex64, device="cuda")
    Ng = torch.empty(shp, dtype=torch.int32, device="cuda")
    f = lambda: bs.bs_grid_visibilities(ctx, n, w.du, uvd, vd, Vg, Ng, flags=fd, chan_avg=avg)
    f()
    torch.cuda.synchronize()
    ks, kf, tot = [], [], []
    for _ in range(5):
        f()
        tm = bs.bs_last_timing(ctx)
        tot.append(tm[0])
        ks.append(tm[1])
        kf.append(tm[2])
    t_wall = time_steps(f, 5, 0, torch)
    ms_s, ms_f, ms = float(np.median(ks)), float(np.median(kf)), float(np.median(tot))
    cells = shp[0] * n * (n // 2 + 1)
    alg = nc * nvis * 9 + cells * 12
    ach = alg / (ms * 1e-3) / 1e9
    t0 = time.perf_counter()
    sub = 24
    rV, rN = oe.grid_visibilities(uv, vd[:sub].cpu().numpy().astype(np.complex128), flags[:sub], n, w.du, avg)
    t_cpu = (time.perf_counter() - t0) * nc / sub
    counts_ok = bool(np.array_equal(Ng[:sub // avg].cpu().numpy(), rN))
    return {
        "value": nc * nvis / t_wall, "unit": "visibility samples/s", "ms_per_call": t_wall * 1e3,
        "kernels_ms": ms, "scatter_ms": ms_s, "output_ms": ms_f,
        "roofline": {"bound": "hbm", "kernel": "k_grid_zero + k_grid_scatter + k_grid_hot + k_grid_fin", "achieved": ach,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": alg, "traffic": TRAFFIC_BYTES.get("grid")},
        "counts_match_oracle_on_24_channels": counts_ok,
        "cpu_oracle": {"value": nc * nvis / t_cpu, "unit": "visibility samples/s", "cores": 1, "kind": "oracle",
                       "sample": f"{sub} of {nc} channels, float64 NumPy, scaled to all channels"},
        "workload": f"{nvis} baselines x {nc} channels -> {shp[0]} x {n} x {n // 2 + 1} cells (4:1 channel collapse)",
    }


def mc_block(bs, ctx, bins, ncand, w, torch, R=64):
    """Monte Carlo of the flagged cube (channels {0,16,31} of every 32): generator + 3D estimate
    + FP64 accumulators per realization, replayed from one captured graph."""
    from paper_2506_10526_amd import synth
    desc = bs.field_desc(w.n, w.nc, bs.BS_K_PHYSICAL, du_lambda=w.du, r_mpc=w.r_mpc,
                         rprime_mpc_per_mhz=w.rprime, dnu_mhz=w.dnu)
    cw = torch.from_numpy(synth.mwa_flags(w.nc, (0, 16, 31)).astype(np.float32)).cuda()
    m = bs.bs_mc_create(ctx, bins, desc, bs.BS_SPLIT_BF16, chan_w=cw)
    try:
        bs.bs_mc_run(m, 7, 0, 2)
        bs.bs_mc_reset(m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bs.bs_mc_run(m, 7, 2, R)
        c, mu, v = bs.bs_mc_stats(m, ncand)
        dt = time.perf_counter() - t0
    finally:
        bs.bs_mc_destroy(m)
    nval = int(np.count_nonzero(c))
    return {"workload": "flagged 256x256x768 cube (channels {0,16,31} mod 32), split-BF16, one hipGraph per realization",
            "realizations": R, "seconds": dt, "ms_per_realization": dt / R * 1e3,
            "products_per_s": nval * w.nc * w.n * w.n * R / dt, "valid_triangles": nval}


def batch_block(bs, ctx, torch, ncubes=64, seed=4):
    """64 seeded cubes of uneven size (n in {128,192,256}, nc in {384,576,768}), 8 log rings, all
    candidate triangles, a seeded subset of 32 nu1 channels with all (nu2, nu3), split-BF16; one
    hipGraph launch for the whole batch (per wave, one persistent contraction launch per tile shape
    in use); tile shapes and pixel chunks per cube shape class from the library's autotuner."""
    rng = np.random.default_rng(seed)
    cubes = []
    for i in range(ncubes):
        n = int(rng.choice([128, 192, 256]))
        nc = int(rng.choice([384, 576, 768]))
        nu1 = sorted(int(x) for x in rng.choice(nc, size=32, replace=False))
        cubes.append((n, nc, 1000 + i, i, nu1))
    desc = bs.field_desc(128, 384, bs.BS_K_CUBIC)
    t0 = time.perf_counter()
    h = bs.bs_batch_create(ctx, cubes, 8, desc, 48.0)
    t_create = time.perf_counter() - t0
    try:
        info = [bs.bs_batch_info(h, i) for i in range(ncubes)]
        tiles = {}
        for i, c in enumerate(cubes):
            tm, tn, m1, k = bs.bs_batch_tile(h, i)
            tiles[f"n={c[0]} nc={c[1]}"] = f"{tm}x{tn}" + (f" rows {m1}x{256 // m1}" if m1 else "") + f", {k} chunk(s)"
        bs.bs_batch_run(h)          # warm-up launch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bs.bs_batch_run(h)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        bs.bs_batch_destroy(h)
    products = sum(x[3] for x in info)
    cand = sum(x[0] * 32 * c[1] * c[1] * c[0] * c[0] for x, c in zip(info, cubes))
    flops = 6.0 * cand
    return {"workload": "64 seeded cubes, n in {128,192,256}, nc in {384,576,768}, 8 log rings, 32 seeded nu1 "
                        "x all (nu2, nu3), split-BF16, ergodic collapse over the nu1 subset",
            "seconds_per_launch": dt, "products": products, "products_per_s": products / dt,
            "mfma_tflops_incl_generation_and_fields": flops / dt / 1e12,
            "waves": 1 + max(x[1] for x in info), "tiles_per_class": dict(sorted(tiles.items())),
            "create_seconds_incl_autotuning": t_create}


def surrogate_block(bs, ctx, bins, ncand, w, torch):
    """Labels (7 flag patterns x 1024 realizations), GPU training with the per-triangle flag summary,
    evaluation against 4096 fresh realizations of config 3's pattern and of two unseen patterns;
    next to 200-realization Monte Carlo and the noise floor of the references."""
    from paper_2506_10526_amd import surrogate, synth
    desc = bs.field_desc(w.n, w.nc, bs.BS_K_PHYSICAL, du_lambda=w.du, r_mpc=w.r_mpc,
                         rprime_mpc_per_mhz=w.rprime, dnu_mhz=w.dnu)
    V = torch.empty((w.nc, w.n, w.nh), dtype=torch.complex64, device="cuda")
    bs.bs_generate_cube(ctx, desc, 1, 0, V)
    B = torch.empty(ncand, dtype=torch.float64, device="cuda")
    N = torch.empty(ncand, dtype=torch.int64, device="cuda")
    bs.bs_estimate_3d(ctx, bins, V, bs.BS_SPLIT_BF16, B, N)
    T3D = N.cpu().numpy()
    pats = dict(surrogate.TRAIN_PATTERNS, **surrogate.UNSEEN_PATTERNS)
    flags = {k: (synth.mwa_flags(w.nc, v) if v else np.ones(w.nc)) for k, v in pats.items()}
    t0 = time.perf_counter()
    ff = surrogate.FlagFeatures(ctx, bins, ncand, T3D, -2.0)
    names = list(surrogate.TRAIN_PATTERNS)
    train = [surrogate.mc_run(ctx, bins, ncand, desc, flags[k], 1024, 100 + i) for i, k in enumerate(names)]
    X, tgt = surrogate.training_set_flag(ff, train, [flags[k] for k in names])
    t_feat = time.perf_counter() - t0 - sum(r.seconds for r in train)
    sur = surrogate.Surrogate(ctx, seed=1)
    try:
        fit = sur.fit(X, tgt, steps=16000, lr=3e-3, cosine=True)
        ref = {k: surrogate.mc_run(ctx, bins, ncand, desc, flags[k], 4096, 5000 + i)
               for i, k in enumerate(("e1", "spread4", "e3"))}
        ref1b = surrogate.mc_run(ctx, bins, ncand, desc, flags["e1"], 4096, 7777)
        m200 = surrogate.mc_run(ctx, bins, ncand, desc, flags["e1"], 200, 3200)
        t0 = time.perf_counter()
        p = {k: surrogate.predict_var_flag(sur, ff, flags[k], bf16=True) for k in ref}
        t_pred = (time.perf_counter() - t0) / len(ref)
    finally:
        sur.close()

    def err(pv, rv):
        ok = np.isfinite(rv) & (rv > 0) & np.isfinite(pv)
        e = np.abs(pv[ok] - rv[ok]) / rv[ok]
        return {"median": float(np.median(e)), "p90": float(np.percentile(e, 90))}
    return {"labels": f"{len(names)} flag patterns ({', '.join(names)}) x 1024 realizations",
            "label_seconds": sum(r.seconds for r in train), "flag_features_seconds": t_feat,
            "train_steps": fit["steps"], "train_seconds": fit["seconds"],
            "predict_ms_bf16_incl_flag_features": t_pred * 1e3,
            "rel_err_vs_mc4096_config3_pattern": err(p["e1"], ref["e1"].var),
            "rel_err_vs_mc4096_unseen_spread4": err(p["spread4"], ref["spread4"].var),
            "rel_err_vs_mc4096_unseen_e3": err(p["e3"], ref["e3"].var),
            "rel_err_mc200_vs_mc4096": err(m200.var, ref["e1"].var), "mc200_seconds": m200.seconds,
            "reference_noise_floor_mc4096_vs_mc4096": err(ref1b.var, ref["e1"].var)}


def full_mabs(bs, ctx, w, Vd, torch):
    """The paper's own workload on the cube (Sec. 6: every combination of three rings and three
    channels): all 133 valid ring triples x all 768^3 channel triples, split-BF16 contraction,
    collapsed to (d1, d2) (non-circular, Sec. 3.2), once unflagged and once with channels
    {0, 16, 31} of every 32 flagged (the counts then carry w1 w2 w3 and N_nu, Sec. 5 / Fig. 2)."""
    from paper_2506_10526_amd import synth
    redges = w.shell_edges(20) / (2 * np.pi * w.du / w.r_mpc)
    rb, rcand = bs.bs_make_bins(ctx, bs.BS_RING_U, w.n, w.nc, redges)
    D = 2 * w.nc - 1
    B = torch.empty((rcand, D, D), dtype=torch.float64, device="cuda")
    N = torch.empty((rcand, D, D), dtype=torch.int64, device="cuda")
    Nn = torch.empty((rcand, D, D), dtype=torch.int32, device="cuda")
    out = {"workload": f"{rcand} ring triples x all {w.nc}^3 channel triples of the {w.n}^2 x {w.nc} cube, split-BF16, "
                       "ergodic collapse to (d1, d2)"}
    for name, cw in (("unflagged", None), ("flagged", synth.mwa_flags(w.nc, (0, 16, 31)))):
        kw = {} if cw is None else {"chan_w": torch.from_numpy(cw.astype(np.float32)).cuda()}
        bs.bs_set_timing(ctx, True)
        torch.cuda.synchronize()
        log(f"[bench] full MABS {name}: {rcand} triples x {w.nc}^3 channel triples")
        t0 = time.perf_counter()
        bs.bs_estimate_mabs(ctx, rb, Vd, bs.BS_SPLIT_BF16, B, N, Nn, collapse=1, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tm = bs.bs_last_timing(ctx)
        tperp_valid = int((N.view(rcand, -1) > 0).any(dim=1).sum().item())
        prods = tperp_valid * float(w.nc) ** 3 * w.n * w.n
        flops = 6.0 * rcand * float(w.nc) ** 3 * w.n * w.n
        out[name] = {"seconds": dt, "contraction_s": tm[1] * 1e-3, "products": prods, "products_per_s": prods / dt,
                     "mfma_TFLOPs_contraction": flops / (tm[1] * 1e-3) / 1e12,
                     "frac_of_bf16_peak": flops / (tm[1] * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                     "valid_triples": tperp_valid}
        log(f"[bench] full MABS {name}: {dt:.2f} s, contraction {tm[1] * 1e-3:.2f} s, "
            f"{out[name]['mfma_TFLOPs_contraction']:.0f} TFLOP/s")
    bs.bs_free_bins(rb)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the library runs on one GPU; sharding over several is not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2506_10526_amd import bs, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration(torch)
        return
    dev = torch.device("cuda:0")
    w = synth.config2()
    edges = w.shell_edges(20)
    log(f"[bench] generating the {w.n}x{w.n}x{w.nc} cube on the GPU (seed {args.seed})")
    stream = torch.cuda.current_stream()
    ctx = bs.bs_create(0, stream.cuda_stream)
    # the seeded cube is generated on the GPU (Philox stream; the oracle's generator makes the same cube)
    gdesc = bs.field_desc(w.n, w.nc, bs.BS_K_PHYSICAL, sigma=w.sigma, f_ng=w.f_ng, pk_index=w.pk_index,
                          du_lambda=w.du, r_mpc=w.r_mpc, rprime_mpc_per_mhz=w.rprime, dnu_mhz=w.dnu)
    Vd = torch.empty((w.nc, w.n, w.nh), dtype=torch.complex64, device=dev)
    bs.bs_generate_cube(ctx, gdesc, args.seed, 0, Vd)
    torch.cuda.synchronize()
    if args.full_mabs:
        print(json.dumps(full_mabs(bs, ctx, w, Vd, torch)))
        bs.bs_destroy(ctx)
        return
    bins, ncand = bs.bs_make_bins(ctx, bs.BS_SHELL_K, w.n, w.nc, edges, du_lambda=w.du, r_mpc=w.r_mpc,
                                  rprime_mpc_per_mhz=w.rprime, dnu_mhz=w.dnu)
    tri, modes = bs.bs_bins_triangles(bins, ncand, 20)
    B = torch.empty(ncand, dtype=torch.float64, device=dev)
    N = torch.empty(ncand, dtype=torch.int64, device=dev)
    nvox = w.nc * w.n * w.n
    bs.bs_set_timing(ctx, True)

    def step(prec):
        return lambda: bs.bs_estimate_3d(ctx, bins, Vd, prec, B, N)

    log("[bench] 3D split-BF16: warmup + timed steps")
    # the timed steps run without the library's kernel events; one more step with them gives the
    # per-kernel times
    bs.bs_set_timing(ctx, False)
    t_split = time_steps(step(bs.BS_SPLIT_BF16), args.steps, args.warmup, torch)
    bs.bs_set_timing(ctx, True)
    step(bs.BS_SPLIT_BF16)()
    tim_split = bs.bs_last_timing(ctx)
    Bs = B.cpu().numpy().copy()
    Nt = N.cpu().numpy().copy()
    count_dev = bs.bs_last_count_dev(ctx)
    count_bound = bs.bs_last_count_bound(ctx)
    log(f"[bench] triangle counts: max |x - rint(x)| = {count_dev:.3e}, max count {Nt.max():.3e}")
    n_valid = int(np.count_nonzero(Nt))
    products = n_valid * nvox
    log(f"[bench] split: {t_split * 1e3:.3f} ms/step, kernels total {tim_split[0]:.3f} contraction {tim_split[1]:.3f} "
        f"fields {tim_split[2]:.3f} ms")
    fp32 = None
    if not args.no_fp32:
        log("[bench] 3D FP32: timed steps")
        bs.bs_set_timing(ctx, False)
        t32 = time_steps(step(bs.BS_FP32), max(3, args.steps // 2), 1, torch)
        bs.bs_set_timing(ctx, True)
        step(bs.BS_FP32)()
        tim32 = bs.bs_last_timing(ctx)
        B32 = B.cpu().numpy()
        ok = Nt > 0
        fp32 = {"value": products / t32, "ms_per_step": t32 * 1e3, "contraction_ms": tim32[1],
                "split_over_fp32": t32 / t_split,
                "max_abs_diff_split_vs_fp32_over_max_B": float(np.max(np.abs(Bs[ok] - B32[ok])) / np.max(np.abs(B32[ok])))}
        log(f"[bench] fp32: {t32 * 1e3:.3f} ms/step, contraction {tim32[1]:.3f} ms")
    # Dominant kernel of the split step: k3_dft, the eta synthesis of every shell field as MFMA
    # GEMMs against twiddle fragments, fused with the pair x field contraction on MFMA.  It is
    # priced against the dense bf16 MFMA peak with its algorithmic split-BF16 work per contracted
    # voxel (reported by the library): 3 bf16 products x 2 flops x 2 (H_j + 1) real modes per
    # field for the synthesis, 3 x 2 x P x F for the contraction (P product rows, F fields), on
    # the M n^2 voxels of the M-point delay grid.
    # Dominant kernel of the split step: k3_dft (eta synthesis of every shell field on MFMA fused
    # with the pair x field contraction).  Priced on the unit of the hot-path scope: the shell
    # fields are read once per voxel, F x 4 bytes (FP32) per voxel of the M-point delay grid
    # (F = 20 non-empty shells, 80 B), HBM-bound; beside it the MFMA view at the method's own
    # split-BF16 work (3 bf16 products = 6 flops per valid triangle per voxel) and the dense
    # equivalent the kernel executes (whole 16-mode steps and 16 x 16 tiles).
    M = int(tim_split[3]) or w.nc
    flops_exec = tim_split[4]
    vox_c = int(tim_split[5]) or M * w.n * w.n
    con_ms = tim_split[1]
    fld_ms = tim_split[2]
    nfields = int(np.count_nonzero(modes))
    byt = 4.0 * nfields * vox_c
    ach = byt / (con_ms * 1e-3) / 1e9
    meth_flops = 6.0 * n_valid * vox_c
    roof = {"bound": "hbm", "kernel": "k3_dft (eta synthesis + contraction, split-BF16 MFMA)", "achieved": ach,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": TRAFFIC_BYTES.get("k3_dft"), "algorithmic_bytes_per_voxel": 4.0 * nfields,
            "voxels_per_launch": vox_c, "delay_grid_M": M, "avg_ms": con_ms, "fields_kernels_ms": fld_ms,
            "mfma_view": {"method_flops_per_voxel": 6.0 * n_valid,
                          "achieved_TFLOPs": meth_flops / (con_ms * 1e-3) / 1e12,
                          "frac_of_bf16_peak": meth_flops / (con_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                          "executed_dense_equivalent_flops_per_voxel": float(flops_exec),
                          "executed_TFLOPs": flops_exec * vox_c / (con_ms * 1e-3) / 1e12}}
    mabs = None
    if not args.no_mabs:
        log("[bench] MABS contraction: 133 ring triples x 8 nu1 rows")
        redges = w.shell_edges(20) / (2 * np.pi * w.du / w.r_mpc)
        rb, rcand = bs.bs_make_bins(ctx, bs.BS_RING_U, w.n, w.nc, redges)
        nu1 = list(range(0, w.nc, 96))
        Bm = torch.empty((rcand, len(nu1), w.nc, w.nc), dtype=torch.float64, device=dev)
        Nm = torch.empty((rcand, len(nu1), w.nc, w.nc), dtype=torch.int64, device=dev)
        res = {}
        precs = (("split_bf16", bs.BS_SPLIT_BF16),) + (() if args.no_mabs_fp32 else (("fp32", bs.BS_FP32),))
        for name, prec in precs:
            f = lambda: bs.bs_estimate_mabs(ctx, rb, Vd, prec, Bm, Nm, nu1=nu1)
            tt = time_steps(f, 2, 1, torch)
            tm = bs.bs_last_timing(ctx)
            nval = int(torch.count_nonzero(Nm).item())
            prods = nval * w.n * w.n
            macs = 3 if prec == bs.BS_SPLIT_BF16 else 1
            flops = 2.0 * macs * rcand * len(nu1) * w.nc * w.nc * w.n * w.n
            peak = BF16_PEAK_TFLOPS if prec == bs.BS_SPLIT_BF16 else FP32_MFMA_PEAK_TFLOPS
            ach = flops / (tm[1] * 1e-3) / 1e12
            res[name] = {"value": prods / tt, "unit": "products/s", "ms_per_call": tt * 1e3,
                         "contraction_ms": tm[1], "products": prods,
                         "roofline": {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                                      "frac": ach / peak, "mfma_flops_per_launch": flops}}
            log(f"[bench] mabs {name}: {tt * 1e3:.1f} ms/call, contraction {tm[1]:.1f} ms, {ach:.0f} TFLOP/s")
        if "fp32" in res:
            res["split_over_fp32"] = res["fp32"]["contraction_ms"] / res["split_bf16"]["contraction_ms"]
        res["workload"] = "133 ring triples (10 rings, k_perp of the 20 shells) x nu1 in {0,96,...,672} x all (nu2, nu3)"
        mabs = res
        bs.bs_free_bins(rb)
        del Bm, Nm
    mdft = None
    if not args.no_mabs_dft:
        log("[bench] Eq. (dft): collapsed MABS of 133 triples -> cylindrical 3D BS")
        mdft = mabs_dft_block(bs, ctx, w, torch)
        log(f"[bench] mabs_dft: {mdft['ms_per_call']:.3f} ms/call (pass n {mdft['pass_n_ms']:.3f}, pass m "
            f"{mdft['pass_m_ms']:.3f}), {mdft['roofline']['achieved']:.0f} GB/s algorithmic")
        mo = mdft["monopole"]
        log(f"[bench] monopole: {mo['ms_per_call']:.3f} ms/call (binning {mo['bin_kernel_ms']:.3f} ms, "
            f"{mo['roofline']['achieved']:.0f} GB/s), {mo['cells_binned']} cells in {mo['bins_filled']} bins")
        mp = mo["multipoles"]
        log(f"[bench] multipoles l<=4: {mp['ms_per_call']:.3f} ms/call (binning {mp['bin_kernel_ms']:.3f} ms, "
            f"{mp['roofline']['achieved']:.0f} GB/s)")
        kg = mo["kpar_grid"]
        log(f"[bench] k_par grid 20x20: {kg['ms_per_call']:.3f} ms/call (binning {kg['bin_kernel_ms']:.3f} ms, "
            f"{kg['roofline']['achieved']:.0f} GB/s)")
    grid = None
    if not args.no_grid:
        log("[bench] Eq. (vg): gridding 262,144 baselines x 768 channels")
        grid = grid_block(bs, ctx, w, torch)
        log(f"[bench] grid: {grid['ms_per_call']:.3f} ms/call (scatter {grid['scatter_ms']:.3f}, output "
            f"{grid['output_ms']:.3f}), {grid['roofline']['achieved']:.0f} GB/s algorithmic")
    dec = None
    if not args.no_grid:
        log("[bench] Eq. (S3): decorrelation factor of the ring triangles, 262,144 baselines")
        dec = decorrelation_block(bs, ctx, w, torch)
        log(f"[bench] decorrelation: {dec['ms_per_call']:.1f} ms/call for {dec['triangles']} ring triangles "
            f"(median D {dec['D_median']:.4f})")
    mc = None
    if not args.no_mc:
        log("[bench] Monte Carlo: 64 flagged realizations from one graph")
        mc = mc_block(bs, ctx, bins, ncand, w, torch)
        log(f"[bench] mc: {mc['ms_per_realization']:.2f} ms/realization")
    batch = None
    if not args.no_batch:
        log("[bench] batch: 64 uneven cubes, one graph launch")
        batch = batch_block(bs, ctx, torch)
        log(f"[bench] batch: {batch['seconds_per_launch']:.2f} s/launch, {batch['products_per_s']:.3e} products/s, "
            f"{batch['mfma_tflops_incl_generation_and_fields']:.0f} TFLOP/s")
    sur = None
    if not args.no_surrogate:
        log("[bench] variance surrogate: labels, training, evaluation against Monte Carlo")
        sur = surrogate_block(bs, ctx, bins, ncand, w, torch)
        log(f"[bench] surrogate: config-3 pattern {sur['rel_err_vs_mc4096_config3_pattern']}, unseen "
            f"{sur['rel_err_vs_mc4096_unseen_spread4']} / {sur['rel_err_vs_mc4096_unseen_e3']}")
    cpu = None
    if not args.no_cpu_baseline:
        Vh = Vd.cpu().numpy()
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        log(f"[bench] CPU oracle baseline: the whole step on {threads} threads")
        cpu = cpu_baseline_allcore(w, Vh, edges, Bs, Nt, threads)
        log(f"[bench] CPU oracle: {cpu['seconds']:.1f} s on {threads} threads")
        log("[bench] CPU oracle baseline: single thread (bounded sample)")
        cpu["single_thread"] = cpu_baseline(w, Vh, edges, Bs, tri)
    out = {
        "metric": "bin-triangle·voxel products/s, split-BF16 MFMA vs FP32 at ≤1e-4 rel err",
        "value": products / t_split,
        "unit": "products/s",
        "value_formed": n_valid * vox_c / t_split,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_split * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 fields, split-bf16 MFMA contraction, f64 sums",
        "data": "synthetic",
        "config": {"workload": "3D BS, 256x256 uv x 768 ch (40 kHz), quadratic field f=0.5, 20 log k-shells "
                               "0.003-1.258 Mpc^-1, all k1>=k2>=k3 candidates",
                   "triangles_candidate": int(ncand), "triangles_valid": n_valid, "voxels": nvox,
                   "products_per_step": products, "parallelism": "single GPU",
                   "products_formed_per_step": n_valid * vox_c,
                   "count_max_dev_from_integer": count_dev, "count_error_bound": count_bound},
        "roofline": roof,
        "kernel_ms": {"step_events": tim_split[0], "contraction": tim_split[1], "fields": tim_split[2]},
        "fp32": fp32,
        "mabs": mabs,
        "mabs_dft": mdft,
        "grid": grid,
        "decorrelation": dec,
        "mc": mc,
        "batch": batch,
        "surrogate": sur,
        "cpu_baseline": cpu,
    }
    bs.bs_free_bins(bins)
    bs.bs_destroy(ctx)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
