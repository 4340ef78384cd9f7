"""Shared helpers for the GPU parity tests (imported by test_gpu_*.py)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2506_10526_amd import bs  # noqa: E402


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def cuda(x: np.ndarray, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x if dtype is None else x.astype(dtype)))
    return t.cuda()


def vis_tensor(V: np.ndarray, precision: int):
    return cuda(V, np.complex128 if precision == bs.BS_FP64 else np.complex64)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# Entries with cond = B_abs / |B_ref| up to KAPPA0 are held to the relative tolerance; beyond
# that (near-zero realisations) the bound is normwise, tol times B_abs.
KAPPA0 = 1e3


def per_bin_errors(Bg, Bref, N, abs_scale):
    """Per-entry error record of the entries with N_tri > 0: rel = |B_gpu - B_ref| / |B_ref|,
    cond = B_abs / |B_ref| and the count (arrays over the valid entries, flattened)."""
    Bg = np.asarray(Bg, dtype=np.float64).ravel()
    Bref = np.asarray(Bref, dtype=np.float64).ravel()
    N = np.asarray(N).ravel()
    ok = N > 0
    err = np.abs(Bg[ok] - Bref[ok])
    ref = np.abs(Bref[ok])
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(ref > 0, err / ref, np.where(err > 0, np.inf, 0.0))
        cond = np.where(ref > 0, np.asarray(abs_scale, dtype=np.float64).ravel()[ok] / ref, np.inf)
    return rel, cond, N[ok], err


def write_per_bin_report(label, Bg, Bref, N, abs_scale, tol, extra=None):
    """Writes the per-bin error table (rel, cond, N_tri per valid entry, plus a summary by
    conditioning band) as JSON into $BS_PER_BIN_DIR when that is set."""
    import json
    import os
    d = os.environ.get("BS_PER_BIN_DIR")
    if not d:
        return
    os.makedirs(d, exist_ok=True)
    rel, cond, n, _ = per_bin_errors(Bg, Bref, N, abs_scale)
    bands = {}
    for name, lo, hi in (("cond<=10", 0, 10), ("10<cond<=1e3", 10, 1e3), ("cond>1e3", 1e3, np.inf)):
        m = (cond > lo) & (cond <= hi) if lo > 0 else cond <= hi
        bands[name] = {"entries": int(m.sum()), "max_rel": float(rel[m].max()) if m.any() else None}
    rep = {"label": label, "tol": tol, "kappa0": KAPPA0, "valid_entries": int(len(rel)), "bands": bands,
           "max_rel_cond_le_kappa0": float(rel[cond <= KAPPA0].max()) if (cond <= KAPPA0).any() else None}
    if len(rel) <= 5000:
        rep["entries"] = [{"rel": float(a), "cond": float(b), "N_tri": int(c)} for a, b, c in zip(rel, cond, n)]
    if extra:
        rep.update(extra)
    safe = "".join(ch if ch.isalnum() or ch in "-_." else "_" for ch in label)
    with open(os.path.join(d, safe + ".json"), "w") as fh:
        json.dump(rep, fh)


def compare_B(Bg, Bref, N, abs_scale, tol, label=""):
    """Per-entry pass criterion: |B_gpu - B_ref| <= max(tol |B_ref|, (tol / KAPPA0) B_abs), with
    B_abs the estimate built from |F1 F2 F3| (so cond = B_abs / |B_ref|).  Entries with
    cond <= KAPPA0 are held to relative error tol; beyond that the bound is normwise, which is
    what floating-point field transforms can deliver (their error is proportional to B_abs).
    Returns (worst relative error of entries with cond <= KAPPA0, worst error / B_abs)."""
    Bg = np.asarray(Bg, dtype=np.float64)
    Bref = np.asarray(Bref, dtype=np.float64)
    ok = N > 0
    assert np.all(np.isnan(Bg[~ok])), f"{label}: B must be NaN where N_tri = 0"
    assert np.all(np.isfinite(Bg[ok])), f"{label}: non-finite B where N_tri > 0"
    err = np.abs(Bg[ok] - Bref[ok])
    ref = np.abs(Bref[ok])
    scale = np.asarray(abs_scale, dtype=np.float64)[ok]
    bound = np.maximum(tol * ref, (tol / KAPPA0) * scale)
    write_per_bin_report(label, Bg, Bref, N, abs_scale, tol)
    bad = err > bound
    assert not bad.any(), (f"{label}: {bad.sum()} entries above max(tol|B|, tol/{KAPPA0:g} B_abs); "
                           f"worst err/bound {float((err / bound).max()):.3g}")
    well = scale <= KAPPA0 * ref
    worst_rel = float((err[well] / ref[well]).max()) if well.any() else 0.0
    worst_norm = float((err / np.maximum(scale, 1e-300)).max()) if err.size else 0.0
    return worst_rel, worst_norm


class Ctx:
    def __init__(self):
        need_gpu()
        self.h = bs.bs_create(0, torch.cuda.current_stream().cuda_stream)

    def close(self):
        bs.bs_destroy(self.h)
