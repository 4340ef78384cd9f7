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
# that (sums that cancel almost completely) the bound is normwise, tol times B_abs.
KAPPA0 = 1e3
# Normwise error floors, as a fraction of B_abs, of the reduced-precision arithmetic.  The
# three-product split-BF16 product has a random relative error of about 2^-16 (the dropped lo*lo
# term and the residuals of the two splits), FP32 fields one FP32 rounding per transform stage;
# such errors average down only as 1 / sqrt(number of contributing terms), so an entry with few
# closed triangles and strong cancellation (cond up to KAPPA0) can miss the relative tolerance
# while its error stays at the floor (tests/test_split_arithmetic.py shows this for the split
# arithmetic alone, with exact accumulation).  Measured maxima over the GPU tests: 4.4e-7 (FP32),
# 1.2e-6 (split-BF16).  Entries that need the floor are counted in the per-bin report.
NORMWISE_FLOOR = {1e-10: 0.0, 1e-5: 1e-6, 1e-4: 3e-6}


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


def write_per_bin_report(label, Bg, Bref, N, abs_scale, tol, extra=None, floor=0.0):
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
    well = cond <= KAPPA0
    rep = {"label": label, "tol": tol, "kappa0": KAPPA0, "normwise_floor": floor, "valid_entries": int(len(rel)),
           "bands": bands, "max_rel_cond_le_kappa0": float(rel[well].max()) if well.any() else None,
           "max_err_over_Babs": float((rel / cond).max()) if len(rel) else None,
           "floor_limited": int((well & (rel > tol)).sum())}
    if len(rel) <= 5000:
        rep["entries"] = [{"rel": float(a), "cond": float(b), "N_tri": int(c)} for a, b, c in zip(rel, cond, n)]
    if extra:
        rep.update(extra)
    safe = "".join(ch if ch.isalnum() or ch in "-_." else "_" for ch in label)
    with open(os.path.join(d, safe + ".json"), "w") as fh:
        json.dump(rep, fh)


def compare_B(Bg, Bref, N, abs_scale, tol, label="", floor=None):
    """Per-entry pass criterion: |B_gpu - B_ref| <= max(tol |B_ref|, floor B_abs) where
    cond <= KAPPA0, and <= tol B_abs beyond, with B_abs the estimate built from |F1 F2 F3|
    (cond = B_abs / |B_ref|): relative error where the sum is not dominated by cancellation,
    normwise error where it is.  floor defaults to NORMWISE_FLOOR[tol]; 0 gives the plain
    relative bar up to KAPPA0.
    Returns (worst relative error of entries with cond <= KAPPA0, worst error / B_abs)."""
    if floor is None:
        floor = NORMWISE_FLOOR.get(tol, 0.0)
    Bg = np.asarray(Bg, dtype=np.float64)
    Bref = np.asarray(Bref, dtype=np.float64)
    ok = N > 0
    assert np.all(np.isnan(Bg[~ok])), f"{label}: B must be NaN where N_tri = 0"
    assert np.all(np.isfinite(Bg[ok])), f"{label}: non-finite B where N_tri > 0"
    err = np.abs(Bg[ok] - Bref[ok])
    ref = np.abs(Bref[ok])
    scale = np.asarray(abs_scale, dtype=np.float64)[ok]
    bound = np.where(scale <= KAPPA0 * ref, np.maximum(tol * ref, floor * scale), tol * scale)
    write_per_bin_report(label, Bg, Bref, N, abs_scale, tol, floor=floor)
    bad = err > bound
    assert not bad.any(), (f"{label}: {bad.sum()} entries above max(tol|B|, {floor:g} B_abs) (cond <= {KAPPA0:g}) "
                           f"or tol B_abs; "
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
