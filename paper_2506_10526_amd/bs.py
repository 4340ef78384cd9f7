"""ctypes binding of libbs (include/bs.h): argument marshalling only.

Every function here has the name of the C entry point it wraps and passes device
pointers (PyTorch tensors' data_ptr()) straight through; all computation happens in
the HIP library.  If libbs.so is missing the import of this module still succeeds, but
every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libbs.so")

BS_OK, BS_EINVAL, BS_ENOMEM, BS_EHIP, BS_ECOUNT, BS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
BS_RING_U, BS_SHELL_K = 0, 1
BS_FP64, BS_FP32, BS_SPLIT_BF16 = 0, 1, 2

EXPORTED = [
    "bs_create", "bs_destroy", "bs_last_error", "bs_set_stream", "bs_make_bins", "bs_bins_triangles",
    "bs_bins_info", "bs_free_bins", "bs_filter_fields", "bs_estimate_mabs", "bs_mabs_dft", "bs_monopole", "bs_monopole_noalloc", "bs_grid_visibilities", "bs_decorrelation", "bs_estimate_3d",
    "bs_set_timing", "bs_last_timing", "bs_last_count_dev", "bs_last_count_bound", "bs_generate_cube", "bs_mc_create", "bs_mc_run",
    "bs_mc_stats", "bs_mc_last", "bs_mc_reset", "bs_mc_destroy", "bs_mlp_create", "bs_mlp_read_state", "bs_mlp_write_state",
    "bs_mlp_set_data", "bs_mlp_loss_grad", "bs_mlp_train", "bs_mlp_predict", "bs_mlp_destroy", "bs_var_features",
    "bs_batch_create", "bs_batch_run", "bs_batch_info", "bs_batch_result", "bs_batch_destroy",
    "bs_batch_tile", "bs_tune_set", "bs_tune_get", "bs_var_flag_proxy", "bs_var_features_flag",
    "bs_multipoles",
    "bs_kpar_grid",
]
BS_MLP_NPARAM, BS_MLP_NSTATE = 133121, 133131
BS_K_CUBIC, BS_K_PHYSICAL = 0, 1


class BsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libbs error {code}: {msg}")
        self.code = code


class bs_bins_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("nc", ctypes.c_int32),
                ("nbins", ctypes.c_int32), ("edges_host", ctypes.POINTER(ctypes.c_double)),
                ("umax", ctypes.c_double), ("du_lambda", ctypes.c_double), ("r_mpc", ctypes.c_double),
                ("rprime_mpc_per_mhz", ctypes.c_double), ("dnu_mhz", ctypes.c_double)]


class bs_weights(ctypes.Structure):
    _fields_ = [("ng", ctypes.c_void_p), ("uv_mask", ctypes.c_void_p), ("chan_w", ctypes.c_void_p)]


class bs_mabs_sel(ctypes.Structure):
    _fields_ = [("n_tri", ctypes.c_int32), ("tri3_host", ctypes.POINTER(ctypes.c_int32)),
                ("n_nu1", ctypes.c_int32), ("nu1_host", ctypes.POINTER(ctypes.c_int32)),
                ("collapse", ctypes.c_int32)]


class bs_field_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nc", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("f_ng", ctypes.c_double), ("pk_index", ctypes.c_double),
                ("du_lambda", ctypes.c_double), ("r_mpc", ctypes.c_double),
                ("rprime_mpc_per_mhz", ctypes.c_double), ("dnu_mhz", ctypes.c_double)]


class bs_batch_cube(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nc", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("realization", ctypes.c_uint64), ("n_nu1", ctypes.c_int32),
                ("nu1_host", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libbs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIBPATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.bs_create.argtypes = [ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.bs_destroy.argtypes = [vp]
    L.bs_destroy.restype = None
    L.bs_last_error.argtypes = [vp]
    L.bs_last_error.restype = ctypes.c_char_p
    L.bs_set_stream.argtypes = [vp, vp]
    L.bs_make_bins.argtypes = [vp, ctypes.POINTER(bs_bins_desc), ctypes.POINTER(vp), ctypes.POINTER(i32)]
    L.bs_bins_triangles.argtypes = [vp, vp, vp]
    L.bs_bins_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.bs_free_bins.argtypes = [vp]
    L.bs_free_bins.restype = None
    L.bs_filter_fields.argtypes = [vp, vp, vp, ctypes.POINTER(bs_weights), i32, i32, vp, vp]
    L.bs_estimate_mabs.argtypes = [vp, vp, vp, ctypes.POINTER(bs_weights), ctypes.POINTER(bs_mabs_sel), i32, dbl,
                                   vp, vp, vp]
    L.bs_estimate_3d.argtypes = [vp, vp, vp, ctypes.POINTER(bs_weights), i32, dbl, vp, vp, vp]
    L.bs_mabs_dft.argtypes = [vp, i32, i32, i32, vp, dbl, vp]
    L.bs_grid_visibilities.argtypes = [vp, i32, i32, dbl, ctypes.c_int64, vp, vp, vp, i32, i32, vp, vp]
    L.bs_monopole.argtypes = [vp, i32, i32, ctypes.POINTER(dbl), dbl, vp, i32, ctypes.POINTER(dbl), vp, vp]
    L.bs_multipoles.argtypes = [vp, i32, i32, ctypes.POINTER(dbl), dbl, vp, i32, ctypes.POINTER(dbl), i32, vp, vp]
    L.bs_kpar_grid.argtypes = [vp, i32, i32, dbl, vp, i32, ctypes.POINTER(dbl), vp, vp]
    L.bs_monopole_noalloc.argtypes = [vp, i32, i32, vp, dbl, vp, i32, vp, vp, vp]
    L.bs_decorrelation.argtypes = [vp, vp, ctypes.c_int64, vp, dbl, dbl, i32, vp]
    L.bs_set_timing.argtypes = [vp, i32]
    L.bs_last_timing.argtypes = [vp, ctypes.POINTER(dbl), i32]
    L.bs_last_count_dev.argtypes = [vp, ctypes.POINTER(dbl)]
    L.bs_last_count_bound.argtypes = [vp, ctypes.POINTER(dbl)]
    u64 = ctypes.c_uint64
    L.bs_generate_cube.argtypes = [vp, ctypes.POINTER(bs_field_desc), u64, u64, vp, vp]
    L.bs_mc_create.argtypes = [vp, vp, ctypes.POINTER(bs_field_desc), ctypes.POINTER(bs_weights), i32, dbl,
                               ctypes.POINTER(vp)]
    L.bs_mc_run.argtypes = [vp, u64, u64, i32, i32]
    L.bs_mc_stats.argtypes = [vp, vp, vp, vp]
    L.bs_mc_last.argtypes = [vp, vp, vp]
    L.bs_mc_reset.argtypes = [vp]
    L.bs_mc_destroy.argtypes = [vp]
    L.bs_mc_destroy.restype = None
    L.bs_mlp_create.argtypes = [vp, u64, i32, ctypes.POINTER(vp)]
    L.bs_mlp_read_state.argtypes = [vp, vp]
    L.bs_mlp_write_state.argtypes = [vp, vp]
    L.bs_mlp_set_data.argtypes = [vp, vp, vp, i32]
    L.bs_mlp_loss_grad.argtypes = [vp, vp, ctypes.POINTER(dbl)]
    L.bs_mlp_train.argtypes = [vp, i32, dbl, i32, ctypes.POINTER(dbl)]
    L.bs_mlp_predict.argtypes = [vp, vp, i32, i32, vp]
    L.bs_mlp_destroy.argtypes = [vp]
    L.bs_mlp_destroy.restype = None
    L.bs_var_features.argtypes = [vp, vp, dbl, dbl, vp, vp]
    L.bs_var_flag_proxy.argtypes = [vp, vp, dbl, vp, vp]
    L.bs_var_features_flag.argtypes = [vp, vp, vp, vp, dbl, vp, vp]
    L.bs_batch_create.argtypes = [vp, ctypes.POINTER(bs_batch_cube), i32, i32, ctypes.POINTER(bs_field_desc), dbl,
                                  ctypes.POINTER(vp)]
    L.bs_batch_run.argtypes = [vp]
    L.bs_batch_info.argtypes = [vp, i32, vp, vp, vp, vp]
    L.bs_batch_result.argtypes = [vp, i32, vp, vp, vp, vp]
    L.bs_batch_destroy.argtypes = [vp]
    L.bs_batch_destroy.restype = None
    L.bs_batch_tile.argtypes = [vp, i32, vp, vp, vp, vp]
    L.bs_tune_set.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32]
    L.bs_tune_get.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp, vp]
    for name in EXPORTED:
        if name not in ("bs_destroy", "bs_last_error", "bs_free_bins", "bs_mc_destroy", "bs_mlp_destroy",
                        "bs_batch_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _check(ctx, rc: int):
    if rc != BS_OK:
        msg = lib().bs_last_error(ctx).decode() if ctx else ""
        raise BsError(rc, msg)


# ---------------------------------------------------------------- entry points
def bs_create(device: int = 0, stream: Optional[int] = None) -> int:
    h = ctypes.c_void_p()
    rc = lib().bs_create(device, stream, ctypes.byref(h))
    if rc != BS_OK:
        raise BsError(rc, "bs_create failed")
    return h.value


def bs_destroy(ctx: int) -> None:
    lib().bs_destroy(ctx)


def bs_last_error(ctx: int) -> str:
    return lib().bs_last_error(ctx).decode()


def bs_set_stream(ctx: int, stream: Optional[int]) -> None:
    _check(ctx, lib().bs_set_stream(ctx, stream))


def bs_make_bins(ctx: Optional[int], kind: int, n: int, nc: int, edges: Sequence[float], umax: float = 0.0,
                 du_lambda: float = 0.0, r_mpc: float = 0.0, rprime_mpc_per_mhz: float = 0.0,
                 dnu_mhz: float = 0.0):
    """Returns (bins handle, n_candidates)."""
    e = (ctypes.c_double * len(edges))(*[float(x) for x in edges])
    d = bs_bins_desc(kind, n, nc, len(edges) - 1, e, umax, du_lambda, r_mpc, rprime_mpc_per_mhz, dnu_mhz)
    h = ctypes.c_void_p()
    nc_ = ctypes.c_int32()
    _check(ctx, lib().bs_make_bins(ctx, ctypes.byref(d), ctypes.byref(h), ctypes.byref(nc_)))
    return h.value, nc_.value


def bs_bins_triangles(bins: int, n_candidates: int, nbins: int):
    """Host copies: (triangles int32 [n][3], modes int64 [nbins]) as nested lists via numpy."""
    import numpy as np
    tri = np.zeros((max(n_candidates, 1), 3), dtype=np.int32)
    modes = np.zeros(max(nbins, 1), dtype=np.int64)
    rc = lib().bs_bins_triangles(bins, tri.ctypes.data, modes.ctypes.data)
    if rc != BS_OK:
        raise BsError(rc, "bs_bins_triangles failed")
    return tri[:n_candidates], modes[:nbins]


def bs_bins_info(bins: int):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    rc = lib().bs_bins_info(bins, ctypes.byref(a), ctypes.byref(b))
    if rc != BS_OK:
        raise BsError(rc, "bs_bins_info failed")
    return a.value, bool(b.value)


def bs_free_bins(bins: int) -> None:
    lib().bs_free_bins(bins)


def _weights(ng=None, uv_mask=None, chan_w=None) -> bs_weights:
    return bs_weights(_ptr(ng), _ptr(uv_mask), _ptr(chan_w))


def bs_filter_fields(ctx: int, bins: int, vis, three_d: int, precision: int, fields, count_fields=None,
                     ng=None, uv_mask=None, chan_w=None) -> None:
    w = _weights(ng, uv_mask, chan_w)
    _check(ctx, lib().bs_filter_fields(ctx, bins, _ptr(vis), ctypes.byref(w), three_d, precision,
                                       _ptr(fields), _ptr(count_fields)))


def bs_estimate_mabs(ctx: int, bins: int, vis, precision: int, B, N_tri, N_nu=None, norm: float = 1.0,
                     tri3=None, nu1=None, collapse: int = 0, ng=None, uv_mask=None, chan_w=None) -> None:
    w = _weights(ng, uv_mask, chan_w)
    tri_arr = nu_arr = None
    ntri = nnu = 0
    if tri3 is not None:
        flat = [int(x) for row in tri3 for x in row]
        ntri = len(flat) // 3
        tri_arr = (ctypes.c_int32 * max(len(flat), 1))(*flat)
    if nu1 is not None:
        nu = [int(x) for x in nu1]
        nnu = len(nu)
        nu_arr = (ctypes.c_int32 * max(nnu, 1))(*nu)
    sel = bs_mabs_sel(ntri, tri_arr, nnu, nu_arr, collapse)
    _check(ctx, lib().bs_estimate_mabs(ctx, bins, _ptr(vis), ctypes.byref(w), ctypes.byref(sel), precision,
                                       float(norm), _ptr(B), _ptr(N_tri), _ptr(N_nu)))


def bs_estimate_3d(ctx: int, bins: int, vis, precision: int, B, N_tri, N_eff=None, norm: float = 1.0,
                   uv_mask=None, chan_w=None, ng=None) -> None:
    w = _weights(ng, uv_mask, chan_w)
    _check(ctx, lib().bs_estimate_3d(ctx, bins, _ptr(vis), ctypes.byref(w), precision, float(norm),
                                     _ptr(B), _ptr(N_tri), _ptr(N_eff)))


def bs_mabs_dft(ctx: int, nc: int, Bbar, out, scale: float = 1.0, circular: bool = False) -> None:
    """Eq. (dft) on a collapsed MABS: Bbar float64 [n_tri][2nc-1][2nc-1] (or [n_tri][nc][nc] when
    circular), out complex128 [n_tri][nc][nc], both on the device."""
    size = nc if circular else 2 * nc - 1
    nt = int(Bbar.shape[0])
    if (tuple(Bbar.shape) != (nt, size, size) or tuple(out.shape) != (nt, nc, nc)
            or not Bbar.is_contiguous() or not out.is_contiguous()):
        raise ValueError("bs_mabs_dft: Bbar must be contiguous [n_tri][%d][%d] and out contiguous [n_tri][%d][%d]"
                         % (size, size, nc, nc))
    _check(ctx, lib().bs_mabs_dft(ctx, int(nc), nt, 1 if circular else 0, _ptr(Bbar), float(scale), _ptr(out)))


def bs_monopole(ctx: int, Bcyl, kperp, kpar_unit: float, k1_edges, mean, count) -> None:
    """Monopole B(k1, mu, t): Bcyl complex128 [n_tri][nc][nc] on the device, kperp [n_tri][3] and
    k1_edges [n_k1 + 1] on the host, mean float64 / count int64 [n_k1][5][5] on the device."""
    nt, nc = int(Bcyl.shape[0]), int(Bcyl.shape[1])
    kp = [float(x) for row in kperp for x in row]
    ke = [float(x) for x in k1_edges]
    nk = len(ke) - 1
    if (tuple(Bcyl.shape) != (nt, nc, nc) or len(kp) != 3 * nt or tuple(mean.shape) != (nk, 5, 5)
            or tuple(count.shape) != (nk, 5, 5) or not Bcyl.is_contiguous() or not mean.is_contiguous()
            or not count.is_contiguous()):
        raise ValueError("bs_monopole: Bcyl [n_tri][nc][nc], kperp [n_tri][3], mean and count [n_k1][5][5]")
    kpa = (ctypes.c_double * max(len(kp), 1))(*kp)
    kea = (ctypes.c_double * len(ke))(*ke)
    _check(ctx, lib().bs_monopole(ctx, nc, nt, kpa, float(kpar_unit), _ptr(Bcyl), nk, kea, _ptr(mean), _ptr(count)))


def bs_multipoles(ctx: int, Bcyl, kperp, kpar_unit: float, k1_edges, lmax: int, moments, count) -> None:
    """Multipole moments B_l^m(k1, mu, t): as bs_monopole, moments float64 [(lmax+1)(lmax+2)/2][n_k1][5][5]
    on the device (l = 0 .. lmax, m = 0 .. l), count int64 [n_k1][5][5]."""
    nt, nc = int(Bcyl.shape[0]), int(Bcyl.shape[1])
    kp = [float(x) for row in kperp for x in row]
    ke = [float(x) for x in k1_edges]
    nk = len(ke) - 1
    nlm = (lmax + 1) * (lmax + 2) // 2
    if (tuple(Bcyl.shape) != (nt, nc, nc) or len(kp) != 3 * nt or tuple(moments.shape) != (nlm, nk, 5, 5)
            or tuple(count.shape) != (nk, 5, 5) or not Bcyl.is_contiguous() or not moments.is_contiguous()
            or not count.is_contiguous()):
        raise ValueError("bs_multipoles: Bcyl [n_tri][nc][nc], kperp [n_tri][3], moments [n_lm][n_k1][5][5], "
                         "count [n_k1][5][5]")
    kpa = (ctypes.c_double * max(len(kp), 1))(*kp)
    kea = (ctypes.c_double * len(ke))(*ke)
    _check(ctx, lib().bs_multipoles(ctx, nc, nt, kpa, float(kpar_unit), _ptr(Bcyl), nk, kea, int(lmax), _ptr(moments),
                                    _ptr(count)))


def bs_kpar_grid(ctx: int, Bcyl, kpar_unit: float, edges, mean, count) -> None:
    """The cylindrical 3D BS binned on a (k_par1, k_par2) grid: Bcyl complex128 [n_tri][nc][nc],
    edges [n_e + 1] (host values), mean float64 [n_tri][n_e][n_e] and count int64 [n_e][n_e] on the
    device."""
    nt, nc = int(Bcyl.shape[0]), int(Bcyl.shape[1])
    ed = [float(x) for x in edges]
    ne = len(ed) - 1
    if (tuple(Bcyl.shape) != (nt, nc, nc) or tuple(mean.shape) != (nt, ne, ne) or tuple(count.shape) != (ne, ne)
            or not Bcyl.is_contiguous() or not mean.is_contiguous() or not count.is_contiguous()):
        raise ValueError("bs_kpar_grid: Bcyl [n_tri][nc][nc], mean [n_tri][n_e][n_e], count [n_e][n_e]")
    eda = (ctypes.c_double * len(ed))(*ed)
    _check(ctx, lib().bs_kpar_grid(ctx, nc, nt, float(kpar_unit), _ptr(Bcyl), ne, eda, _ptr(mean), _ptr(count)))


def bs_monopole_noalloc(ctx: int, Bcyl, kperp, kpar_unit: float, k1_edges, mean, count) -> None:
    """Allocation-free monopole: as bs_monopole, but kperp float64 [n_tri][3] and k1_edges float64
    [n_k1 + 1] are device tensors, and the call only enqueues work on the context's stream."""
    nt, nc = int(Bcyl.shape[0]), int(Bcyl.shape[1])
    nk = int(k1_edges.shape[0]) - 1
    if (tuple(Bcyl.shape) != (nt, nc, nc) or tuple(kperp.shape) != (nt, 3) or tuple(mean.shape) != (nk, 5, 5)
            or tuple(count.shape) != (nk, 5, 5) or not all(t.is_contiguous() for t in (Bcyl, kperp, k1_edges, mean, count))):
        raise ValueError("bs_monopole_noalloc: Bcyl [n_tri][nc][nc], kperp [n_tri][3], mean and count [n_k1][5][5]")
    _check(ctx, lib().bs_monopole_noalloc(ctx, nc, nt, _ptr(kperp), float(kpar_unit), _ptr(Bcyl), nk, _ptr(k1_edges),
                                          _ptr(mean), _ptr(count)))


def bs_decorrelation(ctx: int, rings: int, n_cand: int, uv, du_lambda: float, theta0_rad: float, n_nodes: int = 12):
    """Eq. (S3) decorrelation factor D per candidate ring triangle (host float64 [n_cand]) for the
    baselines uv (device float64 [n_vis][2], wavelengths) gridded with spacing du_lambda."""
    import numpy as np
    nv = int(uv.shape[0])
    if uv.dim() != 2 or int(uv.shape[1]) != 2 or not uv.is_contiguous():
        raise ValueError("bs_decorrelation: uv [n_vis][2]")
    D = np.zeros(max(n_cand, 1), dtype=np.float64)
    _check(ctx, lib().bs_decorrelation(ctx, rings, nv, _ptr(uv), float(du_lambda), float(theta0_rad), int(n_nodes),
                                       D.ctypes.data))
    return D[:n_cand]


def bs_grid_visibilities(ctx: int, n: int, du_lambda: float, uv, vis, Vg, Ng, flags=None, chan_avg: int = 1,
                         precision: int = BS_FP32) -> None:
    """Eq. (vg): uv float64 [n_vis][2], vis complex64 [nc][n_vis], flags uint8 [nc][n_vis] or None;
    Vg complex64 / complex128 (precision BS_FP64) and Ng int32 [nc/chan_avg][n][n/2+1]; all on the device."""
    nc, nv = int(vis.shape[0]), int(vis.shape[1])
    nco = nc // max(chan_avg, 1)
    shp = (nco, n, n // 2 + 1)
    if (tuple(uv.shape) != (nv, 2) or tuple(Vg.shape) != shp or tuple(Ng.shape) != shp
            or (flags is not None and tuple(flags.shape) != (nc, nv))
            or not all(t.is_contiguous() for t in (uv, vis, Vg, Ng) + ((flags,) if flags is not None else ()))):
        raise ValueError("bs_grid_visibilities: uv [n_vis][2], vis/flags [nc][n_vis], Vg/Ng [nc/chan_avg][n][n/2+1]")
    _check(ctx, lib().bs_grid_visibilities(ctx, int(n), nc, float(du_lambda), nv, _ptr(uv), _ptr(vis), _ptr(flags),
                                           int(chan_avg), int(precision), _ptr(Vg), _ptr(Ng)))


def bs_set_timing(ctx: int, enable: bool) -> None:
    _check(ctx, lib().bs_set_timing(ctx, 1 if enable else 0))


def bs_last_timing(ctx: int):
    out = (ctypes.c_double * 6)()
    _check(ctx, lib().bs_last_timing(ctx, out, 6))
    return list(out)


def bs_last_count_dev(ctx: int) -> float:
    d = ctypes.c_double()
    _check(ctx, lib().bs_last_count_dev(ctx, ctypes.byref(d)))
    return d.value


def bs_last_count_bound(ctx: int) -> float:
    d = ctypes.c_double()
    _check(ctx, lib().bs_last_count_bound(ctx, ctypes.byref(d)))
    return d.value


def field_desc(n: int, nc: int, kind: int = BS_K_CUBIC, sigma: float = 0.5, f_ng: float = 0.5,
               pk_index: float = -2.0, du_lambda: float = 1.0, r_mpc: float = 1.0,
               rprime_mpc_per_mhz: float = 1.0, dnu_mhz: float = 1.0) -> bs_field_desc:
    return bs_field_desc(n, nc, kind, sigma, f_ng, pk_index, du_lambda, r_mpc, rprime_mpc_per_mhz, dnu_mhz)


def bs_generate_cube(ctx: int, desc: bs_field_desc, seed: int, realization: int, vis, chan_w=None) -> None:
    """vis: complex64 device tensor [nc][n][n/2+1] (written)."""
    _check(ctx, lib().bs_generate_cube(ctx, ctypes.byref(desc), seed, realization, _ptr(chan_w), _ptr(vis)))


_mc_ctx = {}


def bs_mc_create(ctx: int, bins: int, desc: bs_field_desc, precision: int, norm: float = 1.0,
                 uv_mask=None, chan_w=None) -> int:
    w = bs_weights(None, _ptr(uv_mask), _ptr(chan_w))
    h = ctypes.c_void_p()
    _check(ctx, lib().bs_mc_create(ctx, bins, ctypes.byref(desc), ctypes.byref(w), precision, norm, ctypes.byref(h)))
    _mc_ctx[h.value] = ctx
    return h.value


def bs_mc_run(mc: int, seed: int, first_realization: int, count: int, use_graph: bool = True) -> None:
    _check(_mc_ctx.get(mc), lib().bs_mc_run(mc, seed, first_realization, count, 1 if use_graph else 0))


def bs_mc_stats(mc: int, n_cand: int):
    """(count int64, mean float64, var float64) per candidate triangle, as NumPy arrays."""
    import numpy as np
    cnt = np.zeros(n_cand, dtype=np.int64)
    mean = np.zeros(n_cand, dtype=np.float64)
    var = np.zeros(n_cand, dtype=np.float64)
    _check(_mc_ctx.get(mc), lib().bs_mc_stats(mc, cnt.ctypes.data, mean.ctypes.data, var.ctypes.data))
    return cnt, mean, var


def bs_mc_last(mc: int, n_cand: int):
    import numpy as np
    B = np.zeros(n_cand, dtype=np.float64)
    N = np.zeros(n_cand, dtype=np.int64)
    _check(_mc_ctx.get(mc), lib().bs_mc_last(mc, B.ctypes.data, N.ctypes.data))
    return B, N


def bs_mc_reset(mc: int) -> None:
    _check(_mc_ctx.get(mc), lib().bs_mc_reset(mc))


def bs_mc_destroy(mc: int) -> None:
    lib().bs_mc_destroy(mc)
    _mc_ctx.pop(mc, None)


_mlp_ctx = {}


def bs_mlp_create(ctx: int, seed: int, max_batch: int) -> int:
    h = ctypes.c_void_p()
    _check(ctx, lib().bs_mlp_create(ctx, seed, max_batch, ctypes.byref(h)))
    _mlp_ctx[h.value] = ctx
    return h.value


def bs_mlp_read_state(mlp: int):
    """Host copy (float32 [BS_MLP_NSTATE]) of the parameters followed by the normalisation."""
    import numpy as np
    out = np.zeros(BS_MLP_NSTATE, dtype=np.float32)
    _check(_mlp_ctx.get(mlp), lib().bs_mlp_read_state(mlp, out.ctypes.data))
    return out


def bs_mlp_write_state(mlp: int, state) -> None:
    import numpy as np
    st = np.ascontiguousarray(state, dtype=np.float32)
    assert st.size == BS_MLP_NSTATE
    _check(_mlp_ctx.get(mlp), lib().bs_mlp_write_state(mlp, st.ctypes.data))


def bs_mlp_set_data(mlp: int, X, t) -> None:
    _check(_mlp_ctx.get(mlp), lib().bs_mlp_set_data(mlp, _ptr(X), _ptr(t), int(t.shape[0])))


def bs_mlp_loss_grad(mlp: int, grad=None) -> float:
    loss = ctypes.c_double()
    _check(_mlp_ctx.get(mlp), lib().bs_mlp_loss_grad(mlp, _ptr(grad), ctypes.byref(loss)))
    return loss.value


def bs_mlp_train(mlp: int, steps: int, lr: float, cosine: bool = False) -> float:
    loss = ctypes.c_double()
    _check(_mlp_ctx.get(mlp), lib().bs_mlp_train(mlp, steps, lr, 1 if cosine else 0, ctypes.byref(loss)))
    return loss.value


def bs_mlp_predict(mlp: int, X, y, bf16: bool = False) -> None:
    _check(_mlp_ctx.get(mlp), lib().bs_mlp_predict(mlp, _ptr(X), int(X.shape[0]), 1 if bf16 else 0, _ptr(y)))


def bs_mlp_destroy(mlp: int) -> None:
    lib().bs_mlp_destroy(mlp)
    _mlp_ctx.pop(mlp, None)


def bs_var_features(bins: int, n_cand: int, T3D=None, pk_index: float = -2.0, rho: float = 1.0):
    """(X float32 [n_cand][4], baseline float64 [n_cand] or None) for 3D candidate triangles."""
    import numpy as np
    X = np.zeros((n_cand, 4), dtype=np.float32)
    base = np.zeros(n_cand, dtype=np.float64) if T3D is not None else None
    T = None if T3D is None else np.ascontiguousarray(T3D, dtype=np.int64)
    rc = lib().bs_var_features(bins, None if T is None else T.ctypes.data, pk_index, rho, X.ctypes.data,
                               None if base is None else base.ctypes.data)
    if rc != BS_OK:
        raise BsError(rc, "bs_var_features failed")
    return X, base


def bs_var_flag_proxy(ctx: int, bins: int, n_cand: int, pk_index: float = -2.0, chan_w=None):
    """G float64 [n_cand]: mean over closed triangles of P_w P_w P_w (chan_w: host array or None)."""
    import numpy as np
    G = np.zeros(n_cand, dtype=np.float64)
    w = None if chan_w is None else np.ascontiguousarray(chan_w, dtype=np.float32)
    _check(ctx, lib().bs_var_flag_proxy(ctx, bins, pk_index, None if w is None else w.ctypes.data, G.ctypes.data))
    return G


def bs_var_features_flag(bins: int, n_cand: int, T3D, G, G1, rho3: float):
    """(X float32 [n_cand][4], baseline float64 [n_cand]) with the per-triangle flag summary."""
    import numpy as np
    X = np.zeros((n_cand, 4), dtype=np.float32)
    base = np.zeros(n_cand, dtype=np.float64)
    T = np.ascontiguousarray(T3D, dtype=np.int64)
    Gc = np.ascontiguousarray(G, dtype=np.float64)
    G1c = np.ascontiguousarray(G1, dtype=np.float64)
    rc = lib().bs_var_features_flag(bins, T.ctypes.data, Gc.ctypes.data, G1c.ctypes.data, rho3, X.ctypes.data,
                                    base.ctypes.data)
    if rc != BS_OK:
        raise BsError(rc, "bs_var_features_flag failed")
    return X, base


_batch = {}


def bs_batch_create(ctx: int, cubes, nrings: int, field: bs_field_desc, budget_gib: float = 64.0) -> int:
    """cubes: sequence of (n, nc, seed, realization, nu1 list or None)."""
    arr = (bs_batch_cube * len(cubes))()
    keep = []
    for i, (n, nc, seed, real, nu1) in enumerate(cubes):
        if nu1 is None:
            arr[i] = bs_batch_cube(n, nc, seed, real, 0, None)
        else:
            a = (ctypes.c_int32 * len(nu1))(*nu1)
            keep.append(a)
            arr[i] = bs_batch_cube(n, nc, seed, real, len(nu1), ctypes.cast(a, ctypes.POINTER(ctypes.c_int32)))
    h = ctypes.c_void_p()
    _check(ctx, lib().bs_batch_create(ctx, arr, len(cubes), nrings, ctypes.byref(field), budget_gib, ctypes.byref(h)))
    _batch[h.value] = (ctx, [(c[0], c[1]) for c in cubes])
    return h.value


def bs_batch_run(batch: int) -> None:
    _check(_batch[batch][0], lib().bs_batch_run(batch))


def bs_batch_info(batch: int, cube: int):
    """(n_candidates, wave, pixel_chunks, products) of one cube."""
    a, b, c_, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(_batch[batch][0], lib().bs_batch_info(batch, cube, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c_),
                                                 ctypes.byref(d)))
    return a.value, b.value, c_.value, d.value


def bs_batch_tile(batch: int, cube: int):
    """(tile_m, tile_n, m1, pixel_chunks) of the contraction of one cube."""
    v = [ctypes.c_int32() for _ in range(4)]
    _check(_batch[batch][0], lib().bs_batch_tile(batch, cube, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def bs_tune_set(ctx: int, n: int, nc: int, n_nu1: int, nrings: int, tile_m: int, m1: int, kchunks: int) -> None:
    _check(ctx, lib().bs_tune_set(ctx, n, nc, n_nu1, nrings, tile_m, m1, kchunks))


def bs_tune_get(ctx: int, n: int, nc: int, n_nu1: int, nrings: int):
    """(tile_m, tile_n, m1, pixel_chunks) cached for a cube shape class; zeros when none."""
    v = [ctypes.c_int32() for _ in range(4)]
    _check(ctx, lib().bs_tune_get(ctx, n, nc, n_nu1, nrings, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def bs_batch_result(batch: int, cube: int):
    """(Bbar [n_cand][2nc-1][2nc-1], N_nu [2nc-1][2nc-1], T_perp [n_cand], triangles [n_cand][3])."""
    import numpy as np
    ncand = bs_batch_info(batch, cube)[0]
    n, nc = _batch[batch][1][cube]
    D = 2 * nc - 1
    B = np.zeros((ncand, D, D), dtype=np.float64)
    Nnu = np.zeros((D, D), dtype=np.int32)
    T = np.zeros(ncand, dtype=np.int64)
    tri = np.zeros((ncand, 3), dtype=np.int32)
    _check(_batch[batch][0], lib().bs_batch_result(batch, cube, B.ctypes.data, Nnu.ctypes.data, T.ctypes.data,
                                                   tri.ctypes.data))
    return B, Nnu, T, tri


def bs_batch_destroy(batch: int) -> None:
    lib().bs_batch_destroy(batch)
    _batch.pop(batch, None)
