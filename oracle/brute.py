"""Direct enumeration of closed grid triangles (tiny grids only).

Oracle (test infrastructure only; see the package docstring).

Sec. 3.2 of Gill & Bharadwaj 2025: directly correlating all grid-point triplets
that form closed triangles costs O(Nc^3 Nt^4); the FFT route reaches the same
sum.  Here the sum is written out: for every U1 in bin b1 and U2 in bin b2 the
third side is U3 = -U1 - U2 (mod the grid), and the triangle is kept when U3 is
in bin b3.  The data sum is sum X1 X2 X3 with X = W_g V_g; the count is the
number of kept triangles with all three cells sampled (unit weights).
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np

from .bins import Bins, RING_U, SHELL_K
from .estimator import Weights, delay_transform, symmetrize_columns


def full_plane(xh: np.ndarray, n: int) -> np.ndarray:
    """Expand a [..., n, n//2+1] half plane to [..., n, n] with X(u, v) = conj X(-u, -v)."""
    nh = n // 2 + 1
    out = np.zeros(xh.shape[:-1] + (n,), dtype=np.result_type(xh.dtype, np.complex128))
    out[..., :nh] = xh
    neg = (-np.arange(n)) % n
    for v in range(nh, n):
        out[..., :, v] = np.conj(xh[..., neg, n - v])
    return out


def full_volume(xh: np.ndarray, n: int) -> np.ndarray:
    """Expand [nc][n][n//2+1] to [nc][n][n] with X(e, u, v) = conj X(-e, -u, -v)."""
    nc = xh.shape[0]
    nh = n // 2 + 1
    out = np.zeros((nc, n, n), dtype=np.complex128)
    out[:, :, :nh] = xh
    ne = (-np.arange(nc)) % nc
    nu = (-np.arange(n)) % n
    for v in range(nh, n):
        out[:, :, v] = np.conj(xh[ne][:, nu, n - v])
    return out


def _lut_full_ring(bins: Bins) -> np.ndarray:
    n = bins.n
    nh = n // 2 + 1
    out = np.full((n, n), -1, dtype=np.int32)
    out[:, :nh] = bins.lut
    neg = (-np.arange(n)) % n
    for v in range(nh, n):
        out[:, v] = bins.lut[neg, n - v]
    return out


def _lut_full_shell(bins: Bins) -> np.ndarray:
    n, nc = bins.n, bins.nc
    nh = n // 2 + 1
    out = np.full((nc, n, n), -1, dtype=np.int32)
    out[:, :, :nh] = bins.lut
    ne = (-np.arange(nc)) % nc
    nu = (-np.arange(n)) % n
    for v in range(nh, n):
        out[:, :, v] = bins.lut[ne][:, nu, n - v]
    return out


def _enumerate(lut: np.ndarray, b1: int, b2: int, b3: int):
    """All closed index triangles (flat indices) with sides in bins b1, b2, b3 of `lut`."""
    shape = lut.shape
    c1 = np.argwhere(lut == b1)
    c2 = np.argwhere(lut == b2)
    if len(c1) == 0 or len(c2) == 0:
        return (np.zeros(0, np.int64),) * 3
    dims = np.asarray(shape)
    c3 = (-(c1[:, None, :] + c2[None, :, :])) % dims
    keep = lut[tuple(c3[..., d] for d in range(len(shape)))] == b3
    i1, i2 = np.nonzero(keep)
    f1 = np.ravel_multi_index(tuple(c1[i1].T), shape)
    f2 = np.ravel_multi_index(tuple(c2[i2].T), shape)
    f3 = np.ravel_multi_index(tuple(c3[i1, i2].T), shape)
    return f1, f2, f3


def brute_mabs(bins: Bins, vis: np.ndarray, weights: Optional[Weights], tri3, nus) -> Tuple[complex, int]:
    """(sum of X1 X2 X3 over closed triangles, number of sampled closed triangles)."""
    assert bins.kind == RING_U
    n, nc = bins.n, bins.nc
    w = weights or Weights()
    X = symmetrize_columns(w.data_weight(nc, n) * vis, n)
    Y = w.unit_weight(nc, n)
    lut = _lut_full_ring(bins)
    f1, f2, f3 = _enumerate(lut, *(int(b) for b in tri3))
    x = [full_plane(X[int(nu)], n).ravel() for nu in nus]
    y = [full_plane(Y[int(nu)].astype(np.complex128), n).real.ravel() for nu in nus]
    s = complex(np.sum(x[0][f1] * x[1][f2] * x[2][f3]))
    c = int(np.rint(np.sum(y[0][f1] * y[1][f2] * y[2][f3])))
    return s, c


def brute_3d(bins: Bins, vis: np.ndarray, weights: Optional[Weights], tri3) -> Tuple[complex, int]:
    """3D analogue over the delay-transformed cube and |k| shells."""
    assert bins.kind == SHELL_K
    n = bins.n
    w = weights or Weights()
    vt = delay_transform(vis, w)
    lut = _lut_full_shell(bins)
    m = w.uv_unit(n)
    mfull = full_plane(m.astype(np.complex128), n).real
    f1, f2, f3 = _enumerate(lut, *(int(b) for b in tri3))
    x = full_volume(vt, n).ravel()
    yv = np.broadcast_to(mfull[None], lut.shape).ravel()
    s = complex(np.sum(x[f1] * x[f2] * x[f3]))
    c = int(np.rint(np.sum(yv[f1] * yv[f2] * yv[f3])))
    return s, c


def closed_triangles(bins: Bins, tri3):
    """Closed triangles of a bin triple as flat indices into the full grid (used by theory)."""
    lut = _lut_full_ring(bins) if bins.kind == RING_U else _lut_full_shell(bins)
    return _enumerate(lut, *(int(b) for b in tri3)), lut.shape
