"""Exact integer triangle counts by pair convolution (ring and shell bins).

Oracle (test infrastructure only; see the package docstring).

The number of closed grid triangles of a bin triple (Sec. 3.2: the count that Eq. iFT_I
produces as N_pix^2 sum_theta I1 I2 I3, and its 3D analogue) is, written out,

    T(a, b, c) = #{(k1, k2, k3) : k_i in S_i sampled, k1 + k2 + k3 = 0 (mod the grid)}

where S_i is the set of Fourier cells of bin i over the FULL grid (both Hermitian halves).
Grouping by k1 + k2 gives T(a, b, c) = sum over k3 in S_c of C_ab(-k3), with the pair count

    C_ab(k) = #{(k1, k2) : k1 in S_a, k2 in S_b, k1 + k2 = k}   (a cyclic convolution).

C_ab is computed with the convolution theorem in float64 (fftn of both indicators, product,
ifftn).  Every cell of C_ab is an integer between 0 and min(|S_a|, |S_b|); the float64 result
deviates from it by about eps * log2(N) * sqrt(|S_a| |S_b|) (1e-8 for the largest shells of
the 256^2 x 768 cube), so rounding each cell gives the integer exactly, which is checked
(largest deviation returned and required below 1e-3).  The sum over S_c is then taken in
int64: the count is exact, with no rounding of a large floating-point sum.  This is independent
of the triple-sum route of estimator.py (different transforms, no field products), and it is
pinned against brute-force enumeration on tiny grids.
"""
from __future__ import annotations

from typing import Dict, Optional, Tuple

import numpy as np

from .bins import Bins, RING_U, SHELL_K, signed_index

try:  # scipy.fft runs the same transforms on several threads; numpy.fft otherwise
    import scipy.fft as _sfft
except Exception:  # pragma: no cover
    _sfft = None

ROUND_TOL = 1e-3   # largest accepted |C - rint(C)| of a pair-count cell


def _fftn(x, workers):
    return _sfft.fftn(x, workers=workers) if _sfft is not None else np.fft.fftn(x)


def _ifftn(x, workers):
    return _sfft.ifftn(x, workers=workers) if _sfft is not None else np.fft.ifftn(x)


def full_indicator(bins: Bins, b: int, uv_unit: Optional[np.ndarray] = None) -> np.ndarray:
    """0/1 float64 indicator of the sampled cells of bin b over the full grid.

    The half-plane LUT (v >= 0) is expanded with the mirror cell (-k) of every stored cell; the
    uv occupancy (uv_unit [n][n//2+1], 0/1) is expanded the same way."""
    n = bins.n
    nh = n // 2 + 1
    qu = signed_index(n)
    if bins.kind == RING_U:
        lut = bins.lut
        full = np.zeros((n, n))
        sel = (lut == b).astype(np.float64)
        if uv_unit is not None:
            sel = sel * (np.asarray(uv_unit) > 0)
        full[:, :nh] = sel
        # cell (u, v) for v > n/2 is the mirror of (-u, n - v)
        for v in range(nh, n):
            full[:, v] = sel[(-qu) % n, n - v]
        return full
    assert bins.kind == SHELL_K
    nc = bins.nc
    qe = signed_index(nc)
    sel = (bins.lut == b).astype(np.float64)
    if uv_unit is not None:
        sel = sel * (np.asarray(uv_unit) > 0)[None]
    full = np.zeros((nc, n, n))
    full[:, :, :nh] = sel
    for v in range(nh, n):
        full[:, :, v] = sel[(-qe) % nc][:, (-qu) % n, n - v]
    return full


def pair_count(ia: np.ndarray, ib: np.ndarray, workers: int = 1,
               fa: Optional[np.ndarray] = None, fb: Optional[np.ndarray] = None) -> Tuple[np.ndarray, float]:
    """C_ab(k) = sum_k1 1_a(k1) 1_b(k - k1) (cyclic), rounded per cell to int64.

    Returns (C as int64, largest |C - rint(C)| before rounding).  fa, fb: precomputed fftn of
    the indicators (optional)."""
    fa = _fftn(ia, workers) if fa is None else fa
    fb = _fftn(ib, workers) if fb is None else fb
    c = _ifftn(fa * fb, workers)
    r = np.rint(c.real)
    dev = float(max(np.abs(c.real - r).max(), np.abs(c.imag).max())) if c.size else 0.0
    return r.astype(np.int64), dev


def exact_counts(bins: Bins, uv_unit: Optional[np.ndarray] = None, tri: Optional[np.ndarray] = None,
                 workers: int = 1) -> Tuple[np.ndarray, float]:
    """Exact int64 count of closed grid triangles for each bin triple of `tri` (default: all
    candidates), with unit weights on the uv occupancy `uv_unit` (None: every cell of the support).

    Ring bins give the per-channel-triple count T_perp of the MABS with separable unit weights
    (channel weights multiply it); shell bins give T3D of the 3D estimator.
    Returns (counts [ntri] int64, largest pair-count rounding deviation)."""
    tri = bins.triangles if tri is None else np.asarray(tri).reshape(-1, 3)
    out = np.zeros(len(tri), dtype=np.int64)
    if len(tri) == 0:
        return out, 0.0
    ind: Dict[int, np.ndarray] = {}
    fft: Dict[int, np.ndarray] = {}

    def indicator(b):
        if b not in ind:
            ind[b] = full_indicator(bins, b, uv_unit)
        return ind[b]

    def spectrum(b):
        if b not in fft:
            fft[b] = _fftn(indicator(b), workers)
        return fft[b]

    # group triangles by their (b1, b2) pair: one pair convolution serves every third bin
    groups: Dict[Tuple[int, int], list] = {}
    for t, (a, b, c) in enumerate(tri):
        groups.setdefault((int(a), int(b)), []).append((t, int(c)))
    dev = 0.0
    shape = indicator(int(tri[0][0])).shape
    neg = tuple((-np.arange(s)) % s for s in shape)
    for (a, b), items in groups.items():
        C, d = pair_count(None, None, workers, fa=spectrum(a), fb=spectrum(b))
        dev = max(dev, d)
        Cneg = C[np.ix_(*neg)]          # C_ab(-k)
        for t, c in items:
            out[t] = int(np.sum(Cneg[indicator(c) > 0], dtype=np.int64))
    if dev > ROUND_TOL:
        raise ArithmeticError(f"pair count off an integer by {dev}")
    return out, dev
