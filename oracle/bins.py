"""Ring and shell binning of the Fourier grid, and candidate bin triangles.

Oracle (test infrastructure only; see the package docstring).

Follows Sec. 3.2 of Gill & Bharadwaj 2025 (annular rings a_m of the uv plane,
Fig. 1) and, for the 3D bispectrum, spherical shells in |k| with
k = (k_perp, k_par) of Sec. 2 (k_perp = 2 pi U / r, Sec. 2.1; k_par from the
delay axis as in Eq. (dft)).  Triangles are ordered k1 >= k2 >= k3 by bin
index (Sec. 2.2, shape parameterisation Eq. (shape)).

Readings where the paper is silent:
* bins are half-open, e_j <= x < e_{j+1};
* the uv support is 1 <= |U| <= umax cells with umax = floor((n-1)/3) by default,
  which drops the uv DC and makes closure mod n equal to true closure;
* Nyquist rows/columns (q = -n/2) are never in support; along the delay axis
  the Nyquist plane is excluded as well;
* |k| is evaluated as sqrt(cperp^2 (qu^2+qv^2) + cpar^2 qeta^2) with
  cperp = 2 pi du / r and cpar = 2 pi / (r' nc dnu), in that operation order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

RING_U = 0
SHELL_K = 1


def signed_index(n: int) -> np.ndarray:
    """Signed FFT index q of bin i: i for i < n/2, i - n otherwise (so q(n/2) = -n/2)."""
    i = np.arange(n, dtype=np.int64)
    return np.where(i < (n + 1) // 2, i, i - n)


def _uv_q2(n: int):
    """(qu, qv) integer grids on the [n][n//2+1] half plane."""
    qu = signed_index(n)[:, None]
    qv = np.arange(n // 2 + 1, dtype=np.int64)[None, :]
    return qu, qv


def uv_support(n: int, umax: float) -> np.ndarray:
    """Boolean [n][nh]: 1 <= |U| <= umax and no Nyquist row/column."""
    qu, qv = _uv_q2(n)
    r = np.sqrt((qu * qu + qv * qv).astype(np.float64))
    sup = (r >= 1.0) & (r <= umax)
    if n % 2 == 0:
        sup &= (qu != -n // 2) & (qv != n // 2)
    return sup


def bin_index(x: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """Half-open bin of x in edges: j with e_j <= x < e_{j+1}, else -1."""
    j = np.searchsorted(edges, x, side="right") - 1
    j = np.where((j >= 0) & (j < len(edges) - 1), j, -1)
    return j.astype(np.int32)


def half_weight(n: int) -> np.ndarray:
    """Multiplicity of each half-plane column in the full grid: 1 for v = 0 (and n/2), else 2."""
    nh = n // 2 + 1
    w = np.full(nh, 2, dtype=np.int64)
    w[0] = 1
    if n % 2 == 0:
        w[-1] = 1
    return w


@dataclass
class Bins:
    kind: int
    n: int
    nc: int
    edges: np.ndarray
    umax: float
    lut: np.ndarray          # ring: [n][nh]; shell: [nc][n][nh]; int32 bin or -1
    modes: np.ndarray        # [nbins] int64, modes over the full Fourier grid
    triangles: np.ndarray    # [ncand][3] int32, b1 >= b2 >= b3
    true_closure: bool       # True when closure mod the grid equals true closure
    eta_max: int = 0         # largest |q_eta| in any shell (shells only)

    @property
    def nbins(self) -> int:
        return len(self.edges) - 1

    @property
    def nh(self) -> int:
        return self.n // 2 + 1


def shell_kmag(n: int, nc: int, du: float, r_mpc: float, rprime: float, dnu: float) -> np.ndarray:
    """|k| in Mpc^-1 on the [nc][n][nh] grid (delay axis first)."""
    cperp = 2.0 * math.pi * du / r_mpc
    cpar = 2.0 * math.pi / (rprime * nc * dnu)
    qu, qv = _uv_q2(n)
    qe = signed_index(nc)[:, None, None]
    s_perp = (qu * qu + qv * qv)[None, :, :].astype(np.float64)
    s_par = (qe * qe).astype(np.float64)
    kp2 = (cperp * cperp) * s_perp
    kl2 = (cpar * cpar) * s_par
    return np.sqrt(kp2 + kl2)


def candidate_triangles(edges: np.ndarray, nonempty: np.ndarray, true_closure: bool) -> np.ndarray:
    """Sorted bin triples b1 >= b2 >= b3 over non-empty bins.

    Under true closure a triangle with |k1| in bin b1 needs |k1| <= |k2| + |k3|,
    hence e_{b1} < e_{b2+1} + e_{b3+1}; triples failing that can never close and
    are dropped.  With mod-grid aliasing (a umax override) no triple is dropped.
    """
    nb = len(edges) - 1
    out = []
    for b1 in range(nb):
        if not nonempty[b1]:
            continue
        for b2 in range(b1 + 1):
            if not nonempty[b2]:
                continue
            for b3 in range(b2 + 1):
                if not nonempty[b3]:
                    continue
                if true_closure and not (edges[b2 + 1] + edges[b3 + 1] > edges[b1]):
                    continue
                out.append((b1, b2, b3))
    return np.asarray(out, dtype=np.int32).reshape(-1, 3)


def make_bins(kind: int, n: int, nc: int, edges, umax: Optional[float] = None,
              du: float = 1.0, r_mpc: float = 1.0, rprime: float = 1.0, dnu: float = 1.0) -> Bins:
    """Bin plan: per-cell bin LUT, per-bin mode counts and candidate triangles."""
    edges = np.asarray(edges, dtype=np.float64)
    if edges.ndim != 1 or len(edges) < 2 or not np.all(np.diff(edges) > 0) or not np.all(np.isfinite(edges)):
        raise ValueError("edges must be finite and strictly increasing")
    if umax is None:
        umax = float((n - 1) // 3)
    sup = uv_support(n, umax)
    hw = half_weight(n)
    if kind == RING_U:
        qu, qv = _uv_q2(n)
        r = np.sqrt((qu * qu + qv * qv).astype(np.float64))
        lut = np.where(sup, bin_index(r, edges), -1).astype(np.int32)
        modes = np.array([(hw[None, :] * (lut == b)).sum() for b in range(len(edges) - 1)], dtype=np.int64)
        true_closure = 3 * umax < n
        eta_max = 0
    elif kind == SHELL_K:
        k = shell_kmag(n, nc, du, r_mpc, rprime, dnu)
        lut = bin_index(k, edges)
        lut = np.where(sup[None, :, :], lut, -1)
        qe = signed_index(nc)
        if nc % 2 == 0:
            lut[qe == -nc // 2] = -1
        lut = lut.astype(np.int32)
        modes = np.array([(hw[None, None, :] * (lut == b)).sum() for b in range(len(edges) - 1)],
                         dtype=np.int64)
        in_any = (lut >= 0).any(axis=(1, 2))
        eta_max = int(np.abs(qe[in_any]).max()) if in_any.any() else 0
        true_closure = (3 * umax < n) and (3 * eta_max < nc)
    else:
        raise ValueError("kind must be RING_U or SHELL_K")
    tri = candidate_triangles(edges, modes > 0, true_closure)
    return Bins(kind=kind, n=n, nc=nc, edges=edges, umax=float(umax), lut=lut, modes=modes,
                triangles=tri, true_closure=bool(true_closure), eta_max=eta_max)
