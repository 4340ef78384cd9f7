"""Decorrelation of non-closed baseline triplets by the primary beam (Eq. S3), as it enters the
gridded estimator.

Oracle (test infrastructure only; see the package docstring).

Sec. 3.1 (Eq. S3): the three-visibility correlation of baselines U1, U2, U3 + dU, where
U1 + U2 + U3 = 0, is the closed-triangle one times exp(-pi^2 theta_0^2 |dU|^2 / 3), theta_0 =
0.6 theta_F.  Sec. 3.2 grids each visibility to its nearest grid point (Eq. vg) and correlates
the gridded values at three grid points that close; the baselines behind them generally do not
close: with offsets delta_i = U_i - U_g from their grid points, a closed grid triangle correlates
baseline triplets whose non-closure is dU = delta_1 + delta_2 + delta_3 (Sec. 4 quotes the factor
0.89 for a typical |dU|^2 = dU_g^2 / 2).  With the cell-average weight W_g = 1/N_g, the expected
value of the estimator of a bin triangle is the true MABS times

    D = mean over the closed grid triangles T of the bin (all three cells sampled) of
        mean over the baseline triplets (i, j, k) of T's three cells of exp(-a |delta_i + delta_j + delta_k|^2),

a = pi^2 theta_0^2 / 3.  This module writes D out by enumeration (tiny grids only): the grid
assignment follows Eq. vg as in estimator.grid_visibilities (nearest point, a point with q_v < 0
stands for (-q_u, -q_v) with the baseline reversed, so its offset is negated; a point on the line
q_v = 0 also enters at (-q_u, 0) reversed), and the cells of the full plane with v > n/2 are the
mirrors of stored cells, with negated offsets.  Dividing an estimate by D corrects the
decorrelation bias (largest for the smallest rings, where Sec. 5 sees deviations).
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

from .bins import Bins, RING_U
from .brute import closed_triangles


def decorrelation_rate(theta0: float) -> float:
    """a of exp(-a |dU|^2) in Eq. S3 (dU in wavelengths): pi^2 theta_0^2 / 3."""
    return math.pi ** 2 * theta0 ** 2 / 3.0


def cell_offsets(n: int, uv: np.ndarray, du: float) -> Dict[int, np.ndarray]:
    """Offsets delta = U - U_g (wavelengths) of the baselines gridded into each cell of the FULL
    n x n plane (flat index u * n + v), with the Eq. vg reading of grid_visibilities."""
    uv = np.asarray(uv, dtype=np.float64)
    q = np.rint(uv / du).astype(np.int64)
    d = uv - du * q
    neg = q[:, 1] < 0
    q[neg] = -q[neg]
    d[neg] = -d[neg]
    keep = (np.abs(q[:, 0]) < n // 2) & (np.abs(q[:, 1]) < n // 2)
    half: Dict[tuple, List[np.ndarray]] = {}
    for (qu, qv), dd in zip(q[keep], d[keep]):
        half.setdefault((int(qu) % n, int(qv)), []).append(dd)
        if qv == 0:   # the reversed baseline on the stored line q_v = 0
            half.setdefault((int(-qu) % n, 0), []).append(-dd)
    full: Dict[int, np.ndarray] = {}
    for (iu, iv), lst in half.items():
        arr = np.array(lst)
        full[iu * n + iv] = arr
        if iv > 0:   # the mirror cell (-u, -v) of the full plane: reversed baselines
            full[((-iu) % n) * n + (n - iv)] = -arr
    return full


def decorrelation_factor(bins: Bins, uv: np.ndarray, du: float, theta0: float) -> np.ndarray:
    """D per candidate ring triangle (NaN where no closed grid triangle has all cells sampled)."""
    assert bins.kind == RING_U
    a = decorrelation_rate(theta0)
    offs = cell_offsets(bins.n, uv, du)
    out = np.full(len(bins.triangles), np.nan)
    for t, tri in enumerate(bins.triangles):
        (f1, f2, f3), _ = closed_triangles(bins, tri)
        vals = []
        for c1, c2, c3 in zip(f1, f2, f3):
            if int(c1) not in offs or int(c2) not in offs or int(c3) not in offs:
                continue
            d1, d2, d3 = offs[int(c1)], offs[int(c2)], offs[int(c3)]
            s = d1[:, None, None, :] + d2[None, :, None, :] + d3[None, None, :, :]
            vals.append(float(np.mean(np.exp(-a * np.sum(s * s, axis=-1)))))
        if vals:
            out[t] = float(np.mean(vals))
    return out
