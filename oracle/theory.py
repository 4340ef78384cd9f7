"""Closed forms that pin the estimator: quadratic-field bispectrum, N_nu sampling.

Oracle (test infrastructure only; see the package docstring).

Quadratic non-Gaussian field (Gill & Bharadwaj 2025, Sec. 4, Eq. mb1):
delta = g + f (g^2 - <g^2>), g Gaussian with <|g~(k)|^2> = N_vox P(k), P(0) = 0.
With unnormalised DFTs and <d~1 d~2 d~3> = N_vox B(k1,k2,k3) for k1+k2+k3 = 0
(all k_i != 0), Wick's theorem gives exactly

    B = 2 f [P1 P2 + P2 P3 + P3 P1]  +  (8 f^3 / N_vox) sum_q P(q) P(q - k1) P(q + k3).

The first term is the paper's first-order result, Eq. (bsana); the second is the
one-loop term (the f^2 terms vanish: they are odd moments of g).

Estimator expectations:
* 3D:   E[B_hat(b)] = mean of B over the closed grid triangles of bin triple b.
* MABS: B_A(U1,U2,U3; dnu1, dnu2) = nc^-2 sum_{a,b} exp(+2 pi i (a dnu1 + b dnu2)/nc)
        B((U1,a), (U2,b), (U3,-a-b)), the discrete inverse of Eq. (dft)
        (Sec. 2.2, Eq. 3dbs_mabs) on a periodic channel axis;
        E[B_hat_A(b; nu)] = mean over closed 2D triangles of B_A.

Sampling N_nu(dnu1, dnu2) (Sec. 5, Fig. 2): the number of channel triplets
(nu3 + dnu1, nu3 + dnu2, nu3) inside the band with all three channels unflagged.
"""
from __future__ import annotations

import numpy as np

from .bins import Bins, RING_U, SHELL_K, signed_index
from .brute import closed_triangles


def power_spectrum_full(kmag_full: np.ndarray, index: float, sigma: float) -> np.ndarray:
    """P on the full grid: A |k|^index with P(0) = 0 and (1/N_vox) sum_k P(k) = sigma^2."""
    with np.errstate(divide="ignore"):
        p = np.where(kmag_full > 0, kmag_full ** index, 0.0)
    return p * (sigma * sigma * p.size / p.sum())


def kmag_full_cubic(nc: int, n: int) -> np.ndarray:
    """|k| on the full [nc][n][n] grid with k = 2 pi (q_nu/nc, q_u/n, q_v/n)."""
    qe = signed_index(nc)[:, None, None] / nc
    qu = signed_index(n)[None, :, None] / n
    qv = signed_index(n)[None, None, :] / n
    return 2.0 * np.pi * np.sqrt(qe ** 2 + qu ** 2 + qv ** 2)


class QuadraticBispectrum:
    """Exact discrete bispectrum of the quadratic field on a periodic grid."""

    def __init__(self, p_full: np.ndarray, f: float):
        self.P = np.asarray(p_full, dtype=np.float64)
        self.shape = self.P.shape
        self.N = self.P.size
        self.f = f
        self.Pflat = self.P.ravel()
        self._Phat = np.fft.fftn(self.P)
        self._loop = {}

    def _loop_table(self, k1_flat: int) -> np.ndarray:
        """L[k3] = sum_q P(q) P(q - k1) P(q + k3) for one k1, all k3 (flat)."""
        if k1_flat not in self._loop:
            k1 = np.unravel_index(k1_flat, self.shape)
            g = self.P * np.roll(self.P, shift=k1, axis=tuple(range(self.P.ndim)))  # P(q) P(q - k1)
            corr = np.fft.ifftn(np.conj(np.fft.fftn(g)) * self._Phat).real
            self._loop[k1_flat] = corr.ravel()
        return self._loop[k1_flat]

    def __call__(self, k1: np.ndarray, k2: np.ndarray, k3: np.ndarray, loop: bool = True) -> np.ndarray:
        """B for arrays of flat indices with k1 + k2 + k3 = 0 on the grid."""
        p1, p2, p3 = self.Pflat[k1], self.Pflat[k2], self.Pflat[k3]
        out = 2.0 * self.f * (p1 * p2 + p2 * p3 + p3 * p1)
        if loop and self.f != 0.0:
            lt = np.empty(len(k1))
            for u in np.unique(k1):
                sel = k1 == u
                lt[sel] = self._loop_table(int(u))[k3[sel]]
            out = out + (8.0 * self.f ** 3 / self.N) * lt
        return out


def expected_3d(bins: Bins, qb: QuadraticBispectrum, tri3, loop: bool = True) -> float:
    """E[B_hat_3D] for one bin triple: mean of B over its closed grid triangles."""
    assert bins.kind == SHELL_K
    (f1, f2, f3), shape = closed_triangles(bins, tri3)
    assert shape == qb.shape
    if len(f1) == 0:
        return float("nan")
    return float(np.mean(qb(f1, f2, f3, loop=loop)))


def expected_mabs(bins: Bins, qb: QuadraticBispectrum, tri3, dnu1: int, dnu2: int, loop: bool = True) -> float:
    """E[B_hat_A] for one ring triple at channel separations (dnu1, dnu2), periodic channels."""
    assert bins.kind == RING_U
    nc, n = bins.nc, bins.n
    (g1, g2, g3), shape2 = closed_triangles(bins, tri3)
    if len(g1) == 0:
        return float("nan")
    a = np.arange(nc)
    A, Bq = np.meshgrid(a, a, indexing="ij")
    A, Bq = A.ravel(), Bq.ravel()
    C = (-(A + Bq)) % nc
    phase = np.exp(2j * np.pi * (A * dnu1 + Bq * dnu2) / nc)
    total = 0.0
    plane = n * n
    for u1, u2, u3 in zip(g1, g2, g3):
        k1 = A * plane + u1
        k2 = Bq * plane + u2
        k3 = C * plane + u3
        total += float(np.real(np.sum(phase * qb(k1, k2, k3, loop=loop)))) / (nc * nc)
    return total / len(g1)


def n_nu(nc: int, chan_w=None, circular: bool = False) -> np.ndarray:
    """N_nu(dnu1, dnu2) = sum_nu3 w(nu3 + dnu1) w(nu3 + dnu2) w(nu3) (Sec. 5, Fig. 2).

    Non-circular: [2nc-1][2nc-1] indexed by dnu + nc - 1; circular: [nc][nc] mod nc.
    """
    w = np.ones(nc) if chan_w is None else (np.asarray(chan_w) > 0).astype(np.int64)
    w = w.astype(np.int64)
    if circular:
        out = np.zeros((nc, nc), dtype=np.int64)
        for d1 in range(nc):
            for d2 in range(nc):
                out[d1, d2] = int(np.sum(np.roll(w, -d1) * np.roll(w, -d2) * w))
        return out
    size = 2 * nc - 1
    out = np.zeros((size, size), dtype=np.int64)
    for d1 in range(-(nc - 1), nc):
        # g(nu3) = w(nu3 + d1) w(nu3), zero where nu3 + d1 leaves the band
        g = np.zeros(nc, dtype=np.int64)
        lo, hi = max(0, -d1), min(nc, nc - d1)
        g[lo:hi] = w[lo + d1:hi + d1] * w[lo:hi]
        # out[d2] = sum_nu3 g(nu3) w(nu3 + d2): a full cross-correlation
        out[d1 + nc - 1, :] = np.correlate(w, g, mode="full")
    return out


def n_nu_unflagged_closed_form(nc: int, d1: int, d2: int) -> int:
    """nc - max(0, d1, d2) + min(0, d1, d2), and 0 when that is not positive."""
    return max(0, nc - max(0, d1, d2) + min(0, d1, d2))
