"""FFT-route estimators for the MABS and the 3D bispectrum, in float64.

Oracle (test infrastructure only; see the package docstring).

MABS (Gill & Bharadwaj 2025, Sec. 3.2):
  * D(l_m, nu, theta): inverse FT of W_g V_g restricted to ring a_m (Eq. iFT);
  * I(l_m, nu, theta): inverse FT of W_g N_g restricted to ring a_m (Eq. iFT_I),
    where W_g N_g is the unit-weight sampling indicator [N_g > 0];
  * B_A = (1/A) sum_theta D1 D2 D3 / sum_theta I1 I2 I3 (Eq. estimator_t).
  The grid-unit normalisation used here: with NumPy's ifft (1/N_pix),
  sum_theta D1 D2 D3 = N_pix^-2 sum over closed triangles of X1 X2 X3 and
  sum_theta I1 I2 I3 = N_pix^-2 * (number of closed triangles), so
  N_tri = N_pix^2 S_I and B = norm * N_pix * S_D / N_tri is the average of
  X1 X2 X3 / N_pix over closed grid triangles (Sec. 3.2, the paragraph after
  Eq. estimator_t).  `norm` stands for 1/A.
  Ergodic collapse to (dnu1, dnu2) = (nu1 - nu3, nu2 - nu3) averages the
  per-triplet estimates (Sec. 3.2, the paragraph before Eq. dft), and Eq. (dft)
  takes the collapsed MABS to the cylindrical 3D BS by a 2D DFT over the
  separations (mabs_dft).

3D bispectrum: the delay transform along frequency is applied to the weighted
cube, the 3D grid is split into |k| shells, each shell is inverse-FFT'd to a
real field and the same triple-product estimator is formed over voxels.  This
regroups the paper's MABS -> Eq. (dft) route by 3D |k| shells (the identity is
checked in tests/test_oracle_pins.py).  Flagged channels enter through
rho3 = mean_nu w(nu)^3: N_eff = T3D * rho3 and B = norm * N_vox * S_D / N_eff.

Weights (Sec. 3.2, Eq. vg): W_g = 1/N_g on filled cells, 0 on empty ones.
Separable form: uv occupancy m(U) times channel weight w(nu) in {0, 1}.
Non-Hermitian v = 0 (and Nyquist) columns are symmetrised as
(X(u) + conj X(-u)) / 2 before the inverse transform.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Iterable, Optional, Tuple

import numpy as np

from .bins import Bins, RING_U, SHELL_K

COUNT_TOL = 1e-3   # largest |x - round(x)| accepted before rounding a count


@dataclass
class Weights:
    """Exactly one of (ng) or (uv_mask, chan_w) is used; all None means unit weights."""
    ng: Optional[np.ndarray] = None        # [nc][n][nh] cell counts N_g
    uv_mask: Optional[np.ndarray] = None   # [n][nh] occupancy 0/1
    chan_w: Optional[np.ndarray] = None    # [nc] channel weight 0/1

    def separable(self) -> bool:
        return self.ng is None

    def data_weight(self, nc: int, n: int) -> np.ndarray:
        """W_g[nu][u][v]."""
        nh = n // 2 + 1
        if self.ng is not None:
            ng = np.asarray(self.ng, dtype=np.float64)
            with np.errstate(divide="ignore"):
                return np.where(ng > 0, 1.0 / ng, 0.0)
        m = np.ones((n, nh)) if self.uv_mask is None else np.asarray(self.uv_mask, dtype=np.float64)
        w = np.ones(nc) if self.chan_w is None else np.asarray(self.chan_w, dtype=np.float64)
        return w[:, None, None] * m[None, :, :]

    def unit_weight(self, nc: int, n: int) -> np.ndarray:
        """W_g N_g = [N_g > 0] on [nu][u][v]."""
        if self.ng is not None:
            return (np.asarray(self.ng) > 0).astype(np.float64)
        return (self.data_weight(nc, n) > 0).astype(np.float64)

    def uv_unit(self, n: int) -> np.ndarray:
        nh = n // 2 + 1
        return np.ones((n, nh)) if self.uv_mask is None else (np.asarray(self.uv_mask) > 0).astype(np.float64)

    def chan(self, nc: int) -> np.ndarray:
        return np.ones(nc) if self.chan_w is None else np.asarray(self.chan_w, dtype=np.float64)


def symmetrize_columns(x: np.ndarray, n: int) -> np.ndarray:
    """Replace the self-conjugate half-plane columns (v = 0, and v = n/2 for even n)
    by (X(u) + conj X(-u)) / 2 along the u axis (second-to-last)."""
    x = np.array(x, dtype=np.complex128, copy=True)
    neg = (-np.arange(n)) % n
    cols = [0] + ([n // 2] if n % 2 == 0 else [])
    for c in cols:
        col = x[..., :, c]
        x[..., :, c] = 0.5 * (col + np.conj(col[..., neg]))
    return x


def round_counts(x: np.ndarray) -> Tuple[np.ndarray, float]:
    """Round float triangle counts to int64; returns (counts, max |x - round(x)|)."""
    r = np.rint(x)
    dev = float(np.max(np.abs(x - r))) if x.size else 0.0
    return r.astype(np.int64), dev


# ---------------------------------------------------------------------------
# MABS
# ---------------------------------------------------------------------------
def grid_visibilities(uv: np.ndarray, vis: np.ndarray, flags: Optional[np.ndarray], n: int, du: float,
                      chan_avg: int = 1):
    """Eq. (vg): nearest-grid-point gridding of visibilities on the n x n uv grid of spacing du.

    Visibility i has baseline uv[i] (wavelengths, the same in every channel) and values vis[nu][i];
    F = 1 - flags[nu][i] (flags nonzero = flagged, None = nothing flagged).  Its grid point is
    q = rint(U / du) per axis; a grid point with q_v < 0 stands for (-q_u, -q_v) with the
    visibility conjugated (V(-U) = V*(U) for a real sky), so that the grid is the half plane
    q_v >= 0 stored as [nu][q_u mod n][q_v].  That half plane holds both halves of the line
    q_v = 0, so a visibility on it enters at (q_u, 0) and, conjugated, at (-q_u, 0) (the same
    cell twice for q_u = 0), as its mirror baseline would.  Grid points with |q_u| or |q_v| >= n/2
    are dropped.
    V_g = sum of F V and N_g = sum of F over the visibilities of a grid point; chan_avg consecutive
    channels are gridded together (the channel collapse of Sec. 4).
    Returns (V_g [nc / chan_avg][n][n/2+1] complex128, N_g int64 of the same shape).
    """
    vis = np.asarray(vis)
    nc, nvis = vis.shape
    nco = nc // chan_avg
    nh = n // 2 + 1
    q = np.rint(np.asarray(uv, dtype=np.float64) / du).astype(np.int64)
    neg = q[:, 1] < 0
    q[neg] = -q[neg]
    keep = (np.abs(q[:, 0]) < n // 2) & (np.abs(q[:, 1]) < n // 2)
    cell = (q[:, 0] % n) * nh + q[:, 1]
    F = np.ones((nc, nvis)) if flags is None else 1.0 - (np.asarray(flags) != 0)
    V = np.where(neg[None, :], np.conj(vis), vis).astype(np.complex128) * F
    # the mirror entries of the line q_v = 0
    line = keep & (q[:, 1] == 0)
    cell = np.concatenate([cell, (-q[line, 0]) % n * nh])
    keep = np.concatenate([keep, np.ones(int(line.sum()), dtype=bool)])
    V = np.concatenate([V, np.conj(V[:, line])], axis=1)
    F = np.concatenate([F, F[:, line]], axis=1)
    Vg = np.zeros((nco, n * nh), dtype=np.complex128)
    Ng = np.zeros((nco, n * nh), dtype=np.int64)
    for c in range(nco * chan_avg):
        o = c // chan_avg
        np.add.at(Vg[o], cell[keep], V[c][keep])
        np.add.at(Ng[o], cell[keep], F[c][keep].astype(np.int64))
    return Vg.reshape(nco, n, nh), Ng.reshape(nco, n, nh)


class MabsFields:
    """Lazily computed ring-filtered fields D_b(nu) and I_b(nu) (Eqs. iFT, iFT_I)."""

    def __init__(self, bins: Bins, vis: np.ndarray, weights: Optional[Weights] = None):
        assert bins.kind == RING_U
        self.bins = bins
        self.n, self.nc = bins.n, bins.nc
        self.vis = np.asarray(vis)
        self.w = weights or Weights()
        self.W = self.w.data_weight(self.nc, self.n)
        self.Y = self.w.unit_weight(self.nc, self.n)
        self._d: Dict[int, np.ndarray] = {}
        self._i: Dict[int, np.ndarray] = {}

    def data(self, b: int) -> np.ndarray:
        """D_b[nu][x][y], real, for all channels."""
        if b not in self._d:
            ring = (self.bins.lut == b).astype(np.float64)
            x = ring[None] * self.W * self.vis
            x = symmetrize_columns(x, self.n)
            self._d[b] = np.fft.irfft2(x, s=(self.n, self.n), axes=(1, 2))
        return self._d[b]

    def count(self, b: int) -> np.ndarray:
        """I_b[nu][x][y]: inverse FT of the unit-weight indicator on ring b."""
        if b not in self._i:
            ring = (self.bins.lut == b).astype(np.float64)
            y = symmetrize_columns(ring[None] * self.Y, self.n)
            self._i[b] = np.fft.irfft2(y, s=(self.n, self.n), axes=(1, 2))
        return self._i[b]


def triple_sum(a: np.ndarray, b: np.ndarray, c: np.ndarray) -> np.ndarray:
    """S[i][j][k] = sum_p a[i,p] b[j,p] c[k,p] for a [n1][P], b [n2][P], c [n3][P]."""
    out = np.empty((a.shape[0], b.shape[0], c.shape[0]))
    for i in range(a.shape[0]):
        out[i] = (a[i][None, :] * b) @ c.T
    return out


def estimate_mabs(bins: Bins, vis: np.ndarray, weights: Optional[Weights] = None,
                  tri: Optional[np.ndarray] = None, nu1: Optional[Iterable[int]] = None,
                  norm: float = 1.0, fields: Optional[MabsFields] = None):
    """Full MABS over all (nu2, nu3) for each triangle and each nu1 in `nu1`.

    Returns (B [nt][n1][nc][nc], N_tri [nt][n1][nc][nc], S_D, max count deviation).
    B is NaN where N_tri = 0.
    """
    f = fields or MabsFields(bins, vis, weights)
    tri = bins.triangles if tri is None else np.asarray(tri).reshape(-1, 3)
    nu1 = np.arange(bins.nc) if nu1 is None else np.asarray(list(nu1), dtype=np.int64)
    npix = bins.n * bins.n
    nt = len(tri)
    S = np.empty((nt, len(nu1), bins.nc, bins.nc))
    N = np.empty((nt, len(nu1), bins.nc, bins.nc), dtype=np.int64)
    dev = 0.0
    for t, (b1, b2, b3) in enumerate(tri):
        d1 = f.data(b1).reshape(bins.nc, -1)[nu1]
        d2 = f.data(b2).reshape(bins.nc, -1)
        d3 = f.data(b3).reshape(bins.nc, -1)
        S[t] = triple_sum(d1, d2, d3)
        i1 = f.count(b1).reshape(bins.nc, -1)[nu1]
        i2 = f.count(b2).reshape(bins.nc, -1)
        i3 = f.count(b3).reshape(bins.nc, -1)
        cnt, dv = round_counts(float(npix) * float(npix) * triple_sum(i1, i2, i3))
        N[t] = cnt
        dev = max(dev, dv)
    with np.errstate(invalid="ignore", divide="ignore"):
        B = np.where(N > 0, norm * npix * S / np.where(N > 0, N, 1), np.nan)
    return B, N, S, dev


def mabs_entry(fields: MabsFields, tri3, nu) -> Tuple[float, int, float]:
    """One MABS entry (b1,b2,b3; nu1,nu2,nu3): (S_D, N_tri, S_I) computed directly."""
    b1, b2, b3 = (int(x) for x in tri3)
    n1, n2, n3 = (int(x) for x in nu)
    sd = float(np.sum(fields.data(b1)[n1] * fields.data(b2)[n2] * fields.data(b3)[n3]))
    si = float(np.sum(fields.count(b1)[n1] * fields.count(b2)[n2] * fields.count(b3)[n3]))
    npix = fields.n * fields.n
    return sd, int(np.rint(npix * npix * si)), si


def collapse_mabs(B: np.ndarray, N: np.ndarray, circular: bool = False):
    """Ergodic collapse of a full MABS [nt][nc][nc][nc] to (dnu1, dnu2).

    Non-circular: Bbar[t][d1 + nc - 1][d2 + nc - 1] is the mean of B(nu3 + d1, nu3 + d2, nu3)
    over nu3 with all three channels inside [0, nc) and N_tri > 0; N_nu counts those
    nu3 and Ntot sums their N_tri.  Circular: channel indices are taken mod nc and the
    output is [nt][nc][nc] indexed by (d1 mod nc, d2 mod nc).
    """
    nt, nc = B.shape[0], B.shape[1]
    size = nc if circular else 2 * nc - 1
    Bbar = np.full((nt, size, size), np.nan)
    Nnu = np.zeros((nt, size, size), dtype=np.int64)
    Ntot = np.zeros((nt, size, size), dtype=np.int64)
    drange = range(0, nc) if circular else range(-(nc - 1), nc)
    for t in range(nt):
        for d1 in drange:
            for d2 in drange:
                acc, cnt, tot = 0.0, 0, 0
                for n3 in range(nc):
                    a, b = n3 + d1, n3 + d2
                    if circular:
                        a, b = a % nc, b % nc
                    elif not (0 <= a < nc and 0 <= b < nc):
                        continue
                    if N[t, a, b, n3] > 0:
                        acc += B[t, a, b, n3]
                        cnt += 1
                        tot += int(N[t, a, b, n3])
                i1 = d1 if circular else d1 + nc - 1
                i2 = d2 if circular else d2 + nc - 1
                Nnu[t, i1, i2] = cnt
                Ntot[t, i1, i2] = tot
                if cnt:
                    Bbar[t, i1, i2] = acc / cnt
    return Bbar, Nnu, Ntot


def mabs_dft(Bbar: np.ndarray, scale: float = 1.0, circular: bool = False) -> np.ndarray:
    """Eq. (dft): 2D DFT of the collapsed MABS over the separations (n, m) channels.

    out[t][a][b] = scale * sum_{n,m} exp(-2 pi i (n a + m b) / nc) Bbar_t(n, m), with n and m
    over the half-open range [-nc/2, nc/2), i.e. -h .. nc - 1 - h for h = nc // 2: one period,
    each separation once (the printed limits would count the end separation +-nc/2 twice).
    a, b in [0, nc) index k_par = 2 pi a / (r' B_bw) (a >= nc/2 are the negative frequencies).
    scale stands for (r^2 r' dnu_c)^2.  Bbar is a collapse from collapse_mabs: non-circular
    [nt][2nc-1][2nc-1] (separation d at d + nc - 1) or circular [nt][nc][nc] (d at d mod nc).
    Separations with no sampled triplet (NaN) contribute nothing.
    """
    Bbar = np.asarray(Bbar, dtype=np.float64)
    size = Bbar.shape[1]
    nc = size if circular else (size + 1) // 2
    h = nc // 2
    d = np.arange(-h, nc - h)
    idx = d % nc if circular else d + nc - 1
    A = Bbar[:, idx][:, :, idx]
    A = np.where(np.isnan(A), 0.0, A)
    a = np.arange(nc)
    # phase (a d mod nc) / nc taken exactly in integers before the exponential
    E = np.exp(-2j * np.pi * (np.outer(a, d) % nc) / nc)
    return scale * np.matmul(np.matmul(E, A), E.T)


# Shape bins of the monopole: 5 linear bins over [0.5, 1] in mu and in t (Sec. 5)
SHAPE_EDGES = (0.5, 0.6, 0.7, 0.8, 0.9, 1.0)


def triangle_shape(kperp: np.ndarray, kpar1: np.ndarray, kpar2: np.ndarray):
    """Size and shape (k1, mu, t) of cylindrical triangles (Eq. shape).

    Sides k_i = sqrt(kperp_i^2 + kpar_i^2) with kpar3 = -(kpar1 + kpar2) (the three wave vectors
    close), relabelled so that k1 >= k2 >= k3; t = k2 / k1 and mu = -k1.k2 / (k1 k2) where closure
    gives k1.k2 = (k3^2 - k1^2 - k2^2) / 2, i.e. mu = (k1^2 + k2^2 - k3^2) / (2 k1 k2).  mu and t
    are clamped to [0.5, 1] (their range for a closed triangle; ring-averaged kperp need not close
    exactly).  kperp: [..., 3]; kpar1, kpar2 broadcast against kperp[..., 0].
    """
    kpar3 = -(kpar1 + kpar2)
    s = np.stack([kperp[..., 0] * kperp[..., 0] + kpar1 * kpar1,
                  kperp[..., 1] * kperp[..., 1] + kpar2 * kpar2,
                  kperp[..., 2] * kperp[..., 2] + kpar3 * kpar3], axis=-1)
    s = -np.sort(-s, axis=-1)
    k1, k2 = np.sqrt(s[..., 0]), np.sqrt(s[..., 1])
    mu = ((s[..., 0] + s[..., 1]) - s[..., 2]) / (2.0 * (k1 * k2))
    t = k2 / k1
    return k1, np.clip(mu, 0.5, 1.0), np.clip(t, 0.5, 1.0)


def shape_bin(x: np.ndarray) -> np.ndarray:
    """Bin of mu or t in [0.5, 1]: half-open [e_j, e_j+1), the last bin closed at 1."""
    return np.minimum(np.searchsorted(np.asarray(SHAPE_EDGES), x, side="right") - 1, 4)


def bs_monopole(Bcyl: np.ndarray, kperp: np.ndarray, kpar_unit: float, k1_edges: np.ndarray):
    """Monopole B(k1, mu, t) of cylindrical 3D BS estimates (Sec. 2.2 Eq. shape, Sec. 5).

    Bcyl: [nt][nc][nc] complex, the output of Eq. (dft) for nt ring triples, index a of the
    first separation and b of the second (k_par = kpar_unit * a', a' = a for 2a < nc, else a - nc);
    kperp: [nt][3] the k_perp of the three rings.  Without redshift-space distortion the BS does
    not depend on the orientation, so the monopole of a (k1, mu, t) bin is the mean of Re B over
    every cylindrical cell whose triangle falls in it: k1 bins half-open on k1_edges (cells
    outside are dropped), 5 x 5 shape bins (shape_bin).  Returns (mean [nk][5][5], NaN where
    empty, and the cell count [nk][5][5]).
    """
    Bcyl = np.asarray(Bcyl)
    nt, nc = Bcyl.shape[0], Bcyl.shape[1]
    k1_edges = np.asarray(k1_edges, dtype=np.float64)
    nk = len(k1_edges) - 1
    a = np.arange(nc)
    kp = kpar_unit * np.where(2 * a < nc, a, a - nc).astype(np.float64)
    sums = np.zeros(nk * 25)
    counts = np.zeros(nk * 25, dtype=np.int64)
    for t in range(nt):
        kpt = np.broadcast_to(np.asarray(kperp[t], dtype=np.float64), (nc, nc, 3))
        k1, mu, tt = triangle_shape(kpt, kp[:, None], kp[None, :])
        j = np.searchsorted(k1_edges, k1, side="right") - 1
        ok = (j >= 0) & (j < nk)
        idx = (j * 25 + shape_bin(mu) * 5 + shape_bin(tt))[ok]
        sums += np.bincount(idx, weights=np.real(Bcyl[t])[ok], minlength=nk * 25)
        counts += np.bincount(idx, minlength=nk * 25)
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.where(counts > 0, sums / np.maximum(counts, 1), np.nan)
    return mean.reshape(nk, 5, 5), counts.reshape(nk, 5, 5)


def kpar_bins(kpar: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """Bin of each k_par on increasing edges: half-open [e_i, e_i+1), the last bin closed at its
    top edge; -1 outside."""
    edges = np.asarray(edges, dtype=np.float64)
    ne = len(edges) - 1
    i = np.searchsorted(edges, kpar, side="right") - 1
    i = np.where(kpar == edges[-1], ne - 1, i)
    return np.where((i >= 0) & (i < ne), i, -1)


def bs_kpar_grid(Bcyl: np.ndarray, kpar_unit: float, edges: np.ndarray):
    """Cylindrical 3D BS of each ring triple binned on a (k_par1, k_par2) grid (Sec. 5, Fig. 4).

    Cell (a, b) of Eq. (dft)'s output has k_par1 = kpar_unit a', k_par2 = kpar_unit b' (a' = a for
    2a < nc, else a - nc); the same edges bin both axes (kpar_bins) and a bin's value is the mean of
    Re B over its cells.  Returns (mean [nt][ne][ne], NaN where empty, and the cell count [ne][ne],
    which does not depend on the triangle)."""
    Bcyl = np.asarray(Bcyl)
    nt, nc = Bcyl.shape[0], Bcyl.shape[1]
    ne = len(edges) - 1
    a = np.arange(nc)
    kp = kpar_unit * np.where(2 * a < nc, a, a - nc).astype(np.float64)
    ib = kpar_bins(kp, edges)
    ok = (ib[:, None] >= 0) & (ib[None, :] >= 0)
    idx = (ib[:, None] * ne + ib[None, :])[ok]
    counts = np.bincount(idx, minlength=ne * ne)
    mean = np.full((nt, ne * ne), np.nan)
    for t in range(nt):
        sums = np.bincount(idx, weights=np.real(Bcyl[t])[ok], minlength=ne * ne)
        with np.errstate(invalid="ignore", divide="ignore"):
            mean[t] = np.where(counts > 0, sums / np.maximum(counts, 1), np.nan)
    return mean.reshape(nt, ne, ne), counts.reshape(ne, ne).astype(np.int64)


COLLINEAR_TOL = 1e-9   # mu above 1 - COLLINEAR_TOL: collinear sides, azimuth undefined


def triangle_orientation(kperp: np.ndarray, kpar1: np.ndarray, kpar2: np.ndarray):
    """Line-of-sight direction p = (p_x, p_y, p_z) in the frame of a cylindrical triangle (Eq. orient).

    The sides are sorted as in triangle_shape (k1 >= k2 >= k3, vectors k_1, k_2 of the two largest
    sides, kpar3 = -(kpar1 + kpar2)).  The frame puts k_1 along z and k_2 in the x-z plane with a
    positive x component, k_2 / k2 = (sqrt(1 - mu^2), 0, -mu); the line of sight then has
    p_z = mu_1 = kpar(k_1) / k1 and mu_2 = kpar(k_2) / k2 = -mu p_z + sqrt(1 - mu^2) p_x (Eq. orient),
    so p_x = (mu_2 + mu p_z) / sqrt(1 - mu^2) and p_y = +sqrt(1 - p_x^2 - p_z^2) (the mirror image,
    p_y -> -p_y, describes the same triangle; the sign is taken positive).  mu is the clamped shape
    parameter of triangle_shape; p_x is clamped to |p_x| <= sqrt(1 - p_z^2) (ring-averaged kperp need
    not close exactly).  Where the sides are collinear the azimuth is undefined; numerically that is
    taken as mu > 1 - COLLINEAR_TOL (mu from the closure formula, the same numbers as the shape
    bins): there sqrt(1 - mu^2) < 4.5e-5 and the rounding of mu (~1e-16) would make p_x arbitrary,
    so p_x and p_y are returned as NaN.  Returns (p_x, p_y, p_z)."""
    kpar3 = -(kpar1 + kpar2)
    kp = np.stack(np.broadcast_arrays(kpar1, kpar2, kpar3), axis=-1).astype(np.float64)
    s = np.stack([kperp[..., 0] * kperp[..., 0] + kp[..., 0] * kp[..., 0],
                  kperp[..., 1] * kperp[..., 1] + kp[..., 1] * kp[..., 1],
                  kperp[..., 2] * kperp[..., 2] + kp[..., 2] * kp[..., 2]], axis=-1)
    order = np.argsort(-s, axis=-1, kind="stable")
    s_sorted = np.take_along_axis(s, order, axis=-1)
    kp_sorted = np.take_along_axis(kp, order, axis=-1)
    k1, k2 = np.sqrt(s_sorted[..., 0]), np.sqrt(s_sorted[..., 1])
    mu = np.clip(((s_sorted[..., 0] + s_sorted[..., 1]) - s_sorted[..., 2]) / (2.0 * (k1 * k2)), 0.5, 1.0)
    pz = kp_sorted[..., 0] / k1
    mu2 = kp_sorted[..., 1] / k2
    sq = np.sqrt(np.maximum(1.0 - mu * mu, 0.0))
    defined = mu <= 1.0 - COLLINEAR_TOL
    with np.errstate(invalid="ignore", divide="ignore"):
        px = np.where(defined, (mu2 + mu * pz) / np.where(defined, sq, 1.0), np.nan)
    st = np.sqrt(np.maximum(1.0 - pz * pz, 0.0))
    px = np.clip(px, -st, st)
    py = np.sqrt(np.maximum(1.0 - pz * pz - px * px, 0.0))
    py = np.where(np.isnan(px), np.nan, py)
    return px, py, pz


def lm_pairs(lmax: int):
    """(l, m) in the order of the moments: l = 0 .. lmax, m = 0 .. l."""
    return [(l, m) for l in range(lmax + 1) for m in range(l + 1)]


def bs_multipoles(Bcyl: np.ndarray, kperp: np.ndarray, kpar_unit: float, k1_edges: np.ndarray, lmax: int):
    """Multipole moments B_l^m(k1, mu, t) of cylindrical 3D BS estimates (Eqs. orient, bs_lm).

    Eq. bs_lm integrates [Y_l^m(p)]* B over the orientations p of the line of sight; a (k1, mu, t)
    bin samples orientations through its cells, so the integral over the sphere is taken as 4 pi
    times the mean over the bin's cells:
        B_l^m = sqrt(4 pi (2l + 1)) mean over cells of Re[Y_l^m(p)]* Re B,
    where the real part of Y* is the mean over the two mirror orientations (p_y and -p_y) that a
    cylindrical cell stands for (Y_l^m from scipy.special, Condon-Shortley phase).  m < 0 follows
    from B_l^-m = (-1)^m B_l^m.  Cells whose sides are collinear (mu > 1 - COLLINEAR_TOL, azimuth
    undefined) add the azimuthal mean, 0, to m > 0.  l = 0 is the monopole (bs_monopole).  Bins and cells as in
    bs_monopole.  Returns (moments [n_lm][nk][5][5] in lm_pairs order, NaN where the bin is empty,
    and the cell count [nk][5][5])."""
    from scipy.special import sph_harm_y
    Bcyl = np.asarray(Bcyl)
    nt, nc = Bcyl.shape[0], Bcyl.shape[1]
    k1_edges = np.asarray(k1_edges, dtype=np.float64)
    nk = len(k1_edges) - 1
    pairs = lm_pairs(lmax)
    a = np.arange(nc)
    kp = kpar_unit * np.where(2 * a < nc, a, a - nc).astype(np.float64)
    sums = np.zeros((len(pairs), nk * 25))
    counts = np.zeros(nk * 25, dtype=np.int64)
    for t in range(nt):
        kpt = np.broadcast_to(np.asarray(kperp[t], dtype=np.float64), (nc, nc, 3))
        k1, mu, tt = triangle_shape(kpt, kp[:, None], kp[None, :])
        px, py, pz = triangle_orientation(kpt, kp[:, None], kp[None, :])
        j = np.searchsorted(k1_edges, k1, side="right") - 1
        ok = (j >= 0) & (j < nk)
        idx = (j * 25 + shape_bin(mu) * 5 + shape_bin(tt))[ok]
        counts += np.bincount(idx, minlength=nk * 25)
        theta = np.arccos(np.clip(pz[ok], -1.0, 1.0))
        collinear = np.isnan(px[ok])
        phi = np.where(collinear, 0.0, np.arctan2(np.nan_to_num(py[ok]), np.nan_to_num(px[ok])))
        re_b = np.real(Bcyl[t])[ok]
        for i, (l, m) in enumerate(pairs):
            y = np.real(np.conj(sph_harm_y(l, m, theta, phi)))
            if m > 0:
                y = np.where(collinear, 0.0, y)
            sums[i] += np.bincount(idx, weights=np.sqrt(4 * np.pi * (2 * l + 1)) * y * re_b, minlength=nk * 25)
    with np.errstate(invalid="ignore", divide="ignore"):
        mom = np.where(counts[None, :] > 0, sums / np.maximum(counts, 1)[None, :], np.nan)
    return mom.reshape(len(pairs), nk, 5, 5), counts.reshape(nk, 5, 5)


# ---------------------------------------------------------------------------
# 3D bispectrum
# ---------------------------------------------------------------------------
def delay_transform(vis: np.ndarray, weights: Optional[Weights] = None) -> np.ndarray:
    """Vt[eta][u][v] = sum_nu w(nu) m(U) V(U, nu) exp(-2 pi i eta nu / nc) (forward DFT over nu)."""
    w = weights or Weights()
    if not w.separable():
        raise NotImplementedError("3D estimator needs separable weights")
    nc, n = vis.shape[0], vis.shape[1]
    x = symmetrize_columns(np.asarray(vis) * w.data_weight(nc, n), n)
    return np.fft.fft(x, axis=0)


class ShellFields:
    """Lazily computed shell-filtered real fields F_j and count fields I_j over (eta, u, v)."""

    def __init__(self, bins: Bins, vis: np.ndarray, weights: Optional[Weights] = None):
        assert bins.kind == SHELL_K
        self.bins = bins
        self.w = weights or Weights()
        self.vt = delay_transform(vis, self.w)
        self.m = self.w.uv_unit(bins.n)
        self.shape = (bins.nc, bins.n, bins.n)
        self._f: Dict[int, np.ndarray] = {}
        self._i: Dict[int, np.ndarray] = {}

    def data(self, j: int) -> np.ndarray:
        if j not in self._f:
            x = (self.bins.lut == j) * self.vt
            self._f[j] = np.fft.irfftn(x, s=self.shape, axes=(0, 1, 2))
        return self._f[j]

    def count(self, j: int) -> np.ndarray:
        if j not in self._i:
            y = ((self.bins.lut == j) * self.m[None]).astype(np.float64)
            self._i[j] = np.fft.irfftn(y, s=self.shape, axes=(0, 1, 2))
        return self._i[j]

    def drop(self, keep: Iterable[int] = ()):
        keep = set(keep)
        for d in (self._f, self._i):
            for k in list(d):
                if k not in keep:
                    del d[k]


def rho3(weights: Optional[Weights], nc: int) -> float:
    """rho3 = (1/nc) sum_nu w(nu)^3 (flag correction of the 3D normaliser)."""
    w = (weights or Weights()).chan(nc)
    return float(np.mean(w ** 3))


def estimate_3d(bins: Bins, vis: np.ndarray, weights: Optional[Weights] = None,
                tri: Optional[np.ndarray] = None, norm: float = 1.0,
                fields: Optional[ShellFields] = None, counts: Optional[np.ndarray] = None):
    """3D bispectrum per candidate triangle.

    counts: the triangle counts T3D of `tri` when already known (e.g. the exact integers of
    oracle.counts.exact_counts); otherwise they come from the count fields, rounded.
    Returns (B [nt], T3D [nt] int64, N_eff [nt], S_D [nt], max count deviation).
    """
    f = fields or ShellFields(bins, vis, weights)
    tri = bins.triangles if tri is None else np.asarray(tri).reshape(-1, 3)
    nvox = bins.nc * bins.n * bins.n
    nt = len(tri)
    S = np.empty(nt)
    SI = np.empty(nt)
    for t, (a, b, c) in enumerate(tri):
        S[t] = np.sum(f.data(a) * f.data(b) * f.data(c))
        if counts is None:
            SI[t] = np.sum(f.count(a) * f.count(b) * f.count(c))
    if counts is None:
        T, dev = round_counts(float(nvox) * float(nvox) * SI)
    else:
        T, dev = np.asarray(counts, dtype=np.int64).reshape(nt), 0.0
    neff = T.astype(np.float64) * rho3(weights, bins.nc)
    with np.errstate(invalid="ignore", divide="ignore"):
        B = np.where(T > 0, norm * nvox * S / np.where(neff > 0, neff, 1.0), np.nan)
    return B, T, neff, S, dev
