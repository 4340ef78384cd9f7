"""Seeded synthetic inputs for the bispectrum estimator (host side, NumPy).

This module builds the gridded visibility cubes that both the GPU library and
the CPU oracle consume.  It holds none of the estimator's arithmetic: it only
makes a non-Gaussian sky field, Fourier-transforms each channel into a
Hermitian half-plane uv grid, and builds the weight/flag arrays that go with it.

What it generates (Gill & Bharadwaj 2025, Sec. 4 "Validating the estimator"):

* a Gaussian random field g with power spectrum P(k) proportional to k^-2
  (Sec. 4, first paragraph), normalised so that the field variance is sigma_g^2;
* the quadratic non-Gaussian transform delta = g + f (g^2 - <g^2>) of Eq. (mb1);
* per-channel visibilities V(U, nu) = 2D DFT of delta over the sky pixels,
  stored as the half plane v >= 0 (the uv grid of Eq. (vg) with every cell
  sampled once, so the cell-average weight is 1);
* the MWA-like periodic channel flags of Sec. 4 (24 sub-bands of 32 channels).

Discrete conventions: forward DFTs are unnormalised (NumPy), the uv cell
vector is (q_u, q_v) with signed FFT indices, and the field is laid out
channel-major as delta[nu][x][y] so that V[nu][u][v] = rfft2(delta[nu]).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Physical constants of the MWA-shaped set-up (Sec. 3.1, Sec. 4, Sec. 5).
# --------------------------------------------------------------------------
THETA_F_DEG = 24.68                      # MWA primary-beam FWHM (Sec. 3.1)
THETA0_RAD = 0.6 * math.radians(THETA_F_DEG)   # theta_0 = 0.6 theta_F (Sec. 3.1)
DU_G = math.sqrt(math.log(2.0)) / (math.pi * THETA0_RAD)  # uv grid spacing (Sec. 3.2)
R_MPC = 711.0 / 0.077                    # comoving distance from l = 711 <-> k_perp = 0.077 (Sec. 5, Fig. 4)
RPRIME_MPC_PER_MHZ = 0.68 / 0.04         # 0.68 Mpc per 40 kHz channel (Sec. 4)
DNU_MHZ = 0.04                           # channel width (Sec. 4)
NC_MWA = 768                             # channels (Sec. 4)
K_EDGES_MPC = (0.003, 1.258)             # k range of the 3D results (Sec. 5, Sec. 6)


def default_umax(n: int) -> int:
    """Largest |U| (cells) for which closure mod n equals true closure: 3*umax < n."""
    return (n - 1) // 3


def signed_freq(n: int) -> np.ndarray:
    """Signed integer index of each FFT bin: i for i < n/2, else i - n."""
    i = np.arange(n)
    return np.where(i < (n + 1) // 2, i, i - n).astype(np.int64)


# --------------------------------------------------------------------------
# Power spectrum grids
# --------------------------------------------------------------------------
def kmag_cubic(nc: int, n: int) -> np.ndarray:
    """|k| on a [nc][n][n//2+1] half grid with cubic voxels: k = 2 pi (q_nu/nc, q_x/n, q_y/n)."""
    qn = signed_freq(nc)[:, None, None] / nc
    qx = signed_freq(n)[None, :, None] / n
    qy = np.arange(n // 2 + 1)[None, None, :] / n
    return 2.0 * math.pi * np.sqrt(qn ** 2 + qx ** 2 + qy ** 2)


def kmag_physical(nc: int, n: int, du: float = DU_G, r_mpc: float = R_MPC,
                  rprime: float = RPRIME_MPC_PER_MHZ, dnu: float = DNU_MHZ) -> np.ndarray:
    """|k| in Mpc^-1 on a [nc][n][n//2+1] half grid.

    k_perp = 2 pi dU_g |U| / r (Sec. 2.1, l = 2 pi U = r k_perp) and
    k_par = 2 pi a / (r' B_bw) with B_bw = nc * dnu (Eq. (dft) definitions).
    """
    kpar = 2.0 * math.pi * signed_freq(nc)[:, None, None] / (rprime * nc * dnu)
    ku = 2.0 * math.pi * du * signed_freq(n)[None, :, None] / r_mpc
    kv = 2.0 * math.pi * du * np.arange(n // 2 + 1)[None, None, :] / r_mpc
    return np.sqrt(kpar ** 2 + ku ** 2 + kv ** 2)


def power_law_half(kmag: np.ndarray, index: float = -2.0) -> np.ndarray:
    """Unnormalised P(k) = |k|^index on a half grid, with P(0) = 0."""
    with np.errstate(divide="ignore"):
        p = np.where(kmag > 0, kmag ** index, 0.0)
    return p


def _half_to_full_sum(p_half: np.ndarray, n_last: int) -> float:
    """Sum of a Hermitian-even quantity over the full grid, given its half grid."""
    s = p_half.sum()
    inner = p_half[..., 1:(n_last + 1) // 2].sum() if n_last > 2 else 0.0
    return float(s + inner)


# --------------------------------------------------------------------------
# Fields and cubes
# --------------------------------------------------------------------------
def gaussian_field(p_half_unnorm: np.ndarray, shape: Tuple[int, int, int], sigma: float,
                   rng: np.random.Generator) -> np.ndarray:
    """Gaussian field g[nu][x][y] with <|g~(k)|^2> = N_vox P(k) and Var g = sigma^2.

    g = irfftn(rfftn(white) * sqrt(P)), P = A * p_half_unnorm with A fixed by
    (1/N_vox) sum_k P(k) = sigma^2 (the ensemble variance, not the sample one).
    """
    nvox = shape[0] * shape[1] * shape[2]
    total = _half_to_full_sum(p_half_unnorm, shape[2])
    amp = sigma * sigma * nvox / total
    white = rng.standard_normal(shape)
    gk = np.fft.rfftn(white) * np.sqrt(amp * p_half_unnorm)
    return np.fft.irfftn(gk, s=shape, axes=(0, 1, 2))


def quadratic_field(g: np.ndarray, f: float) -> np.ndarray:
    """delta = g + f (g^2 - <g^2>) of Eq. (mb1); <g^2> is the sample mean."""
    g2 = g * g
    return g + f * (g2 - g2.mean())


def vis_cube(delta: np.ndarray) -> np.ndarray:
    """V[nu][u][v] = 2D DFT of delta[nu] over the sky pixels, half plane v >= 0."""
    return np.fft.rfft2(delta, axes=(1, 2))


def mwa_flags(nc: int, flagged_mod32: Sequence[int] = (0, 16, 31)) -> np.ndarray:
    """Channel weights w(nu) in {0,1}: zero for nu mod 32 in `flagged_mod32` (Sec. 4)."""
    w = np.ones(nc, dtype=np.float64)
    sel = np.isin(np.arange(nc) % 32, np.asarray(flagged_mod32))
    w[sel] = 0.0
    return w


def disk_mask(n: int, umax: Optional[float] = None) -> np.ndarray:
    """uv occupancy [n][n//2+1] uint8: 1 where 1 <= |U| <= umax (the sampled disk)."""
    if umax is None:
        umax = default_umax(n)
    qu = signed_freq(n)[:, None].astype(np.float64)
    qv = np.arange(n // 2 + 1)[None, :].astype(np.float64)
    r = np.sqrt(qu ** 2 + qv ** 2)
    return ((r >= 1.0) & (r <= umax)).astype(np.uint8)


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------
@dataclass
class Workload:
    """One synthetic cube: sizes, field recipe and binning."""
    name: str
    n: int
    nc: int
    kind: str                 # "cubic" (grid-unit k) or "physical" (Mpc^-1)
    sigma: float = 0.5
    f_ng: float = 0.5
    pk_index: float = -2.0
    flags_mod32: Tuple[int, ...] = ()
    du: float = DU_G
    r_mpc: float = R_MPC
    rprime: float = RPRIME_MPC_PER_MHZ
    dnu: float = DNU_MHZ
    extra: dict = field(default_factory=dict)

    @property
    def nh(self) -> int:
        return self.n // 2 + 1

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nc, self.n, self.n)

    def kmag_half(self) -> np.ndarray:
        if self.kind == "cubic":
            return kmag_cubic(self.nc, self.n)
        return kmag_physical(self.nc, self.n, self.du, self.r_mpc, self.rprime, self.dnu)

    def chan_w(self) -> np.ndarray:
        if not self.flags_mod32:
            return np.ones(self.nc, dtype=np.float64)
        return mwa_flags(self.nc, self.flags_mod32)

    def ring_edges(self, nbins: int = 8) -> np.ndarray:
        """Log-spaced ring edges in cells: geomspace(1, umax+1, nbins+1)."""
        return np.geomspace(1.0, default_umax(self.n) + 1.0, nbins + 1)

    def shell_edges(self, nbins: int = 20) -> np.ndarray:
        """Log-spaced |k| shell edges in Mpc^-1 over the range of Sec. 5."""
        return np.geomspace(K_EDGES_MPC[0], K_EDGES_MPC[1], nbins + 1)


def config1() -> Workload:
    """64x64 uv x 16 channels, cubic voxels, 8 log rings (MABS parity case)."""
    return Workload("mabs64x16", n=64, nc=16, kind="cubic")


def config2() -> Workload:
    """256x256 uv x 768 channels of 40 kHz at the MWA set-up (Sec. 4)."""
    return Workload("mwa256x768", n=256, nc=NC_MWA, kind="physical")


def config3() -> Workload:
    """Config 2 with channels {0,16,31} of every 32-channel block flagged."""
    return Workload("mwa256x768_flagged", n=256, nc=NC_MWA, kind="physical",
                    flags_mod32=(0, 16, 31))


def make_cube(w: Workload, seed: int, dtype=np.complex128) -> np.ndarray:
    """Seeded visibility cube V[nc][n][n//2+1] for workload `w` (flags applied)."""
    rng = np.random.default_rng(seed)
    p = power_law_half(w.kmag_half(), w.pk_index)
    g = gaussian_field(p, w.shape, w.sigma, rng)
    delta = quadratic_field(g, w.f_ng)
    v = vis_cube(delta)
    cw = w.chan_w()
    if np.any(cw != 1.0):
        v = v * cw[:, None, None]
    return np.ascontiguousarray(v.astype(dtype))


def small_workload(n: int, nc: int, kind: str = "cubic", **kw) -> Workload:
    """A tiny cube for brute-force and Monte Carlo tests."""
    return Workload(f"tiny{n}x{nc}", n=n, nc=nc, kind=kind, **kw)


def collapsed_mabs(nt: int, nc: int, seed: int, circular: bool = False, gap_frac: float = 0.01) -> np.ndarray:
    """Seeded stand-in for an ergodically collapsed MABS over channel separations (d1, d2):
    float64 [nt][S][S] with S = 2nc - 1 (d at d + nc - 1) or S = nc when circular (d at d mod nc).

    Values are standard normal.  NaN marks separations with no channel triplet: in the
    non-circular layout every (d1, d2) with |d2 - d1| >= nc, plus a random gap_frac of the rest
    in both layouts (separations that flagged channels leave unsampled)."""
    rng = np.random.default_rng(seed)
    size = nc if circular else 2 * nc - 1
    B = rng.standard_normal((nt, size, size))
    if not circular:
        d = np.arange(size) - (nc - 1)
        B[:, np.abs(d[None, :] - d[:, None]) >= nc] = np.nan
    B[rng.random((nt, size, size)) < gap_frac] = np.nan
    return B


def uv_tracks(nvis: int, seed: int, umin: float, umax: float) -> np.ndarray:
    """Seeded stand-in for a baseline distribution (the MWA baselines are not available): float64
    [nvis][2] baselines in wavelengths, radius log-uniform in [umin, umax] (number density falling
    as 1/U^2 in the plane, denser at short baselines like a compact array) and uniform angle."""
    rng = np.random.default_rng(seed)
    r = np.exp(rng.uniform(math.log(umin), math.log(umax), size=nvis))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=nvis)
    return np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1)


def rfi_flags(nc: int, nvis: int, seed: int, rate: float, chan_w: Optional[np.ndarray] = None) -> np.ndarray:
    """uint8 [nc][nvis] flags: whole channels where chan_w is 0 (periodic band flags) plus a random
    `rate` of (channel, baseline) samples (RFI)."""
    rng = np.random.default_rng(seed)
    f = (rng.random((nc, nvis)) < rate).astype(np.uint8)
    if chan_w is not None:
        f[np.asarray(chan_w) == 0, :] = 1
    return f
