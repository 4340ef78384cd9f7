"""Counter-based seeded visibility cubes: the definition the batched Monte Carlo follows.

Oracle (test infrastructure only; see the package docstring).  The GPU library has its own
implementation of the same definition; the two share no code.

Field recipe (Gill & Bharadwaj 2025, Sec. 4): a Gaussian random field g with power spectrum
P(k) proportional to k^index (index = -2 in the paper), P(0) = 0, normalised so that the
ensemble variance of g is sigma^2; the quadratic non-Gaussian field of Eq. (mb1),
delta = g + f (g^2 - <g^2>) with <g^2> the sample mean; per-channel visibilities
V[z] = 2D DFT of delta[z] on the half plane v >= 0, times the channel weight w(z).

Random numbers: Philox4x64-10 (Salmon, Moraes, Dror & Shaw 2011, "Parallel random numbers:
as easy as 1, 2, 3", SC'11), key = (seed, realization), counter = (c, 0, 0, 0).  Block c
gives the white-noise values of voxels 4c .. 4c+3 of the row-major [nc][n][n] grid
(i = (z n + x) n + y):
    u_j = ((x_j >> 40) + 1/2) 2^-24                        (24-bit uniforms in (0, 1))
    white[4c]   = sqrt(-2 ln u_0) cos(2 pi u_1),  white[4c+1] = sqrt(-2 ln u_0) sin(2 pi u_1)
    white[4c+2] = sqrt(-2 ln u_2) cos(2 pi u_3),  white[4c+3] = sqrt(-2 ln u_2) sin(2 pi u_3)
(the Box-Muller transform).  Then g = irfftn(rfftn(white) sqrt(A P)) with
A = sigma^2 N_vox / sum_k P(k) over the full grid, so that <|g~(k)|^2> = N_vox A P(k).

Wave vectors: "cubic" k = 2 pi (q_z / nc, q_x / n, q_y / n); "physical" (Mpc^-1)
k_par = 2 pi q_z / (r' nc dnu) (Eq. dft's delay conjugate) and k_perp = 2 pi dU_g |q| / r
(Sec. 2.1, l = 2 pi U = r k_perp).
"""
from __future__ import annotations

import numpy as np

# Philox4x64 round multipliers and Weyl key increments (Salmon et al. 2011, Table 2 / Sec. 5)
_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a: np.ndarray, b: np.uint64):
    """(high, low) 64-bit halves of the 128-bit product a * b, from 32-bit limbs."""
    al, ah = a & _LO32, a >> _S32
    bl, bh = b & _LO32, b >> _S32
    ll, lh, hl, hh = al * bl, al * bh, ah * bl, ah * bh
    mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, a * b


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds.  ctr: four uint64 arrays (broadcastable), key: two uint64."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) for x in ctr)
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0, k1 = k0 + _W0, k1 + _W1
            h0, l0 = _mulhilo64(c0, _M0)
            h1, l1 = _mulhilo64(c2, _M1)
            c0, c1, c2, c3 = h1 ^ c1 ^ k0, l1, h0 ^ c3 ^ k1, l0
    return c0, c1, c2, c3


def uniforms24(x: np.ndarray) -> np.ndarray:
    """Top 24 bits of a 64-bit word as a uniform in (0, 1): ((x >> 40) + 1/2) 2^-24."""
    return ((x >> np.uint64(40)).astype(np.float64) + 0.5) * 2.0 ** -24


def white_noise(nvox: int, seed: int, realization: int) -> np.ndarray:
    """Standard normal white noise of length nvox (a multiple of 4), as defined above."""
    assert nvox % 4 == 0
    c = np.arange(nvox // 4, dtype=np.uint64)
    z = np.zeros_like(c)
    x = philox4x64_10((c, z, z, z), (np.uint64(seed), np.uint64(realization)))
    u = [uniforms24(v) for v in x]
    r01 = np.sqrt(-2.0 * np.log(u[0]))
    r23 = np.sqrt(-2.0 * np.log(u[2]))
    out = np.empty((nvox // 4, 4))
    out[:, 0] = r01 * np.cos(2 * np.pi * u[1])
    out[:, 1] = r01 * np.sin(2 * np.pi * u[1])
    out[:, 2] = r23 * np.cos(2 * np.pi * u[3])
    out[:, 3] = r23 * np.sin(2 * np.pi * u[3])
    return out.ravel()


def _signed(m: int) -> np.ndarray:
    i = np.arange(m)
    return np.where(i < (m + 1) // 2, i, i - m).astype(np.float64)


def k_squared(n: int, nc: int, kind: str, du: float = 1.0, r_mpc: float = 1.0,
              rprime: float = 1.0, dnu: float = 1.0, full: bool = True) -> np.ndarray:
    """|k|^2 on the [nc][n][n] grid (full) or its half [nc][n][n/2+1]."""
    if kind == "cubic":
        cz, cxy = 2 * np.pi / nc, 2 * np.pi / n
    else:
        cz, cxy = 2 * np.pi / (rprime * nc * dnu), 2 * np.pi * du / r_mpc
    qz = _signed(nc)[:, None, None] * cz
    qx = _signed(n)[None, :, None] * cxy
    qy = (_signed(n) if full else np.arange(n // 2 + 1, dtype=np.float64))[None, None, :] * cxy
    return qz ** 2 + qx ** 2 + qy ** 2


def generate_cube(n: int, nc: int, kind: str, seed: int, realization: int, sigma: float = 0.5,
                  f: float = 0.5, index: float = -2.0, chan_w=None, du: float = 1.0, r_mpc: float = 1.0,
                  rprime: float = 1.0, dnu: float = 1.0) -> np.ndarray:
    """Visibility cube V[nc][n][n/2+1] (complex128) of one seeded realization."""
    shape = (nc, n, n)
    nvox = nc * n * n
    kw = dict(du=du, r_mpc=r_mpc, rprime=rprime, dnu=dnu)
    k2f = k_squared(n, nc, kind, full=True, **kw)
    with np.errstate(divide="ignore"):
        pf = np.where(k2f > 0, k2f ** (index / 2), 0.0)
    amp = sigma * sigma * nvox / pf.sum()
    k2h = k_squared(n, nc, kind, full=False, **kw)
    with np.errstate(divide="ignore"):
        ph = np.where(k2h > 0, k2h ** (index / 2), 0.0)
    white = white_noise(nvox, seed, realization).reshape(shape)
    g = np.fft.irfftn(np.fft.rfftn(white) * np.sqrt(amp * ph), s=shape, axes=(0, 1, 2))
    g2 = g * g
    delta = g + f * (g2 - g2.mean())
    V = np.fft.rfft2(delta, axes=(1, 2))
    if chan_w is not None:
        V = V * np.asarray(chan_w, dtype=np.float64)[:, None, None]
    return V
