"""Plain FP64 reference of the learned variance surrogate: a 4 -> 256 -> 256 -> 256 -> 1 MLP.

Oracle (test infrastructure only; see the package docstring).  The surrogate is not part of the
paper: the paper estimates error bars from the scatter of many independent realizations
(Sec. 4: 250 realizations; Sec. 5: the sigma bands of the results).  The network maps a
triangle's bin centres and a flag summary to log Var(B_hat), and is trained on Monte Carlo
variances of the 3D estimator.

Definitions (everything below is written out plainly; numpy.matmul is the only primitive):
  parameter vector theta = [W1 (256x4), b1, W2 (256x256), b2, W3 (256x256), b3, w4 (1x256), b4],
    row-major, 133,121 numbers;
  normalisation: x' = (x - mu_x) / s_x per input, target t' = (t - mu_t) / s_t;
  z1 = x' W1^T + b1, h1 = silu(z1), silu(z) = z / (1 + e^-z);  likewise h2, h3;
  y' = h3 w4^T + b4;  prediction t = mu_t + s_t y';
  loss L = mean over the batch of (y' - t')^2;
  Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    theta -= lr * (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps) at step k = 1, 2, ...
    with the learning rate of step k of a K-step run lr_k = lr (1 + cos(pi (k-1) / K)) / 2;
Features of a triangle (b1, b2, b3) of |k| shells with edges e: log of the geometric bin centres
sqrt(e_j e_{j+1}) (Mpc^-1) and rho = mean channel weight sum_nu w(nu) / nc.
Target: log Var(B_hat) minus the Gaussian-shaped baseline log(N_vox / T3D) + n_s sum_i log k_i
(the variance of a triangle average scales as P1 P2 P3 N_vox / T3D, P ~ k^n_s), so that the
network learns the smooth correction (non-Gaussian terms, flag leakage) rather than the
22 decades the variance itself spans over the shells.
"""
from __future__ import annotations

import numpy as np

IN, HID = 4, 256
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("w4", (1, HID)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)   # 133121


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, s in SHAPES:
        k = int(np.prod(s))
        out[name] = theta[o:o + k].reshape(s)
        o += k
    return out


INIT_KEY1 = 0x4D4C50   # second Philox key word of the initialisation stream


def init_params(seed: int) -> np.ndarray:
    """theta_j = a_j (2 u_j - 1) with a_j = 1 / sqrt(fan_in) of the layer parameter j belongs to
    (weights and biases alike) and u_j the 24-bit uniform of word j % 4 of Philox4x64-10 block
    (j // 4, 0, 0, 0) under key (seed, 0x4D4C50) (the generator's definitions)."""
    from .generator import philox4x64_10, uniforms24
    nblk = (NPARAM + 3) // 4
    c = np.arange(nblk, dtype=np.uint64)
    z = np.zeros_like(c)
    x = philox4x64_10((c, z, z, z), (np.uint64(seed), np.uint64(INIT_KEY1)))
    u = np.stack([uniforms24(v) for v in x], axis=1).ravel()[:NPARAM]
    a = np.concatenate([np.full(int(np.prod(s)), 1.0 / np.sqrt(s[1] if len(s) == 2 else (IN if name == "b1" else HID)))
                        for name, s in SHAPES])
    return a * (2.0 * u - 1.0)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta: np.ndarray, x: np.ndarray, keep: bool = False):
    """Network output y' for normalised inputs x (batch x 4)."""
    p = unpack(theta)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(z2)
    z3 = h2 @ p["W3"].T + p["b3"]
    h3 = silu(z3)
    y = (h3 @ p["w4"].T)[:, 0] + p["b4"][0]
    if keep:
        return y, (x, z1, h1, z2, h2, z3, h3)
    return y


def loss_and_grad(theta: np.ndarray, x: np.ndarray, t: np.ndarray):
    """L = mean (y' - t')^2 and dL/dtheta by the chain rule, layer by layer."""
    p = unpack(theta)
    y, (x, z1, h1, z2, h2, z3, h3) = forward(theta, x, keep=True)
    B = x.shape[0]
    r = y - t
    L = float(np.mean(r * r))
    dy = 2.0 * r / B                              # dL/dy'
    g = {}
    g["w4"] = (dy @ h3)[None, :]
    g["b4"] = np.array([dy.sum()])
    dz3 = np.outer(dy, p["w4"][0]) * dsilu(z3)
    g["W3"] = dz3.T @ h2
    g["b3"] = dz3.sum(0)
    dz2 = (dz3 @ p["W3"]) * dsilu(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"]) * dsilu(z1)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return L, np.concatenate([g[name].ravel() for name, _ in SHAPES])


class Adam:
    def __init__(self, n: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.k = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta: np.ndarray, g: np.ndarray) -> np.ndarray:
        self.k += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.k)
        vh = self.v / (1 - self.b2 ** self.k)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def normalisation(x: np.ndarray, t: np.ndarray):
    """(mu_x, s_x, mu_t, s_t): per-column mean and standard deviation (1 where it is zero)."""
    mx, sx = x.mean(0), x.std(0)
    sx = np.where(sx > 0, sx, 1.0)
    mt, st = float(t.mean()), float(t.std())
    return mx, sx, mt, (st if st > 0 else 1.0)


def features(edges: np.ndarray, tri: np.ndarray, rho: float) -> np.ndarray:
    """(log k1, log k2, log k3, rho) per triangle, k the geometric centre of each shell."""
    c = np.log(np.sqrt(edges[:-1] * edges[1:]))
    tri = np.asarray(tri)
    return np.column_stack([c[tri[:, 0]], c[tri[:, 1]], c[tri[:, 2]], np.full(len(tri), rho)])


def baseline_log_var(edges: np.ndarray, tri: np.ndarray, T3D: np.ndarray, nvox: int, index: float) -> np.ndarray:
    """log(N_vox / T3D) + index * sum_i log k_i per triangle (-inf where T3D = 0)."""
    c = np.log(np.sqrt(edges[:-1] * edges[1:]))
    tri = np.asarray(tri)
    T = np.asarray(T3D, dtype=np.float64)
    with np.errstate(divide="ignore"):
        out = np.log(nvox / np.where(T > 0, T, 1.0)) + index * c[tri].sum(1)
    return np.where(T > 0, out, -np.inf)


# ------------------------------------------------------------------------------------------------
# Flag-aware inputs.  Flags multiply the cube by w(nu) along frequency; the delay transform of the
# product is the circular convolution of each line's transform with w~ / nc (Sec. 2.2 delay
# transform, Sec. 4 flagging), so a Gaussian field of power P is seen with the power
#     P_w(k_perp, eta) = sum_q c_q P(k_perp, eta - q),   c_q = |w~(q)|^2 / nc^2,
# w~ the unnormalised DFT of w.  The Gaussian variance of a triangle average is proportional to the
# mean over its closed triangles of P_w(k1) P_w(k2) P_w(k3) (times N_vox / T3D, divided by rho3^2
# for the N_eff normalisation); G below is that mean.
def window_power_weights(chan_w: np.ndarray) -> np.ndarray:
    """c_q = |sum_nu w(nu) e^(-2 pi i q nu / nc)|^2 / nc^2 for q = 0 .. nc-1."""
    w = np.asarray(chan_w, dtype=np.float64)
    nc = len(w)
    nu = np.arange(nc)
    wt = np.array([np.sum(w * np.exp(-2j * np.pi * q * nu / nc)) for q in range(nc)])
    return np.abs(wt) ** 2 / nc ** 2


def windowed_power(n: int, nc: int, du: float, r_mpc: float, rprime: float, dnu: float, chan_w,
                   pk_index: float, rel_cut: float = 1e-13) -> np.ndarray:
    """P_w on the [nc][n][n//2+1] delay grid (delay axis first, signed index order of the FFT):
    P(k) = |k|^pk_index with P(0) = 0, |k| as for the shell bins; the sum over q skips the c_q
    below rel_cut * c_0 (exactly zero for periodic masks up to rounding)."""
    from .bins import shell_kmag
    k = shell_kmag(n, nc, du, r_mpc, rprime, dnu)
    with np.errstate(divide="ignore"):
        P = np.where(k > 0, k ** pk_index, 0.0)
    c = window_power_weights(np.ones(nc) if chan_w is None else chan_w)
    out = np.zeros_like(P)
    for q in range(nc):
        if c[q] > rel_cut * c[0]:
            out += c[q] * np.roll(P, q, axis=0)     # out[i] += c_q P[i - q mod nc]
    return out


def flag_proxy(bins, du: float, r_mpc: float, rprime: float, dnu: float, chan_w, pk_index: float,
               counts=None) -> np.ndarray:
    """G_t = mean over the closed triangles of candidate t of P_w(k1) P_w(k2) P_w(k3), by the 3D
    estimator's FFT route on a cube whose delay transform is P_w (NaN where T3D = 0)."""
    from .estimator import estimate_3d
    Pw = windowed_power(bins.n, bins.nc, du, r_mpc, rprime, dnu, chan_w, pk_index)
    V = np.fft.ifft(Pw, axis=0)
    B, T, _, _, _ = estimate_3d(bins, V, None, counts=counts)
    return B * float(bins.nc * bins.n * bins.n)


def features_flag(edges: np.ndarray, tri: np.ndarray, G: np.ndarray, G1: np.ndarray, rho3: float) -> np.ndarray:
    """(log k1, log k2, log k3, log(G / G1) - 2 log rho3) per triangle (NaN where G or G1 <= 0)."""
    c = np.log(np.sqrt(edges[:-1] * edges[1:]))
    tri = np.asarray(tri)
    G = np.asarray(G, dtype=np.float64)
    G1 = np.asarray(G1, dtype=np.float64)
    ok = (G > 0) & (G1 > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(ok, np.log(np.where(ok, G, 1.0) / np.where(ok, G1, 1.0)) - 2.0 * np.log(rho3), np.nan)
    return np.column_stack([c[tri[:, 0]], c[tri[:, 1]], c[tri[:, 2]], f])


def baseline_flag(T3D: np.ndarray, nvox: int, G: np.ndarray, rho3: float) -> np.ndarray:
    """log(N_vox / T3D) + log G - 2 log rho3 per triangle (-inf where T3D = 0 or G <= 0)."""
    T = np.asarray(T3D, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    ok = (T > 0) & (G > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.log(nvox / np.where(ok, T, 1.0)) + np.log(np.where(ok, G, 1.0)) - 2.0 * np.log(rho3)
    return np.where(ok, out, -np.inf)


def train(theta: np.ndarray, x: np.ndarray, t: np.ndarray, steps: int, lr: float = 1e-3, cosine: bool = False):
    """Full-batch Adam on normalised data; returns (theta, losses)."""
    opt = Adam(theta.size, lr=lr)
    losses = []
    for k in range(steps):
        if cosine:
            opt.lr = lr * 0.5 * (1.0 + np.cos(np.pi * k / steps))
        L, g = loss_and_grad(theta, x, t)
        losses.append(L)
        theta = opt.step(theta, g)
    return theta, losses
