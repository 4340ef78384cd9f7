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
