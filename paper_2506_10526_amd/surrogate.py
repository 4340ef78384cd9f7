"""Variance surrogate pipeline over the C ABI (argument marshalling and orchestration only).

Monte Carlo labels (bs_mc_*) -> features (bs_var_features) -> training on the GPU (bs_mlp_*) ->
prediction of per-triangle Var(B_hat), with the plain Monte Carlo as fallback and reference.

Flag patterns (channels flagged in every 32-channel block; Sec. 4 describes edge and centre
flagging of every 1.28 MHz sub-band): the family "e" flags the centre channel 16 and the e outermost
channels at each edge (e = 1 is the three-channel pattern of the flagged workload, e = 4 the paper's
other reading), plus a centre block and an evenly spaced pattern.

The flag summary fed to the network is per triangle: log(G / G1) - 2 log rho3, with G the mean over
the triangle's closed triangles of the window-convolved power P_w P_w P_w (bs_var_flag_proxy: flags
fold power from low |k| into shells of high k_par through the window's spectrum) and G1 the same
without flags; the network's output is added to the Gaussian log variance with flags,
log(N_vox / T3D) + log G - 2 log rho3 (bs_var_features_flag).
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Dict, Optional, Sequence

import numpy as np

from . import bs, synth


def edge_flags(e: int) -> tuple:
    """Channels (mod 32) flagged in flag-family member e."""
    return tuple(sorted(set(range(e)) | {16} | set(range(32 - e, 32))))


# training patterns (channels mod 32) and two patterns kept out of training
TRAIN_PATTERNS = {"none": (), "e0": edge_flags(0), "e1": edge_flags(1), "e2": edge_flags(2), "e4": edge_flags(4),
                  "centre3": (15, 16, 17), "every8": (0, 8, 16, 24)}
UNSEEN_PATTERNS = {"e3": edge_flags(3), "spread4": (3, 11, 19, 26)}


@dataclass
class McResult:
    count: np.ndarray
    mean: np.ndarray
    var: np.ndarray
    rho: float
    seconds: float
    realizations: int


def mc_run(ctx: int, bins: int, ncand: int, desc, chan_w: np.ndarray, R: int, seed: int,
           precision: int = bs.BS_SPLIT_BF16, first: int = 0) -> McResult:
    """R realizations through the 3D estimator; per-triangle mean and variance."""
    import torch
    cw = torch.from_numpy(np.ascontiguousarray(chan_w, dtype=np.float32)).cuda()
    m = bs.bs_mc_create(ctx, bins, desc, precision, chan_w=cw)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bs.bs_mc_run(m, seed, first, R)
        c, mu, v = bs.bs_mc_stats(m, ncand)
        dt = time.perf_counter() - t0
    finally:
        bs.bs_mc_destroy(m)
    return McResult(c, mu, v, float(np.mean(chan_w)), dt, R)


class Surrogate:
    """The MLP on the GPU plus the baseline that turns its output into a variance."""

    def __init__(self, ctx: int, seed: int = 1, max_batch: int = 8192):
        self.ctx = ctx
        self.h = bs.bs_mlp_create(ctx, seed, max_batch)

    def close(self):
        if self.h:
            bs.bs_mlp_destroy(self.h)
            self.h = None

    def fit(self, X: np.ndarray, target: np.ndarray, steps: int, lr: float, cosine: bool = True) -> Dict:
        import torch
        Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
        td = torch.from_numpy(np.ascontiguousarray(target, dtype=np.float32)).cuda()
        bs.bs_mlp_set_data(self.h, Xd, td)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = bs.bs_mlp_train(self.h, steps, lr, cosine)
        dt = time.perf_counter() - t0
        return {"steps": steps, "seconds": dt, "final_loss": loss}

    def predict_log(self, X: np.ndarray, bf16: bool = False) -> np.ndarray:
        import torch
        Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
        y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        bs.bs_mlp_predict(self.h, Xd, y, bf16)
        torch.cuda.synchronize()
        return y.cpu().numpy().astype(np.float64)


class FlagFeatures:
    """Per-pattern inputs of the flag-aware surrogate (G1, the unflagged proxy, computed once)."""

    def __init__(self, ctx: int, bins: int, ncand: int, T3D: np.ndarray, pk_index: float = -2.0):
        self.ctx, self.bins, self.ncand, self.T3D, self.pk = ctx, bins, ncand, np.asarray(T3D), pk_index
        self.G1 = bs.bs_var_flag_proxy(ctx, bins, ncand, pk_index, None)

    def __call__(self, chan_w: np.ndarray):
        """(X [ncand][4], baseline [ncand]) for channel weights chan_w."""
        G = bs.bs_var_flag_proxy(self.ctx, self.bins, self.ncand, self.pk, chan_w)
        return bs.bs_var_features_flag(self.bins, self.ncand, self.T3D, G, self.G1, float(np.mean(np.asarray(chan_w) ** 3)))


def training_set_flag(ff: FlagFeatures, runs: Sequence[McResult], weights: Sequence[np.ndarray]):
    """Stack (flag-aware features, log Var - baseline) over Monte Carlo runs, valid triangles only."""
    Xs, ts = [], []
    for r, w in zip(runs, weights):
        X, base = ff(w)
        ok = (ff.T3D > 0) & (r.count > 1) & np.isfinite(r.var) & (r.var > 0) & np.isfinite(base)
        Xs.append(X[ok])
        ts.append(np.log(r.var[ok]) - base[ok])
    return np.concatenate(Xs), np.concatenate(ts)


def predict_var_flag(sur: "Surrogate", ff: FlagFeatures, chan_w: np.ndarray, bf16: bool = False) -> np.ndarray:
    X, base = ff(chan_w)
    y = sur.predict_log(X, bf16)
    with np.errstate(invalid="ignore"):
        return np.where((ff.T3D > 0) & np.isfinite(base), np.exp(y + base), np.nan)


def training_set(bins: int, ncand: int, T3D: np.ndarray, runs: Sequence[McResult], pk_index: float):
    """Stack (features, log Var - baseline) over Monte Carlo runs, valid triangles only."""
    Xs, ts = [], []
    for r in runs:
        X, base = bs.bs_var_features(bins, ncand, T3D, pk_index, r.rho)
        ok = (T3D > 0) & (r.count > 1) & np.isfinite(r.var) & (r.var > 0)
        Xs.append(X[ok])
        ts.append(np.log(r.var[ok]) - base[ok])
    return np.concatenate(Xs), np.concatenate(ts)


def predict_var(sur: Surrogate, bins: int, ncand: int, T3D: np.ndarray, rho: float, pk_index: float,
                bf16: bool = False) -> np.ndarray:
    X, base = bs.bs_var_features(bins, ncand, T3D, pk_index, rho)
    y = sur.predict_log(X, bf16)
    with np.errstate(invalid="ignore"):
        return np.where(T3D > 0, np.exp(y + base), np.nan)
