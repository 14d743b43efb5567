"""Learned initialisation of inserted Gaussians.

A small network (32 -> 64 -> 64 -> 7, GELU, BF16 MFMA with FP32 accumulate,
all in libgsmap's kernels) maps the features of an insertion candidate - its
3x3 keyframe colours, its inverse depth and statistics of its 8 nearest
existing Gaussians - to the initial log-scales (sorted descending), opacity
logit and colour of the new Gaussian.  It is trained on converged
parameters that the plain mapper itself produced; heuristic initialisation
remains the fallback (insert_gaussians without mlp_out).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import raster as R

N_PARAMS = 6727
SIZES = ((32, 64), (64, 64), (64, 7))


def init_weights(seed=0):
    """He-normal weights, zero biases, as one FP32 vector."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in SIZES:
        parts.append(rng.normal(0.0, math.sqrt(2.0 / i), size=i * o))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


class InitMLP:
    """Device-resident network with Adam state."""

    def __init__(self, weights=None, seed=0, device="cuda"):
        w = init_weights(seed) if weights is None else np.asarray(weights, np.float32)
        assert w.size == N_PARAMS
        self.w = torch.from_numpy(w.copy()).to(device)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.g = torch.zeros_like(self.w)
        self.step = 0
        # Feature / target normalisation (set by fit_normalisation).
        self.x_mu = torch.zeros(32, device=device)
        self.x_sd = torch.ones(32, device=device)
        self.t_mu = torch.zeros(7, device=device)
        self.t_sd = torch.ones(7, device=device)

    def fit_normalisation(self, x, t):
        self.x_mu, self.x_sd = x.mean(0), x.std(0).clamp_min(1e-6)
        self.t_mu, self.t_sd = t.mean(0), t.std(0).clamp_min(1e-6)

    def _xin(self, x):
        return ((x - self.x_mu) / self.x_sd).contiguous()

    def forward_raw(self, x_norm, cache=None):
        y = torch.empty(x_norm.shape[0], 7, device=x_norm.device)
        R.mlp_fwd(self.w, x_norm, y, cache)
        return y

    def predict(self, feats):
        """Initial parameters [M][7] (log-scale 3, opacity logit, RGB 3)."""
        y = self.forward_raw(self._xin(feats))
        return (y * self.t_sd + self.t_mu).contiguous()

    def train_step(self, x, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        """One Adam step on the MSE of normalised targets; returns the loss
        (device tensor)."""
        xn = self._xin(x)
        tn = ((t - self.t_mu) / self.t_sd).contiguous()
        M = xn.shape[0]
        cache = torch.empty(M, 128, device=xn.device)
        y = self.forward_raw(xn, cache)
        dy = torch.empty_like(y)
        loss = torch.zeros(1, dtype=torch.float64, device=xn.device)
        R.mlp_mse(y, tn, dy, loss)
        self.g.zero_()
        R.mlp_bwd(self.w, xn, cache, dy, self.g)
        self.step += 1
        R.mlp_adam(self.w, self.g, self.m, self.v, lr, b1, b2, eps, self.step)
        return loss

    def train(self, x, t, epochs=20, batch=8192, lr=1e-3, seed=0, log=None):
        """Minibatch training on device tensors x [N][32], t [N][7]."""
        g = torch.Generator(device="cpu").manual_seed(seed)
        N = x.shape[0]
        hist = []
        for ep in range(epochs):
            perm = torch.randperm(N, generator=g).to(x.device)
            tot = torch.zeros(1, dtype=torch.float64, device=x.device)
            nb = 0
            for s in range(0, N, batch):
                idx = perm[s:s + batch]
                tot += self.train_step(x[idx], t[idx], lr)
                nb += 1
            hist.append(float(tot) / nb)
            if log:
                log(f"init_mlp: epoch {ep + 1}/{epochs} loss {hist[-1]:.4f}")
        return hist

    def state(self):
        return dict(w=self.w.cpu().numpy(), x_mu=self.x_mu.cpu().numpy(),
                    x_sd=self.x_sd.cpu().numpy(), t_mu=self.t_mu.cpu().numpy(),
                    t_sd=self.t_sd.cpu().numpy())


def targets_from_params(data_rows):
    """Converged parameters [14][k] -> targets [k][7]: log-scales sorted
    descending, opacity logit, RGB."""
    ls = np.sort(data_rows[3:6], axis=0)[::-1]
    return np.concatenate([ls, data_rows[10:11], data_rows[11:14]], 0).T.copy()
