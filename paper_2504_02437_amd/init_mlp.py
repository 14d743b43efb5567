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

    @classmethod
    def load(cls, path=None, device="cuda"):
        """A network saved with np.savez(**state()); by default the one
        trained on 2M pairs from 1200x680 plain-mapper runs."""
        import os
        path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                    "data", "init_mlp_1200x680.npz")
        d = np.load(path)
        net = cls(weights=d["w"], device=device)
        for k in ("x_mu", "x_sd", "t_mu", "t_sd"):
            setattr(net, k, torch.from_numpy(d[k]).to(device))
        return net

    def state(self):
        return dict(w=self.w.cpu().numpy(), x_mu=self.x_mu.cpu().numpy(),
                    x_sd=self.x_sd.cpu().numpy(), t_mu=self.t_mu.cpu().numpy(),
                    t_sd=self.t_sd.cpu().numpy())


def targets_from_params(data_rows):
    """Converged parameters [14][k] -> targets [k][7]: log-scales sorted
    descending, opacity logit, RGB."""
    ls = np.sort(data_rows[3:6], axis=0)[::-1]
    return np.concatenate([ls, data_rows[10:11], data_rows[11:14]], 0).T.copy()


# ---------------------------------------------------------------------------
# Training data from the plain mapper, training, and evaluation.
# ---------------------------------------------------------------------------

def _stream(seed, n_kf, width, height, f, n_gt):
    import synth
    return synth.mapping_stream(seed, n_kf, width, height, f, n_gt)


def collect_pairs(seed, n_kf=40, width=320, height=240, f=260.0,
                  n_gt=100_000, iters_per_kf=10, window=10, device="cuda",
                  log=None):
    """Runs the plain mapper (heuristic initialisation) over one synthetic
    keyframe stream and returns (features [N][32], targets [N][7]) of every
    Gaussian it inserted: the features at insertion time and its parameters
    at the end of the run (log-scales sorted descending, opacity logit,
    RGB)."""
    from .mapper import Mapper, render_images
    st = _stream(seed, n_kf, width, height, f, n_gt)
    imgs = render_images(st.gt, st.cameras, device)
    mp = Mapper(capacity=n_kf * 9 * st.pts[0].shape[0], width=width,
                height=height, window=window, device=device)
    feats, ids = [], []
    for i, cam in enumerate(st.cameras):
        info = mp.add_keyframe(cam, imgs[i], st.pts[i], features=True)
        kept = torch.from_numpy(info["kept"]).to(device)
        k = int(info["kept"].sum())
        n_ins = info["n_after"] - info["n_before"]
        if k != n_ins:
            raise RuntimeError(f"kept mask {k} != inserted {n_ins}")
        feats.append(info["feats"][kept])
        ids.append(torch.arange(info["n_before"], info["n_after"], device=device))
        mp.optimise(iters_per_kf)
        if log and (i + 1) % 10 == 0:
            log(f"collect seed {seed}: kf {i + 1}/{n_kf}, map {mp.params.n()}, "
                f"psnr {mp.psnr():.2f}")
    ids = torch.cat(ids)
    rows = mp.params.data[:, ids]
    ls = torch.sort(rows[3:6], dim=0, descending=True).values
    t = torch.cat([ls, rows[10:11], rows[11:14]], 0).T.contiguous()
    return torch.cat(feats).contiguous(), t


def run_window(seed, mlp=None, n_kf=10, width=320, height=240, f=260.0,
               n_gt=100_000, iters_per_kf=5, extra_iters=100, eval_every=5,
               plateau=None, device="cuda"):
    """Maps a keyframe window with heuristic (mlp=None) or learned
    initialisation; returns the window PSNR curve over iterations.  With
    plateau = (span, gain) the run stops early once the PSNR rose by less
    than `gain` dB over the last `span` iterations."""
    from .mapper import Mapper, render_images
    st = _stream(seed, n_kf, width, height, f, n_gt)
    imgs = render_images(st.gt, st.cameras, device)
    mp = Mapper(capacity=n_kf * 9 * st.pts[0].shape[0], width=width,
                height=height, window=n_kf, device=device)
    curve = []
    for i, cam in enumerate(st.cameras):
        mp.add_keyframe(cam, imgs[i], st.pts[i], mlp=mlp)
        mp.optimise(iters_per_kf)
    cams = st.cameras
    full = imgs.contiguous()
    curve.append((mp.iterations, mp.psnr(cams, full)))
    for _ in range(0, extra_iters, eval_every):
        mp.optimise(eval_every)
        curve.append((mp.iterations, mp.psnr(cams, full)))
        if plateau:
            span, gain = plateau
            back = [p for it, p in curve if it <= curve[-1][0] - span]
            if back and curve[-1][1] - back[-1] < gain:
                break
    return dict(curve=curve, gaussians=mp.params.n())


def iterations_to_reach(curve, target):
    for it, p in curve:
        if p >= target:
            return it
    return None


def compare_at_levels(heuristic, learned, levels):
    """For each PSNR level: the first iteration at which each curve reaches
    it (None when it never does within its run)."""
    return [dict(psnr=float(lv), heuristic=iterations_to_reach(heuristic, lv),
                 learned=iterations_to_reach(learned, lv)) for lv in levels]


def evaluate(net, eval_seeds=(1000, 1001, 1002), eval_kf=10, width=320,
             height=240, f=260.0, n_gt=100_000, max_iters=4000, eval_every=20,
             plateau=(400, 0.05), levels=(8, 10, 12, 14, 16, 18, 20, 22, 24),
             device="cuda", log=None):
    """Heuristic against learned initialisation on held-out scenes, each run
    until its PSNR plateaus (or max_iters): the curves and the iterations
    each needs to reach every PSNR level."""
    out = []
    for s in eval_seeds:
        runs = {}
        for name, m in (("heuristic", None), ("learned", net)):
            runs[name] = run_window(s, m, n_kf=eval_kf, width=width,
                                    height=height, f=f, n_gt=n_gt,
                                    extra_iters=max_iters,
                                    eval_every=eval_every, plateau=plateau,
                                    device=device)["curve"]
        ev = dict(seed=s, heuristic=runs["heuristic"], learned=runs["learned"],
                  levels=compare_at_levels(runs["heuristic"], runs["learned"],
                                           levels))
        out.append(ev)
        if log:
            ch, cm = runs["heuristic"], runs["learned"]
            log(f"eval seed {s}: heuristic {ch[0][1]:.2f} -> {ch[-1][1]:.2f} dB "
                f"in {ch[-1][0]} it., learned {cm[0][1]:.2f} -> {cm[-1][1]:.2f}"
                f" dB in {cm[-1][0]} it.; levels {ev['levels']}")
    return out


def experiment(train_seeds=range(16), eval_seeds=(1000, 1001, 1002),
               n_kf=40, epochs=30, iters_per_kf=10, width=320, height=240,
               f=260.0, n_gt=100_000, eval_kf=10, eval_iters=4000,
               device="cuda", log=None):
    """Collects pairs from the plain mapper on the training seeds, trains the
    network, and compares heuristic vs learned initialisation on the held-out
    seeds over an ``eval_kf``-keyframe window.  Returns (results, network)."""
    X, T = [], []
    for s in train_seeds:
        x, t = collect_pairs(s, n_kf=n_kf, width=width, height=height, f=f,
                             n_gt=n_gt, iters_per_kf=iters_per_kf,
                             device=device, log=log)
        X.append(x)
        T.append(t)
        if log:
            log(f"seed {s}: {x.shape[0]} pairs")
    X = torch.cat(X)
    T = torch.cat(T)
    net = InitMLP(device=device)
    net.fit_normalisation(X, T)
    hist = net.train(X, T, epochs=epochs, batch=8192, lr=1e-3, log=log)
    res = dict(pairs=int(X.shape[0]), train_loss=hist, evals=[],
               setup=dict(width=width, height=height, f=f, n_gt=n_gt,
                          train_seeds=list(train_seeds), n_kf=n_kf,
                          iters_per_kf=iters_per_kf, epochs=epochs,
                          eval_seeds=list(eval_seeds), eval_kf=eval_kf,
                          eval_iters=eval_iters))
    res["evals"] = evaluate(net, eval_seeds, eval_kf=eval_kf, width=width,
                            height=height, f=f, n_gt=n_gt,
                            max_iters=eval_iters, device=device, log=log)
    return res, net


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="learned-initialisation experiment")
    ap.add_argument("--train-seeds", type=int, default=16)
    ap.add_argument("--n-kf", type=int, default=40)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--width", type=int, default=320)
    ap.add_argument("--height", type=int, default=240)
    ap.add_argument("--f", type=float, default=260.0)
    ap.add_argument("--n-gt", type=int, default=100_000)
    ap.add_argument("--eval-iters", type=int, default=4000)
    ap.add_argument("--save", default="")
    ap.add_argument("--evaluate", default="",
                    help="skip training: evaluate the weights in this .npz")
    a = ap.parse_args(argv)
    lg = lambda *x: print(*x, file=sys.stderr, flush=True)
    if a.evaluate:
        net = InitMLP.load(a.evaluate)
        res = dict(weights=a.evaluate,
                   setup=dict(width=a.width, height=a.height, f=a.f,
                              n_gt=a.n_gt, eval_iters=a.eval_iters),
                   evals=evaluate(net, width=a.width, height=a.height, f=a.f,
                                  n_gt=a.n_gt, max_iters=a.eval_iters, log=lg))
        print(json.dumps(res))
        return
    res, net = experiment(train_seeds=range(a.train_seeds), n_kf=a.n_kf,
                          epochs=a.epochs, width=a.width, height=a.height,
                          f=a.f, n_gt=a.n_gt, eval_iters=a.eval_iters, log=lg)
    if a.save:
        np.savez(a.save, **net.state())
    print(json.dumps(res))


if __name__ == "__main__":
    main()
