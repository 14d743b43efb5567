"""Keyframe-window mapping with the rasterizer's kernels (the loop the paper's
mapping back end runs: Map Initialization, Dynamic Insertion and Map
Optimization with Planar Regularization).

For every keyframe: render the current map at the keyframe pose, insert new
Gaussians at the visual-odometry patch pixels whose accumulated alpha does
not exceed ``alpha_skip`` (heuristic or learned initial parameters), then run
window iterations (render, L1 + planar-regulariser gradients, backward, Adam)
over the last ``window`` keyframes; optionally densify on the keyframe
(Eq. 8-9).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import raster as R

LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3)   # mean, log_scale, quat, opacity, rgb


class Mapper:
    def __init__(self, capacity, width, height, window=10, settings=None,
                 lr=LR, lam_color=1.0, lam_reg=1.0, reg_floor=0.01,
                 alpha_skip=0.9, sh_degree=0, device="cuda"):
        self.capacity, self.W, self.H = capacity, width, height
        self.window = window
        self.settings = settings or R.Settings(tile=16)
        self.lr, self.lam_color, self.lam_reg = lr, lam_color, lam_reg
        self.reg_floor, self.alpha_skip = reg_floor, float(np.float32(alpha_skip))
        self.device = device
        # sh_degree > 0: view-dependent colour with (sh_degree + 1)^2 - 1
        # coefficients per channel, zero for new Gaussians.
        self.params = R.ParamBuffer(capacity, device, n=0, sh_degree=sh_degree)
        self.grad = self.params.zeros_like()
        self.m = self.params.zeros_like()
        self.v = self.params.zeros_like()
        self.step = torch.ones(1, dtype=torch.int32, device=device)
        self.kfs = []            # (camera, image [3][H][W] device)
        self._rasts = {}
        self.iterations = 0

    # -- rendering -----------------------------------------------------------
    def _rast(self, cams):
        V = len(cams)
        r = self._rasts.get(V)
        if r is None:
            r = R.Rasterizer(cams, self.capacity, self.settings,
                             device=self.device)
            self._rasts[V] = r
        else:
            r.set_cameras(cams)
        return r

    def render(self, cams):
        r = self._rast(cams)
        r.forward(self.params)
        flags, _ = r.status()
        if flags:
            r.fit_key_capacity(self.params)
            r.forward(self.params)
        return r

    # -- insertion -----------------------------------------------------------
    def candidate_pixels(self, pts):
        """(u, v) of every candidate (patch by patch, 3x3 row-major)."""
        uv = []
        for u, v, _ in np.asarray(pts):
            for p in range(9):
                uv.append((int(u) + p % 3 - 1, int(v) + p // 3 - 1))
        return np.array(uv, np.int64).reshape(-1, 2)

    def add_keyframe(self, cam, image, pts, mlp=None, features=False):
        """Inserts the keyframe's candidates; returns a dict with the count
        before insertion, the kept-candidate mask and (optionally) the
        features of every candidate."""
        r = self.render([cam])
        T = r.T[0].contiguous()
        cam_dev = r.cams_dev
        img = image if torch.is_tensor(image) else torch.from_numpy(
            np.ascontiguousarray(image)).to(self.device)
        pts_d = torch.from_numpy(np.ascontiguousarray(pts, np.float32)).to(self.device)
        C = pts.shape[0] * 9
        feats = mlp_out = None
        if mlp is not None or features:
            feats = torch.empty(C, 32, device=self.device)
            R.knn_features(self.params, cam_dev, self.W, self.H, img, pts_d,
                           False, feats)
        if mlp is not None:
            mlp_out = mlp.predict(feats)
        n0 = self.params.n()
        R.insert_gaussians(self.params, self.m, self.v, cam_dev, self.W,
                           self.H, img, T, pts_d, self.alpha_skip, False,
                           mlp_out)
        uv = self.candidate_pixels(pts)
        Th = T.cpu().numpy().astype(np.float64)
        inside = (uv[:, 0] >= 0) & (uv[:, 0] < self.W) & (uv[:, 1] >= 0) & \
            (uv[:, 1] < self.H)
        d_ok = np.repeat(np.asarray(pts)[:, 2] > 0, 9)
        kept = np.zeros(C, bool)
        kept[inside] = (1.0 - Th[uv[inside, 1], uv[inside, 0]]) <= self.alpha_skip
        kept &= d_ok
        self.kfs.append((cam, img))
        if len(self.kfs) > self.window:
            self.kfs.pop(0)
        return dict(n_before=n0, kept=kept, feats=feats,
                    n_after=self.params.n())

    # -- optimisation --------------------------------------------------------
    def optimise(self, iters):
        cams = [c for c, _ in self.kfs]
        imgs = torch.stack([i for _, i in self.kfs]).contiguous()
        r = self._rast(cams)
        dL = torch.empty_like(imgs)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        for _ in range(iters):
            self.grad.data.zero_()
            loss.zero_()
            r.forward(self.params)
            R.planar_reg(self.params, self.lam_reg, self.reg_floor, self.grad,
                         loss)
            r.backward_l1(self.params, imgs, self.lam_color, self.grad, loss)
            R.adam(self.params, self.grad, self.m, self.v, self.lr, 0.9, 0.999,
                   1e-15, self.step)
            self.step.add_(1)
            self.iterations += 1
        flags, _ = r.status()
        if flags:
            r.fit_key_capacity(self.params)
        return float(loss)

    # -- densification -------------------------------------------------------
    def densify(self, sigma, generator=None):
        """Clarity-enhancing densification (Eq. 8-9) on the latest keyframe:
        splits the Gaussians that dominate more than sigma of its pixels.
        Returns the number split."""
        cam, _ = self.kfs[-1]
        r = self._rast([cam])
        dom = r.forward_dominant(self.params)
        xi = torch.randn(self.capacity, 2, 3, device=self.device,
                         generator=generator)
        n_split = torch.zeros(1, dtype=torch.int32, device=self.device)
        R.densify(self.params, self.m, self.v, dom, sigma, xi, n_split=n_split)
        return int(n_split)

    def psnr(self, cams=None, images=None):
        """Mean PSNR (dB) of the window views (or the given views)."""
        if cams is None:
            cams = [c for c, _ in self.kfs]
            images = torch.stack([i for _, i in self.kfs]).contiguous()
        r = self.render(cams)
        dL = torch.empty_like(images)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        sq = torch.zeros(len(cams), dtype=torch.float64, device=self.device)
        R.loss_l1(r.rgb, images, 1.0, dL, loss, sq)
        mse = sq.cpu().numpy() / (3 * self.W * self.H)
        return float(np.mean(10.0 * np.log10(1.0 / np.maximum(mse, 1e-12))))


def render_images(gaussians, cams, device="cuda", settings=None):
    """Ground-truth keyframe images of a scene, in chunks of 10 views."""
    params = R.ParamBuffer.from_gaussians(gaussians, device=device)
    out = []
    for s in range(0, len(cams), 10):
        chunk = cams[s:s + 10]
        r = R.Rasterizer(chunk, params.capacity, settings or R.Settings(tile=16),
                         device=device)
        r.fit_key_capacity(params)
        r.forward(params)
        out.append(r.rgb.clone())
        del r
    return torch.cat(out, 0)
