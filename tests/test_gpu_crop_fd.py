"""Full gradient check on a 64x64 crop of the 1200x680, 300k-Gaussian room
view: the GPU gradients of all 14 parameter rows of 256 random visible
Gaussians plus the 16 largest contributors against FP64 central differences
of the oracle forward with the decision set frozen."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import gpu_backward, gpu_forward

pytestmark = pytest.mark.gpu

KINDS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")
ROWS = {"mean": 0, "log_scale": 3, "quat": 6, "opacity_logit": 10, "rgb": 11}


def test_crop_gradients_against_fp64_finite_differences():
    w = synth.config3_crop()
    cam = w.cameras[0]
    W = H = 64
    print("case crop fd: gpu", flush=True)
    params, rast = gpu_forward(w, 16)
    p_all = oracle.params64(w.gaussians)
    # Restrict the FP64 model to the Gaussians the crop sees.
    proj_all = oracle.project(p_all, [cam], 16, publish=False)
    vis = np.nonzero(proj_all["tiles"][0] > 0)[0]
    p = {k: np.ascontiguousarray(v[..., vis]) for k, v in p_all.items()}
    proj = oracle.project(p, [cam], 16, publish=False)
    bins = oracle.bin_sort(proj, 16, W, H)
    dec = oracle.decision_buffer(bins, 1, W, H)
    fwd = oracle.forward(proj, bins, p["rgb"], W, H, dec=dec, dec_mode=1)
    # The published-record forward flags FP32-ambiguous pixels: mask them.
    pub = oracle.project(p, [cam], 16, publish=True)
    fpub = oracle.forward(pub, oracle.bin_sort(pub, 16, W, H, emit=False),
                          p["rgb"], W, H)
    mask = (fpub["flags"][0] == 0) & (fwd["nlast"][0] == fpub["nlast"][0])
    rng = np.random.default_rng(3)
    wimg = rng.normal(size=(1, 3, H, W)) * mask[None, None]
    got = gpu_backward(rast, params, wimg.astype(np.float32))
    # Largest contributors: by total blend weight in the crop.
    b = oracle.backward(proj, bins, p["rgb"], W, H, np.ones((1, 3, H, W)),
                        dec=dec, dec_mode=2)
    top = np.argsort(-b["grgb"].sum(0))[:16]
    chosen = np.unique(np.concatenate(
        [rng.choice(len(vis), size=min(256, len(vis)), replace=False), top]))
    print("case crop fd: checking", len(chosen), "of", len(vis), flush=True)

    def loss(pp):
        pr = oracle.project(pp, [cam], 16, publish=False)
        f = oracle.forward(pr, bins, pp["rgb"], W, H, dec=dec, dec_mode=2,
                           nthreads=8)
        return float((f["img"] * wimg).sum())

    scales = {k: np.abs(got[ROWS[k]:ROWS[k] + (p[k].shape[0] if p[k].ndim == 2 else 1),
                            vis]).max() for k in KINDS}
    checked = 0
    for j in chosen:
        g_idx = vis[j]
        for k in KINDS:
            arr = p[k]
            rows = arr.shape[0] if arr.ndim == 2 else 1
            for r in range(rows):
                idx = (r, j) if arr.ndim == 2 else (j,)
                x0 = arr[idx]
                h = 1e-6 * max(1.0, abs(x0))
                pp = {kk: vv.copy() for kk, vv in p.items()}
                pp[k][idx] = x0 + h
                lp = loss(pp)
                pp[k][idx] = x0 - h
                lm = loss(pp)
                fd = (lp - lm) / (2 * h)
                an = float(got[ROWS[k] + r, g_idx])
                tol = 1e-3 * max(abs(fd), 1e-2 * scales[k]) + 1e-9
                assert abs(an - fd) <= tol, (k, r, g_idx, an, fd)
                checked += 1
    print("checked", checked, "partial derivatives", flush=True)
    assert checked == 14 * len(chosen) and len(chosen) >= 256
