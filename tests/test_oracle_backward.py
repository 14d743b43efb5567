"""Pins the oracle's gradients: central finite differences in FP64 with the
decision set (sorted lists, admitted entries, clamps, stop positions) frozen
at the base point, plus single-Gaussian closed forms."""
import math

import numpy as np
import pytest

import oracle
import synth

KINDS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")


def _setup(w, tile=16, bg=(0.0, 0.0, 0.0), seed=0):
    cams = w.cameras
    W, H = cams[0].width, cams[0].height
    p = oracle.params64(w.gaussians)
    proj = oracle.project(p, cams, tile, publish=False)
    bins = oracle.bin_sort(proj, tile, W, H)
    dec = oracle.decision_buffer(bins, len(cams), W, H)
    oracle.forward(proj, bins, p["rgb"], W, H, bg, dec=dec, dec_mode=1)
    rng = np.random.default_rng(seed)
    wimg = rng.normal(size=(len(cams), 3, H, W))
    return p, proj, bins, dec, wimg


def _loss(p, cams, bins, dec, wimg, bg, tile):
    W, H = cams[0].width, cams[0].height
    proj = oracle.project(p, cams, tile, publish=False)
    f = oracle.forward(proj, bins, p["rgb"], W, H, bg, dec=dec, dec_mode=2)
    return float((f["img"] * wimg).sum())


def _analytic(p, proj, bins, dec, wimg, cams, bg):
    W, H = cams[0].width, cams[0].height
    b = oracle.backward(proj, bins, p["rgb"], W, H, wimg, bg, dec=dec,
                        dec_mode=2)
    return oracle.project_bwd(p, cams, b)


def _check_fd(w, bg, n_check=12, tile=16, seed=0):
    cams = w.cameras
    p, proj, bins, dec, wimg = _setup(w, tile, bg, seed)
    grads = _analytic(p, proj, bins, dec, wimg, cams, bg)
    rng = np.random.default_rng(seed + 100)
    n = p["mean"].shape[1]
    visible = np.nonzero(proj["tiles"].sum(0) > 0)[0]
    chosen = rng.choice(visible, size=min(n_check, len(visible)), replace=False)
    worst = 0.0
    for kind in KINDS:
        arr = p[kind]
        rows = arr.shape[0] if arr.ndim == 2 else 1
        scale = np.abs(grads[kind]).max()
        for g in chosen:
            for r in range(rows):
                idx = (r, g) if arr.ndim == 2 else (g,)
                x0 = arr[idx]
                h = 1e-6 * max(1.0, abs(x0))
                pp = {k: v.copy() for k, v in p.items()}
                pp[kind][idx] = x0 + h
                lp = _loss(pp, cams, bins, dec, wimg, bg, tile)
                pp[kind][idx] = x0 - h
                lm = _loss(pp, cams, bins, dec, wimg, bg, tile)
                fd = (lp - lm) / (2 * h)
                an = grads[kind][idx]
                tol = 1e-6 * max(abs(an), 1e-2 * scale) + 1e-9
                err = abs(fd - an)
                worst = max(worst, err / (tol))
                assert err <= tol, (kind, g, r, fd, an)
    return worst


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_finite_differences_all_parameter_kinds(seed):
    w = synth.tiny_scene(seed, n=30, width=40, height=34, f=38.0,
                         log_scale_mu=-1.8)
    _check_fd(w, (0.0, 0.0, 0.0), seed=seed)


def test_finite_differences_with_background():
    w = synth.tiny_scene(7, n=25, width=36, height=30, f=35.0,
                         log_scale_mu=-1.7)
    _check_fd(w, (0.3, 0.55, 0.8), seed=7)


def test_finite_differences_rotated_camera_and_clamp():
    """A rotated, translated camera and Gaussians beyond the 1.3x field of
    view (clamped Jacobian) still match finite differences."""
    rng = np.random.default_rng(11)
    w = synth.tiny_scene(11, n=30, width=40, height=34, f=38.0,
                         log_scale_mu=-1.5)
    g = w.gaussians
    # Push a few Gaussians far to the side, make them big so they still touch
    # the image.
    g.mean[0, :5] = g.mean[2, :5] * 1.2
    g.log_scale[:, :5] = -0.7
    ang = 0.2
    R = np.array([[math.cos(ang), 0, math.sin(ang)], [0, 1, 0],
                  [-math.sin(ang), 0, math.cos(ang)]], np.float32)
    c = w.cameras[0]
    cam = synth.Camera(R, np.array([0.05, -0.02, 0.1], np.float32), c.fx, c.fy,
                       c.cx, c.cy, c.width, c.height)
    w.cameras = [cam]
    _check_fd(w, (0.0, 0.0, 0.0), n_check=15, seed=11)


def test_finite_differences_two_views():
    w = synth.tiny_scene(13, n=25, width=36, height=30, f=35.0,
                         log_scale_mu=-1.8)
    c = w.cameras[0]
    c2 = synth.Camera(c.R, (c.t + np.array([0.1, 0.0, 0.05])).astype(np.float32),
                      c.fx, c.fy, c.cx, c.cy, c.width, c.height)
    w.cameras = [c, c2]
    _check_fd(w, (0.0, 0.0, 0.0), seed=13)


@pytest.mark.parametrize("opl", [0.2, -1.5])
def test_single_gaussian_closed_forms(opl):
    """One Gaussian: C = alpha c + (1 - alpha) bg, so dC/dc = alpha and
    dC/d(opacity) = G (c - bg) where alpha = opacity G is unclamped."""
    W = H = 25
    f = 24.0
    cam = synth.identity_camera(f, f, W, H)
    col = np.array([0.8, 0.3, 0.5])
    bg = (0.1, 0.6, 0.2)
    p = dict(mean=np.array([[0.05], [-0.03], [2.0]]),
             log_scale=np.full((3, 1), -2.3), quat=np.array([[1.0], [0], [0], [0]]),
             opacity_logit=np.array([opl]), rgb=col.reshape(3, 1))
    proj, bins, fwd = oracle.render(p, [cam], tile=8, bg=bg, publish=False)
    u, v = 13, 11
    for ch in range(3):
        dimg = np.zeros((1, 3, H, W))
        dimg[0, ch, v, u] = 1.0
        b = oracle.backward(proj, bins, p["rgb"], W, H, dimg, bg)
        alpha = 1.0 - fwd["T"][0, v, u]
        px, py, A, B, C, o = proj["rec"][0, 0, :6]
        dx, dy = px - u, py - v
        G = math.exp(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy)
        assert alpha == pytest.approx(o * G, rel=1e-14)
        assert b["grgb"][ch, 0] == pytest.approx(alpha, rel=1e-13)
        assert b["gop"][0] == pytest.approx(G * (col[ch] - bg[ch]), rel=1e-12)


def test_clamped_alpha_has_zero_opacity_gradient():
    W = H = 15
    cam = synth.identity_camera(14.0, 14.0, W, H)
    p = dict(mean=np.array([[0.0], [0.0], [2.0]]),
             log_scale=np.full((3, 1), -1.5), quat=np.array([[1.0], [0], [0], [0]]),
             opacity_logit=np.array([8.0]), rgb=np.array([[1.0], [0.5], [0.2]]))
    proj, bins, fwd = oracle.render(p, [cam], tile=8, publish=False)
    c = (W - 1) // 2
    assert 1.0 - fwd["T"][0, c, c] == pytest.approx(oracle.ALPHA_MAX)
    dimg = np.zeros((1, 3, H, W))
    dimg[0, :, c, c] = 1.0
    b = oracle.backward(proj, bins, p["rgb"], W, H, dimg)
    assert b["gop"][0] == 0.0
    np.testing.assert_array_equal(b["g2d"][0, 0], 0.0)
