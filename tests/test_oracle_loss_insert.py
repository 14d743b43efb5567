"""Pins the oracle's loss terms (Eq. 10-11), its Adam step and its keyframe
insertion (Eq. 6 back-projection with the accumulated-alpha mask)."""
import math

import numpy as np
import pytest

import oracle
import synth


def test_l1_closed_form_and_sign_zero():
    rng = np.random.default_rng(0)
    img = rng.uniform(size=(2, 3, 5, 7))
    tgt = rng.uniform(size=(2, 3, 5, 7)).astype(np.float32)
    loss, d = oracle.l1(img, tgt, lam=0.7)
    t64 = tgt.astype(np.float64)
    assert loss == pytest.approx(0.7 * np.abs(img - t64).mean(axis=(1, 2, 3)).sum(),
                                 rel=1e-13)
    np.testing.assert_allclose(d, 0.7 * np.sign(img - t64) / (3 * 5 * 7),
                               rtol=1e-15, atol=0)
    # An image equal to its target: zero loss and sign(0) = 0.
    loss0, d0 = oracle.l1(t64, tgt)
    assert loss0 == 0.0 and np.all(d0 == 0.0)


def test_planar_reg_closed_form():
    s = np.array([[0.05, 0.004, 0.02, 0.03],
                  [0.02, 0.009, 0.02, 0.03],
                  [0.03, 0.5, 0.04, 0.03]])
    val, g = oracle.planar_reg(np.log(s), lam=2.0)
    mins = np.array([0.02, 0.01, 0.02, 0.03])   # the floor applies to #1
    assert val == pytest.approx(2.0 * mins.mean(), rel=1e-13)
    exp_g = np.zeros_like(s)
    exp_g[1, 0] = 2.0 * 0.02 / 4
    # Gaussian 1 sits under the floor: no gradient.  Gaussian 2 ties between
    # axes 0 and 1: the lowest index gets it.  Gaussian 3 ties on all axes.
    exp_g[0, 2] = 2.0 * 0.02 / 4
    exp_g[0, 3] = 2.0 * 0.03 / 4
    np.testing.assert_allclose(g, exp_g, rtol=1e-12, atol=0)


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(1)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    z = np.zeros(50)
    lr = 1e-2
    p1, m1, v1 = oracle.adam(p0, g, z, z, lr, step=1, eps=1e-15)
    np.testing.assert_allclose(p1, p0 - lr * np.sign(g), rtol=0, atol=1e-12)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-12)
    # A second step with the same gradient keeps the unit step size.
    p2, _, _ = oracle.adam(p1, g, m1, v1, lr, step=2, eps=1e-15)
    np.testing.assert_allclose(p2, p0 - 2 * lr * np.sign(g), atol=1e-12)


def _kf(seed=0, W=40, H=30, K=12):
    rng = np.random.default_rng(seed)
    R = np.array([[0.8, 0.0, 0.6], [0.0, 1.0, 0.0], [-0.6, 0.0, 0.8]], np.float32)
    cam = synth.Camera(R, np.array([0.3, -0.1, 0.5], np.float32), 35.0, 36.0,
                       (W - 1) / 2, (H - 1) / 2, W, H)
    T = rng.uniform(0.0, 0.3, size=(H, W))
    img = rng.uniform(size=(3, H, W)).astype(np.float32)
    u = rng.integers(1, W - 1, size=K)
    v = rng.integers(1, H - 1, size=K)
    d = 1.0 / rng.uniform(1, 5, size=K)
    pts = np.stack([u, v, d], 1).astype(np.float32)
    return cam, img, T, pts


def test_insertion_count_order_and_reprojection():
    cam, img, T, pts = _kf()
    out = oracle.insert(cam, img, T, pts, alpha_skip=0.9)
    # Count: candidate pixels with 1 - T <= 0.9.
    exp = []
    for k in range(len(pts)):
        for p in range(9):
            u = int(pts[k, 0]) + p % 3 - 1
            v = int(pts[k, 1]) + p // 3 - 1
            if 1.0 - T[v, u] <= 0.9:
                exp.append(9 * k + p)
    assert out["count"] == len(exp)
    np.testing.assert_array_equal(out["src"], exp)
    # Reprojection of each new mean returns its pixel and the patch depth
    # (within 1e-6: the FP32 rotation is orthonormal only to ~1e-7).
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    for i, s in enumerate(out["src"]):
        k, p = divmod(int(s), 9)
        X = R @ out["mean"][:, i] + t
        u = cam.fx * X[0] / X[2] + cam.cx
        v = cam.fy * X[1] / X[2] + cam.cy
        assert u == pytest.approx(int(pts[k, 0]) + p % 3 - 1, abs=1e-6)
        assert v == pytest.approx(int(pts[k, 1]) + p // 3 - 1, abs=1e-6)
        assert X[2] == pytest.approx(1.0 / np.float64(pts[k, 2]), rel=1e-6)
        uu, vv = int(round(u)), int(round(v))
        np.testing.assert_array_equal(out["rgb"][:, i], img[:, vv, uu])
        # One-pixel footprint: s = z / fx, identity rotation, opacity 0.5.
        np.testing.assert_allclose(np.exp(out["log_scale"][:, i]),
                                   1.0 / np.float64(pts[k, 2]) / np.float32(cam.fx),
                                   rtol=1e-12)
    np.testing.assert_array_equal(out["quat"][0], 1.0)
    np.testing.assert_array_equal(out["quat"][1:], 0.0)
    np.testing.assert_array_equal(out["opacity_logit"], 0.0)


def test_insertion_mask_threshold_and_centre_only():
    cam, img, T, pts = _kf(1)
    T[:] = 0.05           # accumulated alpha 0.95 everywhere: nothing goes in
    assert oracle.insert(cam, img, T, pts)["count"] == 0
    T[:] = 0.5
    assert oracle.insert(cam, img, T, pts)["count"] == 9 * len(pts)
    assert oracle.insert(cam, img, T, pts, centre_only=True)["count"] == len(pts)
    out = oracle.insert(cam, img, T, pts, cap=5)
    assert out["count"] == 9 * len(pts) and out["mean"].shape[1] == 5
