"""Pins of the densification oracle (Eq. 8-9): the dominant Gaussian per
pixel against the brute-force compositor and closed forms, the dominated
pixel counts, and the split rule."""
import math

import numpy as np
import pytest

import oracle
import oracle.brute as brute
from oracle import densify as D
import synth


def _render(w, tile=16):
    p = oracle.params64(w.gaussians)
    c = w.cameras[0]
    proj = oracle.project(p, w.cameras, tile, publish=False)
    bins = oracle.bin_sort(proj, tile, c.width, c.height)
    fwd = oracle.forward(proj, bins, p["rgb"], c.width, c.height)
    return p, proj, fwd


@pytest.mark.parametrize("seed", [11, 12])
def test_dominant_matches_brute_force(seed):
    w = synth.tiny_scene(seed, n=120, width=40, height=30, f=40.0,
                         log_scale_mu=-2.0)
    p, proj, fwd = _render(w)
    _, _, _, dom = brute.composite(proj["rec"], proj["box"], p["rgb"], 40, 30,
                                   with_dominant=True)
    np.testing.assert_array_equal(fwd["dom"], dom)
    assert (fwd["dom"] >= 0).any()


def test_two_stacked_gaussians_closed_form():
    """Front alpha a1, back a2 at the centre pixel: the back one dominates
    exactly when a2 (1 - a1) > a1."""
    for o_front, o_back, want in ((0.3, 0.9, 1), (0.6, 0.9, 0)):
        g = synth.tiny_scene(1, n=2, width=21, height=21, f=30.0).gaussians
        g.mean[:] = np.array([[0.0, 0.0], [0.0, 0.0], [2.0, 3.0]], np.float32)
        g.log_scale[:] = -3.0
        g.quat[:] = np.array([[1.0], [0.0], [0.0], [0.0]], np.float32)
        g.opacity_logit[:] = np.log(np.array([o_front, o_back]) /
                                    (1 - np.array([o_front, o_back]))).astype(np.float32)
        w = synth.Workload("stack", g, [synth.identity_camera(30.0, 30.0, 21, 21)],
                           np.zeros((1, 3, 21, 21), np.float32))
        _, _, fwd = _render(w)
        assert fwd["dom"][0, 10, 10] == want
        a1, a2 = fwd["w1"][0, 10, 10], fwd["w2"][0, 10, 10]
        assert a1 > a2 > 0


def test_dominated_counts():
    dom = np.array([[[-1, 0, 0], [2, 2, 2]]])
    np.testing.assert_array_equal(D.dominated_counts(dom, 4), [2, 0, 3, 0])


def _params(n, cap, seed=0):
    rng = np.random.default_rng(seed)
    p = {"mean": np.zeros((3, cap)), "log_scale": np.zeros((3, cap)),
         "quat": np.zeros((4, cap)), "opacity_logit": np.zeros(cap),
         "rgb": np.zeros((3, cap))}
    p["mean"][:, :n] = rng.normal(size=(3, n))
    p["log_scale"][:, :n] = rng.normal(-2, 0.3, size=(3, n))
    p["quat"][:, :n] = rng.normal(size=(4, n))
    p["opacity_logit"][:n] = rng.normal(size=n)
    p["rgb"][:, :n] = rng.uniform(size=(3, n))
    return p


def test_split_axis_aligned_and_rotated_closed_forms():
    p = _params(3, 6)
    p["quat"][:, 0] = [1, 0, 0, 0]                       # identity
    c, s_ = math.cos(math.pi / 4), math.sin(math.pi / 4)
    p["quat"][:, 1] = [c, 0, 0, s_]                      # 90 degrees about z
    xi = np.random.default_rng(1).normal(size=(6, 2, 3))
    counts = np.array([5, 9, 2])
    out, n, parents, over = D.split(p, 3, 6, counts, 4, xi)
    assert parents == [0, 1] and n == 5 and not over
    s0 = np.exp(p["log_scale"][:, 0])
    np.testing.assert_allclose(out["mean"][:, 0], p["mean"][:, 0] + s0 * xi[0, 0], atol=1e-14)
    np.testing.assert_allclose(out["mean"][:, 3], p["mean"][:, 0] + s0 * xi[0, 1], atol=1e-14)
    s1 = np.exp(p["log_scale"][:, 1])
    rot = np.array([-s1[1] * xi[1, 0, 1], s1[0] * xi[1, 0, 0], s1[2] * xi[1, 0, 2]])
    np.testing.assert_allclose(out["mean"][:, 1], p["mean"][:, 1] + rot, atol=1e-14)
    for slot, parent in ((0, 0), (3, 0), (1, 1), (4, 1)):
        np.testing.assert_allclose(out["log_scale"][:, slot],
                                   p["log_scale"][:, parent] - math.log(1.6))
        np.testing.assert_array_equal(out["rgb"][:, slot], p["rgb"][:, parent])
        assert out["opacity_logit"][slot] == p["opacity_logit"][parent]
    # The untouched Gaussian and the empty tail.
    for k in D.KEYS:
        np.testing.assert_array_equal(out[k][..., 2], p[k][..., 2])
        np.testing.assert_array_equal(out[k][..., 5], p[k][..., 5])


def test_split_threshold_is_strict_and_capacity_bounds_it():
    p = _params(4, 5)
    xi = np.zeros((5, 2, 3))
    counts = np.array([7, 8, 8, 9])
    _, n, parents, over = D.split(p, 4, 5, counts, 7, xi)
    assert parents == [1] and n == 5 and over     # room for one child only
    _, n, parents, over = D.split(_params(4, 8), 4, 8, counts, 7,
                                  np.zeros((8, 2, 3)))
    assert parents == [1, 2, 3] and n == 7 and not over


def test_children_sample_the_parent_covariance():
    """With many draws the children's offsets have the parent's covariance
    R S^2 R^T (statistical check, 4 sigma)."""
    p = _params(1, 40001, seed=3)
    xi = np.random.default_rng(4).normal(size=(1, 2, 3))
    R = D.rotation(p["quat"][:, 0])
    s = np.exp(p["log_scale"][:, 0])
    rng = np.random.default_rng(5)
    offs = []
    for _ in range(4000):
        xi = rng.normal(size=(1, 2, 3))
        out, _, _, _ = D.split(p, 1, 3, np.array([10]), 0, np.concatenate([xi, np.zeros((2, 2, 3))]))
        offs.append(out["mean"][:, 0] - p["mean"][:, 0])
    offs = np.array(offs)
    cov = offs.T @ offs / len(offs)
    ref = R @ np.diag(s * s) @ R.T
    assert np.abs(cov - ref).max() < 4 * np.sqrt(2.0 / len(offs)) * np.abs(ref).max() + 1e-12
