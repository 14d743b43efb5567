"""Pins the learned-initialisation oracle to library routines: torch's BF16
conversion, torch FP64 Linear/GELU and autograd, scipy's KD-tree, central
finite differences and closed-form features."""
import math

import numpy as np
import pytest
import torch

import oracle.mlp as M
import synth


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10 ** rng.uniform(-5, 5, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38]]
                       ).astype(np.float32)
    # 1.00390625 and 1.005859375 sit exactly halfway between BF16 values.
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)


class _RoundGrad(torch.autograd.Function):
    """Identity forward; rounds the incoming gradient to BF16."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return g.float().to(torch.bfloat16).double()


def _ste(x):
    """BF16 rounding in the forward, identity in the backward."""
    r = x.float().to(torch.bfloat16).double()
    return x + (r - x).detach()


def _torch_net(w, x, rounding):
    p = torch.from_numpy(np.asarray(w, np.float64)).requires_grad_(True)
    xs = torch.from_numpy(np.asarray(x, np.float64))
    o = 0
    layers = []
    for i, n in M.SIZES:
        W = p[o:o + i * n].view(i, n)
        o += i * n
        b = p[o:o + n]
        o += n
        layers.append((W, b))
    rnd = _ste if rounding else (lambda a: a)
    rg = _RoundGrad.apply if rounding else (lambda a: a)
    gelu = torch.nn.GELU(approximate="none")
    h = rnd(xs)
    for li, (W, b) in enumerate(layers):
        z = rg(torch.nn.functional.linear(h, rnd(W).T)) + b
        h = rnd(gelu(z)) if li < 2 else z
    return p, h


@pytest.mark.parametrize("rounding", [True, False])
def test_forward_matches_torch_linear_gelu(rounding):
    w = M.init_weights(1)
    x = np.random.default_rng(2).normal(size=(200, 32)).astype(np.float32)
    y, _ = M.forward(w, x, rounding)
    _, yt = _torch_net(w, x, rounding)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("rounding", [True, False])
def test_backward_matches_torch_autograd(rounding):
    w = M.init_weights(3)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(100, 32)).astype(np.float32)
    dy = rng.normal(size=(100, 7))
    y, cache = M.forward(w, x, rounding)
    g = M.backward(w, cache, dy, rounding)
    p, yt = _torch_net(w, x, rounding)
    (yt * torch.from_numpy(dy)).sum().backward()
    np.testing.assert_allclose(g, p.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_backward_matches_central_differences():
    w = M.init_weights(5).astype(np.float64)
    rng = np.random.default_rng(6)
    x = rng.normal(size=(20, 32))
    dy = rng.normal(size=(20, 7))
    _, cache = M.forward(w, x, rounding=False)
    g = M.backward(w, cache, dy, rounding=False)
    for j in rng.choice(M.N_PARAMS, size=60, replace=False):
        h = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        lp = (M.forward(wp, x, False)[0] * dy).sum()
        lm = (M.forward(wm, x, False)[0] * dy).sum()
        assert (lp - lm) / (2 * h) == pytest.approx(g[j], rel=1e-6, abs=1e-8)


def test_gelu_closed_form_points():
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert M.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert M.gelu_grad(np.array([0.0]))[0] == 0.5


def test_knn_matches_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(7)
    means = rng.uniform(-1, 1, size=(3, 3000))
    q = rng.uniform(-1, 1, size=(50, 3))
    idx, dist = M.knn(means, q)
    d, i = cKDTree(means.T).query(q, k=8)
    np.testing.assert_allclose(dist, d, rtol=1e-12)
    np.testing.assert_array_equal(idx, i)


def test_features_closed_form():
    W, H = 20, 16
    cam = synth.identity_camera(30.0, 30.0, W, H)
    img = np.zeros((3, H, W), np.float32)
    img[0] = np.arange(W)[None, :] / W
    img[1] = np.arange(H)[:, None] / H
    img[2] = 0.5
    pts = np.array([[5, 7, 0.5], [0, 0, 0.25]], np.float32)
    means = np.array([[0.0], [0.0], [3.0]])
    rgb = np.array([[0.1], [0.2], [0.3]])
    F, P = M.features(cam, img, pts, means, rgb)
    assert F.shape == (18, 32)
    # Centre candidate of patch 0 is pixel (5, 7): its own neighbourhood.
    c = F[4]
    for q in range(9):
        u, v = 5 + q % 3 - 1, 7 + q // 3 - 1
        np.testing.assert_allclose(c[3 * q:3 * q + 3], img[:, v, u])
    assert c[27] == np.float32(0.5)
    X = P[4]
    np.testing.assert_allclose(X, [(5 - 9.5) / 30 * 2, (7 - 7.5) / 30 * 2, 2.0])
    assert c[28] == pytest.approx(math.log(np.linalg.norm(X - [0, 0, 3])))
    np.testing.assert_allclose(c[29:32], [0.1, 0.2, 0.3])
    # Patch 1 at the image corner: neighbours outside the image are zero.
    corner = F[9 + 0]          # pixel (-1, -1): outside; all its neighbours
    assert np.all(corner[:12] == 0)
    # Empty map: the last four features are zero.
    F0, _ = M.features(cam, img, pts, np.zeros((3, 0)), np.zeros((3, 0)))
    assert np.all(F0[:, 28:] == 0)


def test_mse_gradient():
    rng = np.random.default_rng(8)
    y, t = rng.normal(size=(10, 7)), rng.normal(size=(10, 7))
    v, g = M.mse(y, t)
    assert v == pytest.approx(((y - t) ** 2).mean())
    np.testing.assert_allclose(g, 2 * (y - t) / 70)


def _next_bf16(x):
    """The BF16 neighbour of each BF16 value x away from zero (one ulp)."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64) + (1 << 16)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_forward_magnitude_bounds_one_ulp_flips():
    """Moving any one BF16 hidden activation (layer 1 or 2) by one ulp, as a
    rounding on the other side of a boundary would, changes every output by
    at most 2^-7 of forward_magnitude; and the magnitude bounds |y - b3|."""
    rng = np.random.default_rng(11)
    w = M.init_weights(3)
    w[-7:] = rng.normal(size=7)
    x = rng.normal(size=(20, 32)).astype(np.float32)
    y, c = M.forward(w, x)
    mag = M.forward_magnitude(w, c)
    (_, _), (W2, b2), (W3, b3) = M.unpack(w)
    r = M.bf16
    assert np.all(np.abs(y - b3) <= mag * (1 + 1e-12) + 1e-12)
    worst = 0.0
    for trial in range(300):
        m = rng.integers(20)
        h1, h2 = c["h1"][m].copy(), c["h2"][m].copy()
        if trial % 2:
            i = rng.integers(64)
            h1[i] = _next_bf16(h1[i])
            h2 = r(M.gelu(h1 @ r(W2) + b2))
        else:
            j = rng.integers(64)
            h2[j] = _next_bf16(h2[j])
        d = np.abs(h2 @ r(W3) + b3 - y[m])
        assert np.all(d <= 2 ** -7 * mag[m] * (1 + 1e-9) + 1e-15), (trial, d, mag[m])
        worst = max(worst, float((d / (2 ** -7 * mag[m] + 1e-300)).max()))
    assert worst > 0.05     # the bound is not vacuous


def test_backward_magnitude_bounds_the_gradient():
    """backward_magnitude(|dy|) bounds |backward(dy)| element by element, and
    the bound of a difference of two dy is the magnitude of the difference."""
    rng = np.random.default_rng(12)
    w = M.init_weights(4)
    x = rng.normal(size=(30, 32)).astype(np.float32)
    _, c = M.forward(w, x)
    dy = rng.normal(size=(30, 7)) * 1e-2
    g = M.backward(w, c, dy)
    mg = M.backward_magnitude(w, c, np.abs(dy))
    assert np.all(np.abs(g) <= mg * (1 + 1e-9) + 1e-18)
    dy2 = dy + rng.normal(size=dy.shape) * 1e-4
    d = np.abs(M.backward(w, c, dy2) - g)
    # BF16 rounding of dy and of the hidden gradients: each a relative 2^-8.
    bound = M.backward_magnitude(w, c, np.abs(dy2 - dy)) * (1 + 2 ** -6) + \
        2 ** -6 * (mg + M.backward_magnitude(w, c, np.abs(dy2)))
    assert np.all(d <= bound + 1e-18)
