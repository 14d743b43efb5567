"""Pins the view-dependent colour oracle (real spherical harmonics of the
viewing direction, the colour coefficients c in R^k of the scene
representation): the basis against scipy's complex harmonics, orthonormality
by exact quadrature, the addition theorem, polynomial gradients and the
colour chain by finite differences, the clamp, and the per-view colour
layout of the compositing oracle."""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import sh as S
import synth


def _unit(rng, m):
    d = rng.normal(size=(m, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _real_from_complex(l, m, theta, phi):
    """Real harmonic from scipy's complex one (Condon-Shortley phase
    included): sqrt(2) Re Y_l^m (m > 0), sqrt(2) Im Y_l^|m| (m < 0)."""
    if m == 0:
        return sp.sph_harm_y(l, 0, theta, phi).real
    y = sp.sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2.0) * (y.real if m > 0 else y.imag)


def test_basis_matches_scipy_complex_harmonics():
    d = _unit(np.random.default_rng(0), 200)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = S.basis(3, d)
    j = 0
    for l in range(4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(Y[:, j], _real_from_complex(l, m, theta, phi),
                                       rtol=0, atol=1e-13, err_msg=f"l={l} m={m}")
            j += 1
    assert j == S.n_coeffs(3) == Y.shape[1]


def test_orthonormal_under_exact_quadrature():
    """Gauss-Legendre in cos(theta) times an even phi grid integrates
    products of degree <= 6 exactly: the Gram matrix is the identity."""
    xg, wg = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct * ct)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).ravel()
    Y = S.basis(3, d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-13)


def test_addition_theorem_per_band():
    """sum_m Y_lm(d)^2 = (2l+1)/(4 pi) at every direction."""
    Y = S.basis(3, _unit(np.random.default_rng(1), 100))
    j = 0
    for l in range(4):
        band = Y[:, j:j + 2 * l + 1]
        np.testing.assert_allclose((band ** 2).sum(1), (2 * l + 1) / (4 * np.pi),
                                   rtol=1e-13)
        j += 2 * l + 1


def test_lower_degrees_are_prefixes():
    d = _unit(np.random.default_rng(2), 20)
    full = S.basis(3, d)
    for D in range(3):
        np.testing.assert_array_equal(S.basis(D, d), full[:, :S.n_coeffs(D)])


def test_polynomial_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    d = rng.normal(size=(30, 3))          # off the sphere: plain polynomials
    g = S.basis_grad(3, d)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (S.basis(3, d + e) - S.basis(3, d - e)) / (2 * h)
        np.testing.assert_allclose(g[..., a], fd, rtol=0, atol=1e-8)


def _params(seed, D, n=25, scale=0.15):
    w = synth.tiny_scene(seed, n=n)
    g = synth.with_sh(w.gaussians, seed, D, scale)
    return oracle.params64(g), w.cameras[0]


def _two_views(cam):
    c2 = synth.Camera(np.array([[0.8, 0.0, -0.6], [0.0, 1.0, 0.0],
                                [0.6, 0.0, 0.8]], np.float32),
                      np.array([0.4, -0.1, 0.3], np.float32), cam.fx, cam.fy,
                      cam.cx, cam.cy, cam.width, cam.height)
    return [cam, c2]


def test_degree_zero_is_the_rgb_rows():
    p, cam = _params(4, 0)
    col, raw = S.colours(p, _two_views(cam), 0)
    np.testing.assert_array_equal(col[0], p["rgb"])
    np.testing.assert_array_equal(col[1], p["rgb"])
    # No clamp at degree 0.
    p["rgb"][0, 0] = -0.25
    col, _ = S.colours(p, [cam], 0)
    assert col[0, 0, 0] == -0.25


def test_zero_coefficients_give_the_clamped_base_colour():
    p, cam = _params(5, 2)
    p["sh"][:] = 0.0
    p["rgb"][1, :5] = -0.3
    col, _ = S.colours(p, [cam], 2)
    np.testing.assert_array_equal(col[0], np.maximum(p["rgb"], 0.0))


def test_degree_one_closed_form():
    """Degree 1: raw = rgb + sum_m Y_1m(d) f_m with Y_1 = K1 (-y, z, -x)."""
    p, cam = _params(6, 1)
    o = S.camera_centre(cam)
    v = p["mean"].T - o
    d = v / np.linalg.norm(v, axis=1, keepdims=True)
    K1 = math.sqrt(3 / (4 * math.pi))
    Y = np.stack([-K1 * d[:, 1], K1 * d[:, 2], -K1 * d[:, 0]], 0)  # [3][n]
    want = p["rgb"] + np.einsum("jn,jcn->cn", Y, p["sh"])
    _, raw = S.colours(p, [cam], 1)
    np.testing.assert_allclose(raw[0], want, rtol=0, atol=1e-15)


def test_colour_depends_only_on_the_direction():
    """Moving a mean along its viewing ray leaves its colour unchanged."""
    p, cam = _params(7, 3)
    o = S.camera_centre(cam)
    col, _ = S.colours(p, [cam], 3)
    q = {k: v.copy() for k, v in p.items()}
    q["mean"] = o[:, None] + 1.7 * (p["mean"] - o[:, None])
    col2, _ = S.colours(q, [cam], 3)
    np.testing.assert_allclose(col2, col, rtol=0, atol=1e-14)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_colour_chain_matches_finite_differences(D):
    p, cam = _params(8 + D, D)
    cams = _two_views(cam)
    p["rgb"][:, :3] = -0.6         # clamped in both views: zero gradient
    rng = np.random.default_rng(20 + D)
    gcol = rng.normal(size=(2, 3, p["rgb"].shape[1]))
    _, raw = S.colours(p, cams, D)
    assert (raw < 0).any() and (raw > 0).any()
    d_rgb, d_sh, d_mean = S.colours_bwd(p, cams, D, gcol)
    assert np.all(d_rgb[:, :3] == 0) and np.all(d_sh[:, :, :3] == 0)

    def loss(q):
        return float((S.colours(q, cams, D)[0] * gcol).sum())

    h = 1e-6
    for key, an in (("rgb", d_rgb), ("sh", d_sh), ("mean", d_mean)):
        arr = p[key]
        for idx in list(np.ndindex(arr.shape))[::7]:
            q = {k: v.copy() for k, v in p.items()}
            q[key][idx] = arr[idx] + h
            lp = loss(q)
            q[key][idx] = arr[idx] - h
            lm = loss(q)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - an[idx]) <= 1e-7 * max(1.0, abs(an[idx])), (key, idx, fd, an[idx])


def _render(p, cams, colours, tile=16):
    W, H = cams[0].width, cams[0].height
    proj = oracle.project(p, cams, tile, publish=False)
    bins = oracle.bin_sort(proj, tile, W, H)
    return proj, bins, oracle.forward(proj, bins, colours, W, H)


def test_per_view_colour_layout_of_the_compositing():
    """With per-view colours, view k renders exactly as a shared-colour
    render with view k's colours; equal per-view colours reproduce the
    shared layout bit for bit."""
    p, cam = _params(12, 3, n=40)
    cams = _two_views(cam)
    col, _ = S.colours(p, cams, 3)
    _, _, per = _render(p, cams, col)
    for k in range(2):
        _, _, one = _render(p, cams, col[k])
        np.testing.assert_array_equal(per["img"][k], one["img"][k])
    _, _, shared = _render(p, cams, p["rgb"])
    _, _, same = _render(p, cams, np.stack([p["rgb"]] * 2))
    np.testing.assert_array_equal(same["img"], shared["img"])


def test_per_view_colour_gradients_of_the_compositing():
    """The per-view colour gradient of view k is the shared-layout colour
    gradient of a backward that only sees view k's image gradient."""
    p, cam = _params(13, 2, n=40)
    cams = _two_views(cam)
    W, H = cam.width, cam.height
    col, _ = S.colours(p, cams, 2)
    proj, bins, _ = _render(p, cams, col)
    rng = np.random.default_rng(5)
    dimg = rng.normal(size=(2, 3, H, W))
    per = oracle.backward(proj, bins, col, W, H, dimg)
    assert per["grgb"].shape == (2, 3, p["rgb"].shape[1])
    for k in range(2):
        only = dimg.copy()
        only[1 - k] = 0.0
        one = oracle.backward(proj, bins, col[k], W, H, only)
        np.testing.assert_allclose(per["grgb"][k], one["grgb"], rtol=1e-12,
                                   atol=1e-15)
    # The screen-space and opacity parts do not depend on the layout's
    # bookkeeping, only on the colours.
    np.testing.assert_array_equal(per["gop"], oracle.backward(
        proj, bins, col, W, H, dimg)["gop"])


def test_whole_chain_matches_finite_differences():
    """End to end: projection, per-view colours, compositing, backward and
    chain, with the decisions frozen, against central differences of the
    weighted image sum in every parameter kind including the coefficients."""
    D = 2
    w = synth.tiny_scene(14, n=20, width=36, height=30, f=35.0,
                         log_scale_mu=-1.8)
    g = synth.with_sh(w.gaussians, 14, D, 0.15)
    cams = _two_views(w.cameras[0])
    W, H = cams[0].width, cams[0].height
    p = oracle.params64(g)
    proj = oracle.project(p, cams, 16, publish=False)
    bins = oracle.bin_sort(proj, 16, W, H)
    dec = oracle.decision_buffer(bins, 2, W, H)
    col, _ = S.colours(p, cams, D)
    oracle.forward(proj, bins, col, W, H, dec=dec, dec_mode=1)
    wimg = np.random.default_rng(3).normal(size=(2, 3, H, W))
    bwd = oracle.backward(proj, bins, col, W, H, wimg, dec=dec, dec_mode=2)
    grads = S.chain(p, cams, D, bwd)

    def loss(q):
        pr = oracle.project(q, cams, 16, publish=False)
        c, _ = S.colours(q, cams, D)
        f = oracle.forward(pr, bins, c, W, H, dec=dec, dec_mode=2)
        return float((f["img"] * wimg).sum())

    visible = np.nonzero(proj["tiles"].sum(0) > 0)[0][:6]
    checked = 0
    for key in ("mean", "sh", "rgb", "log_scale"):
        arr = p[key]
        scale = np.abs(grads[key]).max()
        for idx in np.ndindex(arr.shape):
            if idx[-1] not in visible or (key == "sh" and idx[0] % 3):
                continue
            h = 1e-6 * max(1.0, abs(arr[idx]))
            q = {k: v.copy() for k, v in p.items()}
            q[key][idx] = arr[idx] + h
            lp = loss(q)
            q[key][idx] = arr[idx] - h
            lm = loss(q)
            fd = (lp - lm) / (2 * h)
            an = grads[key][idx]
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-2 * scale) + 1e-9, \
                (key, idx, fd, an)
            checked += 1
    assert checked > 60
