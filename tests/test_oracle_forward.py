"""Pins the oracle's compositing (Eq. 3 with the cut-offs) to closed forms,
invariants and a brute-force per-pixel depth sort."""
import math

import numpy as np
import pytest

import oracle
import oracle.brute as brute
import synth


def one_cam(W, H, f):
    return synth.identity_camera(f, f, W, H)


def gauss_set(means, log_scales, opl, rgb, quats=None):
    n = len(means)
    q = np.zeros((4, n))
    q[0] = 1.0
    if quats is not None:
        q = np.asarray(quats, float).T
    return dict(mean=np.asarray(means, float).T.copy(),
                log_scale=np.asarray(log_scales, float).T.copy(),
                quat=q, opacity_logit=np.asarray(opl, float),
                rgb=np.asarray(rgb, float).T.copy())


@pytest.mark.parametrize("opl,l", [(0.5, -2.5), (2.0, -2.0), (-1.0, -2.8)])
def test_single_isotropic_gaussian_closed_form(opl, l):
    W = H = 41
    f = 40.0
    z = 2.0
    c = one_cam(W, H, f)
    col = (0.9, 0.4, 0.1)
    bg = (0.2, 0.3, 0.5)
    p = gauss_set([(0, 0, z)], [(l, l, l)], [opl], [col])
    proj, bins, fwd = oracle.render(p, [c], tile=16, bg=bg, publish=False)
    sig2 = (f * math.exp(l) / z) ** 2 + 0.3
    o = 1.0 / (1.0 + math.exp(-opl))
    r = math.ceil(3 * math.sqrt(sig2 + math.sqrt(0.1)))
    cx = (W - 1) // 2
    lit = 0
    for v in range(H):
        for u in range(W):
            rho2 = (u - cx) ** 2 + (v - cx) ** 2
            inbox = abs(u - cx) <= r and abs(v - cx) <= r
            a = min(float(np.float32(0.99)), o * math.exp(-rho2 / (2 * sig2)))
            if inbox and a >= oracle.ALPHA_MIN:
                lit += 1
                exp_c = [a * col[ch] + (1 - a) * bg[ch] for ch in range(3)]
                exp_t = 1 - a
            else:
                exp_c, exp_t = list(bg), 1.0
            np.testing.assert_allclose(fwd["img"][0, :, v, u], exp_c, atol=1e-12)
            assert fwd["T"][0, v, u] == pytest.approx(exp_t, abs=1e-12)
    # Lattice points with rho^2 <= 2 sigma^2 ln(255 o) inside the box.
    rr = 2 * sig2 * math.log(255 * o)
    us = np.arange(W) - cx
    cnt = ((us[:, None] ** 2 + us[None, :] ** 2 <= rr) &
           (np.abs(us)[:, None] <= r) & (np.abs(us)[None, :] <= r)).sum()
    assert lit == cnt
    assert int((fwd["nlast"] > 0).sum()) == cnt


def test_stack_of_four_opaque_gaussians():
    """Four identical Gaussians of opacity 0.95 centred on one pixel: the
    fourth would take T to 6.25e-6 < 1e-4, so exactly three contribute,
    T_final = 0.05^3 = 1.25e-4 and C = (1 - 1.25e-4) c."""
    W = H = 21
    c = one_cam(W, H, 20.0)
    col = (0.3, 0.6, 0.9)
    opl = math.log(0.95 / 0.05)
    p = gauss_set([(0, 0, 2.0)] * 4, [(-4, -4, -4)] * 4, [opl] * 4, [col] * 4)
    proj, bins, fwd = oracle.render(p, [c], tile=8, publish=False)
    cx = (W - 1) // 2
    o = 1 / (1 + math.exp(-opl))
    assert fwd["nlast"][0, cx, cx] == 3
    assert fwd["T"][0, cx, cx] == pytest.approx((1 - o) ** 3, rel=1e-12)
    assert fwd["T"][0, cx, cx] == pytest.approx(1.25e-4, rel=1e-9)
    np.testing.assert_allclose(fwd["img"][0, :, cx, cx],
                               [0.999875 * x for x in col], rtol=1e-9)


def _scene(seed, n=60, W=48, H=40, f=45.0, mu=-1.8):
    return synth.tiny_scene(seed, n=n, width=W, height=H, f=f,
                            log_scale_mu=mu)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_invariants(seed):
    w = _scene(seed)
    c = w.cameras[0]
    p = oracle.params64(w.gaussians)
    ones = dict(p, rgb=np.ones_like(p["rgb"]))
    proj, bins, f0 = oracle.render(ones, [c], tile=16)
    # Sum of blend weights + T_final = 1 (colour 1, background 0).
    np.testing.assert_allclose(f0["img"][0, 0] + f0["T"][0], 1.0, atol=1e-13)
    assert f0["T"].min() >= oracle.T_MIN
    # Affine in the background with slope T_final.
    bg = (0.3, 0.7, 0.1)
    _, _, f1 = oracle.render(p, [c], tile=16)
    _, _, f2 = oracle.render(p, [c], tile=16, bg=bg)
    for ch in range(3):
        np.testing.assert_allclose(f2["img"][0, ch] - f1["img"][0, ch],
                                   f1["T"][0] * bg[ch], atol=1e-13)
    # Colours in [0, 1] keep the image in [0, 1].
    assert f2["img"].min() >= 0.0 and f2["img"].max() <= 1.0
    # Transmittance is non-increasing along each pixel's list: check that
    # dropping entries from the end of every list can only raise T.
    assert np.all(f1["nlast"] >= 0)


def test_zero_gaussians():
    w = _scene(0, n=4)
    p = oracle.params64(w.gaussians)
    p["mean"][2] = -5.0
    bg = (0.25, 0.5, 0.75)
    _, bins, f = oracle.render(p, w.cameras, tile=16, bg=bg)
    assert bins["n_keys"] == 0
    for ch in range(3):
        assert np.all(f["img"][0, ch] == bg[ch])
    assert np.all(f["T"] == 1.0) and np.all(f["nlast"] == 0)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_tile_path_equals_brute_force(seed):
    w = _scene(seed)
    c = w.cameras[0]
    p = oracle.params64(w.gaussians)
    bg = (0.1, 0.2, 0.3)
    proj, bins, fwd = oracle.render(p, [c], tile=16, bg=bg)
    img, T, cnt = brute.composite(proj["rec"], proj["box"], p["rgb"], c.width,
                                  c.height, bg)
    np.testing.assert_allclose(fwd["img"], img, rtol=0, atol=1e-13)
    np.testing.assert_allclose(fwd["T"], T, rtol=1e-12, atol=0)
    # n_last counts list positions, the brute force counts contributors:
    # both are zero exactly on the same pixels.
    np.testing.assert_array_equal(fwd["nlast"] == 0, cnt == 0)


def test_sampled_pixels_equal_the_whole_brute_force_image():
    """composite_pixels, the per-pixel form used on images too large to
    composite whole, returns the same values as composite at those pixels,
    and agrees with the tile path there."""
    w = _scene(2)
    c = w.cameras[0]
    p = oracle.params64(w.gaussians)
    bg = (0.1, 0.2, 0.3)
    proj, bins, fwd = oracle.render(p, [c], tile=16, bg=bg)
    img, T, _ = brute.composite(proj["rec"], proj["box"], p["rgb"], c.width,
                                c.height, bg)
    rng = np.random.default_rng(7)
    us = rng.integers(0, c.width, 60)
    vs = rng.integers(0, c.height, 60)
    pimg, pT = brute.composite_pixels(proj["rec"], proj["box"], p["rgb"], 0,
                                      us, vs, bg)
    np.testing.assert_array_equal(pimg, img[0][:, vs, us].T)
    np.testing.assert_array_equal(pT, T[0][vs, us])
    np.testing.assert_allclose(pimg, fwd["img"][0][:, vs, us].T, rtol=0,
                               atol=1e-13)


@pytest.mark.parametrize("seed", [0, 4])
def test_tile_size_invariance(seed):
    w = _scene(seed, n=80)
    c = w.cameras[0]
    p = oracle.params64(w.gaussians)
    outs = [oracle.render(p, [c], tile=t)[2] for t in (8, 16, 32)]
    for o in outs[1:]:
        np.testing.assert_array_equal(o["img"], outs[0]["img"])
        np.testing.assert_array_equal(o["T"], outs[0]["T"])


def test_decision_record_and_replay_reproduce_forward():
    w = _scene(5)
    c = w.cameras[0]
    p = oracle.params64(w.gaussians)
    proj = oracle.project(p, [c], 16, publish=False)
    bins = oracle.bin_sort(proj, 16, c.width, c.height)
    dec = oracle.decision_buffer(bins, 1, c.width, c.height)
    f1 = oracle.forward(proj, bins, p["rgb"], c.width, c.height, dec=dec,
                        dec_mode=1)
    f2 = oracle.forward(proj, bins, p["rgb"], c.width, c.height, dec=dec,
                        dec_mode=2)
    np.testing.assert_array_equal(f1["img"], f2["img"])
    np.testing.assert_array_equal(f1["nlast"], f2["nlast"])


def test_work_counters():
    w = _scene(6)
    c = w.cameras[0]
    p = oracle.params64(w.gaussians)
    proj, bins, fwd = oracle.render(p, [c], tile=16)
    cnt = fwd["counters"]
    assert cnt["examined"] >= cnt["inbox"] >= cnt["contributing"] > 0
    _, _, nb = brute.composite(proj["rec"], proj["box"], p["rgb"], c.width,
                               c.height)
    assert cnt["contributing"] == int(nb.sum())


@pytest.mark.parametrize("tile,views", [(8, 1), (16, 2), (32, 1)])
def test_work_counters_equal_an_independent_count(tile, views):
    """All four work counters (examined, in-box, contributing, revisited)
    equal brute.count_pairs, which builds every tile's list from the boxes
    that meet the tile and walks it per pixel, without the oracle's keys,
    sort or ranges.  Dense enough that many pixels stop at T_min, so the
    stop entry's place in the counts is pinned."""
    w = _scene(7, n=200, mu=-1.5)
    cams = [w.cameras[0]]
    c = cams[0]
    for i in range(views - 1):
        t = (c.t + np.array([0.05 * (i + 1), -0.03, 0.02])).astype(np.float32)
        cams.append(synth.Camera(c.R, t, c.fx, c.fy, c.cx, c.cy, c.width,
                                 c.height))
    p = oracle.params64(w.gaussians)
    proj, bins, fwd = oracle.render(p, cams, tile=tile)
    ref = brute.count_pairs(proj["rec"], proj["box"], c.width, c.height, tile)
    assert (fwd["T"] < 1e-3).sum() > 500
    assert fwd["counters"] == ref
    assert ref["examined"] > ref["inbox"] > ref["revisit"] > ref["contributing"] > 0


def test_pixel_walk_against_brute_force():
    """oracle.pixel_walk at every pixel: the contributing entries' weights
    and the transmittance left add to one, their count and the Gaussian of
    largest weight equal the brute-force compositor's, and the walk's
    in-box entries are those whose box holds the pixel, in list order."""
    w = _scene(8, n=150, mu=-1.6)
    c = w.cameras[0]
    p = oracle.params64(w.gaussians)
    proj, bins, fwd = oracle.render(p, [c], tile=16)
    W, H = c.width, c.height
    g, wt, code, cnt = oracle.pixel_walk(proj, bins, W, H, np.arange(W * H))
    _, Tb, nb, domb = brute.composite(proj["rec"], proj["box"], p["rgb"], W, H,
                                      with_dominant=True)
    contrib = (code == oracle.DEC_ADMIT) | (code == oracle.DEC_CLAMP)
    valid = np.arange(g.shape[1])[None, :] < cnt[:, None]
    contrib &= valid
    np.testing.assert_array_equal(contrib.sum(1), nb.reshape(-1))
    np.testing.assert_allclose(wt.sum(1) + Tb.reshape(-1), 1.0, atol=1e-12)
    best = np.where(contrib.any(1), g[np.arange(W * H), np.argmax(wt, 1)], -1)
    np.testing.assert_array_equal(best, domb.reshape(-1))
    np.testing.assert_array_equal(best, fwd["dom"].reshape(-1))
    np.testing.assert_allclose(wt.max(1), fwd["w1"].reshape(-1), rtol=1e-15)
    assert (code[valid] == oracle.DEC_STOP).sum() > 0
    assert np.all(wt[~contrib] == 0)


def test_admit_extent_closed_form_and_containment():
    """An isotropic Gaussian centred on a pixel: the admissible rectangle's
    half-width is the largest integer d with o exp(-d^2 / (2 s^2)) >=
    alpha_min (1 - max(1e-5, ea)).  On a random scene every contributing
    (pixel, Gaussian) pair lies in the Gaussian's rectangle, which lies in its
    integer box."""
    W = H = 101
    cam = one_cam(W, H, 100.0)
    for sigma_world, logit in ((0.02, 1.0), (0.05, -0.5)):
        p = dict(mean=np.array([[0.0], [0.0], [2.0]]),
                 log_scale=np.full((3, 1), math.log(sigma_world)),
                 quat=np.array([[1.0], [0.0], [0.0], [0.0]]),
                 opacity_logit=np.array([logit]), rgb=np.full((3, 1), 0.5))
        proj = oracle.project(p, [cam], 16, publish=False)
        rect = oracle.admit_extent(proj)[0, 0]
        A = proj["rec"][0, 0, 2]
        o = 1.0 / (1.0 + math.exp(-logit))
        s2 = 1.0 / A
        d = 0
        while True:
            nd = d + 1
            ea = 2.0 ** -24 * (4.0 * nd * nd / s2 + 4.0 + 3.0 * abs(math.log(o)))
            if o * math.exp(-0.5 * nd * nd / s2) < oracle.ALPHA_MIN * (1 - max(1e-5, ea)):
                break
            d = nd
        np.testing.assert_array_equal(rect, [50 - d, 50 + d, 50 - d, 50 + d])
    w = _scene(9, n=150, mu=-1.6)
    c = w.cameras[0]
    p = oracle.params64(w.gaussians)
    proj, bins, fwd = oracle.render(p, [c], tile=16)
    rect = oracle.admit_extent(proj)[0]
    box = proj["box"][0]
    has = rect[:, 1] >= rect[:, 0]
    assert np.all(rect[has, 0] >= box[has, 0]) and np.all(rect[has, 1] <= box[has, 1])
    assert np.all(rect[has, 2] >= box[has, 2]) and np.all(rect[has, 3] <= box[has, 3])
    g, wt, code, cnt = oracle.pixel_walk(proj, bins, c.width, c.height,
                                         np.arange(c.width * c.height))
    pix = np.repeat(np.arange(c.width * c.height), g.shape[1]).reshape(g.shape)
    sel = (code == oracle.DEC_ADMIT) | (code == oracle.DEC_CLAMP)
    sel &= np.arange(g.shape[1])[None, :] < cnt[:, None]
    gg, pp = g[sel], pix[sel]
    u, v = pp % c.width, pp // c.width
    r = rect[gg]
    assert np.all((u >= r[:, 0]) & (u <= r[:, 1]) & (v >= r[:, 2]) & (v <= r[:, 3]))
