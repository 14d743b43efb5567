"""Pins of the FP64 structural-similarity oracle (colour loss, Eq. 10)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import ssim as S


def _pair(seed, shape=(2, 3, 13, 17)):
    rng = np.random.default_rng(seed)
    x = rng.uniform(size=shape)
    y = np.clip(x + 0.2 * rng.normal(size=shape), 0.0, 1.0)
    return x, y


def test_window_is_a_normalised_gaussian():
    g = S.window_1d()
    assert g.shape == (11,) and abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, g[::-1])
    r = np.arange(11) - 5
    ref = np.exp(-r * r / (2 * 1.5 ** 2))
    assert np.allclose(g, ref / ref.sum(), rtol=0, atol=1e-16)


def test_identical_images_have_ssim_one_and_zero_gradient():
    x, _ = _pair(1)
    m = S.ssim_map(x, x)
    assert np.abs(m - 1.0).max() < 1e-12
    loss, grad = S.loss_ssim(x, x, 0.2)
    assert abs(loss) < 1e-12 and np.abs(grad).max() < 1e-12


def test_constant_images_match_the_closed_form_away_from_the_border():
    c1, c2 = 0.3, 0.7
    x = np.full((1, 3, 25, 27), c1)
    y = np.full((1, 3, 25, 27), c2)
    m = S.ssim_map(x, y)[..., 5:-5, 5:-5]
    ref = (2 * c1 * c2 + S.C1) / (c1 * c1 + c2 * c2 + S.C1)
    assert np.abs(m - ref).max() < 1e-12


def test_matches_an_independent_library_filter():
    """The same definition through scipy's zero-padded correlation."""
    x, y = _pair(2, (1, 3, 21, 30))
    w = S.window_2d()
    f = lambda a: np.stack([ndimage.correlate(a[0, c], w, mode="constant",
                                              cval=0.0) for c in range(3)])[None]
    mx, my = f(x), f(y)
    vx, vy, cov = f(x * x) - mx * mx, f(y * y) - my * my, f(x * y) - mx * my
    ref = ((2 * mx * my + S.C1) * (2 * cov + S.C2)) / (
        (mx * mx + my * my + S.C1) * (vx + vy + S.C2))
    assert np.abs(S.ssim_map(x, y) - ref).max() < 1e-12


def test_symmetric_and_bounded():
    x, y = _pair(3)
    a, b = S.ssim_map(x, y), S.ssim_map(y, x)
    assert np.abs(a - b).max() < 1e-14
    assert a.max() <= 1.0 + 1e-12


def test_gradient_matches_central_differences():
    x, y = _pair(4)
    lam = 0.2
    _, g = S.loss_ssim(x, y, lam)
    rng = np.random.default_rng(5)
    idx = [tuple(int(rng.integers(0, n)) for n in x.shape) for _ in range(40)]
    # Border and corner pixels too.
    idx += [(0, 0, 0, 0), (1, 2, 12, 16), (0, 1, 0, 16), (1, 0, 12, 0)]
    for i in idx:
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (S.loss_ssim(xp, y, lam)[0] - S.loss_ssim(xm, y, lam)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) * 1e-2 + 1e-9, \
            (i, fd, g[i])


def test_loss_sums_views_of_one_minus_mean_ssim():
    x, y = _pair(6)
    loss, _ = S.loss_ssim(x, y, 0.2)
    m = S.ssim_map(x, y)
    ref = 0.2 * sum(1.0 - m[k].mean() for k in range(x.shape[0]))
    assert abs(loss - ref) < 1e-12


@pytest.mark.parametrize("shape", [(1, 3, 1, 1), (1, 3, 4, 30), (1, 3, 12, 3)])
def test_tiny_and_thin_images(shape):
    """Windows larger than the image: the zero padding still defines every
    sum; identical images still give 1."""
    x, y = _pair(7, shape)
    assert np.isfinite(S.ssim_map(x, y)).all()
    assert np.abs(S.ssim_map(x, x) - 1.0).max() < 1e-12
