"""FP64 oracle of the structural-similarity term of the colour loss.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline are the only callers); shares no code with the GPU library.

The colour loss of the map optimisation (Eq. 10) mixes the L1 photometric
term and a structural-similarity term with weight lambda_photo = 0.2.  As a
loss the similarity enters as 1 - SSIM (it is maximised at 1 for identical
images).  Window, sigma and the stabilising constants are not given in the
paper; the reading is the usual one of the 3D Gaussian Splatting objective
it follows: an 11 x 11 Gaussian window with sigma 1.5 (normalised to sum 1),
C1 = 0.01^2, C2 = 0.03^2, zero padding at the image border (every pixel has
a full window, out-of-image samples are 0), per channel, and the mean over
all pixels and channels of a view.

For one channel, with w the window and * the zero-padded window sum
(mu_x = w * x, m_xx = w * (x x), m_xy = w * (x y), likewise for y):
    var_x = m_xx - mu_x^2,  cov = m_xy - mu_x mu_y
    SSIM = (2 mu_x mu_y + C1)(2 cov + C2) / ((mu_x^2 + mu_y^2 + C1)(var_x + var_y + C2))
Its derivative with respect to the rendered image x goes through the three
window sums that contain x: with S the per-pixel SSIM and A1, A2, B1, B2 its
four factors,
    dS/dmu_x = S (2 mu_y / A1 - 2 mu_y / A2 - 2 mu_x / B1 + 2 mu_x / B2)
    dS/dm_xx = -S / B2,   dS/dm_xy = 2 S / A2,
and each window sum distributes its gradient back through the same (symmetric)
window: dS/dx(p) = sum_q w(q - p) [dS/dmu_x(q) + 2 x(p) dS/dm_xx(q) +
y(p) dS/dm_xy(q)].  Everything here is written out with plain loops over the
121 window offsets, vectorised over pixels only.
"""
from __future__ import annotations

import math

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def window_1d() -> np.ndarray:
    r = WINDOW // 2
    g = np.array([math.exp(-((i - r) ** 2) / (2.0 * SIGMA ** 2))
                  for i in range(WINDOW)])
    return g / g.sum()


def window_2d() -> np.ndarray:
    g = window_1d()
    return np.outer(g, g)


def window_sum(img: np.ndarray) -> np.ndarray:
    """Zero-padded window sum over the last two axes:
    out[..., v, u] = sum_{a, b} w[a, b] img[..., v + a - 5, u + b - 5]."""
    w = window_2d()
    r = WINDOW // 2
    H, W = img.shape[-2:]
    pad = np.zeros(img.shape[:-2] + (H + 2 * r, W + 2 * r))
    pad[..., r:r + H, r:r + W] = img
    out = np.zeros(img.shape, np.float64)
    for a in range(WINDOW):
        for b in range(WINDOW):
            out += w[a, b] * pad[..., a:a + H, b:b + W]
    return out


def _stats(x, y):
    mx, my = window_sum(x), window_sum(y)
    mxx, myy, mxy = window_sum(x * x), window_sum(y * y), window_sum(x * y)
    A1 = 2.0 * mx * my + C1
    A2 = 2.0 * (mxy - mx * my) + C2
    B1 = mx * mx + my * my + C1
    B2 = (mxx - mx * mx) + (myy - my * my) + C2
    return mx, my, A1, A2, B1, B2


def ssim_map(x, y) -> np.ndarray:
    """Per-pixel, per-channel SSIM of images [..., H, W] (FP64)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    _, _, A1, A2, B1, B2 = _stats(x, y)
    return (A1 * A2) / (B1 * B2)


def loss_ssim(x, y, lam=1.0):
    """lam * sum over views of (1 - mean SSIM over 3HW) and its gradient with
    respect to x, for images [V][3][H][W]."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    V = x.shape[0]
    n = x[0].size
    mx, my, A1, A2, B1, B2 = _stats(x, y)
    S = (A1 * A2) / (B1 * B2)
    loss = lam * float(np.sum(1.0 - S.reshape(V, -1).mean(1)))
    d_mu = S * (2.0 * my / A1 - 2.0 * my / A2 - 2.0 * mx / B1 + 2.0 * mx / B2)
    d_mxx = -S / B2
    d_mxy = 2.0 * S / A2
    dS = window_sum(d_mu) + 2.0 * x * window_sum(d_mxx) + y * window_sum(d_mxy)
    grad = -(lam / n) * dS
    return loss, grad
