"""FP64 oracle of view-dependent colour: the Gaussian colour coefficients
c in R^k (Methodology, Scene Representation: the parameters listed after
Eq. 1), read as real spherical harmonics of the viewing direction.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline are the only callers); shares no code with the GPU library.

The paper gives the coefficient vector but not its size or basis.  The
reading follows 3D Gaussian Splatting, which it builds on: per colour channel
the real spherical harmonics of degree 0..D ((D+1)^2 coefficients) evaluated
at the unit direction d from the camera centre o = -R^T t to the mean,

    raw_c = rgb_c + sum_{j >= 1} Y_j(d) f_{j,c},      colour_c = max(raw_c, 0),

where the degree-0 term is carried by the rgb row (it plays the part of
Y_0 f_0 + 1/2 in the 3D Gaussian Splatting form) and j runs over (l, m) in
the order l = 1..D, m = -l..l.  Y_lm is sqrt(2) Re Y_l^m for m > 0,
sqrt(2) Im Y_l^|m| for m < 0 and Y_l^0 for m = 0, with Y_l^m the complex
harmonic carrying the Condon-Shortley phase.  The clamp at zero applies for
D >= 1; D = 0 is the view-independent colour (the rgb rows unchanged, no
clamp).  The gradient passes where raw_c >= 0.

Coefficient layout: sh [K-1][3][n] (K = (D+1)^2), coefficient j >= 1 of
channel c at sh[j-1, c].
"""
from __future__ import annotations

import math

import numpy as np


def n_coeffs(D: int) -> int:
    """Coefficients per channel for degree D."""
    return (D + 1) ** 2


# Normalisation constants of the real harmonics, from
# N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) written out per (l, m).
_K0 = 0.5 / math.sqrt(math.pi)
_K1 = math.sqrt(3.0 / (4.0 * math.pi))
_K2a = 0.5 * math.sqrt(15.0 / math.pi)
_K2b = 0.25 * math.sqrt(5.0 / math.pi)
_K2c = 0.25 * math.sqrt(15.0 / math.pi)
_K3a = 0.25 * math.sqrt(35.0 / (2.0 * math.pi))
_K3b = 0.5 * math.sqrt(105.0 / math.pi)
_K3c = 0.25 * math.sqrt(21.0 / (2.0 * math.pi))
_K3d = 0.25 * math.sqrt(7.0 / math.pi)
_K3e = 0.25 * math.sqrt(105.0 / math.pi)


def basis(D: int, d: np.ndarray) -> np.ndarray:
    """Y_j(d) for j < (D+1)^2 at unit directions d [..., 3] -> [..., K].
    The polynomial forms assume |d| = 1."""
    if not 0 <= D <= 3:
        raise ValueError("degree 0..3")
    d = np.asarray(d, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = [np.full(x.shape, _K0)]
    if D >= 1:
        out += [-_K1 * y, _K1 * z, -_K1 * x]
    if D >= 2:
        out += [_K2a * x * y, -_K2a * y * z, _K2b * (2 * z * z - x * x - y * y),
                -_K2a * x * z, _K2c * (x * x - y * y)]
    if D >= 3:
        out += [-_K3a * y * (3 * x * x - y * y), _K3b * x * y * z,
                -_K3c * y * (4 * z * z - x * x - y * y),
                _K3d * z * (2 * z * z - 3 * x * x - 3 * y * y),
                -_K3c * x * (4 * z * z - x * x - y * y),
                _K3e * z * (x * x - y * y),
                -_K3a * x * (x * x - 3 * y * y)]
    return np.stack(out, -1)


def basis_grad(D: int, d: np.ndarray) -> np.ndarray:
    """Gradient of each polynomial Y_j with respect to (x, y, z), taken with
    the three components independent: [..., K, 3]."""
    d = np.asarray(d, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    o = np.zeros(x.shape)
    g = [(o, o, o)]
    if D >= 1:
        g += [(o, -_K1 + o, o), (o, o, _K1 + o), (-_K1 + o, o, o)]
    if D >= 2:
        g += [(_K2a * y, _K2a * x, o), (o, -_K2a * z, -_K2a * y),
              (-2 * _K2b * x, -2 * _K2b * y, 4 * _K2b * z),
              (-_K2a * z, o, -_K2a * x), (2 * _K2c * x, -2 * _K2c * y, o)]
    if D >= 3:
        g += [(-6 * _K3a * x * y, -3 * _K3a * (x * x - y * y), o),
              (_K3b * y * z, _K3b * x * z, _K3b * x * y),
              (2 * _K3c * x * y, -_K3c * (4 * z * z - x * x - 3 * y * y),
               -8 * _K3c * y * z),
              (-6 * _K3d * x * z, -6 * _K3d * y * z,
               _K3d * (6 * z * z - 3 * x * x - 3 * y * y)),
              (-_K3c * (4 * z * z - 3 * x * x - y * y), 2 * _K3c * x * y,
               -8 * _K3c * x * z),
              (2 * _K3e * x * z, -2 * _K3e * y * z, _K3e * (x * x - y * y)),
              (-3 * _K3a * (x * x - y * y), 6 * _K3a * x * y, o)]
    return np.stack([np.stack(t, -1) for t in g], -2)


def camera_centre(cam) -> np.ndarray:
    """o = -R^T t from the FP32 camera, in FP64."""
    R = np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float32).astype(np.float64)
    return -(R.T @ t)


def _directions(mean, cam):
    """Unit directions from the camera centre to the means [n][3] and the
    reciprocal distances 1 / |mu - o| [n].  A mean at the camera centre
    (never rendered in that view: it lies before the near plane) gets
    direction 0 and reciprocal 0."""
    v = np.asarray(mean, np.float64).T - camera_centre(cam)[None, :]
    r = np.sqrt((v * v).sum(1))
    inv = np.divide(1.0, r, out=np.zeros_like(r), where=r > 0)
    return v * inv[:, None], inv


def colours(p: dict, cams, D: int):
    """Per-view colours [V][3][n] and the unclamped values raw [V][3][n].
    p holds FP64 rows: mean [3][n], rgb [3][n] and, for D >= 1,
    sh [K-1][3][n]."""
    rgb = np.asarray(p["rgb"], np.float64)
    V, n = len(cams), rgb.shape[1]
    if D == 0:
        out = np.broadcast_to(rgb, (V, 3, n)).copy()
        return out, out.copy()
    sh = np.asarray(p["sh"], np.float64)
    raw = np.zeros((V, 3, n))
    for k, cam in enumerate(cams):
        d, _ = _directions(p["mean"], cam)
        Y = basis(D, d)[:, 1:]                       # [n][K-1]
        raw[k] = rgb + np.einsum("nj,jcn->cn", Y, sh)
    return np.maximum(raw, 0.0), raw


def colours_bwd(p: dict, cams, D: int, gcol: np.ndarray):
    """Chain rule of colours() for dL/d colour gcol [V][3][n]: returns
    d_rgb [3][n], d_sh [K-1][3][n] and d_mean [3][n] (through the viewing
    direction), each summed over the views."""
    rgb = np.asarray(p["rgb"], np.float64)
    n = rgb.shape[1]
    gcol = np.asarray(gcol, np.float64)
    if D == 0:
        return gcol.sum(0), np.zeros((0, 3, n)), np.zeros((3, n))
    sh = np.asarray(p["sh"], np.float64)
    _, raw = colours(p, cams, D)
    d_rgb = np.zeros((3, n))
    d_sh = np.zeros_like(sh)
    d_mean = np.zeros((3, n))
    for k, cam in enumerate(cams):
        d, inv_r = _directions(p["mean"], cam)
        g = np.where(raw[k] >= 0.0, gcol[k], 0.0)    # [3][n]
        d_rgb += g
        Y = basis(D, d)[:, 1:]                       # [n][K-1]
        d_sh += np.einsum("nj,cn->jcn", Y, g)
        dY = basis_grad(D, d)[:, 1:, :]               # [n][K-1][3]
        # dL/d(direction), then through d = v / |v|: (I - d d^T) / |v|.
        gd = np.einsum("njx,jcn,cn->nx", dY, sh, g)
        gv = (gd - d * (gd * d).sum(1, keepdims=True)) * inv_r[:, None]
        d_mean += gv.T
    return d_rgb, d_sh, d_mean


def chain(p: dict, cams, D: int, bwd: dict, nthreads: int = 1) -> dict:
    """Parameter gradients of the whole backward for view-dependent colour:
    bwd is the compositing backward run on the per-view colours (its grgb is
    [V][3][n]); the screen-space part goes through the projection backward,
    the colour part through colours_bwd.  Returns the rows of
    ``oracle.project_bwd`` plus "sh" [K-1][3][n]."""
    from . import project_bwd
    d_rgb, d_sh, d_mean = colours_bwd(p, cams, D, bwd["grgb"])
    out = project_bwd(p, cams, dict(bwd, grgb=d_rgb), nthreads)
    out["mean"] = out["mean"] + d_mean
    out["sh"] = d_sh
    return out


def colours_bwd_abs(p: dict, cams, D: int, gcol: np.ndarray):
    """Magnitudes of the terms colours_bwd adds up, for the same per-view
    colour gradients gcol [V][3][n]: every partial derivative and gradient
    by absolute value (the direction chain as |(I - d d^T) / |v|| applied to
    sum_j |dY_j| |f_j| |g|).  Returns d_rgb, d_sh, d_mean magnitudes."""
    rgb = np.asarray(p["rgb"], np.float64)
    n = rgb.shape[1]
    gabs = np.abs(np.asarray(gcol, np.float64))
    if D == 0:
        return gabs.sum(0), np.zeros((0, 3, n)), np.zeros((3, n))
    sh = np.asarray(p["sh"], np.float64)
    _, raw = colours(p, cams, D)
    d_rgb = np.zeros((3, n))
    d_sh = np.zeros_like(sh)
    d_mean = np.zeros((3, n))
    for k, cam in enumerate(cams):
        d, inv_r = _directions(p["mean"], cam)
        g = np.where(raw[k] >= 0.0, gabs[k], 0.0)     # [3][n]
        d_rgb += g
        Y = np.abs(basis(D, d)[:, 1:])                # [n][K-1]
        d_sh += np.einsum("nj,cn->jcn", Y, g)
        dY = np.abs(basis_grad(D, d)[:, 1:, :])       # [n][K-1][3]
        gd = np.einsum("njx,jcn,cn->nx", dY, np.abs(sh), g)
        P = np.abs(np.eye(3)[None] - d[:, :, None] * d[:, None, :])
        d_mean += (np.einsum("nxy,ny->nx", P, gd) * inv_r[:, None]).T
    return d_rgb, d_sh, d_mean


def chain_abs(p: dict, cams, D: int, bwd: dict, nthreads: int = 1) -> dict:
    """Magnitudes of the chain-rule terms of chain() (see
    oracle.project_bwd_abs): the screen-space part through the projection
    backward, the colour part through colours_bwd_abs."""
    from . import project_bwd_abs
    d_rgb, d_sh, d_mean = colours_bwd_abs(p, cams, D, bwd["grgb"])
    out = project_bwd_abs(p, cams, dict(bwd, grgb=d_rgb), nthreads)
    out["mean"] = out["mean"] + d_mean
    out["sh"] = d_sh
    return out
