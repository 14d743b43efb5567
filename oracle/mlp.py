"""FP64 oracle of the learned-initialisation network and its features.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline are the only callers); shares no code with the GPU library.

Network (32 -> 64 -> 64 -> 7, GELU): weights are kept in FP32 and rounded to
BF16 (round to nearest even) where they are used; layer inputs (the features
and each hidden activation) are rounded to BF16; products and sums are FP64
here (FP32 accumulate on the GPU).  Backward: every gradient that enters a
matrix product is rounded to BF16 first; bias gradients and the GELU
derivative are not rounded; the rounding of weights and activations passes
gradients unchanged.  GELU is the exact erf form.

Parameter vector (6727 values): W1 [32][64], b1 [64], W2 [64][64], b2 [64],
W3 [64][7], b3 [7]; a layer computes z = x W + b.

Features of a new Gaussian at candidate pixel (u, v) of a keyframe with
inverse depth d (32 values): the 3x3 neighbourhood's RGB (27, neighbours
row-major, channels interleaved, zero outside the image), d, the mean natural
log of the distances from the back-projected point to its 8 nearest existing
Gaussian means (ties by lower index; a distance floor of 1e-6 m), and the
inverse-distance-weighted mean RGB of those 8 (4 values; zero when the map
is empty).
"""
from __future__ import annotations

import math

import numpy as np

SIZES = ((32, 64), (64, 64), (64, 7))
N_PARAMS = sum(i * o + o for i, o in SIZES)   # 6727


def unpack(w):
    """Splits the parameter vector into [(W, b)] per layer."""
    w = np.asarray(w, np.float64)
    out, o = [], 0
    for i, n in SIZES:
        W = w[o:o + i * n].reshape(i, n)
        o += i * n
        b = w[o:o + n]
        o += n
        out.append((W, b))
    return out


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + \
        z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(w, x, rounding=True):
    """Returns (y [M][7], cache) for features x [M][32]."""
    r = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    (W1, b1), (W2, b2), (W3, b3) = unpack(w)
    xh = r(x)
    z1 = xh @ r(W1) + b1
    h1 = r(gelu(z1))
    z2 = h1 @ r(W2) + b2
    h2 = r(gelu(z2))
    y = h2 @ r(W3) + b3
    return y, dict(x=xh, z1=z1, h1=h1, z2=z2, h2=h2)


def backward(w, cache, dy, rounding=True):
    """Gradient of the parameter vector for dL/dy [M][7]."""
    r = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    (W1, _), (W2, _), (W3, _) = unpack(w)
    dy = np.asarray(dy, np.float64)
    dyh = r(dy)
    dW3 = cache["h2"].T @ dyh
    db3 = dy.sum(0)
    dz2 = (dyh @ r(W3).T) * gelu_grad(cache["z2"])
    dz2h = r(dz2)
    dW2 = cache["h1"].T @ dz2h
    db2 = dz2.sum(0)
    dz1 = (dz2h @ r(W2).T) * gelu_grad(cache["z1"])
    dz1h = r(dz1)
    dW1 = cache["x"].T @ dz1h
    db1 = dz1.sum(0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(),
                           db3])


def forward_magnitude(w, cache):
    """Per output, the magnitude through which a one-ulp change of a BF16
    hidden activation reaches it: sum_j |W3_jk| (|h2_j| + |gelu'(z2_j)|
    sum_i |W2_ij| |h1_i|).  A BF16 rounding of an activation that lands on
    the other side of a rounding boundary (FP32 vs FP64 arithmetic) moves it
    by at most 2^-7 of its magnitude, so the output moves by at most 2^-7
    times this."""
    (W1, _), (W2, _), (W3, _) = unpack(w)
    a2 = np.abs(bf16(W2))
    a3 = np.abs(bf16(W3))
    e2 = np.abs(cache["h2"]) + np.abs(gelu_grad(cache["z2"])) * \
        (np.abs(cache["h1"]) @ a2)
    return e2 @ a3


def backward_magnitude(w, cache, dy):
    """backward() with every factor by absolute value (the BF16 roundings
    kept): for non-negative dy it bounds how far an input change of size dy
    moves each gradient element, and it is the sum of the magnitudes of the
    terms each element adds up."""
    (W1, _), (W2, _), (W3, _) = unpack(w)
    dyh = np.abs(bf16(np.asarray(dy, np.float64)))
    dW3 = np.abs(cache["h2"]).T @ dyh
    db3 = dyh.sum(0)
    dz2 = (dyh @ np.abs(bf16(W3)).T) * np.abs(gelu_grad(cache["z2"]))
    dz2h = np.abs(bf16(dz2))
    dW2 = np.abs(cache["h1"]).T @ dz2h
    db2 = dz2.sum(0)
    dz1 = (dz2h @ np.abs(bf16(W2)).T) * np.abs(gelu_grad(cache["z1"]))
    dz1h = np.abs(bf16(dz1))
    dW1 = np.abs(cache["x"]).T @ dz1h
    db1 = dz1.sum(0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(),
                           db3])


def mse(y, t):
    """Mean over all entries of (y - t)^2 and its gradient."""
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float((d * d).mean()), 2.0 * d / d.size


def init_weights(seed=0):
    """He-style initialisation (the generator the GPU training also uses is
    separate; this one serves the oracle tests)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in SIZES:
        parts.append(rng.normal(0, math.sqrt(2.0 / i), size=i * o))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def knn(means, queries, k=8):
    """Brute force: indices [Q][k] and distances of the k nearest means
    ([3][n]) to each query ([Q][3]), ascending, ties by lower index."""
    m = np.asarray(means, np.float64)
    q = np.asarray(queries, np.float64)
    n = m.shape[1]
    idx = np.zeros((q.shape[0], min(k, n)), np.int64)
    dist = np.zeros((q.shape[0], min(k, n)))
    for i in range(q.shape[0]):
        d2 = ((m - q[i][:, None]) ** 2).sum(0)
        order = np.lexsort((np.arange(n), d2))[:k]
        idx[i] = order
        dist[i] = np.sqrt(d2[order])
    return idx, dist


def features(cam, kf_rgb, pts_uvd, means, rgb, centre_only=False):
    """Features [C][32] of every candidate (patch by patch, the 3x3 pixels
    row-major, or only the centres) and their back-projected points."""
    H, W = cam.height, cam.width
    R = np.asarray(cam.R, np.float32).astype(np.float64)
    t = np.asarray(cam.t, np.float32).astype(np.float64)
    fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    cx, cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))
    img = np.asarray(kf_rgb, np.float32).astype(np.float64)
    cands, pts = [], []
    for k in range(pts_uvd.shape[0]):
        uc, vc, d = (int(pts_uvd[k, 0]), int(pts_uvd[k, 1]),
                     float(np.float32(pts_uvd[k, 2])))
        for p in ([4] if centre_only else range(9)):
            u, v = uc + p % 3 - 1, vc + p // 3 - 1
            f = np.zeros(32)
            for q in range(9):
                uu, vv = u + q % 3 - 1, v + q // 3 - 1
                if 0 <= uu < W and 0 <= vv < H:
                    f[3 * q:3 * q + 3] = img[:, vv, uu]
            f[27] = d
            z = 1.0 / d if d > 0 else 0.0
            xc = np.array([(u - cx) / fx * z, (v - cy) / fy * z, z])
            pts.append(R.T @ (xc - t))
            cands.append(f)
    F = np.array(cands).reshape(-1, 32)
    P = np.array(pts).reshape(-1, 3)
    n = means.shape[1]
    if n > 0 and len(P):
        idx, dist = knn(means, P)
        w = 1.0 / np.maximum(dist, 1e-6)
        F[:, 28] = np.log(np.maximum(dist, 1e-6)).mean(1)
        col = np.asarray(rgb, np.float64)[:, idx]          # [3][C][k]
        F[:, 29:32] = ((col * w[None]).sum(2) / w.sum(1)[None]).T
    return F, P
