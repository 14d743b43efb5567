"""FP64 oracle of clarity-enhancing densification (Eq. 8-9).

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline are the only callers); shares no code with the GPU library.

Eq. 8 picks, for every pixel of the current keyframe, the Gaussian with the
largest blend weight w_m = alpha_m prod_{n<m}(1 - alpha_n) (the forward
oracle returns it as "dom").  Eq. 9 splits the Gaussians whose rendered
pixels overlap the dominant ones by more than a threshold sigma; the overlap
count is garbled in the text and is read as the number of pixels a Gaussian
dominates (strictly more than sigma pixels).  The split itself is not given;
the reading follows the 3D Gaussian Splatting split it builds on: two
children replace the parent, each with mean mu + R(q) (s * xi) for a
standard-normal 3-vector xi (drawn by the caller and passed in, one pair per
Gaussian), log-scale reduced by log(1.6), rotation, opacity and colour
copied.  Child 0 takes the parent's slot, child 1 is appended; children are
appended in ascending parent index, and when the capacity cannot hold every
appended child only the first parents that fit are split (the rest stay
unchanged and the overflow is reported).  Adam moments of both children are
reset to zero.
"""
from __future__ import annotations

import math

import numpy as np

SPLIT_SCALE = 1.6
KEYS = ("mean", "log_scale", "quat", "opacity_logit", "rgb")


def dominated_counts(dom: np.ndarray, n: int) -> np.ndarray:
    """Number of pixels each Gaussian dominates (dom = -1: no Gaussian)."""
    d = np.asarray(dom).ravel()
    return np.bincount(d[d >= 0], minlength=n)[:n]


def rotation(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of the normalised quaternion (w, x, y, z)."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def split(p: dict, n: int, capacity: int, counts: np.ndarray, sigma: int,
          xi: np.ndarray):
    """Splits the Gaussians that dominate more than sigma pixels.

    p: dict of FP64 rows as params64 returns (mean [3][cap], ...), with at
    least `capacity` columns; xi [capacity][2][3].  Returns (new p, new n,
    list of split parents, overflow flag)."""
    out = {k: np.array(v, np.float64, copy=True) for k, v in p.items()}
    eligible = [g for g in range(n) if counts[g] > sigma]
    room = capacity - n
    parents = eligible[:max(0, room)]
    for rank, g in enumerate(parents):
        R = rotation(p["quat"][:, g])
        s = np.exp(p["log_scale"][:, g])
        slots = (g, n + rank)
        for c, slot in enumerate(slots):
            out["mean"][:, slot] = p["mean"][:, g] + R @ (s * xi[g, c])
            out["log_scale"][:, slot] = p["log_scale"][:, g] - math.log(SPLIT_SCALE)
            out["quat"][:, slot] = p["quat"][:, g]
            out["opacity_logit"][slot] = p["opacity_logit"][g]
            out["rgb"][:, slot] = p["rgb"][:, g]
    return out, n + len(parents), parents, len(parents) < len(eligible)
