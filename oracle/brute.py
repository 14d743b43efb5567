"""Brute-force per-pixel compositing in NumPy (test infrastructure only).

For every pixel it gathers every Gaussian whose integer pixel box contains the
pixel, orders them by (FP32 depth, index) with ``numpy.lexsort`` and blends
front to back with the rule of Eq. 3 plus the cut-offs.  It uses no tiles, no
keys and no ranges, so it checks the oracle's binning, sort and tile walk
independently.  Pure Python loops over pixels: composite() only for tiny
scenes, composite_pixels() for a sample of pixels of a large image.
count_pairs() counts the work of a tile walk from the definition of a tile's
list (every Gaussian whose box meets the tile, in (depth, index) order), built
here without keys or a sort of the oracle's.
"""
from __future__ import annotations

import math

import numpy as np


def _blend_pixel(rec_k, box_k, depth_bits, rgb, u, v, alpha_min, T_min,
                 alpha_max):
    """Eq. 3 at pixel (u, v) of one view: every Gaussian whose integer box
    holds the pixel, in (FP32 depth, index) order, blended front to back with
    the cut-offs.  Returns (colour without background, T_final, count,
    dominant Gaussian, its weight)."""
    inb = ((box_k[:, 0] <= u) & (u <= box_k[:, 1]) &
           (box_k[:, 2] <= v) & (v <= box_k[:, 3]))
    cand = np.nonzero(inb)[0]
    order = cand[np.lexsort((cand, depth_bits[cand]))]
    T = 1.0
    C = [0.0, 0.0, 0.0]
    cnt = 0
    wbest, gbest = 0.0, -1
    for g in order:
        px, py, A, B, Cc, o = rec_k[g, :6]
        dx, dy = px - u, py - v
        pw = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
        if pw > 0:
            continue
        a = min(alpha_max, o * math.exp(pw))
        if a < alpha_min:
            continue
        Tn = T * (1.0 - a)
        if Tn < T_min:
            break
        for ch in range(3):
            C[ch] += rgb[ch, g] * a * T
        if a * T > wbest:
            wbest, gbest = a * T, int(g)
        T = Tn
        cnt += 1
    return C, T, cnt, gbest


def _cutoffs(alpha_min, T_min, alpha_max):
    from . import ALPHA_MAX, ALPHA_MIN, T_MIN
    return (ALPHA_MIN if alpha_min is None else alpha_min,
            T_MIN if T_min is None else T_min,
            ALPHA_MAX if alpha_max is None else alpha_max)


def composite(rec, box, rgb, W, H, bg=(0.0, 0.0, 0.0), alpha_min=None,
              T_min=None, alpha_max=None, with_dominant=False):
    """Returns (image, T_final, contributor count) and, with_dominant, also
    the Gaussian of largest blend weight alpha * T per pixel (Eq. 8; first
    on ties, -1 when none)."""
    alpha_min, T_min, alpha_max = _cutoffs(alpha_min, T_min, alpha_max)
    V, n, _ = rec.shape
    img = np.zeros((V, 3, H, W))
    Tf = np.ones((V, H, W))
    ncontrib = np.zeros((V, H, W), np.int64)
    dominant = np.full((V, H, W), -1, np.int64)
    for k in range(V):
        depth_bits = rec[k, :, 6].astype(np.float32).view(np.uint32)
        for v in range(H):
            for u in range(W):
                C, T, cnt, gbest = _blend_pixel(rec[k], box[k], depth_bits,
                                                rgb, u, v, alpha_min, T_min,
                                                alpha_max)
                for ch in range(3):
                    img[k, ch, v, u] = C[ch] + T * bg[ch]
                Tf[k, v, u] = T
                ncontrib[k, v, u] = cnt
                dominant[k, v, u] = gbest
    if with_dominant:
        return img, Tf, ncontrib, dominant
    return img, Tf, ncontrib


def composite_pixels(rec, box, rgb, view, us, vs, bg=(0.0, 0.0, 0.0),
                     alpha_min=None, T_min=None, alpha_max=None):
    """composite() at the listed pixels (us[i], vs[i]) of one view only, for
    images too large to composite whole: colours [m][3] and T_final [m]."""
    alpha_min, T_min, alpha_max = _cutoffs(alpha_min, T_min, alpha_max)
    depth_bits = rec[view, :, 6].astype(np.float32).view(np.uint32)
    m = len(us)
    img = np.zeros((m, 3))
    Tf = np.ones(m)
    for i in range(m):
        C, T, _, _ = _blend_pixel(rec[view], box[view], depth_bits, rgb,
                                  int(us[i]), int(vs[i]), alpha_min, T_min,
                                  alpha_max)
        img[i] = [C[ch] + T * bg[ch] for ch in range(3)]
        Tf[i] = T
    return img, Tf


def count_pairs(rec, box, W, H, tile, alpha_min=None, T_min=None,
                alpha_max=None):
    """Work of walking every pixel's tile list front to back, summed over
    all pixels of all views: examined entries (from the list's start up to
    and including the entry that stops the pixel, or to the list's end),
    in-box entries among them, contributing entries, and in-box entries
    before the pixel's last contributing one (the pairs a backward pass
    walking back from the last contributor revisits).  A tile's list is every
    Gaussian whose integer box meets the tile's pixel rectangle, ordered by
    (FP32 depth bits, index)."""
    alpha_min, T_min, alpha_max = _cutoffs(alpha_min, T_min, alpha_max)
    V, n, _ = rec.shape
    Tx, Ty = -(-W // tile), -(-H // tile)
    tot = dict(examined=0, inbox=0, contributing=0, revisit=0)
    for k in range(V):
        depth_bits = rec[k, :, 6].astype(np.float32).view(np.uint32)
        b = box[k]
        for ty in range(Ty):
            for tx in range(Tx):
                u0, v0 = tx * tile, ty * tile
                u1, v1 = min(W, u0 + tile) - 1, min(H, v0 + tile) - 1
                meets = ((b[:, 0] <= u1) & (b[:, 1] >= u0) & (b[:, 2] <= v1) &
                         (b[:, 3] >= v0) & (b[:, 0] <= b[:, 1]) &
                         (b[:, 2] <= b[:, 3]))
                cand = np.nonzero(meets)[0]
                lst = cand[np.lexsort((cand, depth_bits[cand]))]
                for v in range(v0, v1 + 1):
                    for u in range(u0, u1 + 1):
                        T = 1.0
                        inb_pos = []
                        last = 0
                        for i, g in enumerate(lst):
                            tot["examined"] += 1
                            if not (b[g, 0] <= u <= b[g, 1] and
                                    b[g, 2] <= v <= b[g, 3]):
                                continue
                            tot["inbox"] += 1
                            inb_pos.append(i)
                            px, py, A, B, Cc, o = rec[k, g, :6]
                            dx, dy = px - u, py - v
                            pw = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy
                            if pw > 0:
                                continue
                            a = min(alpha_max, o * math.exp(pw))
                            if a < alpha_min:
                                continue
                            Tn = T * (1.0 - a)
                            if Tn < T_min:
                                break
                            T = Tn
                            tot["contributing"] += 1
                            last = i + 1
                        tot["revisit"] += sum(1 for i in inb_pos if i < last)
    return tot
