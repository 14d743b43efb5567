"""Pins the per-element tolerance of the GPU gradient comparisons.

A parameter gradient is a sum of chain-rule terms (over views, pixels and
the screen-space quantities px, py, A, B, C, opacity and colour); where large
terms cancel, the FP32 screen-space sums' rounding is amplified.  The GPU
comparisons therefore take, per element, 1e-3 of max(|g|, 1e-2 max|g| of its
kind, m), where m is the sum of the absolute values of the terms
(oracle.project_bwd_abs / oracle.sh.chain_abs), and check the screen-space
gradients themselves per element at 1e-3.

Pinned here: the magnitude equals the projection backward assembled column
by column from one-hot calls; it bounds |g|; an FP32 evaluation of the
compositing backward, written here with numpy float32 arithmetic (forward
compositing, transmittance recovered by division from T_final, the running
colour sum, a pairwise sum over each tile's pixels, then a sequential sum
over the tiles in random orders), passes both checks; and planted mistakes in
it (a dropped background term, the transmittance of the wrong entry) fail
them."""
import numpy as np
import pytest

import oracle
from oracle import sh as OS
import synth

F32 = np.float32


def _scene(seed, n=180, W=61, H=47, f=50.0, views=2):
    w = synth.tiny_scene(seed, n=n, width=W, height=H, f=f, log_scale_mu=-1.8)
    rng = np.random.default_rng(seed + 7)
    c = w.cameras[0]
    cams = [c]
    for _ in range(views - 1):
        a = rng.normal(0, 0.08)
        R = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0],
                      [-np.sin(a), 0, np.cos(a)]], np.float32)
        cams.append(synth.Camera(R, rng.normal(0, 0.05, 3).astype(np.float32),
                                 c.fx, c.fy, c.cx, c.cy, c.width, c.height))
    w.cameras = cams
    return w


def fp32_backward(proj, bins, rgb, W, H, dL, bg, order_seed,
                  plant=None):
    """The compositing backward evaluated in FP32 (see the module text).
    Returns g2d [V][n][5], gop [n], grgb [3][n] as float32."""
    rec = proj["rec"].astype(F32)
    box = proj["box"]
    V, n = proj["tiles"].shape
    tile = bins["tile"]
    Tx, Ty = bins["Tx"], bins["Ty"]
    vals, ranges = bins["vals"], bins["ranges"]
    rgb32 = rgb.astype(F32)
    bg32 = np.asarray(bg, F32)
    amin, tmin, amax = F32(1.0 / 255.0), F32(1e-4), F32(0.99)
    parts = []   # (view, gaussian, tile, q, partial)
    for t in range(V * Tx * Ty):
        k, tt = divmod(t, Tx * Ty)
        ty, tx = divmod(tt, Tx)
        s, e = int(ranges[t, 0]), int(ranges[t, 1])
        if s == e:
            continue
        vv, uu = np.meshgrid(np.arange(ty * tile, min(H, (ty + 1) * tile)),
                             np.arange(tx * tile, min(W, (tx + 1) * tile)),
                             indexing="ij")
        u, v = uu.ravel(), vv.ravel()
        uf, vf = u.astype(F32), v.astype(F32)
        g = [dL[k, ch, v, u].astype(F32) for ch in range(3)]
        T = np.ones(u.size, F32)
        live = np.ones(u.size, bool)
        L = e - s
        con = np.zeros((L, u.size), bool)
        clamp = np.zeros((L, u.size), bool)
        AL = np.zeros((L, u.size), F32)
        GG = np.zeros((L, u.size), F32)
        DX = np.zeros((L, u.size), F32)
        DY = np.zeros((L, u.size), F32)
        for i in range(L):
            gi = vals[s + i]
            px, py, A, B, C, o = rec[k, gi, :6]
            b = box[k, gi]
            inb = (u >= b[0]) & (u <= b[1]) & (v >= b[2]) & (v <= b[3])
            dx = px - uf
            dy = py - vf
            pw = F32(-0.5) * (A * dx * dx + C * dy * dy) - B * dx * dy
            G = np.exp(pw)
            og = o * G
            al = np.minimum(amax, og)
            ok = live & inb & (pw <= 0) & (al >= amin)
            Tn = T * (F32(1) - al)
            stop = ok & (Tn < tmin)
            live &= ~stop
            c = ok & ~stop
            con[i], clamp[i] = c, c & (og > amax)
            AL[i], GG[i], DX[i], DY[i] = al, G, dx, dy
            T = np.where(c, Tn, T)
        Tf = T
        Tb = Tf * (bg32[0] * g[0] + bg32[1] * g[1] + bg32[2] * g[2])
        Sg = np.zeros(u.size, F32)
        Tcur = Tf
        for i in range(L - 1, -1, -1):
            gi = vals[s + i]
            px, py, A, B, C, o = rec[k, gi, :6]
            c = con[i]
            if not c.any():
                continue
            alo = np.where(c, AL[i], F32(0))
            rom = F32(1) / (F32(1) - alo)
            Ti = Tcur * rom
            Tnext = Tcur
            Tcur = Ti
            Tw = Tnext if plant == "transmittance" else Ti
            w = alo * Tw
            cg = rgb32[0, gi] * g[0] + rgb32[1, gi] * g[1] + rgb32[2, gi] * g[2]
            diff = cg - Sg
            tb = F32(0) if plant == "background" else Tb * rom
            dal = Ti * diff - tb
            Sg = Sg + alo * diff
            dalm = np.where(c & ~clamp[i], dal, F32(0))
            dpw = dalm * AL[i]
            dx, dy = DX[i], DY[i]
            terms = [-(A * dx + B * dy) * dpw, -(C * dy + B * dx) * dpw,
                     F32(-0.5) * dx * dx * dpw, -dx * dy * dpw,
                     F32(-0.5) * dy * dy * dpw, dalm * GG[i],
                     w * g[0], w * g[1], w * g[2]]
            for q, tq in enumerate(terms):
                parts.append((k, gi, t, q, np.sum(tq, dtype=F32)))
    rng = np.random.default_rng(order_seed)
    order = rng.permutation(len(parts))
    g2d = np.zeros((V, n, 5), F32)
    gop = np.zeros(n, F32)
    grgb = np.zeros((3, n), F32)
    for j in order:
        k, gi, _, q, val = parts[j]
        if q < 5:
            g2d[k, gi, q] = F32(g2d[k, gi, q] + val)
        elif q == 5:
            gop[gi] = F32(gop[gi] + val)
        else:
            grgb[q - 6, gi] = F32(grgb[q - 6, gi] + val)
    return g2d, gop, grgb


def _setup(seed, bg, tile=16, views=2):
    w = _scene(seed, views=views)
    W, H = w.cameras[0].width, w.cameras[0].height
    p = oracle.params64(w.gaussians)
    proj = oracle.project(p, w.cameras, tile, publish=True)
    bins = oracle.bin_sort(proj, tile, W, H)
    fwd = oracle.forward(proj, bins, p["rgb"], W, H, bg)
    rng = np.random.default_rng(seed + 1)
    dL = rng.normal(size=(len(w.cameras), 3, H, W)).astype(np.float32)
    dL *= (fwd["flags"] == 0)[:, None]
    b = oracle.backward(proj, bins, p["rgb"], W, H, dL.astype(np.float64), bg)
    return w, p, proj, bins, dL, b


def _ok(got, ref, mag=None, rtol=1e-3):
    ref = np.asarray(ref, np.float64)
    base = np.maximum(np.abs(ref), 1e-2 * np.abs(ref).max())
    if mag is not None:
        base = np.maximum(base, mag)
    return np.abs(np.asarray(got, np.float64) - ref) <= rtol * base


def _screen_ok(b32, b):
    return (all(_ok(b32["g2d"][..., q], b["g2d"][..., q]).all()
                for q in range(5))
            and _ok(b32["gop"], b["gop"]).all()
            and all(_ok(b32["grgb"][c], b["grgb"][c]).all() for c in range(3)))


def _params_ok(w, p, b32, b):
    ref = oracle.project_bwd(p, w.cameras, b)
    mag = oracle.project_bwd_abs(p, w.cameras, b)
    got = oracle.project_bwd(p, w.cameras, b32)
    return all(_ok(got[k], ref[k], mag[k]).all() for k in ref)


@pytest.mark.parametrize("seed,bg", [(11, (0.0, 0.0, 0.0)),
                                     (12, (0.3, 0.6, 0.1))])
def test_fp32_backward_passes_the_tolerance(seed, bg):
    w, p, proj, bins, dL, b = _setup(seed, bg)
    W, H = w.cameras[0].width, w.cameras[0].height
    assert (np.abs(b["g2d"]) > 0).sum() > 500
    for order in range(3):
        g2d, gop, grgb = fp32_backward(proj, bins, p["rgb"], W, H, dL, bg,
                                       order)
        b32 = dict(g2d=g2d.astype(np.float64), gop=gop.astype(np.float64),
                   grgb=grgb.astype(np.float64))
        assert _screen_ok(b32, b)
        assert _params_ok(w, p, b32, b)


def test_magnitude_is_the_chain_column_by_column():
    """project_bwd_abs equals the sum over views and screen quantities of
    |chain(one-hot input)| x |g2d|, assembled here from one-hot calls of the
    projection backward, and bounds every gradient's absolute value."""
    w, p, proj, bins, dL, b = _setup(13, (0.0, 0.0, 0.0))
    n = p["mean"].shape[1]
    V = len(w.cameras)
    got = oracle.project_bwd_abs(p, w.cameras, b)
    grads = oracle.project_bwd(p, w.cameras, b)
    acc = {k: np.zeros_like(v) for k, v in got.items()}
    z = dict(gop=np.zeros(n), grgb=np.zeros((3, n)))
    for k in range(V):
        for c in range(5):
            g2d = np.zeros((V, n, 5))
            g2d[k, :, c] = np.abs(b["g2d"][k, :, c])
            col = oracle.project_bwd(p, w.cameras, dict(z, g2d=g2d))
            for kind in ("mean", "log_scale", "quat"):
                acc[kind] += np.abs(col[kind])
    o = 1.0 / (1.0 + np.exp(-p["opacity_logit"].reshape(-1)))
    acc["opacity_logit"] = np.abs(b["gop"]) * o * (1 - o)
    acc["rgb"] = np.abs(b["grgb"])
    for kind in got:
        np.testing.assert_allclose(got[kind].reshape(acc[kind].shape),
                                   acc[kind], rtol=1e-12, atol=1e-300)
        assert np.all(got[kind] >= np.abs(grads[kind]) * (1 - 1e-12))
    # Where the terms cancel, the magnitude exceeds |g| (the case the
    # tolerance is for).
    assert np.any(got["log_scale"] > 10 * np.abs(grads["log_scale"]))


def test_sh_magnitudes_bound_and_match_single_terms():
    """colours_bwd_abs bounds colours_bwd's results, and equals their
    absolute values where each is a single term (one view, one channel)."""
    w = synth.tiny_scene(16, n=50, width=40, height=30, f=40.0)
    g = synth.with_sh(w.gaussians, 0, 3, 0.3)
    p = oracle.params64(g)
    cams = w.cameras
    n = g.n
    rng = np.random.default_rng(5)
    gcol = rng.normal(size=(1, 3, n))
    ref = OS.colours_bwd(p, cams, 3, gcol)
    mag = OS.colours_bwd_abs(p, cams, 3, gcol)
    for r, m in zip(ref, mag):
        assert np.all(m >= np.abs(r) * (1 - 1e-12))
    one = np.zeros_like(gcol)
    one[0, 1] = gcol[0, 1]
    r1 = OS.colours_bwd(p, cams, 3, one)
    m1 = OS.colours_bwd_abs(p, cams, 3, one)
    np.testing.assert_allclose(m1[0], np.abs(r1[0]), rtol=1e-12)
    np.testing.assert_allclose(m1[1], np.abs(r1[1]), rtol=1e-12)


@pytest.mark.parametrize("plant", ["background", "transmittance"])
def test_planted_mistakes_fail_the_tolerance(plant):
    """A dropped background term in dL/dalpha, and the colour weight taken
    with the transmittance of the entry behind: each fails the screen-space
    check and the parameter check."""
    bg = (0.3, 0.6, 0.1)
    w, p, proj, bins, dL, b = _setup(14, bg, views=1)
    W, H = w.cameras[0].width, w.cameras[0].height
    g2d, gop, grgb = fp32_backward(proj, bins, p["rgb"], W, H, dL, bg, 0,
                                   plant=plant)
    b32 = dict(g2d=g2d.astype(np.float64), gop=gop.astype(np.float64),
               grgb=grgb.astype(np.float64))
    assert not _screen_ok(b32, b)
    assert not _params_ok(w, p, b32, b)
