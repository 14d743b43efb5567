"""CPU FP64 oracle of the differentiable tile rasterizer.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  It shares no code with the GPU
library, and the GPU library never calls it.

This module marshals numpy arrays into ``liboracle.so`` (plain C, FP64; see
``gsoracle.c`` for the passages of the paper each function follows).  All
parameters are widened exactly from FP32 to FP64 before the call.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

# Thresholds the rasterizer uses, as FP32 values widened to FP64.
ALPHA_MIN = float(np.float32(1.0) / np.float32(255.0))
T_MIN = float(np.float32(1e-4))
ALPHA_MAX = float(np.float32(0.99))
# Decision codes of a (pixel, entry) pair in the forward walk.
DEC_SKIP, DEC_ADMIT, DEC_CLAMP, DEC_STOP = 0, 1, 2, 3
REC_FIELDS = ("px", "py", "A", "B", "C", "opacity", "depth", "radius")

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)
_u32 = C.POINTER(C.c_uint32)
_u64 = C.POINTER(C.c_uint64)
_u8 = C.POINTER(C.c_uint8)
_i64 = C.POINTER(C.c_int64)


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = C.CDLL(os.environ.get("ORACLE_LIB_OVERRIDE", _build.LIB))
        L.or_project.restype = C.c_int
        L.or_project.argtypes = [C.c_int, _d, _d, _d, _d, _d, C.c_int, C.c_int,
                                 _d, _d, _i32, _i32, C.c_int]
        L.or_bin_sort.restype = C.c_int64
        L.or_bin_sort.argtypes = [C.c_int, C.c_int, _i32, _i32, _d, C.c_int,
                                  C.c_int, C.c_int, _u64, _u32, _u64, _u32,
                                  C.c_int64, _u32, C.c_int]
        L.or_forward.restype = C.c_int
        L.or_forward.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                 _d, _i32, _d, C.c_int, _u32, _u32, _d,
                                 C.c_double,
                                 C.c_double, C.c_double, _d, _d, _i32, _u8, _d,
                                 _d, _i64, _u8, C.c_int, C.c_int, _i32, _d, _d,
                                 _d, C.c_int]
        L.or_backward.restype = C.c_int
        L.or_backward.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                  _d, _i32, _d, C.c_int, _u32, _u32, _d,
                                  C.c_double,
                                  C.c_double, C.c_double, _d, _u8, C.c_int,
                                  C.c_int, _d, _d, _d, C.c_int]
        L.or_project_bwd.restype = C.c_int
        L.or_project_bwd.argtypes = [C.c_int, C.c_int, _d, _d, _d, _d, _d, _d,
                                     _d, _d, _d, _d, _d, _d, _d, C.c_int]
        L.or_project_bwd_abs.restype = C.c_int
        L.or_project_bwd_abs.argtypes = [C.c_int, C.c_int, _d, _d, _d, _d,
                                         _d, _d, _d, _d, _d, _d, _d, _d, _d,
                                         C.c_int]
        L.or_pixel_walk.restype = C.c_int
        L.or_pixel_walk.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                    _d, _i32, _u32, _u32, C.c_double,
                                    C.c_double, C.c_double, C.c_int, _i64,
                                    C.c_int, _i32, _d, _u8, _i32]
        L.or_admit_extent.restype = None
        L.or_admit_extent.argtypes = [C.c_int, C.c_int, _d, _i32, C.c_double,
                                      _i32, C.c_int]
        L.or_l1.restype = C.c_double
        L.or_l1.argtypes = [C.c_int, C.c_int, C.c_int, _d, _d, C.c_double, _d]
        L.or_planar_reg.restype = C.c_double
        L.or_planar_reg.argtypes = [C.c_int, _d, C.c_double, C.c_double, _d]
        L.or_adam.restype = None
        L.or_adam.argtypes = [C.c_int64, _d, _d, _d, _d, C.c_double,
                              C.c_double, C.c_double, C.c_double, C.c_int]
        L.or_insert.restype = C.c_int
        L.or_insert.argtypes = [_d, _d, _d, _d, C.c_int, C.c_double, C.c_int,
                                C.c_int, _d, _d, _d, _d, _d, _i32, _d,
                                C.c_double]
        L.or_nearest.restype = None
        L.or_nearest.argtypes = [_d, _d, C.c_int, C.c_int, _d, C.c_int, _d,
                                 C.c_int]
        _LIB = L
    return _LIB


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32), dtype=np.float64)


def cam_array(cam) -> np.ndarray:
    """Camera as 19 doubles (R[9], t[3], fx, fy, cx, cy, near, W, H); every
    real value is the FP32 value the GPU sees, widened exactly."""
    f = lambda x: float(np.float32(x))
    return np.array(list(np.asarray(cam.R, np.float32).astype(np.float64).ravel())
                    + list(np.asarray(cam.t, np.float32).astype(np.float64))
                    + [f(cam.fx), f(cam.fy), f(cam.cx), f(cam.cy), f(cam.near),
                       float(cam.width), float(cam.height)], dtype=np.float64)


def params64(g):
    """FP64 copies of a Gaussians set's planar arrays."""
    out = dict(mean=_f64(g.mean), log_scale=_f64(g.log_scale),
               quat=_f64(g.quat), opacity_logit=_f64(g.opacity_logit),
               rgb=_f64(g.rgb))
    if getattr(g, "sh", None) is not None:
        out["sh"] = _f64(g.sh)
    return out


def project(p, cams, tile=16, publish=True, nthreads=1):
    """Projects every Gaussian into every camera (Eq. 1-2).

    ``p`` is a dict from :func:`params64` (or any dict of FP64 planar arrays).
    Returns rec [V][n][8], cov [V][n][3], box [V][n][4] int32, tiles [V][n].
    """
    L = lib()
    n = p["mean"].shape[1]
    V = len(cams)
    rec = np.zeros((V, n, 8))
    cov = np.zeros((V, n, 3))
    box = np.zeros((V, n, 4), np.int32)
    tiles = np.zeros((V, n), np.int32)
    for k, cam in enumerate(cams):
        ca = cam_array(cam)
        L.or_project(n, _p(p["mean"], _d), _p(p["log_scale"], _d),
                     _p(p["quat"], _d), _p(p["opacity_logit"], _d), _p(ca, _d),
                     tile, 1 if publish else 0, _p(rec[k], _d), _p(cov[k], _d),
                     _p(box[k], _i32), _p(tiles[k], _i32), nthreads)
    return dict(rec=rec, cov=cov, box=box, tiles=tiles)


def bin_sort(proj, tile, W, H, cap=None, emit=True, nthreads=1):
    """Duplicated (tile, depth) keys, stable sort and tile ranges (views
    emitted and sorted on nthreads threads; the result does not depend on
    it)."""
    L = lib()
    V, n = proj["tiles"].shape
    total = int(proj["tiles"].astype(np.int64).sum())
    cap = total if cap is None else cap
    Tx, Ty = (W + tile - 1) // tile, (H + tile - 1) // tile
    keys_emit = np.zeros(max(total, 1), np.uint64) if emit else None
    vals_emit = np.zeros(max(total, 1), np.uint32) if emit else None
    keys = np.zeros(max(total, 1), np.uint64)
    vals = np.zeros(max(total, 1), np.uint32)
    ranges = np.zeros((V * Tx * Ty, 2), np.uint32)
    nk = L.or_bin_sort(V, n, _p(proj["box"], _i32), _p(proj["tiles"], _i32),
                       _p(proj["rec"], _d), tile, W, H, _p(keys_emit, _u64),
                       _p(vals_emit, _u32), _p(keys, _u64), _p(vals, _u32),
                       cap, _p(ranges, _u32), nthreads)
    if nk < 0:
        raise OverflowError("key capacity exceeded")
    out = dict(keys=keys[:nk], vals=vals[:nk], ranges=ranges, n_keys=int(nk),
               Tx=Tx, Ty=Ty, tile=tile)
    if emit:
        out["keys_emit"] = keys_emit[:nk]
        out["vals_emit"] = vals_emit[:nk]
    return out


def _colour_layout(rgb, V, n):
    if rgb.shape == (3, n):
        return 0
    if rgb.shape == (V, 3, n):
        return 1
    raise ValueError(f"colours must be [3][{n}] or [{V}][3][{n}]")


def forward(proj, bins, rgb, W, H, bg=(0.0, 0.0, 0.0), alpha_min=ALPHA_MIN,
            T_min=T_MIN, alpha_max=ALPHA_MAX, dec=None, dec_mode=0,
            nthreads=1):
    """Front-to-back compositing (Eq. 3) over each tile's sorted list; also
    the dominant Gaussian of every pixel (Eq. 8): "dom" (index, -1 if none),
    "w1" its blend weight, "w2" the runner-up weight, "werr" a relative FP32
    error bound of the weights.  rgb is [3][n], or [V][3][n] per view (the
    view-dependent colours of ``oracle.sh.colours``)."""
    L = lib()
    V, n = proj["tiles"].shape
    img = np.zeros((V, 3, H, W))
    T = np.zeros((V, H, W))
    nlast = np.zeros((V, H, W), np.int32)
    flags = np.zeros((V, H, W), np.uint8)
    errb = np.zeros((V, H, W))
    terr = np.zeros((V, H, W))
    cnt = np.zeros(4, np.int64)
    dom = np.zeros((V, H, W), np.int32)
    w1 = np.zeros((V, H, W))
    w2 = np.zeros((V, H, W))
    werr = np.zeros((V, H, W))
    bgv = np.asarray(bg, np.float64)
    Ld = 0 if dec is None else dec.shape[-1]
    rgb = np.ascontiguousarray(rgb, np.float64)
    per_view = _colour_layout(rgb, V, n)
    vals = bins["vals"] if bins["n_keys"] else np.zeros(1, np.uint32)
    rc = L.or_forward(V, W, H, bins["tile"], n, _p(proj["rec"], _d),
                      _p(proj["box"], _i32), _p(rgb, _d), per_view,
                      _p(vals, _u32),
                      _p(bins["ranges"], _u32), _p(bgv, _d), alpha_min, T_min,
                      alpha_max, _p(img, _d), _p(T, _d), _p(nlast, _i32),
                      _p(flags, _u8), _p(errb, _d), _p(terr, _d), _p(cnt, _i64),
                      _p(dec, _u8), Ld, dec_mode, _p(dom, _i32), _p(w1, _d),
                      _p(w2, _d), _p(werr, _d), nthreads)
    if rc != 0:
        raise ValueError("decision buffer too short")
    return dict(img=img, T=T, nlast=nlast, flags=flags, errb=errb, terr=terr,
                dom=dom, w1=w1, w2=w2, werr=werr,
                counters=dict(examined=int(cnt[0]), inbox=int(cnt[1]),
                              contributing=int(cnt[2]), revisit=int(cnt[3])))


def pixel_walk(proj, bins, W, H, pix, alpha_min=ALPHA_MIN, T_min=T_MIN,
               alpha_max=ALPHA_MAX):
    """The forward walk at the listed pixels (flat indices (k H + v) W + u):
    for each, the in-box entries of its tile list up to the stop, as arrays
    (gaussian [m][L], weight alpha T [m][L] (0 if not contributing),
    decision code [m][L], count [m])."""
    L = lib()
    V, n = proj["tiles"].shape
    pix = np.ascontiguousarray(pix, np.int64)
    r = bins["ranges"].astype(np.int64)
    maxw = max(1, int((r[:, 1] - r[:, 0]).max()))
    m = len(pix)
    g = np.zeros((m, maxw), np.int32)
    wt = np.zeros((m, maxw))
    code = np.zeros((m, maxw), np.uint8)
    cnt = np.zeros(m, np.int32)
    vals = bins["vals"] if bins["n_keys"] else np.zeros(1, np.uint32)
    rc = L.or_pixel_walk(V, W, H, bins["tile"], n, _p(proj["rec"], _d),
                         _p(proj["box"], _i32), _p(vals, _u32),
                         _p(bins["ranges"], _u32), alpha_min, T_min, alpha_max,
                         m, _p(pix, _i64), maxw, _p(g, _i32), _p(wt, _d),
                         _p(code, _u8), _p(cnt, _i32))
    if rc != 0:
        raise ValueError("pixel outside the views, or a walk longer than the "
                         "longest tile list")
    return g, wt, code, cnt


def admit_extent(proj, alpha_min=ALPHA_MIN, nthreads=1):
    """Per (view, Gaussian), the pixel rectangle (u_lo, u_hi, v_lo, v_hi)
    of its box outside which no FP32 evaluation of alpha can reach
    alpha_min; (0, -1, 0, -1) when none can."""
    L = lib()
    V, n = proj["tiles"].shape
    rect = np.zeros((V, n, 4), np.int32)
    L.or_admit_extent(V, n, _p(proj["rec"], _d), _p(proj["box"], _i32),
                      alpha_min, _p(rect, _i32), nthreads)
    return rect


def decision_buffer(bins, V, W, H):
    r = bins["ranges"].astype(np.int64)
    L = max(1, int((r[:, 1] - r[:, 0]).max()))
    return np.zeros((V, H, W, L), np.uint8)


def backward(proj, bins, rgb, W, H, dimg, bg=(0.0, 0.0, 0.0),
             alpha_min=ALPHA_MIN, T_min=T_MIN, alpha_max=ALPHA_MAX, dec=None,
             dec_mode=0, nthreads=1):
    """Exact derivative of the compositing with the decision set fixed.
    Returns g2d [V][n][5] (px, py, A, B, C), gop [n] and grgb: [3][n]
    summed over the views, or [V][3][n] when the colours are per view."""
    L = lib()
    V, n = proj["tiles"].shape
    g2d = np.zeros((V, n, 5))
    gop = np.zeros(n)
    bgv = np.asarray(bg, np.float64)
    dimg = np.ascontiguousarray(dimg, np.float64)
    rgb = np.ascontiguousarray(rgb, np.float64)
    per_view = _colour_layout(rgb, V, n)
    grgb = np.zeros(rgb.shape)
    Ld = 0 if dec is None else dec.shape[-1]
    vals = bins["vals"] if bins["n_keys"] else np.zeros(1, np.uint32)
    rc = L.or_backward(V, W, H, bins["tile"], n, _p(proj["rec"], _d),
                       _p(proj["box"], _i32), _p(rgb, _d), per_view,
                       _p(vals, _u32),
                       _p(bins["ranges"], _u32), _p(bgv, _d), alpha_min, T_min,
                       alpha_max, _p(dimg, _d), _p(dec, _u8), Ld, dec_mode,
                       _p(g2d, _d), _p(gop, _d), _p(grgb, _d), nthreads)
    if rc != 0:
        raise ValueError("decision buffer too short")
    return dict(g2d=g2d, gop=gop, grgb=grgb)


def project_bwd(p, cams, bwd, nthreads=1):
    """Chain rule from the screen-space gradients to the 14 parameter rows."""
    L = lib()
    n = p["mean"].shape[1]
    camd = np.stack([cam_array(c) for c in cams])
    out = dict(mean=np.zeros((3, n)), log_scale=np.zeros((3, n)),
               quat=np.zeros((4, n)), opacity_logit=np.zeros(n),
               rgb=np.zeros((3, n)))
    L.or_project_bwd(len(cams), n, _p(p["mean"], _d), _p(p["log_scale"], _d),
                     _p(p["quat"], _d), _p(p["opacity_logit"], _d),
                     _p(camd, _d), _p(bwd["g2d"], _d), _p(bwd["gop"], _d),
                     _p(bwd["grgb"], _d), _p(out["mean"], _d),
                     _p(out["log_scale"], _d), _p(out["quat"], _d),
                     _p(out["opacity_logit"], _d), _p(out["rgb"], _d), nthreads)
    return out


def project_bwd_abs(p, cams, bwd, nthreads=1):
    """Magnitude of the chain-rule terms behind each parameter gradient: the
    projection backward with every partial derivative and every screen-space
    gradient taken by absolute value (sum over views and screen quantities
    of |d out / d g2d| |g2d|; |gop| o (1 - o); |grgb|).  It bounds the
    gradient's absolute value, and an error of relative size e in the
    screen-space gradients moves the gradient by at most e times it."""
    L = lib()
    n = p["mean"].shape[1]
    camd = np.stack([cam_array(c) for c in cams])
    out = dict(mean=np.zeros((3, n)), log_scale=np.zeros((3, n)),
               quat=np.zeros((4, n)), opacity_logit=np.zeros(n),
               rgb=np.zeros((3, n)))
    x2d = np.ascontiguousarray(np.abs(bwd["g2d"]), np.float64)
    xop = np.ascontiguousarray(np.abs(bwd["gop"]), np.float64)
    xrgb = np.ascontiguousarray(np.abs(bwd["grgb"]), np.float64)
    if xrgb.shape != (3, n):
        raise ValueError("per-view colour magnitudes go through oracle.sh")
    L.or_project_bwd_abs(len(cams), n, _p(p["mean"], _d),
                         _p(p["log_scale"], _d), _p(p["quat"], _d),
                         _p(p["opacity_logit"], _d), _p(camd, _d),
                         _p(x2d, _d), _p(xop, _d), _p(xrgb, _d),
                         _p(out["mean"], _d), _p(out["log_scale"], _d),
                         _p(out["quat"], _d), _p(out["opacity_logit"], _d),
                         _p(out["rgb"], _d), nthreads)
    return out


def l1(img, target, lam=1.0):
    """Sum over views of lam * mean |img - target| and its gradient."""
    L = lib()
    img = np.ascontiguousarray(img, np.float64)
    tgt = _f64(target)
    V, _, H, W = img.shape
    dimg = np.zeros_like(img)
    loss = L.or_l1(V, H, W, _p(img, _d), _p(tgt, _d), lam, _p(dimg, _d))
    return loss, dimg


def planar_reg(log_scale, lam=1.0, floor=0.01):
    """lam * mean_g max(floor, min_j exp(l_gj)) and its gradient."""
    L = lib()
    ls = np.ascontiguousarray(log_scale, np.float64)
    g = np.zeros_like(ls)
    v = L.or_planar_reg(ls.shape[1], _p(ls, _d), lam, floor, _p(g, _d))
    return v, g


def adam(p, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-15):
    L = lib()
    p = np.ascontiguousarray(p, np.float64).copy()
    m = np.ascontiguousarray(m, np.float64).copy()
    v = np.ascontiguousarray(v, np.float64).copy()
    g = np.ascontiguousarray(g, np.float64)
    L.or_adam(p.size, _p(p, _d), _p(g, _d), _p(m, _d), _p(v, _d), lr, b1, b2,
              eps, step)
    return p, m, v


def nearest(cam, pts_uvd, means, centre_only=False, nthreads=1):
    """Squared distance from each insertion candidate's back-projected point
    to the nearest existing mean (Eq. 7); -1 outside the image or for d <= 0,
    inf for an empty map.  means: [3][n]."""
    L = lib()
    K = pts_uvd.shape[0]
    per = 1 if centre_only else 9
    means = _f64(means).reshape(3, -1)
    out = np.zeros(K * per)
    L.or_nearest(_p(cam_array(cam), _d), _p(_f64(pts_uvd), _d), K,
                 1 if centre_only else 0, _p(means, _d), means.shape[1],
                 _p(out, _d), nthreads)
    return out


def insert(cam, kf_rgb, kf_T, pts_uvd, alpha_skip=0.9, centre_only=False,
           cap=None, cand_d2=None, tau=None):
    """Back-projected, masked insertion of patch pixels (Eq. 6), with the
    accumulated-alpha mask, or with the distance test of Eq. 7 (a candidate
    is kept when cand_d2 > tau^2) when cand_d2 is given."""
    L = lib()
    K = pts_uvd.shape[0]
    cap = 9 * K if cap is None else cap
    ca = cam_array(cam)
    rgb = _f64(kf_rgb)
    T = np.ascontiguousarray(kf_T if kf_T is not None else np.zeros((1,)),
                             np.float64)
    pts = _f64(pts_uvd)
    out = dict(mean=np.zeros((3, cap)), log_scale=np.zeros((3, cap)),
               quat=np.zeros((4, cap)), opacity_logit=np.zeros(cap),
               rgb=np.zeros((3, cap)))
    src = np.zeros(cap, np.int32)
    # The distance threshold is an FP32 setting: square its FP32 value.
    d2 = None if cand_d2 is None else np.ascontiguousarray(cand_d2, np.float64)
    tau2 = 0.0 if tau is None else float(np.float32(tau)) ** 2
    cnt = L.or_insert(_p(ca, _d), _p(rgb, _d), _p(T, _d), _p(pts, _d), K,
                      alpha_skip, 1 if centre_only else 0, cap,
                      _p(out["mean"], _d), _p(out["log_scale"], _d),
                      _p(out["quat"], _d), _p(out["opacity_logit"], _d),
                      _p(out["rgb"], _d), _p(src, _i32),
                      _p(d2, _d), tau2)
    m = min(cnt, cap)
    return dict(count=int(cnt), src=src[:m],
                **{k: v[..., :m] for k, v in out.items()})


def render(p, cams, tile=16, bg=(0.0, 0.0, 0.0), publish=True, nthreads=1):
    """Projection, binning and forward compositing in one call."""
    W, H = cams[0].width, cams[0].height
    proj = project(p, cams, tile, publish, nthreads)
    bins = bin_sort(proj, tile, W, H, emit=False)
    fwd = forward(proj, bins, p["rgb"], W, H, bg, nthreads=nthreads)
    return proj, bins, fwd
