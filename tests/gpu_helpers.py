"""Shared helpers of the GPU parity tests: run the HIP path and the CPU oracle
on identical seeded inputs and compare them at the stated tolerances."""
import numpy as np
import torch

import oracle
from oracle import sh as OS
from paper_2504_02437_amd import raster as R

IMG_TOL = 1e-5       # absolute, per pixel and channel (FP32 vs FP64)
GRAD_RTOL = 1e-3     # relative, with a floor of 1e-2 * max |g| per tensor
MAX_FLAGGED = 1e-3   # fraction of pixels whose decisions are FP32-ambiguous


def gpu_forward(w, tile=16, batch=256, bg=(0.0, 0.0, 0.0), emit_keys=True,
                key_capacity=None, params=None, threads=0, full_box=False):
    if params is None:
        params = R.ParamBuffer.from_gaussians(w.gaussians)
    rast = R.Rasterizer(w.cameras, params.capacity,
                        R.Settings(tile=tile, lds_batch=batch, bg=bg,
                                   emit_keys=emit_keys, block_threads=threads,
                                   full_box=full_box),
                        key_capacity=key_capacity)
    rast.forward(params)
    torch.cuda.synchronize()
    return params, rast


def oracle_colours(w, p64):
    """The oracle's colours: rgb [3][n], or [V][3][n] per view when the
    Gaussians carry view-dependent colour coefficients."""
    D = w.gaussians.sh_degree
    return p64["rgb"] if D == 0 else OS.colours(p64, w.cameras, D)[0]


def oracle_forward(w, tile=16, bg=(0.0, 0.0, 0.0), nthreads=8):
    p64 = oracle.params64(w.gaussians)
    W, H = w.cameras[0].width, w.cameras[0].height
    proj = oracle.project(p64, w.cameras, tile, publish=True, nthreads=nthreads)
    bins = oracle.bin_sort(proj, tile, W, H, emit=False, nthreads=nthreads)
    fwd = oracle.forward(proj, bins, oracle_colours(w, p64), W, H, bg,
                         nthreads=nthreads)
    return p64, proj, bins, fwd


def _unpack(rb):
    return np.stack([rb[..., 0] & 0xFFFF, rb[..., 0] >> 16,
                     rb[..., 1] & 0xFFFF, rb[..., 1] >> 16], -1)


def check_records(rast, proj):
    """Records and integer boxes bit-exact.  Tile counts equal the oracle's
    with whole-box binning; with render boxes a Gaussian touches a subset of
    its tiles."""
    rec = rast.ws.records().cpu().numpy()
    tt = rast.ws.tiles_touched().cpu().numpy()
    if rast.settings.full_box:
        np.testing.assert_array_equal(tt, proj["tiles"])
    else:
        assert np.all(tt <= proj["tiles"]) and np.all((tt > 0) <= (proj["tiles"] > 0))
    vis = proj["tiles"] > 0
    ref = proj["rec"].astype(np.float32)
    got = {"px": rec[..., 0], "py": rec[..., 1], "A": rec[..., 2],
           "B": rec[..., 3], "C": rec[..., 4], "opacity": rec[..., 5],
           "depth": rec[..., 9]}
    for i, name in enumerate(oracle.REC_FIELDS[:7]):
        a = got[name][vis].view(np.uint32)
        b = ref[..., i][vis].view(np.uint32)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, (name, bad[:5], got[name][vis][bad[:5]],
                               ref[..., i][vis][bad[:5]])
    bu = rec[..., 10].view(np.int32)
    bv = rec[..., 11].view(np.int32)
    box = np.stack([bu & 0xFFFF, bu >> 16, bv & 0xFFFF, bv >> 16], -1)
    np.testing.assert_array_equal(box[vis], proj["box"][vis])


def render_box_lists(rast, bins):
    """The oracle's tile lists restricted to the entries whose GPU render box
    meets the tile (order kept): (keys, vals, ranges)."""
    T = rast.settings.tile
    Tx, Ty = rast.ws.tiles_x, rast.ws.tiles_y
    keys, vals = bins["keys"], bins["vals"]
    tile = (keys >> np.uint64(32)).astype(np.int64)
    k = tile // (Tx * Ty)
    rem = tile % (Tx * Ty)
    ty, tx = rem // Tx, rem % Tx
    rb = _unpack(rast.ws.render_box().cpu().numpy())[k, vals.astype(np.int64)]
    meet = ((rb[:, 0] <= tx * T + T - 1) & (rb[:, 1] >= tx * T) &
            (rb[:, 2] <= ty * T + T - 1) & (rb[:, 3] >= ty * T))
    n_tiles = bins["ranges"].shape[0]
    counts = np.bincount(tile[meet], minlength=n_tiles)
    ends = np.cumsum(counts)
    ranges = np.stack([ends - counts, ends], -1).astype(np.uint32)
    return keys[meet], vals[meet], ranges


def check_sort(rast, bins):
    """Ranges, keys and values bit-exact: equal to the oracle's with
    whole-box binning, and to the oracle's lists restricted by the render
    boxes otherwise."""
    flags, nk = rast.status()
    assert flags == 0
    if rast.settings.full_box:
        keys, vals, ranges = bins["keys"], bins["vals"], bins["ranges"]
    else:
        keys, vals, ranges = render_box_lists(rast, bins)
    assert nk == len(vals)
    np.testing.assert_array_equal(rast.ws.ranges().cpu().numpy().view(np.uint32),
                                  ranges)
    np.testing.assert_array_equal(rast.ws.vals_sorted(nk).cpu().numpy().view(np.uint32),
                                  vals)
    if rast.settings.emit_keys:
        np.testing.assert_array_equal(
            rast.ws.keys_sorted(nk).cpu().numpy().view(np.uint64), keys)


def last_contributors(nlast, ranges, vals, T, Tx, Ty):
    """Gaussian index of each pixel's last contributing entry (-1 if none)."""
    V, H, W = nlast.shape
    kk, vv, uu = np.meshgrid(np.arange(V), np.arange(H), np.arange(W),
                             indexing="ij")
    tile = (kk * Ty + vv // T) * Tx + uu // T
    start = ranges[tile, 0].astype(np.int64)
    pos = start + nlast.astype(np.int64) - 1
    out = np.full(nlast.shape, -1, np.int64)
    has = nlast > 0
    out[has] = vals[pos[has]]
    return out


def check_forward(rast, fwd, bins=None, max_flagged=MAX_FLAGGED):
    mask = fwd["flags"] == 0
    assert 1.0 - mask.mean() <= max_flagged, 1.0 - mask.mean()
    img = rast.rgb.cpu().numpy()
    T = rast.T.cpu().numpy()
    nl = rast.nlast.cpu().numpy()
    m3 = np.broadcast_to(mask[:, None], img.shape)
    err = np.abs(img - fwd["img"])[m3]
    assert err.max(initial=0.0) <= IMG_TOL, err.max()
    terr = np.abs(T - fwd["T"])[mask]
    assert terr.max(initial=0.0) <= IMG_TOL, terr.max()
    if rast.settings.full_box:
        np.testing.assert_array_equal(nl[mask], fwd["nlast"][mask])
    elif bins is not None:
        # n_last indexes shorter lists: compare the identity of each pixel's
        # last contributing Gaussian instead.
        _, nk = rast.status()
        tsz, Tx, Ty = rast.settings.tile, rast.ws.tiles_x, rast.ws.tiles_y
        got = last_contributors(nl, rast.ws.ranges().cpu().numpy().view(np.uint32),
                                rast.ws.vals_sorted(nk).cpu().numpy().view(np.uint32),
                                tsz, Tx, Ty)
        ref = last_contributors(fwd["nlast"], bins["ranges"], bins["vals"],
                                tsz, Tx, Ty)
        np.testing.assert_array_equal(got[mask], ref[mask])
    return mask, float(err.max(initial=0.0))


def check_grads(got, ref, n, rtol=GRAD_RTOL, names=None, mag=None):
    """got: [14 + coefficient rows][cap] GPU gradients; ref: dict of oracle
    gradients (with "sh" [K-1][3][n] for view-dependent colour).  Every
    element within rtol of max(|ref|, 1e-2 of its kind's largest |ref|, m),
    where m (mag, the same rows as ref; oracle.project_bwd_abs or
    oracle.sh.chain_abs) is the sum of the absolute values of the chain-rule
    terms the element adds up: where large terms cancel, rounding of the FP32
    screen-space sums of relative size e moves the result by up to e m.
    Without mag the bar is plain (as on small scenes).  Returns the worst
    relative error per kind and how many elements needed the m term."""
    worst = {}
    relaxed = 0
    rows = dict(R.ROWS)
    if "sh" in ref:
        rows["sh"] = (14, got.shape[0])
    for name, (a, b) in rows.items():
        if names and name not in names:
            continue
        r = np.asarray(ref[name]).reshape(b - a, -1)
        g = got[a:b, :n]
        scale = np.abs(r).max()
        base = np.maximum(np.abs(r), 1e-2 * scale)
        err = np.abs(g - r)
        if mag is not None:
            m = np.asarray(mag[name]).reshape(b - a, -1)
            relaxed += int(((err > rtol * base) & (err <= rtol * m)).sum())
            base = np.maximum(base, m)
        tol = rtol * base + 1e-30
        rel = err / tol
        worst[name] = float(rel.max(initial=0.0)) * rtol
        bad = np.argwhere(rel > 1.0)
        assert bad.size == 0, (name, bad[:5], g[tuple(bad[0])],
                               r[tuple(bad[0])])
    worst["elements_within_magnitude_only"] = relaxed
    return worst


def _check_rows(name, got, ref, rtol):
    """Per element within rtol of max(|ref|, 1e-2 of the row group's largest
    |ref|)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    tol = rtol * np.maximum(np.abs(ref), 1e-2 * np.abs(ref).max()) + 1e-30
    rel = np.abs(got - ref) / tol
    bad = np.argwhere(rel > 1.0)
    assert bad.size == 0, (name, bad[:5], got[tuple(bad[0])], ref[tuple(bad[0])])
    return float(rel.max(initial=0.0)) * rtol


def check_screen_grads(rast, grad, b, n, rtol=GRAD_RTOL):
    """The compositing backward's own sums, read from the workspace before the
    projection backward consumes them: dL/d(px, py, A, B, C) per view and
    quantity, dL/d opacity summed over the views, and dL/d colour (the
    caller's colour rows, or per view with view-dependent colour), each per
    element against the oracle's."""
    g2d = rast.ws.grad2d().cpu().numpy()[:, :, :n]          # [V][5][n]
    worst = {}
    for q, name in enumerate(("px", "py", "A", "B", "C")):
        worst[name] = _check_rows(name, g2d[:, q], b["g2d"][:, :, q], rtol)
    worst["opacity"] = _check_rows(
        "opacity", rast.ws.grad_opacity().cpu().numpy()[:n], b["gop"], rtol)
    if b["grgb"].ndim == 3:
        col = rast.ws.grad_colour().cpu().numpy()[:, :, :n]
    else:
        a, z = R.ROWS["rgb"]
        col = grad.data[a:z, :n].cpu().numpy()
    for c in range(3):
        worst[f"colour{c}"] = _check_rows(f"colour{c}", col[..., c, :],
                                          b["grgb"][..., c, :], rtol)
    return worst


def gpu_backward(rast, params, dL):
    grad = params.zeros_like()
    rast.backward(params, torch.from_numpy(np.ascontiguousarray(dL)).cuda(), grad)
    torch.cuda.synchronize()
    return grad.data.cpu().numpy()


def gpu_backward_screen(rast, params, dL=None, target=None, lam=1.0,
                        check=None):
    """The compositing backward (fed with dL, or with the L1 term fused in
    against target: gs_render_bwd_l1), then the projection backward.  check
    (optional) is called with the gradient buffer between the two, while the
    workspace still holds the screen-space sums.  Returns (parameter
    gradients, check's result, fused loss or None)."""
    grad = params.zeros_like()
    S = rast.settings
    loss = None
    if target is None:
        R.render_bwd_pixels(rast.ws, params, S,
                            torch.from_numpy(np.ascontiguousarray(dL)).cuda(),
                            rast.T, rast.nlast, grad)
    else:
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        R.render_bwd_l1(rast.ws, params, S, rast.rgb, target, lam, rast.T,
                        rast.nlast, grad, loss)
    torch.cuda.synchronize()
    screen = check(grad) if check else None
    R.project_bwd(rast.ws, params, rast.cams_dev, grad)
    torch.cuda.synchronize()
    return (grad.data.cpu().numpy(), screen,
            None if loss is None else float(loss))


def oracle_backward(w, p64, proj, bins, dL, bg=(0.0, 0.0, 0.0), nthreads=8,
                    full=False):
    """Oracle parameter gradients; with full=True also the chain magnitudes
    (see check_grads) and the screen-space sums: (ref, mag, screen)."""
    W, H = w.cameras[0].width, w.cameras[0].height
    b = oracle.backward(proj, bins, oracle_colours(w, p64), W, H,
                        dL.astype(np.float64), bg, nthreads=nthreads)
    D = w.gaussians.sh_degree
    if D:
        ref = OS.chain(p64, w.cameras, D, b, nthreads=nthreads)
        mag = OS.chain_abs(p64, w.cameras, D, b, nthreads=nthreads) if full else None
    else:
        ref = oracle.project_bwd(p64, w.cameras, b, nthreads=nthreads)
        mag = oracle.project_bwd_abs(p64, w.cameras, b, nthreads=nthreads) if full else None
    if full:
        return ref, mag, b
    return ref


def masked_dL(rng, mask, shape, scale=1.0):
    dL = (rng.normal(size=shape) * scale).astype(np.float32)
    dL *= mask[:, None].astype(np.float32)
    return dL
