"""Shared helpers of the GPU parity tests: run the HIP path and the CPU oracle
on identical seeded inputs and compare them at the stated tolerances."""
import numpy as np
import torch

import oracle
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


def oracle_forward(w, tile=16, bg=(0.0, 0.0, 0.0), nthreads=8):
    p64 = oracle.params64(w.gaussians)
    W, H = w.cameras[0].width, w.cameras[0].height
    proj = oracle.project(p64, w.cameras, tile, publish=True, nthreads=nthreads)
    bins = oracle.bin_sort(proj, tile, W, H, emit=False)
    fwd = oracle.forward(proj, bins, p64["rgb"], W, H, bg, nthreads=nthreads)
    return p64, proj, bins, fwd


def check_records(rast, proj):
    rec = rast.ws.records().cpu().numpy()
    tt = rast.ws.tiles_touched().cpu().numpy()
    np.testing.assert_array_equal(tt, proj["tiles"])
    vis = tt > 0
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


def check_sort(rast, bins):
    flags, nk = rast.status()
    assert flags == 0
    assert nk == bins["n_keys"]
    ranges = rast.ws.ranges().cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(ranges, bins["ranges"])
    vals = rast.ws.vals_sorted(nk).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(vals, bins["vals"])
    keys = rast.ws.keys_sorted(nk).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(keys, bins["keys"])


def check_forward(rast, fwd, max_flagged=MAX_FLAGGED):
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
    np.testing.assert_array_equal(nl[mask], fwd["nlast"][mask])
    return mask, float(err.max(initial=0.0))


def check_grads(got, ref, n, rtol=GRAD_RTOL, names=None):
    """got: [14][cap] GPU gradients; ref: dict of oracle gradients."""
    worst = {}
    for name, (a, b) in R.ROWS.items():
        if names and name not in names:
            continue
        r = np.asarray(ref[name]).reshape(b - a, -1)
        g = got[a:b, :n]
        scale = np.abs(r).max()
        tol = rtol * np.maximum(np.abs(r), 1e-2 * scale) + 1e-30
        rel = np.abs(g - r) / tol
        worst[name] = float(rel.max(initial=0.0)) * rtol
        bad = np.argwhere(rel > 1.0)
        assert bad.size == 0, (name, bad[:5], g[tuple(bad[0])], r[tuple(bad[0])])
    return worst


def gpu_backward(rast, params, dL):
    grad = params.zeros_like()
    rast.backward(params, torch.from_numpy(np.ascontiguousarray(dL)).cuda(), grad)
    torch.cuda.synchronize()
    return grad.data.cpu().numpy()


def oracle_backward(w, p64, proj, bins, dL, bg=(0.0, 0.0, 0.0), nthreads=8):
    W, H = w.cameras[0].width, w.cameras[0].height
    b = oracle.backward(proj, bins, p64["rgb"], W, H, dL.astype(np.float64), bg,
                        nthreads=nthreads)
    return oracle.project_bwd(p64, w.cameras, b, nthreads=nthreads)


def masked_dL(rng, mask, shape, scale=1.0):
    dL = (rng.normal(size=shape) * scale).astype(np.float32)
    dL *= mask[:, None].astype(np.float32)
    return dL
