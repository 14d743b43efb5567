"""GPU checks of the differentiation capability (torch.autograd.Function),
keyframe insertion, the loss terms and the Adam step against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import (check_grads, gpu_forward, masked_dL, oracle_backward,
                         oracle_forward)
from paper_2504_02437_amd import raster as R

pytestmark = pytest.mark.gpu


def test_autograd_function_matches_oracle_gradient():
    w = synth.tiny_scene(31, n=250, width=64, height=48, f=55.0,
                         log_scale_mu=-2.0)
    print("case autograd", flush=True)
    p64, proj, bins, fwd = oracle_forward(w, 16)
    mask = fwd["flags"][0] == 0
    params = R.ParamBuffer.from_gaussians(w.gaussians)
    rast = R.Rasterizer(w.cameras, params.capacity, R.Settings(tile=16))
    data = params.data.requires_grad_(True)
    rgb, T, nlast = R.Rasterize.apply(data, rast, params)
    wimg = masked_dL(np.random.default_rng(1), mask[None], (1, 3, 48, 64))
    loss = (rgb * torch.from_numpy(wimg).cuda()).sum()
    loss.backward()
    got = data.grad.detach().cpu().numpy()
    ref = oracle_backward(w, p64, proj, bins, wimg)
    check_grads(got, ref, w.gaussians.n)


def test_autograd_refits_an_overflowing_key_capacity():
    """A workspace too small for the keys would truncate the tile lists: the
    autograd forward reads the status word, refits the workspace to the key
    count and renders again, so image and gradient match the oracle."""
    w = synth.tiny_scene(33, n=250, width=64, height=48, f=55.0,
                         log_scale_mu=-2.0)
    print("case autograd overflow refit", flush=True)
    p64, proj, bins, fwd = oracle_forward(w, 16)
    mask = fwd["flags"][0] == 0
    params = R.ParamBuffer.from_gaussians(w.gaussians)
    rast = R.Rasterizer(w.cameras, params.capacity, R.Settings(tile=16),
                        key_capacity=16)
    data = params.data.requires_grad_(True)
    rgb, T, nlast = R.Rasterize.apply(data, rast, params)
    assert rast.status()[0] == 0
    img = rgb.detach().cpu().numpy()[0]
    assert np.abs(img - fwd["img"][0])[:, mask].max() <= 1e-5
    wimg = masked_dL(np.random.default_rng(1), mask[None], (1, 3, 48, 64))
    (rgb * torch.from_numpy(wimg).cuda()).sum().backward()
    check_grads(data.grad.detach().cpu().numpy(),
                oracle_backward(w, p64, proj, bins, wimg), w.gaussians.n)


@pytest.mark.parametrize("change", ["forward", "cameras", "workspace"])
def test_autograd_backward_refuses_stale_state(change):
    """The backward recomputes from the rasterizer's current lists: after
    another forward, a camera change or a workspace rebuild it raises instead
    of returning gradients of another render."""
    w = synth.tiny_scene(34, n=120, width=48, height=40, f=45.0)
    print("case autograd stale", change, flush=True)
    params = R.ParamBuffer.from_gaussians(w.gaussians)
    rast = R.Rasterizer(w.cameras, params.capacity, R.Settings(tile=16))
    data = params.data.requires_grad_(True)
    rgb, _, _ = R.Rasterize.apply(data, rast, params)
    if change == "forward":
        rast.forward(params)
    elif change == "cameras":
        rast.set_cameras(w.cameras)
    else:
        rast.ws = R.Workspace(rast.V, rast.W, rast.H, 16, params.capacity,
                              1 << 16)
        rast.fit_key_capacity(params)
    with pytest.raises(RuntimeError, match="before the backward"):
        rgb.sum().backward()


def test_autograd_function_against_fp32_finite_differences():
    """Central differences of the GPU forward itself (FP32, step 1e-3
    relative).  The alpha and transmittance cut-offs are discontinuities that
    no output reveals (one pixel crossing alpha_min moves the loss by
    ~alpha_min), so this check runs with cut-offs of 1e-30 / 1e-35 where
    every remaining decision (boxes, render boxes, sorted lists, stop
    positions) is checked frozen; the cut-off rules are covered by the oracle's frozen-decision
    differences and the parity tests.  FP32 rounding of the image gives the
    differences an absolute noise of about 5e-4, hence the floor."""
    w = synth.tiny_scene(32, n=60, width=48, height=40, f=45.0,
                         log_scale_mu=-1.6)
    print("case autograd fd", flush=True)
    params = R.ParamBuffer.from_gaussians(w.gaussians)
    rast = R.Rasterizer(w.cameras, params.capacity,
                        R.Settings(tile=16, alpha_min=1e-30, T_min=1e-35))
    wimg = torch.from_numpy(np.random.default_rng(2).normal(
        size=(1, 3, 40, 48)).astype(np.float32)).cuda()
    data = params.data.requires_grad_(True)
    rgb, _, nl0 = R.Rasterize.apply(data, rast, params)
    (rgb * wimg).sum().backward()
    g = data.grad.detach().clone()
    nl0 = nl0.clone()

    def decisions():
        nk = rast.status()[1]
        return (rast.ws.tiles_touched().clone(), rast.ws.ranges().clone(),
                rast.ws.vals_sorted(nk).clone(),
                rast.ws.records()[..., 10:12].clone(),
                rast.ws.render_box().clone())

    rast.forward(params)
    dec0 = decisions()
    rng = np.random.default_rng(3)
    checked = 0
    with torch.no_grad():
        for _ in range(60):
            row = int(rng.integers(0, 14))
            col = int(rng.integers(0, w.gaussians.n))
            x0 = float(params.data[row, col])
            h = 1e-3 * max(1.0, abs(x0))
            vals = []
            ok = True
            for sgn in (1, -1):
                params.data[row, col] = x0 + sgn * h
                out, _, nl = rast.forward(params)
                ok &= bool(torch.equal(nl, nl0))
                d = decisions()
                ok &= all(a.shape == b.shape and bool(torch.equal(a, b))
                          for a, b in zip(d, dec0))
                vals.append(float((out * wimg).double().sum()))
            params.data[row, col] = x0
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            an = float(g[row, col])
            scale = float(g[row].abs().max())
            assert abs(fd - an) <= 2e-2 * max(abs(an), 1e-2 * scale) + 2e-3, \
                (row, col, fd, an)
            checked += 1
    assert checked >= 30


def test_insert_gaussians_matches_oracle():
    rng = np.random.default_rng(41)
    W, H = 96, 64
    R_ = np.array([[0.8, 0.0, 0.6], [0.0, 1.0, 0.0], [-0.6, 0.0, 0.8]],
                  np.float32)
    cam = synth.Camera(R_, np.array([0.3, -0.1, 0.5], np.float32), 80.0, 82.0,
                       (W - 1) / 2, (H - 1) / 2, W, H)
    kT = rng.uniform(0.0, 0.25, size=(H, W)).astype(np.float32)
    img = rng.uniform(size=(3, H, W)).astype(np.float32)
    K = 96
    pts = np.stack([rng.integers(0, W, K), rng.integers(0, H, K),
                    1.0 / rng.uniform(1, 5, K)], 1).astype(np.float32)
    n0, cap = 1000, 1600
    base = synth.tiny_scene(41, n=n0)
    params = R.ParamBuffer.from_gaussians(base.gaussians, capacity=cap)
    m = params.zeros_like()
    v = params.zeros_like()
    m.data.fill_(7.0)
    v.data.fill_(7.0)
    cam_dev = R.cameras_to_device([cam])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nins = torch.zeros(1, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    print("case insert", flush=True)
    R.insert_gaussians(params, m, v, cam_dev, W, H, dev(img), dev(kT),
                       dev(pts), alpha_skip=float(np.float32(0.9)),
                       n_inserted_dev=nins, status_dev=status)
    torch.cuda.synchronize()
    ref = oracle.insert(cam, img, kT.astype(np.float64), pts,
                        alpha_skip=float(np.float32(0.9)))
    cnt = ref["count"]
    assert int(nins.item()) == cnt and params.n() == n0 + cnt
    assert int(status.item()) == 0
    got = params.data[:, n0:n0 + cnt].cpu().numpy()
    np.testing.assert_allclose(got[0:3], ref["mean"], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(got[3:6], ref["log_scale"], rtol=1e-6, atol=1e-7)
    np.testing.assert_array_equal(got[6:10], ref["quat"])
    np.testing.assert_array_equal(got[10], ref["opacity_logit"])
    np.testing.assert_array_equal(got[11:14], ref["rgb"])
    assert torch.all(m.data[:, n0:n0 + cnt] == 0) and torch.all(v.data[:, n0:n0 + cnt] == 0)
    assert torch.all(m.data[:, :n0] == 7.0)
    # Fill to capacity: the overflow is flagged and nothing is written past it.
    big = np.tile(pts, (4, 1))
    kT[:] = 1.0
    R.insert_gaussians(params, m, v, cam_dev, W, H, dev(img), dev(kT),
                       dev(big), n_inserted_dev=nins, status_dev=status)
    torch.cuda.synchronize()
    assert params.n() == cap and int(status.item()) & 2
    assert int(nins.item()) == 9 * 4 * K - sum(
        1 for k in range(4 * K) for p in range(9)
        if not (0 <= int(big[k, 0]) + p % 3 - 1 < W and
                0 <= int(big[k, 1]) + p // 3 - 1 < H))


def test_loss_reg_adam_match_oracle():
    rng = np.random.default_rng(51)
    print("case loss/reg/adam", flush=True)
    img = rng.uniform(size=(2, 3, 30, 40)).astype(np.float32)
    tgt = rng.uniform(size=(2, 3, 30, 40)).astype(np.float32)
    tgt[0, 0, 0, :5] = img[0, 0, 0, :5]          # sign(0) = 0 cases
    dL = torch.empty(2, 3, 30, 40, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    sq = torch.zeros(2, dtype=torch.float64, device="cuda")
    R.loss_l1(torch.from_numpy(img).cuda(), torch.from_numpy(tgt).cuda(), 0.8,
              dL, loss, sq)
    ref_loss, ref_d = oracle.l1(img.astype(np.float64), tgt, 0.8)
    assert float(loss) == pytest.approx(ref_loss, rel=1e-6)
    np.testing.assert_allclose(dL.cpu().numpy(), ref_d, rtol=1e-6)
    np.testing.assert_allclose(
        sq.cpu().numpy(),
        ((img.astype(np.float64) - tgt) ** 2).sum(axis=(1, 2, 3)), rtol=1e-6)
    w = synth.tiny_scene(52, n=500)
    w.gaussians.log_scale[:, :50] = np.log(0.005)       # under the floor
    w.gaussians.log_scale[1, 50:60] = w.gaussians.log_scale[0, 50:60]  # ties
    params = R.ParamBuffer.from_gaussians(w.gaussians, capacity=600)
    grad = params.zeros_like()
    reg = torch.zeros(1, dtype=torch.float64, device="cuda")
    R.planar_reg(params, 2.0, 0.01, grad, reg)
    # The floor is an FP32 argument of the API: give the oracle the same value.
    ref_v, ref_g = oracle.planar_reg(w.gaussians.log_scale.astype(np.float64),
                                     2.0, float(np.float32(0.01)))
    assert float(reg) == pytest.approx(ref_v, rel=1e-12)
    np.testing.assert_allclose(grad.data[3:6, :500].cpu().numpy(), ref_g,
                               rtol=1e-6, atol=0)
    # Adam on the live entries only, two steps.
    g = torch.from_numpy(rng.normal(size=(14, 600)).astype(np.float32)).cuda()
    grad.data.copy_(g)
    m = params.zeros_like()
    v = params.zeros_like()
    p0 = params.data.clone()
    lr = (1e-2, 2e-2, 3e-2, 4e-2, 5e-2)
    for step in (1, 2):
        R.adam(params, grad, m, v, lr, 0.9, 0.999, 1e-15, step)
    torch.cuda.synchronize()
    rows = [0, 0, 0, 1, 1, 1, 2, 2, 2, 2, 3, 4, 4, 4]
    p = p0.cpu().numpy().astype(np.float64)
    gg = g.cpu().numpy().astype(np.float64)
    for r in range(14):
        pr, mr, vr = p[r, :500], np.zeros(500), np.zeros(500)
        for step in (1, 2):
            pr, mr, vr = oracle.adam(pr, gg[r, :500], mr, vr, lr[rows[r]], step)
        np.testing.assert_allclose(params.data[r, :500].cpu().numpy(), pr,
                                   rtol=0, atol=1e-6)
    assert torch.equal(params.data[:, 500:], p0[:, 500:])


def test_bulk_insertion_fills_a_400k_capacity():
    """Keyframe insertions grow a 50k map to exactly its 400k capacity: every
    call before the last inserts all its candidates (fully transparent
    keyframe), the last one reports the overflow and stops at the capacity,
    and the grown map renders."""
    W, H = 1200, 680
    cam = synth.room_camera()
    g = synth.room_gaussians(np.random.default_rng([3, 2]), 50_000)
    cap = 400_000
    params = R.ParamBuffer.from_gaussians(g, capacity=cap)
    cam_dev = R.cameras_to_device([cam])
    kT = torch.ones(H, W, device="cuda")
    img = torch.rand(3, H, W, device="cuda")
    rng = np.random.default_rng(4)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    nins = torch.zeros(1, dtype=torch.int32, device="cuda")
    n, K = 50_000, 7281
    print("case bulk insertion", flush=True)
    while n < cap:
        pts = np.stack([rng.integers(1, W - 1, K), rng.integers(1, H - 1, K),
                        1.0 / rng.uniform(1, 5, K)], 1).astype(np.float32)
        R.insert_gaussians(params, None, None, cam_dev, W, H, img, kT,
                           torch.from_numpy(pts).cuda(), n_inserted_dev=nins,
                           status_dev=status)
        torch.cuda.synchronize()
        assert int(nins.item()) == 9 * K
        full = n + 9 * K > cap
        n = min(n + 9 * K, cap)
        assert params.n() == n
        assert bool(int(status.item()) & 2) == full
    rast = R.Rasterizer([cam], cap, R.Settings(tile=16))
    rast.fit_key_capacity(params)
    rast.forward(params)
    torch.cuda.synchronize()
    assert rast.status()[0] == 0
    T = rast.T.cpu().numpy()
    assert np.isfinite(T).all() and T.min() >= 0.0 and T.max() <= 1.0
