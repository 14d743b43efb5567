"""GPU learned-initialisation kernels vs the FP64 oracle: kNN features,
the BF16-MFMA forward and backward, the MSE gradient, Adam, training and
MLP-driven insertion."""
import numpy as np
import pytest
import torch

import oracle
import oracle.mlp as OM
import synth
from paper_2504_02437_amd import init_mlp as IM
from paper_2504_02437_amd import raster as R

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _kf(seed, W=120, H=90, K=40):
    rng = np.random.default_rng(seed)
    w = synth.room_gaussians(rng, 20000)
    cam = synth.room_camera(W, H, 80.0)
    img = rng.uniform(size=(3, H, W)).astype(np.float32)
    pts = np.stack([rng.integers(0, W, K), rng.integers(0, H, K),
                    1.0 / rng.uniform(1, 4, K)], 1).astype(np.float32)
    return w, cam, img, pts


@pytest.mark.parametrize("centre_only", [False, True])
def test_knn_features_match_oracle(centre_only):
    g, cam, img, pts = _kf(1)
    print("case knn", centre_only, flush=True)
    params = R.ParamBuffer.from_gaussians(g)
    C = pts.shape[0] * (1 if centre_only else 9)
    feats = torch.empty(C, 32, device="cuda")
    kidx = torch.empty(C, 8, dtype=torch.int32, device="cuda")
    kd = torch.empty(C, 8, device="cuda")
    R.knn_features(params, R.cameras_to_device([cam]), cam.width, cam.height,
                   _dev(img), _dev(pts), centre_only, feats, kidx, kd)
    torch.cuda.synchronize()
    F, P = OM.features(cam, img, pts, g.mean.astype(np.float64),
                       g.rgb.astype(np.float64), centre_only)
    idx, dist = OM.knn(g.mean.astype(np.float64), P)
    np.testing.assert_array_equal(kidx.cpu().numpy(), idx)
    np.testing.assert_allclose(kd.cpu().numpy(), dist, rtol=1e-6)
    np.testing.assert_allclose(feats.cpu().numpy(), F, rtol=1e-6, atol=1e-7)


def test_knn_features_equal_distances_take_the_lower_index():
    """The second half of the map repeats the first, so every neighbour
    comes as a pair at the same distance (indices i and i + 10000, staged in
    different chunks and read by different lanes): the lower index first."""
    g, cam, img, pts = _kf(3, K=23)
    g.mean[:, 10000:] = g.mean[:, :10000]
    print("case knn ties", flush=True)
    params = R.ParamBuffer.from_gaussians(g)
    C = pts.shape[0] * 9
    feats = torch.empty(C, 32, device="cuda")
    kidx = torch.empty(C, 8, dtype=torch.int32, device="cuda")
    kd = torch.empty(C, 8, device="cuda")
    R.knn_features(params, R.cameras_to_device([cam]), cam.width, cam.height,
                   _dev(img), _dev(pts), False, feats, kidx, kd)
    torch.cuda.synchronize()
    F, P = OM.features(cam, img, pts, g.mean.astype(np.float64),
                       g.rgb.astype(np.float64), False)
    idx, _ = OM.knn(g.mean.astype(np.float64), P)
    assert np.all(idx[:, 1::2] == idx[:, 0::2] + 10000)
    np.testing.assert_array_equal(kidx.cpu().numpy(), idx)
    np.testing.assert_allclose(feats.cpu().numpy(), F, rtol=1e-6, atol=1e-7)


def test_knn_features_full_map_sampled():
    """The densification workload's shape: 96 patches x 9 candidates against
    a 300k-Gaussian map (spare capacity as in mapping), one launch; sampled
    patches (corners included) against the brute-force oracle."""
    rng = np.random.default_rng(7)
    W, H = 1200, 680
    g = synth.room_gaussians(rng, 300000)
    cam = synth.room_camera(W, H, 600.0)
    img = rng.uniform(size=(3, H, W)).astype(np.float32)
    pts = np.stack([rng.integers(0, W, 96), rng.integers(0, H, 96),
                    1.0 / rng.uniform(1, 5, 96)], 1).astype(np.float32)
    pts[0, :2] = (0, 0)
    pts[95, :2] = (W - 1, H - 1)
    print("case knn full", flush=True)
    params = R.ParamBuffer.from_gaussians(g, capacity=450000)
    feats = torch.empty(96 * 9, 32, device="cuda")
    kidx = torch.empty(96 * 9, 8, dtype=torch.int32, device="cuda")
    kd = torch.empty(96 * 9, 8, device="cuda")
    R.knn_features(params, R.cameras_to_device([cam]), W, H, _dev(img),
                   _dev(pts), False, feats, kidx, kd)
    torch.cuda.synchronize()
    sel = np.array([0, 13, 41, 77, 95])
    F, P = OM.features(cam, img, pts[sel], g.mean.astype(np.float64),
                       g.rgb.astype(np.float64), False)
    idx, dist = OM.knn(g.mean.astype(np.float64), P)
    rows = (sel[:, None] * 9 + np.arange(9)).ravel()
    np.testing.assert_array_equal(kidx.cpu().numpy()[rows], idx)
    np.testing.assert_allclose(kd.cpu().numpy()[rows], dist, rtol=1e-6)
    np.testing.assert_allclose(feats.cpu().numpy()[rows], F, rtol=1e-6, atol=1e-7)


def test_knn_features_small_and_empty_map():
    g, cam, img, pts = _kf(2, K=5)
    params = R.ParamBuffer.from_gaussians(g.subset(np.arange(5)), capacity=64)
    feats = torch.empty(45, 32, device="cuda")
    R.knn_features(params, R.cameras_to_device([cam]), cam.width, cam.height,
                   _dev(img), _dev(pts), False, feats)
    F, _ = OM.features(cam, img, pts, g.mean[:, :5].astype(np.float64),
                       g.rgb[:, :5].astype(np.float64))
    np.testing.assert_allclose(feats.cpu().numpy(), F, rtol=1e-6, atol=1e-7)
    params.n_dev.zero_()
    R.knn_features(params, R.cameras_to_device([cam]), cam.width, cam.height,
                   _dev(img), _dev(pts), False, feats)
    assert torch.all(feats[:, 28:] == 0)


def _io(seed, M):
    rng = np.random.default_rng(seed)
    w = OM.init_weights(seed)
    w[-7:] = rng.normal(size=7)
    x = rng.normal(size=(M, 32)).astype(np.float32)
    return w, x, rng


def _y_tol(w, rc):
    """Per-output bar of 2 BF16 ulps: a hidden activation whose BF16
    rounding falls on the other side of a boundary in FP32 vs FP64 moves by
    one ulp (2^-7 of its magnitude), which reaches output k through at most
    oracle.mlp.forward_magnitude; FP32 accumulation adds 1e-6 relative."""
    (_, _), (_, _), (_, b3) = OM.unpack(w)
    mag = OM.forward_magnitude(w, rc)
    return 2 ** -7 * mag + 1e-6 * (mag + np.abs(b3))


@pytest.mark.parametrize("M", [1, 63, 64, 200, 1000])
def test_mlp_forward_matches_oracle(M):
    w, x, _ = _io(3, M)
    print("case mlp fwd", M, flush=True)
    y = torch.empty(M, 7, device="cuda")
    cache = torch.empty(M, 128, device="cuda")
    R.mlp_fwd(_dev(w), _dev(x), y, cache)
    ref, rc = OM.forward(w, x)
    got = y.cpu().numpy()
    tol = _y_tol(w, rc)
    assert np.all(np.abs(got - ref) <= tol), (np.abs(got - ref) / tol).max()
    np.testing.assert_allclose(cache.cpu().numpy()[:, :64], rc["z1"],
                               rtol=1e-5, atol=1e-5 * np.abs(rc["z1"]).max())


@pytest.mark.parametrize("M", [64, 300])
def test_mlp_backward_matches_oracle(M):
    """The oracle runs the whole step on its own (forward, MSE, backward);
    the GPU's gradient may differ only through the forward's per-output bar
    (which moves dL/dy by at most 2 tol / (7 M)) and BF16 rounding flips of
    dL/dy and of the hidden gradients (2^-6 of the terms' magnitudes)."""
    w, x, rng = _io(4, M)
    print("case mlp bwd", M, flush=True)
    t = rng.normal(size=(M, 7)).astype(np.float32)
    y = torch.empty(M, 7, device="cuda")
    cache = torch.empty(M, 128, device="cuda")
    R.mlp_fwd(_dev(w), _dev(x), y, cache)
    dy = torch.empty_like(y)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    R.mlp_mse(y, _dev(t), dy, loss)
    dw = torch.zeros(IM.N_PARAMS, device="cuda")
    R.mlp_bwd(_dev(w), _dev(x), cache, dy, dw)
    ref_y, rc = OM.forward(w, x)
    ref_loss, ref_dy = OM.mse(ref_y, t)
    tol_y = _y_tol(w, rc)
    r = np.abs(ref_y - t)
    assert abs(float(loss) - ref_loss) <= ((2 * r + tol_y) * tol_y).sum() / r.size
    ddy = 2.0 * tol_y / r.size
    ref_g = OM.backward(w, rc, ref_dy)
    bound = OM.backward_magnitude(w, rc, ddy) * (1 + 2 ** -6) + 2 ** -6 * (
        OM.backward_magnitude(w, rc, np.abs(ref_dy)) +
        OM.backward_magnitude(w, rc, np.abs(ref_dy) + ddy))
    got = dw.cpu().numpy()
    bad = np.nonzero(np.abs(got - ref_g) > bound + 1e-12)[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], ref_g[bad[:5]], bound[bad[:5]])


def test_mlp_adam_step_matches_oracle():
    rng = np.random.default_rng(5)
    w = rng.normal(size=IM.N_PARAMS).astype(np.float32)
    g = rng.normal(size=IM.N_PARAMS).astype(np.float32)
    wd, gd = _dev(w), _dev(g)
    m = torch.zeros_like(wd)
    v = torch.zeros_like(wd)
    for step in (1, 2):
        R.mlp_adam(wd, gd, m, v, 1e-3, 0.9, 0.999, 1e-8, step)
    p, mm, vv = w.astype(np.float64), np.zeros(IM.N_PARAMS), np.zeros(IM.N_PARAMS)
    for step in (1, 2):
        p, mm, vv = oracle.adam(p, g, mm, vv, 1e-3, step, eps=1e-8)
    np.testing.assert_allclose(wd.cpu().numpy(), p, atol=1e-6)


def test_training_fits_a_smooth_function():
    """The project's own kernels train the network: the loss on a smooth
    synthetic regression falls by an order of magnitude."""
    rng = np.random.default_rng(6)
    x = rng.normal(size=(16384, 32)).astype(np.float32)
    A = rng.normal(size=(32, 7)) / 6
    t = np.tanh(x @ A).astype(np.float32)
    net = IM.InitMLP(seed=7)
    xd, td = _dev(x), _dev(t)
    net.fit_normalisation(xd, td)
    hist = net.train(xd, td, epochs=30, batch=4096, lr=3e-3)
    print("training loss", hist[0], hist[-1], flush=True)
    assert hist[-1] < 0.1 * hist[0]


def test_insert_with_mlp_output():
    g, cam, img, pts = _kf(8, K=30)
    params = R.ParamBuffer.from_gaussians(g, capacity=g.n + 300)
    rng = np.random.default_rng(9)
    mlp_out = rng.normal(size=(270, 7)).astype(np.float32)
    kT = rng.uniform(0.0, 0.3, size=(cam.height, cam.width)).astype(np.float32)
    R.insert_gaussians(params, None, None, R.cameras_to_device([cam]),
                       cam.width, cam.height, None, _dev(kT), _dev(pts),
                       mlp_out=_dev(mlp_out))
    torch.cuda.synchronize()
    ref = oracle.insert(cam, img, kT.astype(np.float64), pts,
                        alpha_skip=float(np.float32(0.9)))
    n0 = g.n
    assert params.n() == n0 + ref["count"]
    got = params.data[:, n0:n0 + ref["count"]].cpu().numpy()
    src = ref["src"]
    np.testing.assert_allclose(got[0:3], ref["mean"], rtol=1e-6, atol=1e-6)
    np.testing.assert_array_equal(got[3:6], mlp_out[src, 0:3].T)
    np.testing.assert_array_equal(got[10], mlp_out[src, 3])
    np.testing.assert_array_equal(got[11:14], mlp_out[src, 4:7].T)
