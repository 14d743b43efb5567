"""The library's own window graph (gs_window_build / gs_window_run): one
mapping iteration captured behind the C ABI and replayed.  Every replay
matches the same calls made eagerly from the same state, and on the
benchmark's 10-view window the replayed iteration matches the oracle:
image, loss and every parameter gradient; the Adam node applies the
gradient the graph produced with the device step count, which it advances."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import (check_forward, check_grads, gpu_forward,
                         oracle_backward, oracle_forward)
from paper_2504_02437_amd import raster as R

pytestmark = pytest.mark.gpu

LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3)
B1, B2, EPS = 0.9, 0.999, 1e-15
# The Adam kernel takes the betas as FP32 settings: 1 - 0.999f is 1.3e-5 off
# 1 - 0.999, so the check below uses the FP32 values.
B1F, B2F = float(np.float32(B1)), float(np.float32(B2))


def _state(params, rast, target):
    return dict(params=params, rast=rast, grad=params.zeros_like(),
                m=params.zeros_like(), v=params.zeros_like(), target=target,
                loss=torch.zeros(1, dtype=torch.float64, device="cuda"),
                sq=torch.zeros(rast.V, dtype=torch.float64, device="cuda"),
                step=torch.ones(1, dtype=torch.int32, device="cuda"))


def _eager(st):
    """The calls the window graph captures, made one by one."""
    p, r = st["params"], st["rast"]
    st["grad"].data.zero_()
    st["loss"].zero_()
    st["sq"].zero_()
    r.forward(p)
    R.planar_reg(p, 1.0, 0.01, st["grad"], st["loss"])
    R.render_bwd_l1(r.ws, p, r.settings, r.rgb, st["target"], 1.0, r.T,
                    r.nlast, st["grad"], st["loss"], st["sq"])
    R.project_bwd(r.ws, p, r.cams_dev, st["grad"])
    R.adam(p, st["grad"], st["m"], st["v"], LR, B1, B2, EPS, st["step"])
    st["step"].add_(1)


def _graph(st):
    return R.WindowGraph(st["rast"], st["params"], st["grad"], st["target"],
                         st["loss"], lam_l1=1.0, lam_reg=1.0, reg_floor=0.01,
                         m=st["m"], v=st["v"], lr=LR, beta1=B1, beta2=B2,
                         eps=EPS, step=st["step"], sqerr=st["sq"])


def _snap(st):
    r = st["rast"]
    return dict(params=st["params"].data.clone(), m=st["m"].data.clone(),
                v=st["v"].data.clone(), step=st["step"].clone(),
                grad=st["grad"].data.clone(), rgb=r.rgb.clone(), T=r.T.clone(),
                nlast=r.nlast.clone(), loss=st["loss"].clone(),
                sq=st["sq"].clone())


def _restore(st, s):
    st["params"].data.copy_(s["params"])
    st["m"].data.copy_(s["m"])
    st["v"].data.copy_(s["v"])
    st["step"].copy_(s["step"])
    torch.cuda.synchronize()


@pytest.mark.parametrize("degree", [0, 1])
def test_window_graph_replays_match_eager_calls(degree):
    """Two views of a small scene, tile 16: three replays, each from the
    state an eager iteration started from, with the program's own eager work
    between them.  Image, transmittance, n_last and step count are
    identical; the losses agree to FP64 atomic order, parameters and moments
    to FP32 atomic order.  Degree 1 adds the view-dependent colour's
    backward after the projection backward, and its coefficient rows to the
    Adam step."""
    w = synth.tiny_scene(71, n=800, width=96, height=72, f=80.0,
                         log_scale_mu=-2.0)
    w.gaussians = synth.with_sh(w.gaussians, 3, degree, 0.05)
    c = w.cameras[0]
    w.cameras = [c, synth.Camera(c.R, (c.t + np.array([0.05, 0.0, 0.02])
                                       ).astype(np.float32),
                                 c.fx, c.fy, c.cx, c.cy, c.width, c.height)]
    params = R.ParamBuffer.from_gaussians(w.gaussians, capacity=1000)
    rast = R.Rasterizer(w.cameras, params.capacity, R.Settings(tile=16))
    tgt = torch.from_numpy(np.random.default_rng(6).uniform(
        size=(2, 3, 72, 96)).astype(np.float32)).cuda()
    st = _state(params, rast, tgt)
    starts, eager = [], []
    for _ in range(3):
        starts.append(_snap(st))
        _eager(st)
        torch.cuda.synchronize()
        eager.append(_snap(st))
    _restore(st, starts[0])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = _graph(st)
    torch.cuda.synchronize()
    # The capture enqueued nothing: the state is untouched.
    assert torch.equal(st["params"].data, starts[0]["params"])
    for i in range(3):
        print("case window replay", degree, i, flush=True)
        _restore(st, starts[i])
        g.run(stream)
        torch.cuda.synchronize()
        got = _snap(st)
        for k in ("rgb", "T", "nlast", "step"):
            assert torch.equal(got[k], eager[i][k]), (i, k)
        torch.testing.assert_close(got["loss"], eager[i]["loss"], rtol=1e-12,
                                   atol=0)
        torch.testing.assert_close(got["sq"], eager[i]["sq"], rtol=1e-12,
                                   atol=0)
        for k in ("params", "m", "v"):
            torch.testing.assert_close(got[k], eager[i][k], rtol=1e-5,
                                       atol=1e-7)
        st["rast"].count_pairs(st["params"])
        torch.cuda.synchronize()
    g.close()


def test_window_graph_build_errors_leave_the_stream_usable():
    """A setting the calls reject is reported at build time (nothing
    captured), and the stream then runs eager work as before."""
    w = synth.tiny_scene(72, n=200, width=64, height=48, f=60.0)
    params = R.ParamBuffer.from_gaussians(w.gaussians)
    rast = R.Rasterizer(w.cameras, params.capacity, R.Settings(tile=16))
    tgt = torch.zeros(1, 3, 48, 64, device="cuda")
    st = _state(params, rast, tgt)
    rast.settings.lds_batch = 300
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with pytest.raises(R.L.GsError, match="lds_batch"):
            _graph(st)
        rast.settings.lds_batch = 256
        # Parameters of another capacity than the workspace's are refused
        # before anything is captured.
        other = R.ParamBuffer.from_gaussians(w.gaussians,
                                             capacity=params.capacity + 64)
        st_other = dict(st, params=other, grad=other.zeros_like(),
                        m=other.zeros_like(), v=other.zeros_like())
        with pytest.raises(R.L.GsError, match="capacity"):
            _graph(st_other)
        rast.forward(params)
    torch.cuda.synchronize()
    assert float(rast.T.min()) > 0


def test_window_graph_on_the_benchmark_window_against_the_oracle():
    """The benchmark's workload and launch shape (10 views, 1200x680, 300k
    Gaussians, 32/256/256), run three times from the same state through the
    library's graph: the image and its decisions match the oracle, the loss
    (L1 and planar terms) too, every parameter gradient per element as in
    the other full-size tests (the oracle's L1 gradient from its own image,
    targets 1e-4 away from it, FP32-ambiguous pixels given zero gradient on
    both sides), and the Adam node's output follows from the graph's own
    gradient, moments and step count."""
    w = synth.config2()
    print("case window graph oracle", flush=True)
    p64, proj, bins, fwd = oracle_forward(w, 32, nthreads=16)
    V, _, H, W = fwd["img"].shape
    mask = fwd["flags"] == 0
    tgt = np.random.default_rng(22).uniform(size=fwd["img"].shape).astype(np.float32)
    near = np.abs(fwd["img"] - tgt) < 1e-4
    tgt[near] = (fwd["img"][near] + 1e-4).astype(np.float32)
    _, dL = oracle.l1(fwd["img"], tgt, 1.0)
    dL *= mask[:, None]
    unfl = np.broadcast_to(mask[:, None], fwd["img"].shape)
    l1_ref = np.abs(fwd["img"] - tgt)[unfl].sum() / (3.0 * H * W)
    reg_ref, greg = oracle.planar_reg(p64["log_scale"], 1.0, 0.01)
    ref, mag, _ = oracle_backward(w, p64, proj, bins, dL, nthreads=16,
                                  full=True)
    ref = dict(ref, log_scale=ref["log_scale"] + greg)
    mag = dict(mag, log_scale=mag["log_scale"] + np.abs(greg))
    print("case window graph gpu", flush=True)
    params, rast = gpu_forward(w, 32, 256, threads=256, emit_keys=False,
                               key_capacity=int(1.25 * len(bins["vals"])))
    check_forward(rast, fwd, bins)
    # FP32-ambiguous pixels: target = the (deterministic) GPU image, so the
    # fused L1 term gives them sign 0, as the oracle's masked gradient.
    gtgt = torch.where(torch.from_numpy(mask).cuda()[:, None],
                       torch.from_numpy(tgt).cuda(), rast.rgb)
    st = _state(params, rast, gtgt)
    start = _snap(st)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = _graph(st)
    n = w.gaussians.n
    images = None
    for i in range(3):
        print("case window graph replay", i, flush=True)
        _restore(st, start)
        g.run(stream)
        torch.cuda.synchronize()
        got = _snap(st)
        assert int(got["step"]) == int(start["step"]) + 1
        if images is None:
            images = (got["rgb"], got["T"], got["nlast"])
            check_forward(rast, fwd, bins)
        else:
            for a, b in zip(images, (got["rgb"], got["T"], got["nlast"])):
                assert torch.equal(a, b)
        loss = float(got["loss"])
        assert abs(loss - (l1_ref + reg_ref)) <= V * 1e-5 + 1e-9 * reg_ref, \
            (loss, l1_ref, reg_ref)
        gg = got["grad"].cpu().numpy()
        worst = check_grads(gg, ref, n, mag=mag)
        print("window graph worst grad rel err", worst, flush=True)
        # Adam from the graph's own gradient (FP64 here, FP32 on the GPU).
        s = int(start["step"])
        g64 = gg[:, :n].astype(np.float64)
        m1 = B1F * start["m"][:, :n].cpu().numpy() + (1 - B1F) * g64
        v1 = B2F * start["v"][:, :n].cpu().numpy() + (1 - B2F) * g64 * g64
        np.testing.assert_allclose(got["m"][:, :n].cpu().numpy(), m1,
                                   rtol=1e-5, atol=1e-12)
        np.testing.assert_allclose(got["v"][:, :n].cpu().numpy(), v1,
                                   rtol=1e-5, atol=1e-20)
        lr = np.repeat(np.asarray(LR), [3, 3, 4, 1, 3])[:, None]
        step = lr * (m1 / (1 - B1F ** s)) / (np.sqrt(v1 / (1 - B2F ** s)) + EPS)
        p1 = start["params"][:, :n].cpu().numpy().astype(np.float64) - step
        np.testing.assert_allclose(got["params"][:, :n].cpu().numpy(), p1,
                                   rtol=1e-6, atol=1e-6 * lr.max())
        rast.count_pairs(params)
        torch.cuda.synchronize()
    g.close()
