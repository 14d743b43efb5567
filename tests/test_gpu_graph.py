"""One whole mapping iteration (project, bin, sort, render, L1 + planar
gradients, backward, projection backward, Adam with a device step count)
captured as a HIP graph and replayed, with the L1 term as a separate pass
and fused into the backward: every replay matches the same iteration run
eagerly from the same state."""
import numpy as np
import pytest
import torch

import synth
from paper_2504_02437_amd import raster as R

pytestmark = pytest.mark.gpu

LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3)


def _setup():
    w = synth.tiny_scene(61, n=800, width=96, height=72, f=80.0,
                         log_scale_mu=-2.0)
    c = w.cameras[0]
    c2 = synth.Camera(c.R, (c.t + np.array([0.05, 0.0, 0.02])).astype(np.float32),
                      c.fx, c.fy, c.cx, c.cy, c.width, c.height)
    w.cameras = [c, c2]
    params = R.ParamBuffer.from_gaussians(w.gaussians, capacity=1000)
    rast = R.Rasterizer(w.cameras, params.capacity, R.Settings(tile=16))
    st = dict(params=params, rast=rast, grad=params.zeros_like(),
              m=params.zeros_like(), v=params.zeros_like(),
              target=torch.from_numpy(np.random.default_rng(6).uniform(
                  size=(2, 3, 72, 96)).astype(np.float32)).cuda(),
              dL=torch.empty(2, 3, 72, 96, device="cuda"),
              loss=torch.zeros(1, dtype=torch.float64, device="cuda"),
              step=torch.ones(1, dtype=torch.int32, device="cuda"))
    return w, st


def _iteration(st, fused=False):
    p, r = st["params"], st["rast"]
    st["grad"].data.zero_()
    st["loss"].zero_()
    r.forward(p)
    R.planar_reg(p, 1.0, 0.01, st["grad"], st["loss"])
    if fused:
        # The benchmark's iteration: the L1 term fused into the backward.
        r.backward_l1(p, st["target"], 1.0, st["grad"], st["loss"])
    else:
        R.loss_l1(r.rgb, st["target"], 1.0, st["dL"], st["loss"])
        r.backward(p, st["dL"], st["grad"])
    R.adam(p, st["grad"], st["m"], st["v"], LR, 0.9, 0.999, 1e-15, st["step"])
    st["step"].add_(1)


def _snapshot(st):
    return [st[k].data.clone() for k in ("params", "m", "v")] + \
        [st["step"].clone(), st["rast"].rgb.clone(), st["loss"].clone()]


def _restore(st, snap):
    for k, t in zip(("params", "m", "v"), snap[:3]):
        st[k].data.copy_(t)
    st["step"].copy_(snap[3])


@pytest.mark.parametrize("fused", [False, True])
def test_graph_replays_match_eager_iterations(fused):
    w, st = _setup()
    start = _snapshot(st)
    eager = []
    for _ in range(3):
        _iteration(st, fused)
        eager.append(_snapshot(st))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _iteration(st, fused)                  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    _restore(st, start)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        _iteration(st, fused)
    torch.cuda.synchronize()
    _restore(st, start)
    torch.cuda.synchronize()
    for i in range(3):
        print("case graph replay", i, flush=True)
        # Each replay starts from the state the eager run had before its
        # iteration i (atomics make the states differ in the last bits).
        _restore(st, start if i == 0 else eager[i - 1])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = _snapshot(st)
        # The forward is deterministic: the replayed image is bit-identical.
        assert torch.equal(got[4], eager[i][4]), i
        assert torch.equal(got[3], eager[i][3]), i
        # The loss: the fused L1 sum is formed in a fixed order, the planar
        # term with FP64 atomics (last bits).
        torch.testing.assert_close(got[5], eager[i][5], rtol=1e-12, atol=0)
        # Gradients are summed with float atomics: the parameters agree to
        # rounding.
        for a, b in zip(got[:3], eager[i][:3]):
            torch.testing.assert_close(a, b, rtol=1e-5, atol=1e-7)
        # Eager work of the program itself between replays.
        st["rast"].count_pairs(st["params"])
        torch.cuda.synchronize()
