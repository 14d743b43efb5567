"""gs_insert_distance_noalloc (the distance-tested insertion with its scratch
in the library's static device array) against gs_insert_distance with a
caller scratch, through the C ABI: two calls in a row on the same map, the
second with fewer candidates, give bit-identical parameters, moments, live
counts, inserted counts and status; too many candidates are refused before
any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from paper_2504_02437_amd import _lib as L
from paper_2504_02437_amd import raster as R

pytestmark = pytest.mark.gpu


def _noalloc(params, m, v, cam_dev, W, H, img, pts, tau, nins, status):
    return L.lib().gs_insert_distance_noalloc(
        C.byref(params.struct()), C.byref(m.struct()), C.byref(v.struct()),
        C.c_void_p(cam_dev.data_ptr()), W, H, C.c_void_p(img.data_ptr()),
        C.c_void_p(pts.data_ptr()), pts.shape[0], C.c_float(tau), 0, None,
        C.c_void_p(nins.data_ptr()), C.c_void_p(status.data_ptr()), None)


def _setup(seed, n0, cap):
    w = synth.config1(seed=seed, n=n0)
    cam = w.cameras[0]
    params = R.ParamBuffer.from_gaussians(w.gaussians, capacity=cap)
    return w, cam, params


def test_noalloc_insertion_equals_the_scratch_entry_point():
    n0, cap = 40_000, 40_000 + 2 * 864 + 100
    w, cam, base = _setup(5, n0, cap)
    W, H = cam.width, cam.height
    rng = np.random.default_rng(7)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    cam_dev = R.cameras_to_device([cam])
    img = dev(rng.uniform(size=(3, H, W)).astype(np.float32))
    sides = []
    for _ in range(2):
        p = R.ParamBuffer.from_gaussians(w.gaussians, capacity=cap)
        m, v = p.zeros_like(), p.zeros_like()
        m.data.fill_(2.0)
        v.data.fill_(3.0)
        sides.append((p, m, v))
    tau = 0.03
    for call, K in enumerate((96, 40)):
        print("case no-alloc insertion call", call, "patches", K, flush=True)
        pts = dev(np.stack([rng.integers(0, W, K), rng.integers(0, H, K),
                            1.0 / rng.uniform(1, 5, K)], 1).astype(np.float32))
        outs = []
        for i, (p, m, v) in enumerate(sides):
            nins = torch.full((1,), -7, dtype=torch.int32, device="cuda")
            status = torch.zeros(1, dtype=torch.int32, device="cuda")
            if i == 0:
                R.insert_distance(p, m, v, cam_dev, W, H, img, pts, tau,
                                  n_inserted_dev=nins, status_dev=status)
            else:
                assert _noalloc(p, m, v, cam_dev, W, H, img, pts, tau, nins,
                                status) == L.GS_OK
            torch.cuda.synchronize()
            outs.append((p.data.cpu().numpy(), m.data.cpu().numpy(),
                         v.data.cpu().numpy(), p.n(), int(nins), int(status)))
        a, b = outs
        assert a[3] == b[3] and a[4] == b[4] and a[5] == b[5] == 0
        assert a[4] > 0, "the case inserts something"
        for x, y in zip(a[:3], b[:3]):
            np.testing.assert_array_equal(x, y)
    assert sides[0][0].n() > n0


def test_noalloc_insertion_refuses_too_many_candidates():
    w, cam, p = _setup(6, 1000, 2000)
    m, v = p.zeros_like(), p.zeros_like()
    before = p.data.clone()
    pts = torch.zeros(7282, 3, device="cuda")   # 9 x 7282 > 65536
    nins = torch.zeros(1, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = _noalloc(p, m, v, R.cameras_to_device([cam]), cam.width, cam.height,
                  torch.zeros(3, cam.height, cam.width, device="cuda"), pts,
                  0.01, nins, status)
    assert rc == L.GS_E_CAPACITY
    assert b"static scratch" in L.lib().gs_last_error()
    torch.cuda.synchronize()
    assert torch.equal(p.data, before) and p.n() == 1000
