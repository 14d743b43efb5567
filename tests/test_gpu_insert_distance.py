"""GPU insertion with the distance test of Eq. 7 against the oracle: the
nearest squared distances are bit-exact (same FP64 expression), so the kept
set and its order are exact; inserted parameters match as in the
alpha-masked insertion; empty maps and capacity overflow."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2504_02437_amd import raster as R

pytestmark = pytest.mark.gpu


def _case(seed, n0, cap, K=96, centre_only=False, tau_q=0.5, scene=None):
    """scene: None for a 96x64 camera over a tiny scene, else a workload
    whose first camera and Gaussians are used (n0 = all of them)."""
    rng = np.random.default_rng(seed)
    if scene is None:
        W, H = 96, 64
        R_ = np.array([[0.8, 0.0, 0.6], [0.0, 1.0, 0.0], [-0.6, 0.0, 0.8]],
                      np.float32)
        cam = synth.Camera(R_, np.array([0.3, -0.1, 0.5], np.float32), 80.0,
                           82.0, (W - 1) / 2, (H - 1) / 2, W, H)
        gauss = synth.tiny_scene(seed, n=max(n0, 1)).gaussians
    else:
        cam = scene.cameras[0]
        W, H = cam.width, cam.height
        gauss = scene.gaussians
    img = rng.uniform(size=(3, H, W)).astype(np.float32)
    pts = np.stack([rng.integers(-1, W + 1, K), rng.integers(-1, H + 1, K),
                    1.0 / rng.uniform(1, 5, K)], 1).astype(np.float32)
    params = R.ParamBuffer.from_gaussians(gauss, capacity=cap)
    params.n_dev.fill_(n0)
    means = params.data[0:3, :n0].cpu().numpy()
    d2 = oracle.nearest(cam, pts, means, centre_only=centre_only, nthreads=16)
    inside = d2 >= 0
    finite = inside & np.isfinite(d2)
    tau = float(np.float32(np.sqrt(np.quantile(d2[finite], tau_q)))) if finite.any() else 1.0
    m, v = params.zeros_like(), params.zeros_like()
    m.data.fill_(3.0)
    v.data.fill_(3.0)
    nins = torch.zeros(1, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    scratch = R.insert_distance(params, m, v, R.cameras_to_device([cam]), W, H,
                                dev(img), dev(pts), tau, centre_only=centre_only,
                                n_inserted_dev=nins, status_dev=status)
    torch.cuda.synchronize()
    bits = scratch.cpu().numpy().view(np.uint64)
    got_d2 = bits.view(np.float64)
    tested = bits != np.uint64(0xFFFFFFFFFFFFFFFF)
    if n0 > 0:
        np.testing.assert_array_equal(tested, inside)
        np.testing.assert_array_equal(got_d2[inside], d2[inside])
    else:
        assert not tested.any()
    ref = oracle.insert(cam, img, None, pts, centre_only=centre_only,
                        cand_d2=d2, tau=tau, cap=cap - n0)
    cnt = ref["count"]
    assert int(nins.item()) == cnt
    k = min(cnt, cap - n0)
    assert params.n() == n0 + k
    assert bool(int(status.item()) & 2) == (cnt > cap - n0)
    got = params.data[:, n0:n0 + k].cpu().numpy()
    np.testing.assert_allclose(got[0:3], ref["mean"], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(got[3:6], ref["log_scale"], rtol=1e-6, atol=1e-7)
    np.testing.assert_array_equal(got[6:10], ref["quat"])
    np.testing.assert_array_equal(got[10], ref["opacity_logit"])
    np.testing.assert_array_equal(got[11:14], ref["rgb"])
    assert torch.all(m.data[:, n0:n0 + k] == 0)
    assert torch.all(m.data[:, :n0] == 3.0)
    return cnt


@pytest.mark.parametrize("centre_only", [False, True])
def test_distance_insertion_matches_oracle(centre_only):
    print("case insert distance", centre_only, flush=True)
    cnt = _case(51, 3000, 5000, centre_only=centre_only)
    assert cnt > 0


def test_distance_insertion_into_an_empty_map():
    print("case insert distance empty", flush=True)
    cnt = _case(52, 0, 2000)
    assert cnt > 0


def test_distance_insertion_overflow():
    print("case insert distance overflow", flush=True)
    _case(53, 3000, 3010, tau_q=0.1)


def test_distance_insertion_full_size():
    """The benchmark's insertion workload: 96 patches x 9 candidates on the
    1200x680 room view, tested against all 300k Gaussians of the map."""
    w = synth.config1()
    n = w.gaussians.n
    print("case insert distance full size", flush=True)
    cnt = _case(52, n, n + 96 * 9, scene=w)
    assert cnt > 0
