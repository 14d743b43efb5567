"""Pins of the oracle's distance-tested insertion (Eq. 7, read as "farther
than tau"): nearest distances against a k-d tree, the strict threshold, the
empty map and agreement of the candidate order with the alpha-masked
insertion."""
import numpy as np
from scipy.spatial import cKDTree

import oracle
import synth


def _setup(seed=0, K=40, n=500):
    rng = np.random.default_rng(seed)
    W, H = 64, 48
    cam = synth.identity_camera(50.0, 52.0, W, H, (0.1, -0.2, 0.3))
    pts = np.stack([rng.integers(-1, W + 1, K), rng.integers(-1, H + 1, K),
                    1.0 / rng.uniform(1, 4, K)], 1).astype(np.float32)
    pts[3, 2] = -0.5                       # a bad depth
    means = rng.normal(size=(3, n)).astype(np.float32) * 2.0
    rgb = rng.uniform(size=(3, H, W)).astype(np.float32)
    return cam, pts, means, rgb


def _points(cam, pts, centre_only=False):
    """Back-projected candidates via the alpha-masked insertion with a fully
    transparent keyframe (every candidate inside the image kept)."""
    T = np.ones((cam.height, cam.width), np.float32)
    ins = oracle.insert(cam, np.zeros((3, cam.height, cam.width)), T, pts,
                        alpha_skip=0.9, centre_only=centre_only)
    return ins


def test_nearest_matches_a_kd_tree():
    cam, pts, means, _ = _setup()
    d2 = oracle.nearest(cam, pts, means)
    ins = _points(cam, pts)
    tree = cKDTree(means.T.astype(np.float64))
    dist, _ = tree.query(ins["mean"].T)
    got = d2[ins["src"]]           # src: patch * 9 + pixel
    np.testing.assert_allclose(np.sqrt(got), dist, rtol=1e-12, atol=1e-12)
    # Candidates outside the image or with a bad depth are -1.
    outside = np.setdiff1d(np.arange(d2.size), ins["src"])
    assert np.all(d2[outside] == -1.0)


def test_threshold_is_strict_and_orders_like_the_alpha_insertion():
    cam, pts, means, rgb = _setup(1)
    d2 = oracle.nearest(cam, pts, means)
    inside = d2 >= 0
    tau = float(np.float32(np.sqrt(np.median(d2[inside]))))
    ins = oracle.insert(cam, rgb, None, pts, cand_d2=d2, tau=tau)
    want = np.nonzero(d2 > np.float64(np.float32(tau)) ** 2)[0]
    np.testing.assert_array_equal(ins["src"], want)
    # A point exactly on an existing mean is never inserted at tau = 0.
    ins0 = oracle.insert(cam, rgb, None, pts, cand_d2=np.where(d2 >= 0, 0.0, -1.0),
                         tau=0.0)
    assert ins0["count"] == 0
    # The inserted parameters are those of the alpha-masked path.
    all_ins = _points(cam, pts)
    sel = np.searchsorted(all_ins["src"], ins["src"])
    np.testing.assert_array_equal(ins["mean"], all_ins["mean"][:, sel])


def test_empty_map_inserts_every_candidate():
    cam, pts, _, rgb = _setup(2)
    d2 = oracle.nearest(cam, pts, np.zeros((3, 0), np.float32))
    assert np.all((d2 == -1.0) | np.isinf(d2))
    ins = oracle.insert(cam, rgb, None, pts, cand_d2=d2, tau=1e30)
    assert ins["count"] == _points(cam, pts)["count"]


def test_centre_only_candidates():
    cam, pts, means, rgb = _setup(3)
    d2 = oracle.nearest(cam, pts, means, centre_only=True)
    full = oracle.nearest(cam, pts, means)
    np.testing.assert_array_equal(d2, full.reshape(-1, 9)[:, 4])
