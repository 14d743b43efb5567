"""Pins the oracle's key emission, stable sort and tile ranges to textbook
routines (numpy's stable argsort / lexsort) and to brute-force tile scans."""
import numpy as np
import pytest

import oracle
import synth


def _multi_view(seed=0, V=3, n=400):
    rng = np.random.default_rng(seed)
    w = synth.tiny_scene(seed, n=n, width=70, height=45, f=60.0)
    cams = [w.cameras[0]]
    for _ in range(V - 1):
        c = w.cameras[0]
        t = (c.t + rng.normal(0, 0.1, 3)).astype(np.float32)
        cams.append(synth.Camera(c.R, t, c.fx, c.fy, c.cx, c.cy, c.width,
                                 c.height))
    return w, cams


@pytest.mark.parametrize("tile,threads", [(8, 1), (16, 1), (32, 1), (8, 3),
                                          (16, 8)])
def test_sort_matches_stable_argsort_and_lexsort(tile, threads):
    """Views are emitted and sorted in parallel: the result is the single
    stable sort of all keys whatever the thread count."""
    w, cams = _multi_view(V=5 if threads > 1 else 3)
    p = oracle.params64(w.gaussians)
    W, H = cams[0].width, cams[0].height
    proj = oracle.project(p, cams, tile)
    b = oracle.bin_sort(proj, tile, W, H, nthreads=threads)
    assert b["n_keys"] == int(proj["tiles"].sum())
    order = np.argsort(b["keys_emit"], kind="stable")
    np.testing.assert_array_equal(b["keys"], b["keys_emit"][order])
    np.testing.assert_array_equal(b["vals"], b["vals_emit"][order])
    # The order is exactly lexicographic in (view-tile, depth bits, index).
    tid = (b["keys_emit"] >> np.uint64(32)).astype(np.int64)
    dep = (b["keys_emit"] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    lex = np.lexsort((b["vals_emit"], dep, tid))
    np.testing.assert_array_equal(b["vals"], b["vals_emit"][lex])


def test_emitted_keys_cover_exactly_the_touched_tiles():
    w, cams = _multi_view(seed=1)
    tile = 8
    p = oracle.params64(w.gaussians)
    W, H = cams[0].width, cams[0].height
    Tx, Ty = -(-W // tile), -(-H // tile)
    proj = oracle.project(p, cams, tile)
    b = oracle.bin_sort(proj, tile, W, H)
    n = p["mean"].shape[1]
    tid = (b["keys_emit"] >> np.uint64(32)).astype(np.int64)
    dep = (b["keys_emit"] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    pos = 0
    for k in range(len(cams)):
        for g in range(n):
            nt = proj["tiles"][k, g]
            if nt == 0:
                continue
            bx = proj["box"][k, g]
            expect = []
            for ty in range(Ty):
                for tx in range(Tx):
                    x0, y0 = tx * tile, ty * tile
                    if x0 <= bx[1] and x0 + tile - 1 >= bx[0] and \
                            y0 <= bx[3] and y0 + tile - 1 >= bx[2]:
                        expect.append((k * Ty + ty) * Tx + tx)
            got = tid[pos:pos + nt]
            np.testing.assert_array_equal(got, expect)
            np.testing.assert_array_equal(b["vals_emit"][pos:pos + nt], g)
            d32 = np.float32(proj["rec"][k, g, 6]).view(np.uint32)
            assert np.all(dep[pos:pos + nt] == d32)
            pos += nt
    assert pos == b["n_keys"]


def test_ranges_partition_the_sorted_list():
    w, cams = _multi_view(seed=2)
    tile = 16
    p = oracle.params64(w.gaussians)
    W, H = cams[0].width, cams[0].height
    proj = oracle.project(p, cams, tile)
    b = oracle.bin_sort(proj, tile, W, H)
    r = b["ranges"].astype(np.int64)
    assert r[0, 0] == 0 and r[-1, 1] == b["n_keys"]
    np.testing.assert_array_equal(r[1:, 0], r[:-1, 1])
    tid = (b["keys"] >> np.uint64(32)).astype(np.int64)
    for t in range(r.shape[0]):
        assert np.all(tid[r[t, 0]:r[t, 1]] == t)
    # Per-tile count = number of boxes overlapping the tile (brute force).
    Tx = -(-W // tile)
    Ty = -(-H // tile)
    for t in range(0, r.shape[0], 5):
        k, tt = divmod(t, Tx * Ty)
        ty, tx = divmod(tt, Tx)
        bx = proj["box"][k]
        ok = (proj["tiles"][k] > 0) & (bx[:, 0] <= tx * tile + tile - 1) & \
            (bx[:, 1] >= tx * tile) & (bx[:, 2] <= ty * tile + tile - 1) & \
            (bx[:, 3] >= ty * tile)
        assert r[t, 1] - r[t, 0] == ok.sum()


def test_capacity_overflow_is_reported():
    w, cams = _multi_view(seed=3, V=1)
    p = oracle.params64(w.gaussians)
    proj = oracle.project(p, cams, 16)
    with pytest.raises(OverflowError):
        oracle.bin_sort(proj, 16, cams[0].width, cams[0].height,
                        cap=int(proj["tiles"].sum()) - 1)


def test_empty_scene():
    w = synth.tiny_scene(0, n=5)
    p = oracle.params64(w.gaussians)
    p["mean"][2] = -1.0   # all behind the camera
    proj = oracle.project(p, w.cameras, 16)
    b = oracle.bin_sort(proj, 16, w.cameras[0].width, w.cameras[0].height)
    assert b["n_keys"] == 0
    assert np.all(b["ranges"] == 0)


def test_equal_depth_ties_keep_index_order():
    """Gaussians on the plane z = 2 seen by an identity camera share the FP32
    depth exactly, so within a tile every key ties: the stable sort must keep
    them in ascending index order, and compositing follows that order."""
    w = synth.tiny_scene(21, n=60, width=40, height=32, f=38.0,
                         log_scale_mu=-1.6)
    w.gaussians.mean[2, :] = 2.0
    p = oracle.params64(w.gaussians)
    c = w.cameras[0]
    proj = oracle.project(p, [c], 16)
    assert np.all(proj["rec"][0, proj["tiles"][0] > 0, 6] == 2.0)
    b = oracle.bin_sort(proj, 16, c.width, c.height)
    r = b["ranges"].astype(np.int64)
    for t in range(r.shape[0]):
        seg = b["vals"][r[t, 0]:r[t, 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)
    import oracle.brute as brute
    f = oracle.forward(proj, b, p["rgb"], c.width, c.height)
    img, _, _ = brute.composite(proj["rec"], proj["box"], p["rgb"], c.width,
                                c.height)
    np.testing.assert_allclose(f["img"], img, atol=1e-13)
