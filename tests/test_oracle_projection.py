"""Pins the oracle's projection (Eq. 1-2) to closed forms and invariants."""
import math

import numpy as np
import pytest

import oracle
import synth


def one(mean, log_scale, quat=(1.0, 0.0, 0.0, 0.0), opl=0.0, rgb=(1, 1, 1)):
    return dict(mean=np.array(mean, float).reshape(3, 1),
                log_scale=np.array(log_scale, float).reshape(3, 1),
                quat=np.array(quat, float).reshape(4, 1),
                opacity_logit=np.array([opl], float),
                rgb=np.array(rgb, float).reshape(3, 1))


def cam(W=101, H=81, f=50.0, R=None, t=(0.0, 0.0, 0.0)):
    R = np.eye(3) if R is None else R
    return synth.Camera(np.asarray(R, np.float32), np.asarray(t, np.float32),
                        f, f, (W - 1) / 2.0, (H - 1) / 2.0, W, H)


def rand_rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def proj1(p, c, tile=16, publish=False):
    out = oracle.project(p, [c], tile, publish)
    return {k: v[0, 0] for k, v in out.items()}


@pytest.mark.parametrize("z,l", [(2.0, -3.0), (1.3, -2.2), (4.0, -1.0)])
def test_on_axis_isotropic(z, l):
    rng = np.random.default_rng(1)
    q = rng.normal(size=4)
    c = cam()
    r = proj1(one((0, 0, z), (l, l, l), q, opl=0.3), c)
    f = float(np.float32(c.fx))
    sig2 = (f * math.exp(l) / z) ** 2 + 0.3
    a, b, cc = r["cov"]
    assert a == pytest.approx(sig2, rel=1e-12)
    assert cc == pytest.approx(sig2, rel=1e-12)
    assert abs(b) < 1e-12 * sig2
    px, py, A, B, Cc, o, depth, rad = r["rec"]
    assert A == pytest.approx(1 / sig2, rel=1e-12)
    assert Cc == pytest.approx(1 / sig2, rel=1e-12)
    assert abs(B) < 1e-12 / sig2
    assert rad == math.ceil(3 * math.sqrt(sig2 + math.sqrt(0.1)))
    assert (px, py) == (c.cx, c.cy)
    assert depth == z
    assert o == pytest.approx(1 / (1 + math.exp(-0.3)), rel=1e-15)


def test_off_axis_isotropic_rotated_camera():
    """Isotropic Sigma = s^2 I gives Sigma2D = s^2 J J^T + 0.3 I for any
    world-to-camera rotation, with J evaluated at the camera-space mean."""
    rng = np.random.default_rng(2)
    for _ in range(20):
        Rk = rand_rot(rng).astype(np.float32)
        tk = rng.normal(size=3).astype(np.float32)
        c = cam(R=Rk, t=tk)
        tcam = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.4, 0.4), 1.0]) \
            * rng.uniform(1.0, 5.0)
        R64 = Rk.astype(np.float64)
        mu = R64.T @ (tcam - tk.astype(np.float64))
        l = rng.uniform(-3, -1)
        r = proj1(one(mu, (l, l, l)), c)
        # Recover the exact camera-space point the oracle sees.
        t = R64 @ mu + tk.astype(np.float64)
        f = float(np.float32(c.fx))
        J = np.array([[f / t[2], 0, -f * t[0] / t[2] ** 2],
                      [0, f / t[2], -f * t[1] / t[2] ** 2]])
        # W is the FP32 rotation, orthonormal only to ~1e-7, so keep W W^T.
        S2 = math.exp(2 * l) * J @ (R64 @ R64.T) @ J.T + 0.3 * np.eye(2)
        a, b, cc = r["cov"]
        np.testing.assert_allclose([a, b, cc], [S2[0, 0], S2[0, 1], S2[1, 1]],
                                   rtol=1e-9, atol=1e-12)
        assert r["rec"][0] == pytest.approx(f * t[0] / t[2] + c.cx, rel=1e-12)
        assert r["rec"][1] == pytest.approx(f * t[1] / t[2] + c.cy, rel=1e-12)
        assert r["rec"][6] == pytest.approx(t[2], rel=1e-14)


@pytest.mark.parametrize("theta", [0.3, 1.1, -0.7, 2.5])
def test_anisotropic_about_optical_axis(theta):
    """q = (cos th/2, 0, 0, sin th/2) is a rotation by th about z; on the axis
    Sigma2D = (f/z)^2 Rz diag(s1^2, s2^2) Rz^T + 0.3 I."""
    s = np.array([0.05, 0.012, 0.03])
    z = 2.0
    q = (math.cos(theta / 2), 0, 0, math.sin(theta / 2))
    c = cam()
    r = proj1(one((0, 0, z), np.log(s), q), c)
    f = float(np.float32(c.fx))
    co, si = math.cos(theta), math.sin(theta)
    k = (f / z) ** 2
    exp_a = k * (s[0] ** 2 * co ** 2 + s[1] ** 2 * si ** 2) + 0.3
    exp_b = k * (s[0] ** 2 - s[1] ** 2) * co * si
    exp_c = k * (s[0] ** 2 * si ** 2 + s[1] ** 2 * co ** 2) + 0.3
    np.testing.assert_allclose(r["cov"], [exp_a, exp_b, exp_c], rtol=1e-12,
                               atol=1e-14)


@pytest.mark.parametrize("theta", [0.4, -1.2])
def test_anisotropic_about_x_axis(theta):
    """q = (cos th/2, sin th/2, 0, 0): on the axis only the image-plane block
    of Rx diag(s^2) Rx^T is seen: diag(s1^2, cos^2 s2^2 + sin^2 s3^2)."""
    s = np.array([0.02, 0.05, 0.011])
    z = 1.7
    q = (math.cos(theta / 2), math.sin(theta / 2), 0, 0)
    c = cam()
    r = proj1(one((0, 0, z), np.log(s), q), c)
    f = float(np.float32(c.fx))
    k = (f / z) ** 2
    co, si = math.cos(theta), math.sin(theta)
    np.testing.assert_allclose(
        r["cov"], [k * s[0] ** 2 + 0.3, 0.0,
                   k * (co ** 2 * s[1] ** 2 + si ** 2 * s[2] ** 2) + 0.3],
        rtol=1e-12, atol=1e-12)


def test_quaternion_sign_and_scale_invariance():
    w = synth.tiny_scene(3, n=30)
    c = w.cameras[0]
    p = oracle.params64(w.gaussians)
    base = oracle.project(p, [c], 8, publish=True)
    neg = dict(p, quat=-p["quat"])
    sc = dict(p, quat=3.7 * p["quat"])
    on = oracle.project(neg, [c], 8, publish=True)
    os_ = oracle.project(sc, [c], 8, publish=True)
    np.testing.assert_array_equal(on["rec"], base["rec"])
    np.testing.assert_array_equal(on["box"], base["box"])
    np.testing.assert_allclose(os_["cov"], base["cov"], rtol=1e-13)


def test_isotropic_rotation_invariance():
    rng = np.random.default_rng(5)
    c = cam()
    for _ in range(10):
        mu = (rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(1, 4))
        l = rng.uniform(-3, -1)
        r1 = proj1(one(mu, (l, l, l), rng.normal(size=4)), c)
        r2 = proj1(one(mu, (l, l, l), rng.normal(size=4)), c)
        np.testing.assert_allclose(r1["cov"], r2["cov"], rtol=1e-12, atol=1e-13)


def test_conic_inverts_covariance():
    w = synth.config0()
    p = oracle.params64(w.gaussians)
    out = oracle.project(p, w.cameras, 16, publish=False)
    keep = out["tiles"][0] > 0
    a, b, c = out["cov"][0, keep].T
    A, B, C = out["rec"][0, keep, 2:5].T
    np.testing.assert_allclose(a * A + b * B, 1.0, atol=1e-12)
    np.testing.assert_allclose(a * B + b * C, 0.0, atol=1e-12)
    np.testing.assert_allclose(b * B + c * C, 1.0, atol=1e-12)


def test_near_plane_and_nonfinite_cull():
    c = cam()
    assert proj1(one((0, 0, 0.2), (-3, -3, -3)), c)["tiles"] == 0
    assert proj1(one((0, 0, 0.1), (-3, -3, -3)), c)["tiles"] == 0
    assert proj1(one((0, 0, 0.25), (-3, -3, -3)), c)["tiles"] > 0
    assert proj1(one((np.nan, 0, 2.0), (-3, -3, -3)), c)["tiles"] == 0
    assert proj1(one((0, 0, 2.0), (np.inf, -3, -3)), c)["tiles"] == 0
    assert proj1(one((0, 0, 2.0), (-3, -3, -3), (0, 0, 0, 0)), c)["tiles"] == 0
    # Far outside the image: empty box.
    assert proj1(one((50.0, 0, 2.0), (-3, -3, -3)), c)["tiles"] == 0


def test_fov_clamp_of_jacobian():
    """A large Gaussian whose mean is far off to the side: the Jacobian uses
    the clamped x = 1.3 * W / (2 fx) * z."""
    c = cam(W=101, H=81, f=50.0)
    z = 2.0
    limx = 1.3 * (101 / (2 * 50.0))
    x = 2.0 * limx * z
    l = math.log(3.0)
    r = proj1(one((x, 0, z), (l, l, l)), c)
    assert r["tiles"] > 0
    f = 50.0
    J = np.array([[f / z, 0, -f * (limx * z) / z ** 2], [0, f / z, 0]])
    S2 = 9.0 * J @ J.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(r["cov"], [S2[0, 0], S2[0, 1], S2[1, 1]],
                               rtol=1e-12)


def test_box_and_tile_count_against_tile_scan():
    w = synth.config0()
    p = oracle.params64(w.gaussians)
    c = w.cameras[0]
    for tile in (8, 16, 32):
        out = oracle.project(p, [c], tile, publish=True)
        Tx, Ty = -(-c.width // tile), -(-c.height // tile)
        tx = np.arange(Tx)
        ty = np.arange(Ty)
        for g in range(0, p["mean"].shape[1], 97):
            b = out["box"][0, g]
            if out["tiles"][0, g] == 0:
                continue
            # A tile is touched when its pixel rectangle meets the box.
            hx = (tx * tile <= b[1]) & (np.minimum(tx * tile + tile - 1, c.width - 1) >= b[0])
            hy = (ty * tile <= b[3]) & (np.minimum(ty * tile + tile - 1, c.height - 1) >= b[2])
            assert out["tiles"][0, g] == hx.sum() * hy.sum()
            px, r = out["rec"][0, g, 0], out["rec"][0, g, 7]
            # Every pixel within the radius of the mean (in x) lies in the box.
            us = np.arange(c.width)
            inside = (np.abs(us - np.float64(np.float32(px))) <= r - 1e-3)
            assert np.all((us[inside] >= b[0]) & (us[inside] <= b[1]))


def test_publish_rounds_to_fp32():
    w = synth.config0()
    p = oracle.params64(w.gaussians)
    exact = oracle.project(p, w.cameras, 16, publish=False)
    pub = oracle.project(p, w.cameras, 16, publish=True)
    np.testing.assert_array_equal(pub["rec"][..., :7],
                                  exact["rec"][..., :7].astype(np.float32))
    np.testing.assert_array_equal(pub["box"], exact["box"])
