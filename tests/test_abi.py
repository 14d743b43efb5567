"""CPU-side checks of the C ABI: the library loads, exports every function
the header declares, and rejects bad arguments on the host before touching a
GPU."""
import ctypes as C

import pytest

from paper_2504_02437_amd import _lib as L


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = L.declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(L._SIGS) == set(names)


def test_version_and_no_error():
    assert L.lib().gs_version().startswith(b"gsmap")
    assert L.lib().gs_last_error() is not None


def _geo(**kw):
    d = dict(n_views=2, width=100, height=60, tile=16, capacity=1000,
             key_capacity=50000)
    d.update(kw)
    return L.gs_geometry(d["n_views"], d["width"], d["height"], d["tile"],
                         d["capacity"], 0, d["key_capacity"])


def test_workspace_size_host_only():
    size = C.c_size_t()
    assert L.lib().gs_workspace_size(C.byref(_geo()), C.byref(size)) == L.GS_OK
    # records 48 B + tiles 4 B per (view, Gaussian); 20 B per key; grad2d.
    assert size.value >= 2 * 1000 * 52 + 50000 * 20 + 2 * 5 * 1000 * 4
    big = C.c_size_t()
    L.lib().gs_workspace_size(C.byref(_geo(key_capacity=100000)), C.byref(big))
    assert big.value - size.value >= 50000 * 20 - 4 * 256


@pytest.mark.parametrize("kw", [dict(tile=12), dict(n_views=0), dict(width=0),
                                dict(height=20000), dict(capacity=-1),
                                dict(key_capacity=2 ** 31)])
def test_workspace_size_rejects_bad_geometry(kw):
    size = C.c_size_t()
    rc = L.lib().gs_workspace_size(C.byref(_geo(**kw)), C.byref(size))
    assert rc == L.GS_E_INVALID
    assert L.lib().gs_last_error() != b""


def test_calls_reject_null_workspace_without_launching():
    lib = L.lib()
    s = L.gs_settings(16, 256)
    p = L.gs_params()
    assert lib.gs_project_and_bin(None, C.byref(p), None, C.byref(s), None) == L.GS_E_INVALID
    assert lib.gs_sort_tile_keys(None, C.byref(s), None) == L.GS_E_INVALID
    assert lib.gs_render_fwd(None, C.byref(p), C.byref(s), None, None, None,
                             None) == L.GS_E_INVALID
    assert lib.gs_render_bwd(None, C.byref(p), C.byref(s), None, None, None,
                             C.byref(p), None) == L.GS_E_INVALID
    assert lib.gs_project_bwd(None, C.byref(p), None, C.byref(p),
                              None) == L.GS_E_INVALID
    c = (C.c_uint64 * 4)()
    assert lib.gs_count_pairs(None, C.byref(p), C.byref(s), c,
                              None) == L.GS_E_INVALID
    assert lib.gs_read_status(None, None, None, None, 0) == L.GS_E_INVALID


def test_settings_validation():
    lib = L.lib()
    p = L.gs_params()
    good = dict(tile=16, lds_batch=256, alpha_min=1 / 255, T_min=1e-4,
                alpha_max=0.99)
    for bad in (dict(tile=24), dict(lds_batch=300), dict(alpha_min=0.0),
                dict(alpha_max=1.0), dict(T_min=0.0)):
        d = dict(good, **bad)
        s = L.gs_settings(d["tile"], d["lds_batch"])
        s.alpha_min, s.T_min, s.alpha_max = d["alpha_min"], d["T_min"], d["alpha_max"]
        # NULL params are reported first, so pass a fake non-null row set.
        p.mean = p.log_scale = p.quat = p.opacity_logit = p.rgb = 16
        assert lib.gs_loss_l1(None, None, 1, 1, 1, 1.0, None, None, None,
                              None) == L.GS_E_INVALID
        ws = C.c_void_p(0)
        assert lib.gs_sort_tile_keys(ws, C.byref(s), None) == L.GS_E_INVALID


def test_insert_and_adam_reject_bad_arguments():
    lib = L.lib()
    p = L.gs_params()
    lr = (C.c_float * 5)(1, 1, 1, 1, 1)
    assert lib.gs_adam(C.byref(p), C.byref(p), C.byref(p), C.byref(p), lr, 0.9,
                       0.999, 1e-15, 1, None, None) == L.GS_E_INVALID
    assert lib.gs_insert_gaussians(C.byref(p), None, None, None, 10, 10, None,
                                   None, None, 5, 0.9, 0, None, None, None,
                                   None) == L.GS_E_INVALID


def _fake_params(D=0, sh=True):
    p = L.gs_params()
    p.mean = p.log_scale = p.quat = p.opacity_logit = p.rgb = 256
    p.n_dev = 256
    p.capacity = 10
    p.sh_degree = D
    p.sh = 256 if (sh and D) else None
    return p


def test_view_dependent_colour_layout_is_checked_on_the_host():
    """sh_degree outside 0..3, a missing coefficient pointer and gradient or
    moment arrays whose degree differs from the parameters' are rejected
    before anything is launched."""
    lib = L.lib()
    lr = (C.c_float * 6)(1, 1, 1, 1, 1, 1)
    for bad in (_fake_params(4), _fake_params(-1), _fake_params(2, sh=False)):
        assert lib.gs_adam(C.byref(bad), C.byref(bad), C.byref(bad),
                           C.byref(bad), lr, 0.9, 0.999, 1e-15, 1, None,
                           None) == L.GS_E_INVALID
        assert b"sh" in lib.gs_last_error()
    p, q = _fake_params(3), _fake_params(2)
    assert lib.gs_adam(C.byref(p), C.byref(q), C.byref(p), C.byref(p), lr,
                       0.9, 0.999, 1e-15, 1, None, None) == L.GS_E_INVALID
    assert b"sh_degree" in lib.gs_last_error()
    assert lib.gs_adam(C.byref(p), C.byref(p), C.byref(p), C.byref(q), lr,
                       0.9, 0.999, 1e-15, 1, None, None) == L.GS_E_INVALID
    assert lib.gs_densify(C.byref(p), C.byref(q), None, None, 0, 1,
                          C.c_void_p(256), C.c_void_p(256), None, None,
                          None) == L.GS_E_INVALID
    assert b"sh_degree" in lib.gs_last_error()
    assert lib.gs_insert_gaussians(C.byref(p), C.byref(q), None,
                                   C.c_void_p(256), 10, 10, C.c_void_p(256),
                                   C.c_void_p(256), C.c_void_p(256), 5, 0.9, 0,
                                   None, None, None, None) == L.GS_E_INVALID
    assert b"sh_degree" in lib.gs_last_error()


def test_params_struct_layout():
    """gs_params: six pointers, capacity, sh_degree, coefficient pointer."""
    assert C.sizeof(L.gs_params) == 64
    assert L.gs_params.sh_degree.offset == 52 and L.gs_params.sh.offset == 56


def test_parameters_gradients_and_moments_must_not_share_memory():
    """A gradient or moment set that overlaps the parameters (or another such
    set) is rejected on the host: the kernels read one and write the other
    Gaussian by Gaussian."""
    lib = L.lib()
    lr = (C.c_float * 6)(1, 1, 1, 1, 1, 1)

    def rows(base, cap=10):
        q = L.gs_params()
        row = cap * 4
        q.mean, q.log_scale, q.quat = base, base + 3 * row, base + 6 * row
        q.opacity_logit, q.rgb = base + 10 * row, base + 11 * row
        q.n_dev, q.capacity = 1 << 20, cap
        return q

    p, g, m, v = rows(4096), rows(8192), rows(12288), rows(16384)
    overlap = rows(4096 + 40 * 5)      # starts inside p's log_scale rows
    cases = [(overlap, m, v), (g, overlap, v), (g, m, overlap), (g, m, m)]
    for gg, mm, vv in cases:
        assert lib.gs_adam(C.byref(p), C.byref(gg), C.byref(mm), C.byref(vv),
                           lr, 0.9, 0.999, 1e-15, 1, None,
                           None) == L.GS_E_INVALID
        assert b"share memory" in lib.gs_last_error()
    loss = C.c_void_p(1 << 20)
    assert lib.gs_planar_reg(C.byref(p), 1.0, 0.01, C.byref(p), loss,
                             None) == L.GS_E_INVALID
    assert b"share memory" in lib.gs_last_error()
    assert lib.gs_densify(C.byref(p), C.byref(overlap), None, None, 0, 1,
                          C.c_void_p(256), C.c_void_p(256), None, None,
                          None) == L.GS_E_INVALID
    assert b"share memory" in lib.gs_last_error()
    assert lib.gs_insert_gaussians(C.byref(p), C.byref(m), C.byref(m),
                                   C.c_void_p(256), 10, 10, C.c_void_p(256),
                                   C.c_void_p(256), C.c_void_p(256), 5, 0.9, 0,
                                   None, None, None, None) == L.GS_E_INVALID
    assert b"share memory" in lib.gs_last_error()


def test_window_build_rejects_bad_arguments_on_the_host():
    """gs_window_build checks its arguments before it touches the stream:
    NULL out / desc, the null stream and missing buffers are GS_E_INVALID,
    and out is cleared.  run and destroy of a NULL handle are safe."""
    lib = L.lib()
    d = L.gs_window_desc()
    h = C.c_void_p(1234)
    assert lib.gs_window_build(C.byref(d), C.c_void_p(8), None) == L.GS_E_INVALID
    assert lib.gs_window_build(None, C.c_void_p(8), C.byref(h)) == L.GS_E_INVALID
    assert h.value is None
    assert lib.gs_window_build(C.byref(d), None, C.byref(h)) == L.GS_E_INVALID
    assert b"null stream" in lib.gs_last_error()
    assert lib.gs_window_build(C.byref(d), C.c_void_p(8), C.byref(h)) == L.GS_E_INVALID
    assert b"required" in lib.gs_last_error()
    assert lib.gs_window_run(None, None) == L.GS_E_INVALID
    assert lib.gs_window_destroy(None) == L.GS_OK
