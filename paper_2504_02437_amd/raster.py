"""Python surface of the rasterizer: device buffers, workspaces and the calls
of the C ABI under the same names, plus a torch.autograd.Function.

PyTorch is used for device memory and streams only.  Every computation runs
in libgsmap's HIP kernels; this module marshals pointers and sizes.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L

ROWS = {"mean": (0, 3), "log_scale": (3, 6), "quat": (6, 10),
        "opacity_logit": (10, 11), "rgb": (11, 14)}
ALPHA_MIN = float(np.float32(1.0) / np.float32(255.0))
T_MIN = float(np.float32(1e-4))
ALPHA_MAX = float(np.float32(0.99))


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _require_cuda(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def sh_rows(degree: int) -> int:
    """Rows of view-dependent colour coefficients for a degree (0..3)."""
    return 3 * ((degree + 1) ** 2 - 1)


class ParamBuffer:
    """Gaussian parameters (or gradients / optimiser moments of the same
    layout) as one FP32 device tensor [14 + sh_rows(sh_degree)][capacity]
    whose rows are mean 0-2, log_scale 3-5, quat 6-9 (w, x, y, z),
    opacity_logit 10, rgb 11-13 and, from row 14, the view-dependent colour
    coefficients (row 14 + 3 (j - 1) + c: coefficient j of channel c), plus a
    device int32 live count."""

    def __init__(self, capacity: int, device="cuda", n: int = 0, data=None,
                 n_dev=None, sh_degree: int = 0):
        if not 0 <= sh_degree <= 3:
            raise ValueError("sh_degree must be 0..3")
        self.capacity = int(capacity)
        self.sh_degree = int(sh_degree)
        rows = 14 + sh_rows(self.sh_degree)
        self.data = (torch.zeros(rows, self.capacity, dtype=torch.float32,
                                 device=device) if data is None else data)
        assert self.data.shape == (rows, self.capacity)
        self.n_dev = (torch.tensor([n], dtype=torch.int32, device=device)
                      if n_dev is None else n_dev)

    @classmethod
    def from_gaussians(cls, g, capacity=None, device="cuda"):
        n = g.n
        cap = n if capacity is None else int(capacity)
        if cap < n:
            raise ValueError("capacity below the Gaussian count")
        D = getattr(g, "sh_degree", 0)
        host = np.zeros((14 + sh_rows(D), cap), np.float32)
        host[0:3, :n] = g.mean
        host[3:6, :n] = g.log_scale
        host[6:10, :n] = g.quat
        host[10, :n] = g.opacity_logit
        host[11:14, :n] = g.rgb
        if D:
            host[14:, :n] = np.asarray(g.sh, np.float32).reshape(-1, n)
        return cls(cap, device, n, torch.from_numpy(host).to(device),
                   sh_degree=D)

    def zeros_like(self, share_count=True):
        return ParamBuffer(self.capacity, self.data.device,
                           data=torch.zeros_like(self.data),
                           n_dev=self.n_dev if share_count else None,
                           sh_degree=self.sh_degree)

    def row(self, name):
        if name == "sh":
            return self.data[14:]
        a, b = ROWS[name]
        return self.data[a:b]

    def n(self) -> int:
        return int(self.n_dev.item())

    def struct(self) -> L.gs_params:
        base = self.data.data_ptr()
        stride = self.capacity * 4
        return L.gs_params(base + 0 * stride, base + 3 * stride,
                           base + 6 * stride, base + 10 * stride,
                           base + 11 * stride, self.n_dev.data_ptr(),
                           self.capacity, self.sh_degree,
                           base + 14 * stride if self.sh_degree else 0)

    def to_numpy(self):
        """Live rows as numpy; "sh" is [K-1][3][n] when sh_degree > 0."""
        n = self.n()
        h = self.data[:, :n].cpu().numpy()
        out = {k: (h[a:b] if b - a > 1 else h[a]) for k, (a, b) in ROWS.items()}
        if self.sh_degree:
            out["sh"] = h[14:].reshape(-1, 3, n)
        return out


def camera_struct(cam) -> L.gs_camera:
    c = L.gs_camera()
    c.R[:] = [float(x) for x in np.asarray(cam.R, np.float32).ravel()]
    c.t[:] = [float(x) for x in np.asarray(cam.t, np.float32).ravel()]
    c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
    c.near_z = getattr(cam, "near", 0.2)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def cameras_to_device(cams, device="cuda") -> torch.Tensor:
    """gs_camera[V] packed into a device uint8 tensor."""
    arr = (L.gs_camera * len(cams))(*[camera_struct(c) for c in cams])
    host = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
    return torch.from_numpy(host).to(device)


@dataclass
class Settings:
    tile: int = 16
    lds_batch: int = 256
    bg: tuple = (0.0, 0.0, 0.0)
    alpha_min: float = ALPHA_MIN
    T_min: float = T_MIN
    alpha_max: float = ALPHA_MAX
    emit_keys: bool = False
    block_threads: int = 0
    full_box: bool = False   # render whole integer boxes (no render-box cut)

    def struct(self) -> L.gs_settings:
        s = L.gs_settings()
        s.tile, s.lds_batch = self.tile, self.lds_batch
        s.bg[:] = list(self.bg)
        s.alpha_min, s.T_min, s.alpha_max = (self.alpha_min, self.T_min,
                                             self.alpha_max)
        s.flags = ((L.GS_FLAG_EMIT_KEYS if self.emit_keys else 0) |
                   (L.GS_FLAG_FULL_BOX if self.full_box else 0))
        s.block_threads = self.block_threads
        return s


class Workspace:
    """A caller-owned device buffer carved by the library for one geometry."""

    def __init__(self, n_views, width, height, tile, capacity, key_capacity,
                 device="cuda", stream=None):
        self.geo = L.gs_geometry(n_views, width, height, tile, capacity, 0,
                                 int(key_capacity))
        size = C.c_size_t()
        L.call("gs_workspace_size", C.byref(self.geo), C.byref(size))
        self.bytes = size.value
        self.buf = torch.empty(self.bytes + 256, dtype=torch.uint8, device=device)
        off = (-self.buf.data_ptr()) % 256
        self.base = self.buf.data_ptr() + off
        self.handle = C.c_void_p()
        L.call("gs_workspace_create", C.byref(self.geo), C.c_void_p(self.base),
               C.c_size_t(self.bytes), _stream(stream), C.byref(self.handle))
        v = L.gs_workspace_view()
        L.call("gs_workspace_get_view", self.handle, C.byref(v))
        self.view = v
        self.tiles_x, self.tiles_y = v.tiles_x, v.tiles_y
        self.generation = 0

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                L.lib().gs_workspace_destroy(h)
            except Exception:
                pass
            self.handle = None

    def _slice(self, ptr, dtype, count):
        start = ptr - self.buf.data_ptr()
        nbytes = count * torch.tensor([], dtype=dtype).element_size()
        return self.buf[start:start + nbytes].view(dtype)

    @property
    def n_tiles(self):
        return self.geo.n_views * self.tiles_x * self.tiles_y

    def records(self):
        """[V][capacity][12] float32 view of the projected records."""
        V, cap = self.geo.n_views, self.geo.capacity
        return self._slice(self.view.records, torch.float32, V * cap * 12).view(
            V, cap, 12)

    def tiles_touched(self):
        V, cap = self.geo.n_views, self.geo.capacity
        return self._slice(self.view.tiles_touched, torch.int32, V * cap).view(V, cap)

    def render_box(self):
        """[V][capacity][2] int32 packed render boxes."""
        V, cap = self.geo.n_views, self.geo.capacity
        return self._slice(self.view.render_box, torch.int32, V * cap * 2).view(
            V, cap, 2)

    def ranges(self):
        return self._slice(self.view.ranges, torch.int32, self.n_tiles * 2).view(
            self.n_tiles, 2)

    def vals_sorted(self, n):
        return self._slice(self.view.vals_sorted, torch.int32, n)

    def keys_sorted(self, n):
        return self._slice(self.view.keys_sorted, torch.int64, n)

    def grad2d(self):
        V, cap = self.geo.n_views, self.geo.capacity
        return self._slice(self.view.grad2d, torch.float32, V * 5 * cap).view(
            V, 5, cap)

    def grad_opacity(self):
        return self._slice(self.view.grad_opacity, torch.float32,
                           self.geo.capacity)

    def grad_colour(self):
        V, cap = self.geo.n_views, self.geo.capacity
        return self._slice(self.view.grad_colour, torch.float32,
                           V * 3 * cap).view(V, 3, cap)


# ---- The C ABI under its own names ---------------------------------------

def project_and_bin(ws, params, cams_dev, settings, stream=None):
    L.call("gs_project_and_bin", ws.handle, C.byref(params.struct()),
           _ptr(cams_dev), C.byref(settings.struct()), _stream(stream))
    ws.generation += 1


def sort_tile_keys(ws, settings, stream=None):
    L.call("gs_sort_tile_keys", ws.handle, C.byref(settings.struct()),
           _stream(stream))


def render_fwd(ws, params, settings, out_rgb, out_T, out_nlast, stream=None):
    for t, nm in ((out_rgb, "out_rgb"), (out_T, "out_T"), (out_nlast, "out_nlast")):
        _require_cuda(t, nm)
    V, H, W = ws.geo.n_views, ws.geo.height, ws.geo.width
    if out_rgb.numel() != V * 3 * H * W or out_T.numel() != V * H * W or \
            out_nlast.numel() != V * H * W:
        raise ValueError("output sizes do not match the workspace geometry")
    if out_rgb.dtype != torch.float32 or out_T.dtype != torch.float32 or \
            out_nlast.dtype != torch.int32:
        raise ValueError("outputs must be float32, float32, int32")
    L.call("gs_render_fwd", ws.handle, C.byref(params.struct()),
           C.byref(settings.struct()), _ptr(out_rgb), _ptr(out_T),
           _ptr(out_nlast), _stream(stream))


def render_dominant(ws, params, settings, out_rgb, out_T, out_nlast, out_dom,
                    stream=None):
    """render_fwd that also writes each pixel's dominant Gaussian (Eq. 8)."""
    for t, nm in ((out_rgb, "out_rgb"), (out_T, "out_T"),
                  (out_nlast, "out_nlast"), (out_dom, "out_dom")):
        _require_cuda(t, nm)
    V, H, W = ws.geo.n_views, ws.geo.height, ws.geo.width
    if out_dom.numel() != V * H * W or out_dom.dtype != torch.int32:
        raise ValueError("out_dom must be int32 [V][H][W]")
    L.call("gs_render_dominant", ws.handle, C.byref(params.struct()),
           C.byref(settings.struct()), _ptr(out_rgb), _ptr(out_T),
           _ptr(out_nlast), _ptr(out_dom), _stream(stream))


def densify_scratch(capacity, device="cuda"):
    return torch.empty(capacity + (capacity + 1023) // 1024 + 4,
                       dtype=torch.int32, device=device)


def densify(params, m, v, dom, sigma, xi, scratch=None, n_split=None,
            status=None, stream=None):
    """Splits the Gaussians dominating more than sigma pixels of dom (Eq. 9).
    xi: [capacity][2][3] float32 standard-normal draws.  Returns the scratch
    buffer (its first `capacity` entries hold the dominated-pixel counts)."""
    _require_cuda(dom, "dom")
    if dom.dtype != torch.int32:
        raise ValueError("dom must be int32")
    cap = params.capacity
    if xi.shape != (cap, 2, 3) or xi.dtype != torch.float32 or not xi.is_contiguous():
        raise ValueError("xi must be contiguous float32 [capacity][2][3]")
    if scratch is None:
        scratch = densify_scratch(cap, params.data.device)
    L.call("gs_densify", C.byref(params.struct()),
           C.byref(m.struct()) if m is not None else None,
           C.byref(v.struct()) if v is not None else None, _ptr(dom),
           int(dom.numel()), int(sigma), _ptr(xi), _ptr(scratch),
           _ptr(n_split), _ptr(status), _stream(stream))
    return scratch


def count_pairs(ws, params, settings, counts_dev, stream=None):
    """Adds (examined, in-box, contributing, revisited) pair counts of the
    forward walk to counts_dev (int64[4] device tensor)."""
    if counts_dev.dtype != torch.int64 or counts_dev.numel() < 4:
        raise ValueError("counts_dev must be an int64 tensor of 4 elements")
    L.call("gs_count_pairs", ws.handle, C.byref(params.struct()),
           C.byref(settings.struct()), _ptr(counts_dev), _stream(stream))


def render_bwd(ws, params, cams_dev, settings, dL_drgb, T_final, n_last, grad,
               stream=None):
    """The whole backward: gs_render_bwd (pixel pass) then gs_project_bwd."""
    render_bwd_pixels(ws, params, settings, dL_drgb, T_final, n_last, grad,
                      stream)
    project_bwd(ws, params, cams_dev, grad, stream)


def render_bwd_pixels(ws, params, settings, dL_drgb, T_final, n_last, grad,
                      stream=None):
    V, H, W = ws.geo.n_views, ws.geo.height, ws.geo.width
    for t, nm, cnt in ((dL_drgb, "dL_drgb", V * 3 * H * W),
                       (T_final, "T_final", V * H * W),
                       (n_last, "n_last", V * H * W)):
        _require_cuda(t, nm)
        if t.numel() != cnt:
            raise ValueError(f"{nm} size does not match the workspace geometry")
    L.call("gs_render_bwd", ws.handle, C.byref(params.struct()),
           C.byref(settings.struct()), _ptr(dL_drgb), _ptr(T_final),
           _ptr(n_last), C.byref(grad.struct()), _stream(stream))


def render_bwd_l1(ws, params, settings, rgb, target, lam, T_final, n_last,
                  grad, loss_dev, sqerr_dev=None, stream=None):
    """gs_render_bwd_l1: the compositing backward with the L1 term fused in
    (dL/dC formed per pixel from the forward's image and the target; the
    loss is added to loss_dev)."""
    V, H, W = ws.geo.n_views, ws.geo.height, ws.geo.width
    for t, nm, cnt in ((rgb, "rgb", V * 3 * H * W), (target, "target", V * 3 * H * W),
                       (T_final, "T_final", V * H * W),
                       (n_last, "n_last", V * H * W)):
        _require_cuda(t, nm)
        if t.numel() != cnt:
            raise ValueError(f"{nm} size does not match the workspace geometry")
    if loss_dev.dtype != torch.float64:
        raise ValueError("loss_dev must be float64")
    L.call("gs_render_bwd_l1", ws.handle, C.byref(params.struct()),
           C.byref(settings.struct()), _ptr(rgb), _ptr(target), float(lam),
           _ptr(T_final), _ptr(n_last), C.byref(grad.struct()),
           _ptr(loss_dev), _ptr(sqerr_dev), _stream(stream))


def project_bwd(ws, params, cams_dev, grad, stream=None):
    L.call("gs_project_bwd", ws.handle, C.byref(params.struct()),
           _ptr(cams_dev), C.byref(grad.struct()), _stream(stream))


def loss_l1(rgb, target, lam, dL_drgb, loss_dev, sqerr_dev=None, stream=None):
    V, _, H, W = rgb.shape
    for t, nm in ((rgb, "rgb"), (target, "target"), (dL_drgb, "dL_drgb")):
        _require_cuda(t, nm)
        if t.shape != rgb.shape or t.dtype != torch.float32:
            raise ValueError(f"{nm} must be float32 of shape {tuple(rgb.shape)}")
    if loss_dev.dtype != torch.float64:
        raise ValueError("loss_dev must be float64")
    L.call("gs_loss_l1", _ptr(rgb), _ptr(target), V, H, W, float(lam),
           _ptr(dL_drgb), _ptr(loss_dev), _ptr(sqerr_dev), _stream(stream))


def loss_colour(rgb, target, lam_l1, lam_ssim, dL_drgb, loss_dev,
                sqerr_dev=None, ssim_dev=None, scratch=None, stream=None):
    """gs_loss_colour: lam_l1 * L1 + lam_ssim * (1 - SSIM), gradient written
    to dL_drgb.  Returns the scratch buffer."""
    V, _, H, W = rgb.shape
    for t, nm in ((rgb, "rgb"), (target, "target"), (dL_drgb, "dL_drgb")):
        _require_cuda(t, nm)
        if t.shape != rgb.shape or t.dtype != torch.float32:
            raise ValueError(f"{nm} must be float32 of shape {tuple(rgb.shape)}")
    if scratch is None:
        scratch = ssim_scratch(rgb)
    L.call("gs_loss_colour", _ptr(rgb), _ptr(target), V, H, W, float(lam_l1),
           float(lam_ssim), _ptr(dL_drgb), _ptr(loss_dev), _ptr(sqerr_dev),
           _ptr(ssim_dev), _ptr(scratch), _stream(stream))
    return scratch


def ssim_scratch(rgb):
    """Scratch buffer gs_loss_ssim needs for images shaped like `rgb`."""
    return torch.empty((3,) + tuple(rgb.shape), dtype=torch.float32,
                       device=rgb.device)


def loss_ssim(rgb, target, lam, dL_drgb, loss_dev, ssim_dev=None, scratch=None,
              stream=None):
    """ADDS lam * sum_views (1 - mean SSIM) to loss_dev and its gradient to
    dL_drgb (after loss_l1, which writes dL_drgb)."""
    V, _, H, W = rgb.shape
    for t, nm in ((rgb, "rgb"), (target, "target"), (dL_drgb, "dL_drgb")):
        _require_cuda(t, nm)
        if t.shape != rgb.shape or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"{nm} must be contiguous float32 of shape {tuple(rgb.shape)}")
    if loss_dev.dtype != torch.float64:
        raise ValueError("loss_dev must be float64")
    if scratch is None:
        scratch = ssim_scratch(rgb)
    if scratch.numel() < 3 * rgb.numel() or scratch.dtype != torch.float32:
        raise ValueError("scratch must hold 3 * rgb.numel() float32")
    L.call("gs_loss_ssim", _ptr(rgb), _ptr(target), V, H, W, float(lam),
           _ptr(dL_drgb), _ptr(loss_dev), _ptr(ssim_dev), _ptr(scratch),
           _stream(stream))


def planar_reg(params, lam, floor, grad, loss_dev, stream=None):
    L.call("gs_planar_reg", C.byref(params.struct()), float(lam), float(floor),
           C.byref(grad.struct()), _ptr(loss_dev), _stream(stream))


def adam(params, grad, m, v, lr, beta1, beta2, eps, step, stream=None):
    """Adam step; `step` is an int, or an int32 device tensor holding the
    step count (read on the device, so graph replays see its current
    value).  lr: rates of mean, log_scale, quat, opacity_logit, rgb and,
    for view-dependent colour, the coefficients (default rgb's / 20)."""
    lr = [float(x) for x in lr]
    if len(lr) == 5:
        lr.append(lr[4] / 20.0)
    lr_arr = (C.c_float * 6)(*lr)
    if isinstance(step, torch.Tensor):
        if step.dtype != torch.int32 or not step.is_cuda:
            raise ValueError("a device step count must be an int32 device tensor")
        s_host, s_dev = 0, _ptr(step)
    else:
        s_host, s_dev = int(step), None
    L.call("gs_adam", C.byref(params.struct()), C.byref(grad.struct()),
           C.byref(m.struct()), C.byref(v.struct()), lr_arr, float(beta1),
           float(beta2), float(eps), s_host, s_dev, _stream(stream))


class WindowGraph:
    """One mapping iteration over a rasterizer's window captured as a HIP
    graph by the library (gs_window_build): clear grad / loss / sqerr,
    project and bin, sort, render, planar regulariser (lam_reg > 0 or
    floor given), backward with the fused L1 term, projection backward and,
    with m, v and step (an int32 device tensor), the Adam step that also
    advances step.  The graph keeps the buffers' addresses: keep them alive
    and rebuild after replacing any (for instance after fit_key_capacity
    rebuilt the workspace)."""

    def __init__(self, rast, params, grad, target, loss, lam_l1=1.0,
                 lam_reg=0.0, reg_floor=0.01, m=None, v=None, lr=None,
                 beta1=0.9, beta2=0.999, eps=1e-15, step=None, sqerr=None,
                 planar_reg=True, stream=None):
        _require_cuda(target, "target")
        _require_cuda(loss, "loss")
        if target.shape != rast.rgb.shape or target.dtype != torch.float32:
            raise ValueError("target must be float32 of the rendered shape")
        if loss.dtype != torch.float64 or loss.numel() < 1:
            raise ValueError("loss must be a float64 device tensor")
        if sqerr is not None and (sqerr.dtype != torch.float64 or
                                  sqerr.numel() < rast.V):
            raise ValueError("sqerr must hold n_views float64")
        d = L.gs_window_desc()
        d.ws = rast.ws.handle
        d.params = params.struct()
        d.cams = _ptr(rast.cams_dev)
        d.settings = rast.settings.struct()
        d.out_rgb, d.out_T, d.out_nlast = (_ptr(rast.rgb), _ptr(rast.T),
                                           _ptr(rast.nlast))
        d.target = _ptr(target)
        d.lambda_l1, d.lambda_reg, d.reg_floor = lam_l1, lam_reg, reg_floor
        d.loss_dev = _ptr(loss)
        d.sqerr_dev = _ptr(sqerr) if sqerr is not None else None
        d.grad = grad.struct()
        flags = L.GS_WINDOW_PLANAR_REG if planar_reg else 0
        if m is not None:
            if step is None or step.dtype != torch.int32 or not step.is_cuda:
                raise ValueError("the Adam step needs an int32 device step")
            lr = [float(x) for x in lr]
            if len(lr) == 5:
                lr.append(lr[4] / 20.0)
            d.adam_m, d.adam_v = m.struct(), v.struct()
            d.lr = (C.c_float * 6)(*lr)
            d.beta1, d.beta2, d.eps = beta1, beta2, eps
            d.step_dev = _ptr(step)
            flags |= L.GS_WINDOW_ADAM
        d.flags = flags
        self._keep = (rast, params, grad, target, loss, m, v, step, sqerr)
        self.handle = C.c_void_p()
        st = torch.cuda.current_stream() if stream is None else stream
        L.call("gs_window_build", C.byref(d), C.c_void_p(st.cuda_stream),
               C.byref(self.handle))

    def run(self, stream=None):
        st = torch.cuda.current_stream() if stream is None else stream
        L.call("gs_window_run", self.handle, C.c_void_p(st.cuda_stream))

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            L.lib().gs_window_destroy(h)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def insert_gaussians(params, m, v, cam_dev, width, height, kf_rgb, kf_T, pts,
                     alpha_skip=0.9, centre_only=False, mlp_out=None,
                     n_inserted_dev=None, status_dev=None, stream=None):
    n_pts = 0 if pts is None else pts.shape[0]
    L.call("gs_insert_gaussians", C.byref(params.struct()),
           C.byref(m.struct()) if m is not None else None,
           C.byref(v.struct()) if v is not None else None, _ptr(cam_dev),
           int(width), int(height), _ptr(kf_rgb), _ptr(kf_T), _ptr(pts), n_pts,
           float(alpha_skip), 1 if centre_only else 0, _ptr(mlp_out),
           _ptr(n_inserted_dev), _ptr(status_dev), _stream(stream))


def insert_distance(params, m, v, cam_dev, width, height, kf_rgb, pts, tau,
                    centre_only=False, mlp_out=None, scratch=None,
                    n_inserted_dev=None, status_dev=None, stream=None):
    """Insertion with the distance test of Eq. 7.  Returns the scratch
    tensor (int64 view of each candidate's nearest squared distance bits)."""
    n_pts = 0 if pts is None else pts.shape[0]
    C_ = n_pts * (1 if centre_only else 9)
    if scratch is None:
        scratch = torch.empty(max(C_, 1), dtype=torch.int64,
                              device=params.data.device)
    L.call("gs_insert_distance", C.byref(params.struct()),
           C.byref(m.struct()) if m is not None else None,
           C.byref(v.struct()) if v is not None else None, _ptr(cam_dev),
           int(width), int(height), _ptr(kf_rgb), _ptr(pts), n_pts,
           float(tau), 1 if centre_only else 0, _ptr(mlp_out), _ptr(scratch),
           _ptr(n_inserted_dev), _ptr(status_dev), _stream(stream))
    return scratch


def knn_features(params, cam_dev, width, height, kf_rgb, pts, centre_only,
                 feats, knn_idx=None, knn_dist=None, stream=None):
    n_pts = 0 if pts is None else pts.shape[0]
    L.call("gs_knn_features", C.byref(params.struct()), _ptr(cam_dev),
           int(width), int(height), _ptr(kf_rgb), _ptr(pts), n_pts,
           1 if centre_only else 0, _ptr(feats), _ptr(knn_idx),
           _ptr(knn_dist), _stream(stream))


def mlp_fwd(weights, x, y, cache=None, stream=None):
    L.call("gs_mlp_fwd", _ptr(weights), _ptr(x), int(x.shape[0]), _ptr(y),
           _ptr(cache), _stream(stream))


def mlp_mse(y, target, dy, loss_dev=None, stream=None):
    L.call("gs_mlp_mse", _ptr(y), _ptr(target), int(y.shape[0]), _ptr(dy),
           _ptr(loss_dev), _stream(stream))


def mlp_bwd(weights, x, cache, dy, dweights, stream=None):
    L.call("gs_mlp_bwd", _ptr(weights), _ptr(x), _ptr(cache), _ptr(dy),
           int(x.shape[0]), _ptr(dweights), _stream(stream))


def mlp_adam(weights, dweights, m, v, lr, beta1, beta2, eps, step,
             stream=None):
    L.call("gs_mlp_adam", _ptr(weights), _ptr(dweights), _ptr(m), _ptr(v),
           float(lr), float(beta1), float(beta2), float(eps), int(step),
           _stream(stream))


def read_status(ws, stream=None, clear=False):
    flags = C.c_int32()
    nk = C.c_int64()
    rc = L.lib().gs_read_status(ws.handle, _stream(stream), C.byref(flags),
                                C.byref(nk), 1 if clear else 0)
    if rc not in (L.GS_OK, L.GS_E_OVERFLOW):
        L.check(rc)
    return flags.value, nk.value


# ---- Convenience: one rasterizer over a fixed set of views ---------------

def default_key_capacity(capacity, n_views):
    return int(min(2 ** 31 - 1, max(1 << 20, 48 * capacity * n_views)))


class Rasterizer:
    """Project, bin, sort and render a ParamBuffer into a fixed set of views,
    holding the workspace and the per-pixel outputs of the last forward."""

    def __init__(self, cams, capacity, settings: Settings | None = None,
                 key_capacity=None, device="cuda"):
        self.settings = settings or Settings()
        self.cams = list(cams)
        self.V = len(self.cams)
        self.W, self.H = self.cams[0].width, self.cams[0].height
        for c in self.cams:
            if (c.width, c.height) != (self.W, self.H):
                raise ValueError("all views must share the image size")
        self.capacity = capacity
        kc = default_key_capacity(capacity, self.V) if key_capacity is None \
            else key_capacity
        self.ws = Workspace(self.V, self.W, self.H, self.settings.tile,
                            capacity, kc, device)
        self.cams_dev = cameras_to_device(self.cams, device)
        self.rgb = torch.empty(self.V, 3, self.H, self.W, device=device)
        self.T = torch.empty(self.V, self.H, self.W, device=device)
        self.nlast = torch.empty(self.V, self.H, self.W, dtype=torch.int32,
                                 device=device)
        # Bumped by every forward, camera change and workspace rebuild: a
        # backward checks it against the forward it belongs to.
        self.generation = 0

    def fit_key_capacity(self, params, margin=1.25, stream=None):
        """Projects and bins once; if the keys overflowed the workspace,
        rebuilds it with `margin` times the exact key count.  Returns the key
        count.  (Synchronises the stream.)"""
        project_and_bin(self.ws, params, self.cams_dev, self.settings, stream)
        flags, nk = read_status(self.ws, stream, clear=True)
        if flags & L.GS_STATUS_KEY_OVERFLOW:
            cap = int(min(2 ** 31 - 1, max(1024, int(nk * margin))))
            if nk > cap:
                raise RuntimeError(f"{nk} keys exceed the 2^31 limit")
            self.ws = None
            torch.cuda.empty_cache()
            self.ws = Workspace(self.V, self.W, self.H, self.settings.tile,
                                self.capacity, cap, self.rgb.device)
        self.generation += 1
        return nk

    def set_cameras(self, cams):
        if len(cams) != self.V:
            raise ValueError("view count is fixed per rasterizer")
        self.cams = list(cams)
        self.cams_dev.copy_(cameras_to_device(cams, self.cams_dev.device))
        self.generation += 1

    def forward(self, params, stream=None):
        self.generation += 1
        project_and_bin(self.ws, params, self.cams_dev, self.settings, stream)
        sort_tile_keys(self.ws, self.settings, stream)
        render_fwd(self.ws, params, self.settings, self.rgb, self.T,
                   self.nlast, stream)
        return self.rgb, self.T, self.nlast

    def forward_dominant(self, params, stream=None):
        """forward() plus each pixel's dominant Gaussian (int32 [V][H][W])."""
        dom = torch.empty(self.T.shape, dtype=torch.int32, device=self.T.device)
        self.generation += 1
        project_and_bin(self.ws, params, self.cams_dev, self.settings, stream)
        sort_tile_keys(self.ws, self.settings, stream)
        render_dominant(self.ws, params, self.settings, self.rgb, self.T,
                        self.nlast, dom, stream)
        return dom

    def count_pairs(self, params, stream=None):
        """Work counters of the current sorted lists (run forward first)."""
        c = torch.zeros(4, dtype=torch.int64, device=self.rgb.device)
        count_pairs(self.ws, params, self.settings, c, stream)
        h = c.cpu().tolist()
        return dict(examined=h[0], inbox=h[1], contributing=h[2], revisit=h[3])

    def backward(self, params, dL_drgb, grad, stream=None):
        render_bwd(self.ws, params, self.cams_dev, self.settings,
                   dL_drgb.contiguous(), self.T, self.nlast, grad, stream)

    def backward_l1(self, params, target, lam, grad, loss_dev, sqerr_dev=None,
                    stream=None):
        """The whole backward of the L1 photometric term of the last forward
        (fused into the compositing backward) plus the projection backward;
        adds the loss to loss_dev."""
        render_bwd_l1(self.ws, params, self.settings, self.rgb,
                      target.contiguous(), lam, self.T, self.nlast, grad,
                      loss_dev, sqerr_dev, stream)
        project_bwd(self.ws, params, self.cams_dev, grad, stream)

    def status(self, clear=False):
        return read_status(self.ws, None, clear)


class Rasterize(torch.autograd.Function):
    """Differentiable render: forward keeps only per-pixel state (T_final,
    n_last) and the sorted tile lists; backward recomputes each entry's
    transmittance inside render_bwd."""

    @staticmethod
    def forward(ctx, data, rast: Rasterizer, params: ParamBuffer):
        if data.data_ptr() != params.data.data_ptr():
            raise ValueError("data must be params.data")
        rgb, T, nlast = rast.forward(params)
        # Truncated tile lists would give a wrong image and wrong gradients:
        # on a key overflow, refit the workspace to the exact count and
        # render again (this reads the status word: one stream sync).
        flags, _ = rast.status()
        if flags & L.GS_STATUS_KEY_OVERFLOW:
            rast.fit_key_capacity(params)
            rgb, T, nlast = rast.forward(params)
            flags, _ = rast.status()
            if flags & L.GS_STATUS_KEY_OVERFLOW:
                raise RuntimeError("key capacity exceeded after refitting")
        if flags:
            raise RuntimeError(f"device status {flags} after the forward")
        ctx.rast = rast
        ctx.params = params
        ctx.generation = rast.generation
        ctx.ws, ctx.ws_generation = rast.ws, rast.ws.generation
        ctx.mark_non_differentiable(T, nlast)
        return rgb.clone(), T.clone(), nlast.clone()

    @staticmethod
    def backward(ctx, g_rgb, g_T, g_nlast):
        rast, params = ctx.rast, ctx.params
        if rast.generation != ctx.generation or rast.ws is not ctx.ws or \
                rast.ws.generation != ctx.ws_generation:
            raise RuntimeError("another forward ran on this rasterizer before "
                               "the backward of this one")
        grad = params.zeros_like()
        if g_rgb is None:
            g_rgb = torch.zeros_like(rast.rgb)
        rast.backward(params, g_rgb.contiguous(), grad)
        return grad.data, None, None
