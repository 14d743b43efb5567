// One mapping iteration over a keyframe window as a HIP graph owned behind
// the C ABI (gs_window_build / gs_window_run / gs_window_destroy).
//
// The build captures, on the caller's stream, the same calls an eager
// iteration makes: clear the gradient, loss and squared-error buffers, then
// projection and binning, the per-tile sort, the forward render, the planar
// regulariser's gradient, the compositing backward with the L1 term fused
// in, the projection backward and the Adam step with its device step count
// advanced.  Clearing uses the library's fill kernels (no memset nodes), so
// every node of the graph is a kernel.  The graph holds the caller's device
// pointers; it owns no device memory of its own.

#include <new>

#include "gs_internal.h"

struct gs_window {
  hipGraphExec_t exec;
  int n_views;
};

namespace gs {
namespace {

__global__ void k_add_i32(int32_t* x, int32_t d) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *x += d;
}

size_t rows_of(const gs_params* p) {
  return p->sh_degree > 0 ? (size_t)GS_SH_ROWS(p->sh_degree) : 0;
}

hipError_t zero_rows(const gs_params* g, hipStream_t st) {
  const size_t c = (size_t)(g->capacity > 0 ? g->capacity : 0);
  float* rows[6] = {g->mean, g->log_scale, g->quat, g->opacity_logit, g->rgb,
                    g->sh};
  const size_t n[6] = {3, 3, 4, 1, 3, rows_of(g)};
  for (int i = 0; i < 6; ++i) {
    if (!rows[i] || n[i] == 0 || c == 0) continue;
    const hipError_t e = launch_fill_u32(rows[i], 0u, n[i] * c, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The iteration, enqueued on st (called while st captures).
int enqueue_iteration(const gs_window_desc* d, hipStream_t st) {
  gs_params params = d->params, grad = d->grad, m = d->adam_m, v = d->adam_v;
  int rc = check_hip(zero_rows(&grad, st), "clearing the gradient");
  if (rc) return rc;
  rc = check_hip(launch_fill_u32(d->loss_dev, 0u, 2, st), "clearing the loss");
  if (rc) return rc;
  if (d->sqerr_dev) {
    rc = check_hip(launch_fill_u32(d->sqerr_dev, 0u,
                                   2 * (size_t)d->ws->geo.n_views, st),
                   "clearing the squared errors");
    if (rc) return rc;
  }
  if ((rc = gs_project_and_bin(d->ws, &params, d->cams, &d->settings, st)))
    return rc;
  if ((rc = gs_sort_tile_keys(d->ws, &d->settings, st))) return rc;
  if ((rc = gs_render_fwd(d->ws, &params, &d->settings, d->out_rgb, d->out_T,
                          d->out_nlast, st)))
    return rc;
  if (d->flags & GS_WINDOW_PLANAR_REG) {
    if ((rc = gs_planar_reg(&params, d->lambda_reg, d->reg_floor, &grad,
                            d->loss_dev, st)))
      return rc;
  }
  if ((rc = gs_render_bwd_l1(d->ws, &params, &d->settings, d->out_rgb,
                             d->target, d->lambda_l1, d->out_T, d->out_nlast,
                             &grad, d->loss_dev, d->sqerr_dev, st)))
    return rc;
  if ((rc = gs_project_bwd(d->ws, &params, d->cams, &grad, st))) return rc;
  if (d->flags & GS_WINDOW_ADAM) {
    if ((rc = gs_adam(&params, &grad, &m, &v, d->lr, d->beta1, d->beta2,
                      d->eps, 1, d->step_dev, st)))
      return rc;
    hipLaunchKernelGGL(k_add_i32, dim3(1), dim3(64), 0, st, d->step_dev, 1);
    if ((rc = check_hip(hipGetLastError(), "advancing the step count")))
      return rc;
  }
  return GS_OK;
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" {

GS_API int gs_window_build(const gs_window_desc* d, void* stream,
                           gs_window** out) {
  if (!out) { set_error("out is NULL"); return GS_E_INVALID; }
  *out = nullptr;
  if (!d) { set_error("desc is NULL"); return GS_E_INVALID; }
  if (!stream) {
    set_error("a window graph is captured on a created stream, not the null "
              "stream");
    return GS_E_INVALID;
  }
  if (!d->ws || !d->cams || !d->out_rgb || !d->out_T || !d->out_nlast ||
      !d->target || !d->loss_dev) {
    set_error("window: ws, cams, outputs, target and loss_dev are required");
    return GS_E_INVALID;
  }
  int rc = validate_params(&d->params, "params");
  if (!rc) rc = validate_params(&d->grad, "grad");
  if (!rc) rc = validate_settings(&d->settings);
  if (rc) return rc;
  if (d->flags & ~(GS_WINDOW_PLANAR_REG | GS_WINDOW_ADAM)) {
    set_error("window: unknown flags 0x%x", d->flags);
    return GS_E_INVALID;
  }
  if (d->flags & GS_WINDOW_ADAM) {
    if (!d->step_dev) {
      set_error("window: GS_WINDOW_ADAM needs step_dev");
      return GS_E_INVALID;
    }
    if ((rc = validate_params(&d->adam_m, "adam_m")) ||
        (rc = validate_params(&d->adam_v, "adam_v")))
      return rc;
  }
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cs;
  if ((rc = check_hip(hipStreamIsCapturing(st, &cs), "hipStreamIsCapturing")))
    return rc;
  if (cs != hipStreamCaptureStatusNone) {
    set_error("window: the stream is already capturing");
    return GS_E_INVALID;
  }
  if ((rc = check_hip(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal),
                      "hipStreamBeginCapture")))
    return rc;
  // Every call below is host-checked before it launches anything; on an
  // error the capture is ended and discarded.
  const int rc_iter = enqueue_iteration(d, st);
  hipGraph_t graph = nullptr;
  const hipError_t e_end = hipStreamEndCapture(st, &graph);
  if (rc_iter) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc_iter;
  }
  if ((rc = check_hip(e_end, "hipStreamEndCapture"))) return rc;
  hipGraphExec_t exec = nullptr;
  rc = check_hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0),
                 "hipGraphInstantiate");
  (void)hipGraphDestroy(graph);
  if (rc) return rc;
  gs_window* w = new (std::nothrow) gs_window;
  if (!w) {
    (void)hipGraphExecDestroy(exec);
    set_error("window: out of host memory");
    return GS_E_INVALID;
  }
  w->exec = exec;
  w->n_views = d->ws->geo.n_views;
  *out = w;
  return GS_OK;
}

GS_API int gs_window_run(gs_window* w, void* stream) {
  if (!w || !w->exec) { set_error("window is NULL"); return GS_E_INVALID; }
  return check_hip(hipGraphLaunch(w->exec, (hipStream_t)stream),
                   "hipGraphLaunch");
}

GS_API int gs_window_destroy(gs_window* w) {
  if (!w) return GS_OK;
  int rc = GS_OK;
  if (w->exec) rc = check_hip(hipGraphExecDestroy(w->exec), "hipGraphExecDestroy");
  delete w;
  return rc;
}

}  // extern "C"
