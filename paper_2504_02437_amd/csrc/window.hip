// One mapping iteration over a keyframe window as a HIP graph owned behind
// the C ABI (gs_window_build / gs_window_run / gs_window_destroy).
//
// The build captures, on the caller's stream, the same calls an eager
// iteration makes: clear the gradient, loss and squared-error buffers (the
// same launch forms the per-Gaussian shapes of the projection), then
// projection and binning, the per-tile sort, the forward render, the
// compositing backward with the L1 term fused in (the planar regulariser's
// gradient in extra workgroups of the same launch), the projection backward
// (the L1 tile-loss sum in one extra workgroup) and the Adam step with its
// device step count advanced.  The clearing is one kernel of its own (no memset nodes), which
// also advances the step count, so every node of the graph is a kernel.  The
// graph holds the caller's device pointers; it owns no device memory of its
// own.

#include <new>

#include "gs_internal.h"
#include "shape.h"
#include "tails.h"

struct gs_window {
  hipGraphExec_t exec;
  int n_views;
};

namespace gs {
namespace {

size_t rows_of(const gs_params* p) {
  return p->sh_degree > 0 ? (size_t)GS_SH_ROWS(p->sh_degree) : 0;
}

// The iteration's clearing in one launch: up to kClearJobs 32-bit rows set
// to zero (the gradient rows, the loss and squared-error slots), workgroups
// dealt to the rows in turn, and the Adam step count advanced by one (its
// Adam launch reads the count minus one, so a run still uses the count it
// started with and leaves it advanced).
constexpr int kClearJobs = 8;
constexpr int kClearPer = 4;   // elements per thread
struct ClearArgs {
  uint32_t* p[kClearJobs];
  size_t n[kClearJobs];
  int first[kClearJobs + 1];   // first clearing workgroup of each row
  int jobs;
  int32_t* step;               // advanced by one when not NULL
  // The first shape_blocks workgroups form the per-Gaussian shapes of the
  // projection (256 Gaussians each) instead of clearing.
  int shape_blocks;
  ShapeJob shape;
  // Workgroup 0 also forms the views' FP64 camera constants.
  const gs_camera* cams;
  int V;
  double* camd;
};

__global__ __launch_bounds__(256) void k_clear_iteration(ClearArgs a) {
  if (a.step && blockIdx.x == 0 && threadIdx.x == 0) *a.step += 1;
  cam_d_fill(a.cams, a.V, a.camd);
  if ((int)blockIdx.x < a.shape_blocks) {
    shape_one(a.shape, (int)blockIdx.x * 256 + (int)threadIdx.x);
    return;
  }
  const int b = (int)blockIdx.x - a.shape_blocks;
  int j = 0;
  while (j + 1 < a.jobs && b >= a.first[j + 1]) ++j;
  uint32_t* p = a.p[j];
  const size_t n = a.n[j];
  const size_t base = (size_t)(b - a.first[j]) * 256 * kClearPer + threadIdx.x;
#pragma unroll
  for (int e = 0; e < kClearPer; ++e) {
    const size_t i = base + (size_t)e * 256;
    if (i < n) p[i] = 0u;
  }
}

hipError_t clear_iteration(const gs_window_desc* d, hipStream_t st) {
  const gs_params* g = &d->grad;
  const size_t c = (size_t)(g->capacity > 0 ? g->capacity : 0);
  ClearArgs a;
  a.jobs = 0;
  auto add = [&](void* ptr, size_t n) {
    if (!ptr || n == 0) return;
    a.p[a.jobs] = (uint32_t*)ptr;
    a.n[a.jobs] = n;
    ++a.jobs;
  };
  float* rows[6] = {g->mean, g->log_scale, g->quat, g->opacity_logit, g->rgb,
                    g->sh};
  const size_t nr[6] = {3, 3, 4, 1, 3, rows_of(g)};
  for (int i = 0; i < 6; ++i) add(rows[i], nr[i] * c);
  add(d->loss_dev, 2);
  if (d->sqerr_dev) add(d->sqerr_dev, 2 * (size_t)d->ws->geo.n_views);
  a.step = (d->flags & GS_WINDOW_ADAM) ? d->step_dev : nullptr;
  long long blocks = 0;
  for (int j = 0; j < a.jobs; ++j) {
    a.first[j] = (int)blocks;
    blocks += (long long)((a.n[j] + 256 * kClearPer - 1) / (256 * kClearPer));
    if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  }
  a.first[a.jobs] = (int)blocks;
  if (blocks == 0) {   // nothing to clear; the step count still advances
    a.jobs = 1; a.p[0] = nullptr; a.n[0] = 0; a.first[0] = 0; a.first[1] = 1;
    blocks = 1;
  }
  a.shape = shape_job(d->ws, &d->params);
  a.cams = d->cams;
  a.V = d->ws->geo.n_views;
  a.camd = d->ws->camd;
  a.shape_blocks = (d->params.capacity + 255) / 256;
  blocks += a.shape_blocks;
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_clear_iteration, dim3((unsigned)blocks), dim3(256), 0,
                     st, a);
  return hipGetLastError();
}

// The iteration, enqueued on st (called while st captures).
int enqueue_iteration(const gs_window_desc* d, hipStream_t st) {
  gs_params params = d->params, grad = d->grad, m = d->adam_m, v = d->adam_v;
  int rc = check_hip(clear_iteration(d, st), "clearing the iteration's rows");
  if (rc) return rc;
  // The clearing launch formed the per-Gaussian shapes already.
  if ((rc = project_and_bin_checked(d->ws, &params, d->cams, &d->settings, st,
                                    true)))
    return rc;
  if ((rc = gs_sort_tile_keys(d->ws, &d->settings, st))) return rc;
  if ((rc = gs_render_fwd(d->ws, &params, &d->settings, d->out_rgb, d->out_T,
                          d->out_nlast, st)))
    return rc;
  // The planar regulariser runs as extra workgroups of the compositing
  // backward, and the L1 tile losses are summed by one extra workgroup of the
  // projection backward: two launches fewer than calling the entry points.
  PlanarJob planar;
  const bool reg = (d->flags & GS_WINDOW_PLANAR_REG) != 0;
  if (reg && (rc = planar_checked(&params, d->lambda_reg, d->reg_floor, &grad,
                                  d->loss_dev, &planar)))
    return rc;
  if ((rc = render_bwd_l1_checked(d->ws, &params, &d->settings, d->out_rgb,
                                  d->target, d->lambda_l1, d->out_T,
                                  d->out_nlast, &grad, d->loss_dev,
                                  d->sqerr_dev, st, reg ? &planar : nullptr,
                                  true)))
    return rc;
  const L1ReduceJob l1 = l1_reduce_job(d->ws, d->loss_dev, d->sqerr_dev);
  // The camera constants were formed by the clearing launch.
  if ((rc = project_bwd_checked(d->ws, &params, d->cams, &grad, st, &l1,
                                true)))
    return rc;
  if (d->flags & GS_WINDOW_ADAM) {
    // The clearing launch advanced *step_dev already.
    if ((rc = adam_checked(&params, &grad, &m, &v, d->lr, d->beta1, d->beta2,
                           d->eps, 1, d->step_dev, -1, st)))
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
  // The clearing launch forms the shapes in the workspace's buffer.
  if (d->params.capacity != d->ws->geo.capacity) {
    set_error("window: params.capacity %d differs from the workspace's %d",
              d->params.capacity, d->ws->geo.capacity);
    return GS_E_CAPACITY;
  }
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
