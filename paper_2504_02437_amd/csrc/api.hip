// Host side of the C ABI: argument checks, workspace carving, launches and
// error reporting.  Allocates no device memory.

#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gs_internal.h"
#include "shape.h"
#include "tails.h"

namespace gs {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return GS_OK;
  set_error("%s: %s", what, hipGetErrorString(e));
  return GS_E_HIP;
}

int validate_settings(const gs_settings* s) {
  if (!s) { set_error("settings is NULL"); return GS_E_INVALID; }
  if (s->tile != 8 && s->tile != 16 && s->tile != 32) {
    set_error("tile must be 8, 16 or 32 (got %d)", s->tile);
    return GS_E_INVALID;
  }
  if (s->lds_batch != 128 && s->lds_batch != 256 && s->lds_batch != 512) {
    set_error("lds_batch must be 128, 256 or 512 (got %d)", s->lds_batch);
    return GS_E_INVALID;
  }
  const int bt = s->block_threads;
  const bool bt_ok = bt == 0 || (s->tile == 8 && bt == 64) ||
                     (s->tile == 16 && (bt == 64 || bt == 128 || bt == 256)) ||
                     (s->tile == 32 && (bt == 128 || bt == 256));
  if (!bt_ok) {
    set_error("block_threads %d not supported for tile %d", bt, s->tile);
    return GS_E_INVALID;
  }
  if (!(s->alpha_min > 0.f) || !(s->alpha_max <= 1.f) ||
      !(s->alpha_min < s->alpha_max) || !(s->T_min > 0.f) ||
      !(s->alpha_max < 1.f)) {
    set_error("need 0 < alpha_min < alpha_max < 1 and T_min > 0");
    return GS_E_INVALID;
  }
  return GS_OK;
}

int validate_params(const gs_params* p, const char* what) {
  if (!p) { set_error("%s is NULL", what); return GS_E_INVALID; }
  if (!p->mean || !p->log_scale || !p->quat || !p->opacity_logit || !p->rgb) {
    set_error("%s has a NULL row pointer", what);
    return GS_E_INVALID;
  }
  if (p->capacity < 0) { set_error("%s capacity < 0", what); return GS_E_INVALID; }
  if (p->sh_degree < 0 || p->sh_degree > GS_SH_MAX_DEGREE) {
    set_error("%s sh_degree must be 0..%d (got %d)", what, GS_SH_MAX_DEGREE,
              p->sh_degree);
    return GS_E_INVALID;
  }
  if (p->sh_degree > 0 && !p->sh) {
    set_error("%s has sh_degree %d and a NULL sh pointer", what, p->sh_degree);
    return GS_E_INVALID;
  }
  return GS_OK;
}

// Gradient and moment arrays mirror the parameters' layout.
static int same_layout(const gs_params* p, const gs_params* q, const char* what) {
  if (q && q->sh_degree != p->sh_degree) {
    set_error("%s has sh_degree %d, the parameters %d", what, q->sh_degree,
              p->sh_degree);
    return GS_E_INVALID;
  }
  return GS_OK;
}

// Byte ranges of a parameter set's rows (empty for a NULL row).
static void row_ranges(const gs_params* p, uintptr_t (&r)[6][2]) {
  const size_t c = (size_t)(p->capacity > 0 ? p->capacity : 0) * sizeof(float);
  const void* ptr[6] = {p->mean, p->log_scale, p->quat, p->opacity_logit,
                        p->rgb, p->sh_degree > 0 ? p->sh : nullptr};
  const size_t rows[6] = {3, 3, 4, 1, 3,
                          (size_t)(p->sh_degree > 0 ? GS_SH_ROWS(p->sh_degree)
                                                    : 0)};
  for (int i = 0; i < 6; ++i) {
    r[i][0] = (uintptr_t)ptr[i];
    r[i][1] = ptr[i] ? r[i][0] + rows[i] * c : r[i][0];
  }
}

// Parameters, gradients and moments are read and written in the same
// kernels, one thread per Gaussian and row: two of them must not share
// memory.
static int disjoint(const gs_params* p, const char* pw, const gs_params* q,
                    const char* qw) {
  if (!p || !q) return GS_OK;
  uintptr_t a[6][2], b[6][2];
  row_ranges(p, a);
  row_ranges(q, b);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j)
      if (a[i][0] < a[i][1] && b[j][0] < b[j][1] && a[i][0] < b[j][1] &&
          b[j][0] < a[i][1]) {
        set_error("%s and %s share memory", pw, qw);
        return GS_E_INVALID;
      }
  return GS_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int make_layout(const gs_geometry* g, Layout& L, int& tx, int& ty) {
  if (!g) { set_error("geometry is NULL"); return GS_E_INVALID; }
  if (g->n_views < 1 || g->width < 1 || g->height < 1 || g->width > 16384 ||
      g->height > 16384) {
    set_error("need n_views >= 1 and 1 <= width, height <= 16384");
    return GS_E_INVALID;
  }
  if (g->tile != 8 && g->tile != 16 && g->tile != 32) {
    set_error("tile must be 8, 16 or 32 (got %d)", g->tile);
    return GS_E_INVALID;
  }
  if (g->capacity < 0 || g->key_capacity < 0 ||
      g->key_capacity > (int64_t)0x7fffffff) {
    set_error("need capacity >= 0 and 0 <= key_capacity < 2^31");
    return GS_E_INVALID;
  }
  tx = (g->width + g->tile - 1) / g->tile;
  ty = (g->height + g->tile - 1) / g->tile;
  const size_t V = g->n_views, cap = g->capacity, kc = g->key_capacity;
  const size_t tiles = V * tx * ty;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.records = take(V * cap * sizeof(Record));
  L.tiles_touched = take(V * cap * 4);
  L.rbox = take(V * cap * 8);
  L.depth = take(V * cap * 4);
  L.diff = take(V * (size_t)(ty + 1) * (tx + 1) * 4);
  L.ranges = take(tiles * 8);
  L.cursor = take(tiles * 4);
  L.tile_order = take(tiles * 4);
  L.tile_loss = take(tiles * 16);
  const int ch = bin_chunk(tx, ty);
  L.chunk_counts = take(ch ? V * ((cap + ch - 1) / ch) * (size_t)tx * ty * 4 : 0);
  L.keys_unsorted = take(kc * 8);
  L.vals_sorted = take(kc * 4);
  L.keys_sorted = take(kc * 8);
  L.grad2d = take(V * 5 * cap * 4);
  L.gop = take(cap * 4);
  L.gcol = take(V * 3 * cap * 4);
  L.shape = take(cap * (6 * 8 + 4 + 4));
  L.camd = take(V * kCamDoubles * sizeof(double));
  L.counters = take(sizeof(Counters));
  L.total = off;
  return GS_OK;
}

static int check_ws(const gs_workspace* ws) {
  if (!ws || !ws->base) { set_error("workspace is NULL"); return GS_E_INVALID; }
  return GS_OK;
}

static int finish(hipError_t e, const char* what) { return check_hip(e, what); }

// The render boxes of the last projection hold every pixel whose alpha can
// reach the alpha_min they were formed for; a smaller alpha_min needs larger
// boxes.
static int check_box_alpha(const gs_workspace* ws, const gs_settings* s) {
  if (s->alpha_min < ws->box_alpha_min) {
    set_error("settings.alpha_min %g is below the %g the render boxes were "
              "formed for; project again with these settings",
              (double)s->alpha_min, (double)ws->box_alpha_min);
    return GS_E_INVALID;
  }
  return GS_OK;
}

int render_bwd_l1_checked(gs_workspace* ws, const gs_params* params,
                         const gs_settings* s, const float* out_rgb,
                         const float* target, float lambda,
                         const float* T_final, const int32_t* n_last,
                         gs_params* grad, double* loss_dev, double* sqerr_dev,
                         void* stream, const PlanarJob* planar,
                         bool defer_reduce) {
  g_err[0] = 0;
  if (int rc = check_ws(ws)) return rc;
  if (int rc = validate_params(params, "params")) return rc;
  if (int rc = validate_params(grad, "grad")) return rc;
  if (int rc = validate_settings(s)) return rc;
  if (s->tile != ws->geo.tile) { set_error("settings.tile differs from the workspace's"); return GS_E_INVALID; }
  if (int rc = check_box_alpha(ws, s)) return rc;
  if (!out_rgb || !target || !T_final || !n_last || !loss_dev) {
    set_error("an input is NULL");
    return GS_E_INVALID;
  }
  if (grad->capacity != params->capacity || params->capacity != ws->geo.capacity) {
    set_error("grad / params / workspace capacities differ");
    return GS_E_CAPACITY;
  }
  if (int rc = same_layout(params, grad, "grad")) return rc;
  if (int rc = disjoint(params, "params", grad, "grad")) return rc;
  L1Fused l1{out_rgb, target, lambda, loss_dev, sqerr_dev};
  l1.defer_reduce = defer_reduce;
  return finish(launch_render_bwd(ws, s, nullptr, T_final, n_last, grad->rgb,
                                  params->sh_degree > 0, &l1,
                                  (hipStream_t)stream, planar),
                "render_bwd_l1");
}

int project_bwd_checked(gs_workspace* ws, const gs_params* params,
                        const gs_camera* cams, gs_params* grad, void* stream,
                        const L1ReduceJob* l1, bool cam_table) {
  g_err[0] = 0;
  if (int rc = check_ws(ws)) return rc;
  if (int rc = validate_params(params, "params")) return rc;
  if (int rc = validate_params(grad, "grad")) return rc;
  if (!cams || !params->n_dev) { set_error("an input is NULL"); return GS_E_INVALID; }
  if (grad->capacity != params->capacity || params->capacity != ws->geo.capacity) {
    set_error("grad / params / workspace capacities differ");
    return GS_E_CAPACITY;
  }
  if (int rc = same_layout(params, grad, "grad")) return rc;
  if (int rc = disjoint(params, "params", grad, "grad")) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_project_bwd(ws, params, cams, grad, st, l1, cam_table);
  if (e != hipSuccess) return finish(e, "project_bwd");
  return finish(launch_sh_bwd(ws, params, cams, grad, st),
                "view-dependent colour backward");
}

int planar_checked(const gs_params* params, float lambda, float floor_,
                   gs_params* grad, double* loss_dev, PlanarJob* job) {
  g_err[0] = 0;
  if (int rc = validate_params(params, "params")) return rc;
  if (!grad || !grad->log_scale || !loss_dev || !params->n_dev) { set_error("an argument is NULL"); return GS_E_INVALID; }
  if (grad->capacity != params->capacity) { set_error("capacities differ"); return GS_E_CAPACITY; }
  if (int rc = disjoint(params, "params", grad, "grad")) return rc;
  *job = planar_job(params, lambda, floor_, grad, loss_dev);
  return GS_OK;
}

int project_and_bin_checked(gs_workspace* ws, const gs_params* params,
                            const gs_camera* cams, const gs_settings* s,
                            void* stream, bool shape_done) {
  g_err[0] = 0;
  if (int rc = check_ws(ws)) return rc;
  if (int rc = validate_params(params, "params")) return rc;
  if (int rc = validate_settings(s)) return rc;
  if (!params->n_dev) { set_error("params.n_dev is NULL"); return GS_E_INVALID; }
  if (!cams) { set_error("cams is NULL"); return GS_E_INVALID; }
  if (s->tile != ws->geo.tile) {
    set_error("settings.tile %d differs from the workspace's %d", s->tile,
              ws->geo.tile);
    return GS_E_INVALID;
  }
  if (params->capacity != ws->geo.capacity) {
    set_error("params.capacity %d differs from the workspace's %d",
              params->capacity, ws->geo.capacity);
    return GS_E_CAPACITY;
  }
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_project(ws, params, cams, s, st, shape_done);
  if (e != hipSuccess) return finish(e, "project");
  e = launch_sh_colour(ws, params, cams, st);
  if (e != hipSuccess) return finish(e, "view-dependent colour");
  ws->box_alpha_min = (s->flags & GS_FLAG_FULL_BOX) ? 0.f : s->alpha_min;
  return finish(launch_bin(ws, params, st), "bin");
}

int adam_checked(gs_params* params, const gs_params* grad, gs_params* m,
                 gs_params* v, const float* lr, float beta1, float beta2,
                 float eps, int32_t step, const int32_t* step_dev,
                 int step_bias, void* stream) {
  g_err[0] = 0;
  if (int rc = validate_params(params, "params")) return rc;
  if (int rc = validate_params(grad, "grad")) return rc;
  if (int rc = validate_params(m, "m")) return rc;
  if (int rc = validate_params(v, "v")) return rc;
  if (!lr || !params->n_dev) { set_error("lr or n_dev is NULL"); return GS_E_INVALID; }
  if (!step_dev && step < 1) { set_error("step must be >= 1"); return GS_E_INVALID; }
  if (grad->capacity != params->capacity || m->capacity != params->capacity ||
      v->capacity != params->capacity) {
    set_error("capacities differ");
    return GS_E_CAPACITY;
  }
  if (int rc = same_layout(params, grad, "grad")) return rc;
  if (int rc = disjoint(params, "params", grad, "grad")) return rc;
  if (int rc = same_layout(params, m, "m")) return rc;
  if (int rc = same_layout(params, v, "v")) return rc;
  const gs_params* all[4] = {params, grad, m, v};
  const char* names[4] = {"params", "grad", "m", "v"};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (int rc = disjoint(all[i], names[i], all[j], names[j])) return rc;
  return finish(launch_adam(params, grad, m, v, lr, beta1, beta2, eps, step,
                            step_dev, (hipStream_t)stream, step_bias), "adam");
}

}  // namespace gs

using namespace gs;

extern "C" {

const char* gs_last_error(void) { return g_err; }

const char* gs_version(void) { return "gsmap 0.1 (gfx950)"; }

int gs_workspace_size(const gs_geometry* geo, size_t* bytes) {
  g_err[0] = 0;
  Layout L;
  int tx, ty;
  int rc = make_layout(geo, L, tx, ty);
  if (rc) return rc;
  if (!bytes) { set_error("bytes is NULL"); return GS_E_INVALID; }
  *bytes = L.total;
  return GS_OK;
}

int gs_workspace_create(const gs_geometry* geo, void* device_buffer,
                        size_t bytes, void* stream, gs_workspace** out) {
  g_err[0] = 0;
  if (!out) { set_error("out is NULL"); return GS_E_INVALID; }
  *out = nullptr;
  Layout L;
  int tx, ty;
  int rc = make_layout(geo, L, tx, ty);
  if (rc) return rc;
  if (!device_buffer) { set_error("device_buffer is NULL"); return GS_E_INVALID; }
  if (((uintptr_t)device_buffer & 255) != 0) {
    set_error("device_buffer must be 256-byte aligned");
    return GS_E_INVALID;
  }
  if (bytes < L.total) {
    set_error("workspace needs %zu bytes, got %zu", L.total, bytes);
    return GS_E_CAPACITY;
  }
  gs_workspace* ws = (gs_workspace*)calloc(1, sizeof(gs_workspace));
  if (!ws) { set_error("out of host memory"); return GS_E_INVALID; }
  ws->geo = *geo;
  ws->tiles_x = tx;
  ws->tiles_y = ty;
  ws->base = (char*)device_buffer;
  ws->bytes = bytes;
  ws->L = L;
  char* b = ws->base;
  ws->records = (Record*)(b + L.records);
  ws->tiles_touched = (int32_t*)(b + L.tiles_touched);
  ws->rbox = (int2*)(b + L.rbox);
  ws->depth = (float*)(b + L.depth);
  ws->box_alpha_min = 0.f;
  ws->diff = (int32_t*)(b + L.diff);
  ws->ranges = (uint32_t*)(b + L.ranges);
  ws->cursor = (uint32_t*)(b + L.cursor);
  ws->tile_order = (uint32_t*)(b + L.tile_order);
  ws->tile_loss = (double*)(b + L.tile_loss);
  ws->chunk_counts = (uint32_t*)(b + L.chunk_counts);
  ws->keys_unsorted = (unsigned long long*)(b + L.keys_unsorted);
  ws->vals_sorted = (uint32_t*)(b + L.vals_sorted);
  ws->keys_sorted = (unsigned long long*)(b + L.keys_sorted);
  ws->grad2d = (float*)(b + L.grad2d);
  ws->gop = (float*)(b + L.gop);
  ws->gcol = (float*)(b + L.gcol);
  ws->shape = (double*)(b + L.shape);
  ws->camd = (double*)(b + L.camd);
  ws->counters = (Counters*)(b + L.counters);
  hipStream_t st = (hipStream_t)stream;
  const size_t V = geo->n_views, cap = geo->capacity;
  hipError_t e = launch_fill_u32(ws->diff, 0, V * (size_t)(ty + 1) * (tx + 1), st);
  if (e == hipSuccess) e = launch_fill_u32(ws->grad2d, 0, V * 5 * cap, st);
  if (e == hipSuccess) e = launch_fill_u32(ws->gop, 0, cap, st);
  if (e == hipSuccess) e = launch_fill_u32(ws->gcol, 0, V * 3 * cap, st);
  if (e == hipSuccess) e = launch_fill_u32(ws->counters, 0, sizeof(Counters) / 4, st);
  if (e == hipSuccess) e = launch_fill_u32(ws->ranges, 0, V * tx * ty * 2, st);
  if (e == hipSuccess) e = launch_iota_u32(ws->tile_order, V * tx * ty, st);
  if (e == hipSuccess) e = launch_fill_u32(ws->tiles_touched, 0, V * cap, st);
  if (e != hipSuccess) {
    free(ws);
    return check_hip(e, "workspace clear");
  }
  *out = ws;
  return GS_OK;
}

int gs_workspace_destroy(gs_workspace* ws) {
  free(ws);
  return GS_OK;
}

int gs_workspace_get_view(const gs_workspace* ws, gs_workspace_view* out) {
  g_err[0] = 0;
  if (int rc = check_ws(ws)) return rc;
  if (!out) { set_error("out is NULL"); return GS_E_INVALID; }
  out->records = ws->records;
  out->tiles_touched = ws->tiles_touched;
  out->render_box = (int32_t*)ws->rbox;
  out->ranges = ws->ranges;
  out->vals_sorted = ws->vals_sorted;
  out->keys_sorted = (uint64_t*)ws->keys_sorted;
  out->grad2d = ws->grad2d;
  out->n_keys = (int64_t*)&ws->counters->n_keys;
  out->status = &ws->counters->status;
  out->tiles_x = ws->tiles_x;
  out->tiles_y = ws->tiles_y;
  out->grad_opacity = ws->gop;
  out->grad_colour = ws->gcol;
  return GS_OK;
}

int gs_project_and_bin(gs_workspace* ws, const gs_params* params,
                       const gs_camera* cams, const gs_settings* s,
                       void* stream) {
  return project_and_bin_checked(ws, params, cams, s, stream, false);
}

int gs_sort_tile_keys(gs_workspace* ws, const gs_settings* s, void* stream) {
  g_err[0] = 0;
  if (int rc = check_ws(ws)) return rc;
  if (int rc = validate_settings(s)) return rc;
  return finish(launch_sort(ws, s, (hipStream_t)stream), "sort_tile_keys");
}

int gs_render_fwd(gs_workspace* ws, const gs_params* params,
                  const gs_settings* s, float* out_rgb, float* out_T,
                  int32_t* out_nlast, void* stream) {
  g_err[0] = 0;
  if (int rc = check_ws(ws)) return rc;
  if (int rc = validate_params(params, "params")) return rc;
  if (int rc = validate_settings(s)) return rc;
  if (s->tile != ws->geo.tile) { set_error("settings.tile differs from the workspace's"); return GS_E_INVALID; }
  if (int rc = check_box_alpha(ws, s)) return rc;
  if (!out_rgb || !out_T || !out_nlast) { set_error("an output is NULL"); return GS_E_INVALID; }
  return finish(launch_render_fwd(ws, s, out_rgb, out_T, out_nlast,
                                  (hipStream_t)stream), "render_fwd");
}

int gs_render_dominant(gs_workspace* ws, const gs_params* params,
                       const gs_settings* s, float* out_rgb, float* out_T,
                       int32_t* out_nlast, int32_t* out_dom, void* stream) {
  g_err[0] = 0;
  if (int rc = check_ws(ws)) return rc;
  if (int rc = validate_params(params, "params")) return rc;
  if (int rc = validate_settings(s)) return rc;
  if (s->tile != ws->geo.tile) { set_error("settings.tile differs from the workspace's"); return GS_E_INVALID; }
  if (int rc = check_box_alpha(ws, s)) return rc;
  if (!out_rgb || !out_T || !out_nlast || !out_dom) { set_error("an output is NULL"); return GS_E_INVALID; }
  return finish(launch_render_dominant(ws, s, out_rgb, out_T, out_nlast,
                                       out_dom, (hipStream_t)stream),
                "render_dominant");
}

int gs_densify(gs_params* params, gs_params* adam_m, gs_params* adam_v,
               const int32_t* dom, int64_t n_pixels, int32_t sigma,
               const float* xi, int32_t* scratch, int32_t* n_split_dev,
               int32_t* status_dev, void* stream) {
  g_err[0] = 0;
  if (int rc = validate_params(params, "params")) return rc;
  if (!params->n_dev) { set_error("params.n_dev is NULL"); return GS_E_INVALID; }
  if (adam_m) {
    if (int rc = validate_params(adam_m, "adam_m")) return rc;
  }
  if (adam_v) {
    if (int rc = validate_params(adam_v, "adam_v")) return rc;
  }
  if ((adam_m && adam_m->capacity != params->capacity) ||
      (adam_v && adam_v->capacity != params->capacity)) {
    set_error("Adam moment capacities differ from the parameters'");
    return GS_E_CAPACITY;
  }
  if (int rc = same_layout(params, adam_m, "adam_m")) return rc;
  if (int rc = same_layout(params, adam_v, "adam_v")) return rc;
  if (int rc = disjoint(params, "params", adam_m, "adam_m")) return rc;
  if (int rc = disjoint(params, "params", adam_v, "adam_v")) return rc;
  if (int rc = disjoint(adam_m, "adam_m", adam_v, "adam_v")) return rc;
  if (!xi || !scratch || (n_pixels > 0 && !dom)) { set_error("an argument is NULL"); return GS_E_INVALID; }
  if (n_pixels < 0 || sigma < 0) { set_error("need n_pixels >= 0 and sigma >= 0"); return GS_E_INVALID; }
  return finish(launch_densify(params, adam_m, adam_v, dom, n_pixels, sigma, xi,
                               scratch, n_split_dev, status_dev,
                               (hipStream_t)stream),
                "densify");
}

int gs_count_pairs(gs_workspace* ws, const gs_params* params,
                   const gs_settings* s, uint64_t* counts_dev, void* stream) {
  g_err[0] = 0;
  if (int rc = check_ws(ws)) return rc;
  if (int rc = validate_params(params, "params")) return rc;
  if (int rc = validate_settings(s)) return rc;
  if (s->tile != ws->geo.tile) { set_error("settings.tile differs from the workspace's"); return GS_E_INVALID; }
  if (int rc = check_box_alpha(ws, s)) return rc;
  if (!counts_dev) { set_error("counts_dev is NULL"); return GS_E_INVALID; }
  return finish(launch_count_pairs(ws, s, (unsigned long long*)counts_dev,
                                   (hipStream_t)stream), "count_pairs");
}

int gs_render_bwd(gs_workspace* ws, const gs_params* params,
                  const gs_settings* s,
                  const float* dL_drgb, const float* T_final,
                  const int32_t* n_last, gs_params* grad, void* stream) {
  g_err[0] = 0;
  if (int rc = check_ws(ws)) return rc;
  if (int rc = validate_params(params, "params")) return rc;
  if (int rc = validate_params(grad, "grad")) return rc;
  if (int rc = validate_settings(s)) return rc;
  if (s->tile != ws->geo.tile) { set_error("settings.tile differs from the workspace's"); return GS_E_INVALID; }
  if (int rc = check_box_alpha(ws, s)) return rc;
  if (!dL_drgb || !T_final || !n_last) {
    set_error("an input is NULL");
    return GS_E_INVALID;
  }
  if (grad->capacity != params->capacity || params->capacity != ws->geo.capacity) {
    set_error("grad / params / workspace capacities differ");
    return GS_E_CAPACITY;
  }
  if (int rc = same_layout(params, grad, "grad")) return rc;
  if (int rc = disjoint(params, "params", grad, "grad")) return rc;
  return finish(launch_render_bwd(ws, s, dL_drgb, T_final, n_last, grad->rgb,
                                  params->sh_degree > 0, nullptr,
                                  (hipStream_t)stream),
                "render_bwd");
}

int gs_render_bwd_l1(gs_workspace* ws, const gs_params* params,
                     const gs_settings* s, const float* out_rgb,
                     const float* target, float lambda, const float* T_final,
                     const int32_t* n_last, gs_params* grad, double* loss_dev,
                     double* sqerr_dev, void* stream) {
  return render_bwd_l1_checked(ws, params, s, out_rgb, target, lambda, T_final,
                               n_last, grad, loss_dev, sqerr_dev, stream,
                               nullptr, false);
}

int gs_project_bwd(gs_workspace* ws, const gs_params* params,
                   const gs_camera* cams, gs_params* grad, void* stream) {
  return project_bwd_checked(ws, params, cams, grad, stream, nullptr);
}

int gs_loss_l1(const float* rgb, const float* target, int32_t n_views,
               int32_t height, int32_t width, float lambda, float* dL_drgb,
               double* loss_dev, double* sqerr_dev, void* stream) {
  g_err[0] = 0;
  if (!rgb || !target || !dL_drgb || !loss_dev) { set_error("an argument is NULL"); return GS_E_INVALID; }
  if (n_views < 1 || height < 1 || width < 1) { set_error("bad image size"); return GS_E_INVALID; }
  return finish(launch_loss_l1(rgb, target, n_views, height, width, lambda,
                               dL_drgb, loss_dev, sqerr_dev, (hipStream_t)stream),
                "loss_l1");
}

int gs_loss_ssim(const float* rgb, const float* target, int32_t n_views,
                 int32_t height, int32_t width, float lambda, float* dL_drgb,
                 double* loss_dev, double* ssim_dev, float* scratch,
                 void* stream) {
  g_err[0] = 0;
  if (!rgb || !target || !dL_drgb || !loss_dev || !scratch) { set_error("an argument is NULL"); return GS_E_INVALID; }
  if (n_views < 1 || height < 1 || width < 1 || n_views > 21845) { set_error("bad image size"); return GS_E_INVALID; }
  return finish(launch_loss_ssim(rgb, target, n_views, height, width, lambda,
                                 dL_drgb, loss_dev, ssim_dev, scratch,
                                 (hipStream_t)stream),
                "loss_ssim");
}

int gs_loss_colour(const float* rgb, const float* target, int32_t n_views,
                   int32_t height, int32_t width, float lambda_l1,
                   float lambda_ssim, float* dL_drgb, double* loss_dev,
                   double* sqerr_dev, double* ssim_dev, float* scratch,
                   void* stream) {
  g_err[0] = 0;
  if (!rgb || !target || !dL_drgb || !loss_dev || !scratch) { set_error("an argument is NULL"); return GS_E_INVALID; }
  if (n_views < 1 || height < 1 || width < 1 || n_views > 21845) { set_error("bad image size"); return GS_E_INVALID; }
  return finish(launch_loss_colour(rgb, target, n_views, height, width,
                                   lambda_l1, lambda_ssim, 1, dL_drgb,
                                   loss_dev, sqerr_dev, ssim_dev, scratch,
                                   (hipStream_t)stream),
                "loss_colour");
}

int gs_planar_reg(const gs_params* params, float lambda, float floor_,
                  gs_params* grad, double* loss_dev, void* stream) {
  PlanarJob j;
  if (int rc = planar_checked(params, lambda, floor_, grad, loss_dev, &j))
    return rc;
  return finish(launch_planar_job(j, (hipStream_t)stream), "planar_reg");
}

int gs_adam(gs_params* params, const gs_params* grad, gs_params* m,
            gs_params* v, const float* lr, float beta1, float beta2,
            float eps, int32_t step, const int32_t* step_dev, void* stream) {
  return adam_checked(params, grad, m, v, lr, beta1, beta2, eps, step,
                      step_dev, 0, stream);
}

int gs_insert_gaussians(gs_params* params, gs_params* adam_m, gs_params* adam_v,
                        const gs_camera* cam, int32_t width, int32_t height,
                        const float* kf_rgb, const float* kf_T_final,
                        const float* pts_uvd, int32_t n_pts, float alpha_skip,
                        int32_t centre_only, const float* mlp_out,
                        int32_t* n_inserted_dev, int32_t* status_dev,
                        void* stream) {
  g_err[0] = 0;
  if (int rc = validate_params(params, "params")) return rc;
  if (!params->n_dev || !cam || !kf_T_final || (!kf_rgb && !mlp_out)) {
    set_error("an argument is NULL");
    return GS_E_INVALID;
  }
  if (n_pts < 0 || (long long)n_pts * 9 > 65536) { set_error("need 0 <= n_pts and 9 n_pts <= 65536"); return GS_E_INVALID; }
  if (n_pts > 0 && !pts_uvd) { set_error("pts_uvd is NULL"); return GS_E_INVALID; }
  if (width < 1 || height < 1) { set_error("bad image size"); return GS_E_INVALID; }
  if ((adam_m && adam_m->capacity != params->capacity) ||
      (adam_v && adam_v->capacity != params->capacity)) {
    set_error("moment capacities differ");
    return GS_E_CAPACITY;
  }
  if (adam_m) {
    if (int rc = validate_params(adam_m, "adam_m")) return rc;
    if (int rc = same_layout(params, adam_m, "adam_m")) return rc;
  }
  if (adam_v) {
    if (int rc = validate_params(adam_v, "adam_v")) return rc;
    if (int rc = same_layout(params, adam_v, "adam_v")) return rc;
  }
  if (int rc = disjoint(params, "params", adam_m, "adam_m")) return rc;
  if (int rc = disjoint(params, "params", adam_v, "adam_v")) return rc;
  if (int rc = disjoint(adam_m, "adam_m", adam_v, "adam_v")) return rc;
  return finish(launch_insert(params, adam_m, adam_v, cam, width, height, kf_rgb,
                              kf_T_final, pts_uvd, n_pts, alpha_skip, centre_only,
                              mlp_out, n_inserted_dev, status_dev,
                              (hipStream_t)stream), "insert_gaussians");
}

int gs_insert_distance(gs_params* params, gs_params* adam_m,
                       gs_params* adam_v, const gs_camera* cam, int32_t width,
                       int32_t height, const float* kf_rgb,
                       const float* pts_uvd, int32_t n_pts, float tau,
                       int32_t centre_only, const float* mlp_out,
                       uint64_t* scratch, int32_t* n_inserted_dev,
                       int32_t* status_dev, void* stream) {
  g_err[0] = 0;
  if (int rc = validate_params(params, "params")) return rc;
  if (!params->n_dev || !cam || (!kf_rgb && !mlp_out)) {
    set_error("an argument is NULL");
    return GS_E_INVALID;
  }
  if (n_pts < 0 || (long long)n_pts * 9 > 65536) { set_error("need 0 <= n_pts and 9 n_pts <= 65536"); return GS_E_INVALID; }
  if (n_pts > 0 && (!pts_uvd || !scratch)) { set_error("pts_uvd or scratch is NULL"); return GS_E_INVALID; }
  if (width < 1 || height < 1) { set_error("bad image size"); return GS_E_INVALID; }
  if (!(tau >= 0.f)) { set_error("need tau >= 0"); return GS_E_INVALID; }
  if ((adam_m && adam_m->capacity != params->capacity) ||
      (adam_v && adam_v->capacity != params->capacity)) {
    set_error("moment capacities differ");
    return GS_E_CAPACITY;
  }
  if (adam_m) {
    if (int rc = validate_params(adam_m, "adam_m")) return rc;
    if (int rc = same_layout(params, adam_m, "adam_m")) return rc;
  }
  if (adam_v) {
    if (int rc = validate_params(adam_v, "adam_v")) return rc;
    if (int rc = same_layout(params, adam_v, "adam_v")) return rc;
  }
  if (int rc = disjoint(params, "params", adam_m, "adam_m")) return rc;
  if (int rc = disjoint(params, "params", adam_v, "adam_v")) return rc;
  if (int rc = disjoint(adam_m, "adam_m", adam_v, "adam_v")) return rc;
  return finish(launch_insert_distance(params, adam_m, adam_v, cam, width,
                                       height, kf_rgb, pts_uvd, n_pts, tau,
                                       centre_only, mlp_out,
                                       (unsigned long long*)scratch,
                                       n_inserted_dev, status_dev,
                                       (hipStream_t)stream),
                "insert_distance");
}

int gs_knn_features(const gs_params* params, const gs_camera* cam,
                    int32_t width, int32_t height, const float* kf_rgb,
                    const float* pts_uvd, int32_t n_pts, int32_t centre_only,
                    float* feats, int32_t* knn_idx, float* knn_dist,
                    void* stream) {
  g_err[0] = 0;
  if (int rc = validate_params(params, "params")) return rc;
  if (!params->n_dev || !cam || !kf_rgb || !feats) { set_error("an argument is NULL"); return GS_E_INVALID; }
  if (n_pts < 0 || (long long)n_pts * 9 > 65536) { set_error("need 0 <= n_pts and 9 n_pts <= 65536"); return GS_E_INVALID; }
  if (n_pts > 0 && !pts_uvd) { set_error("pts_uvd is NULL"); return GS_E_INVALID; }
  if (width < 1 || height < 1) { set_error("bad image size"); return GS_E_INVALID; }
  return finish(launch_knn_features(params, cam, width, height, kf_rgb, pts_uvd,
                                    n_pts, centre_only, feats, knn_idx, knn_dist,
                                    (hipStream_t)stream), "knn_features");
}

int gs_mlp_fwd(const float* weights, const float* x, int32_t m, float* y,
               float* cache, void* stream) {
  g_err[0] = 0;
  if (!weights || (m > 0 && (!x || !y))) { set_error("an argument is NULL"); return GS_E_INVALID; }
  if (m < 0) { set_error("m < 0"); return GS_E_INVALID; }
  return finish(launch_mlp_fwd(weights, x, m, y, cache, (hipStream_t)stream), "mlp_fwd");
}

int gs_mlp_mse(const float* y, const float* target, int32_t m, float* dy,
               double* loss_dev, void* stream) {
  g_err[0] = 0;
  if (m > 0 && (!y || !target || !dy)) { set_error("an argument is NULL"); return GS_E_INVALID; }
  if (m < 0) { set_error("m < 0"); return GS_E_INVALID; }
  return finish(launch_mlp_mse(y, target, m, dy, loss_dev, (hipStream_t)stream), "mlp_mse");
}

int gs_mlp_bwd(const float* weights, const float* x, const float* cache,
               const float* dy, int32_t m, float* dweights, void* stream) {
  g_err[0] = 0;
  if (!weights || !dweights || (m > 0 && (!x || !cache || !dy))) { set_error("an argument is NULL"); return GS_E_INVALID; }
  if (m < 0) { set_error("m < 0"); return GS_E_INVALID; }
  return finish(launch_mlp_bwd(weights, x, cache, dy, m, dweights, (hipStream_t)stream), "mlp_bwd");
}

int gs_mlp_adam(float* weights, const float* dweights, float* adam_m,
                float* adam_v, float lr, float beta1, float beta2, float eps,
                int32_t step, void* stream) {
  g_err[0] = 0;
  if (!weights || !dweights || !adam_m || !adam_v) { set_error("an argument is NULL"); return GS_E_INVALID; }
  if (step < 1) { set_error("step must be >= 1"); return GS_E_INVALID; }
  return finish(launch_mlp_adam(weights, dweights, adam_m, adam_v, lr, beta1, beta2,
                                eps, step, (hipStream_t)stream), "mlp_adam");
}

int gs_read_status(gs_workspace* ws, void* stream, int32_t* flags,
                   int64_t* n_keys, int32_t clear) {
  g_err[0] = 0;
  if (int rc = check_ws(ws)) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (int rc = check_hip(hipStreamSynchronize(st), "stream sync")) return rc;
  Counters c;
  if (int rc = check_hip(hipMemcpy(&c, ws->counters, sizeof(c), hipMemcpyDeviceToHost),
                         "read status"))
    return rc;
  if (flags) *flags = c.status;
  if (n_keys) *n_keys = c.n_keys;
  if (clear) {
    if (int rc = check_hip(launch_fill_u32(&ws->counters->status, 0, 1, st), "clear status"))
      return rc;
    if (int rc = check_hip(hipStreamSynchronize(st), "stream sync")) return rc;
  }
  return c.status ? GS_E_OVERFLOW : GS_OK;
}

}  // extern "C"
