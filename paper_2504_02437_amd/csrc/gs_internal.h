// Internal declarations shared by the HIP translation units of libgsmap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsmap.h"

namespace gs {

// One projected (view, Gaussian) record, 48 bytes = three float4:
//   q0 = (px, py, A, B), q1 = (C, opacity, r, g),
//   q2 = (b, depth, u_lo | u_hi << 16, v_lo | v_hi << 16)
// (A, B, C) is the conic: the inverse of the dilated screen covariance.
struct __align__(16) Record {
  float4 q0, q1, q2;
};

// Workspace layout: every region is carved from the caller's device buffer.
struct Layout {
  size_t records, tiles_touched, rbox, depth, diff, ranges, cursor, tile_order,
      tile_loss, chunk_counts,
      keys_unsorted, vals_sorted, keys_sorted, grad2d, gop, gcol, shape,
      camd, counters, total;
};

// Binning works on chunks of Gaussians of one view (one workgroup each) with
// the view's tile counters and coverage difference grid in LDS: 1024
// Gaussians per chunk for grids of up to 1024 tiles, 2048 up to 16384 tiles
// (difference grids of up to that many cells + 257); 0 for larger grids,
// which bin with a global difference grid and per-key global atomics.
constexpr int kGridSlack = 257;
inline int bin_chunk(int tx, int ty) {
  const long long nb = (long long)tx * ty, cells = (long long)(tx + 1) * (ty + 1);
  if (nb <= 1024 && cells <= 1024 + kGridSlack) return 1024;
  if (nb <= 16384 && cells <= 16384 + kGridSlack) return 2048;
  return 0;
}

// Device-side counters block.
struct Counters {
  long long n_keys;
  int status;
  int pad;
};

hipError_t launch_loss_ssim(const float* rgb, const float* target, int V,
                            int H, int W, float lam, float* dL, double* loss,
                            double* ssim, float* scratch, hipStream_t st);
hipError_t launch_loss_colour(const float* rgb, const float* target, int V,
                              int H, int W, float lam_l1, float lam,
                              int fuse_l1, float* dL, double* loss,
                              double* sqerr, double* ssim, float* scratch,
                              hipStream_t st);
hipError_t launch_knn_features(const gs_params* p, const gs_camera* cam, int W,
                               int H, const float* kf_rgb, const float* pts,
                               int n_pts, int centre_only, float* feats,
                               int32_t* knn_idx, float* knn_dist,
                               hipStream_t st);
hipError_t launch_mlp_fwd(const float* w, const float* x, int M, float* y,
                          float* cache, hipStream_t st);
hipError_t launch_mlp_bwd(const float* w, const float* x, const float* cache,
                          const float* dy, int M, float* dw, hipStream_t st);
hipError_t launch_mlp_mse(const float* y, const float* t, int M, float* dy,
                          double* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v,
                           float lr, float b1, float b2, float eps, int step,
                           hipStream_t st);

}  // namespace gs

struct gs_workspace {
  gs_geometry geo;
  int tiles_x, tiles_y;
  char* base;
  size_t bytes;
  gs::Layout L;
  gs::Record* records;
  int32_t* tiles_touched;
  int2* rbox;            // [V][capacity] render boxes (packed 16-bit pairs)
  float* depth;          // [V][capacity] camera-space depth (the key's upper
                         // half), beside the records for coalesced reads
  float box_alpha_min;   // alpha_min the render boxes were formed for
  int32_t* diff;         // [V][Ty + 1][Tx + 1] tile-coverage difference grid
                         // (grids too large for the chunked binning)
  uint32_t* ranges;      // [V * Ty * Tx][2]
  uint32_t* cursor;      // [V * Ty * Tx] tile counts
  uint32_t* tile_order;  // [V * Ty * Tx] tiles by descending key count (the
                         // per-tile kernels take block b -> tile order[b])
  double* tile_loss;     // [V * Ty * Tx][2] fused L1 loss and squared error
                         // of each tile, summed by one small kernel
  uint32_t* chunk_counts;  // [V][chunks][Ty * Tx] keys of each chunk per
                           // tile, then each chunk's offset in the tile
  unsigned long long* keys_unsorted;  // [key_capacity] depth bits << 32 | g
  uint32_t* vals_sorted;
  unsigned long long* keys_sorted;
  float* grad2d;         // [V][5][capacity]
  float* gop;            // [capacity] dL/d opacity summed over views
  double* camd;          // [V][21] FP64 camera constants (shape.h), formed
                         // by the launch before the projection
  float* gcol;           // [V][3][capacity] dL/d colour per view (used with
                         // view-dependent colour)
  double* shape;         // [6][capacity] 3D covariance (upper triangle) of
                         // the last projection, then float opacity
                         // [capacity] and float log2(opacity) [capacity]
  gs::Counters* counters;
};

namespace gs {

void set_error(const char* fmt, ...);
int check_hip(hipError_t e, const char* what);
int validate_settings(const gs_settings* s);
int validate_params(const gs_params* p, const char* what);

// Launchers implemented by the kernel translation units.  They return a
// hipError_t from the launch (hipGetLastError).
// shape_done: the per-Gaussian shapes of p are formed already (shape.h).
hipError_t launch_project(gs_workspace* ws, const gs_params* p,
                          const gs_camera* cams, const gs_settings* s,
                          hipStream_t st, bool shape_done = false);
struct PlanarJob;      // tails.h
struct L1ReduceJob;    // tails.h
// l1: the fused L1 term's tile-loss reduction as one workgroup appended to
// the launch (the window graph), or null.
hipError_t launch_project_bwd(gs_workspace* ws, const gs_params* p,
                              const gs_camera* cams, gs_params* grad,
                              hipStream_t st, const L1ReduceJob* l1 = nullptr,
                              bool cam_table = false);
hipError_t launch_bin(gs_workspace* ws, const gs_params* p, hipStream_t st);
hipError_t launch_sort(gs_workspace* ws, const gs_settings* s, hipStream_t st);
hipError_t launch_render_fwd(gs_workspace* ws, const gs_settings* s,
                             float* rgb, float* T, int32_t* nlast,
                             hipStream_t st);
hipError_t launch_insert_distance(gs_params* p, gs_params* m, gs_params* v,
                                  const gs_camera* cam, int W, int H,
                                  const float* kf_rgb, const float* pts,
                                  int n_pts, float tau, int centre_only,
                                  const float* mlp_out,
                                  unsigned long long* d2bits,
                                  int32_t* n_inserted, int32_t* status,
                                  hipStream_t st);
hipError_t launch_render_dominant(gs_workspace* ws, const gs_settings* s,
                                  float* rgb, float* T, int32_t* nlast,
                                  int32_t* dom, hipStream_t st);
hipError_t launch_densify(gs_params* p, gs_params* m, gs_params* v,
                          const int32_t* dom, long long n_pix, int sigma,
                          const float* xi, int32_t* scratch, int32_t* n_split,
                          int32_t* status, hipStream_t st);
hipError_t launch_count_pairs(gs_workspace* ws, const gs_settings* s,
                              unsigned long long* counts, hipStream_t st);
// The L1 photometric term fused into the compositing backward.
struct L1Fused {
  const float* rgb;
  const float* target;
  float lambda;
  double* loss;
  double* sqerr;
  bool defer_reduce = false;   // the caller reduces the tile losses later
};
// planar: the planar regulariser's workgroups appended to the launch (the
// window graph), or null.
hipError_t launch_render_bwd(gs_workspace* ws, const gs_settings* s,
                             const float* dL, const float* T,
                             const int32_t* nlast, float* grad_rgb,
                             int per_view_colour, const L1Fused* l1,
                             hipStream_t st, const PlanarJob* planar = nullptr);
hipError_t launch_l1_reduce(const gs_workspace* ws, double* loss,
                            double* sqerr, hipStream_t st);
hipError_t launch_sh_colour(gs_workspace* ws, const gs_params* p,
                            const gs_camera* cams, hipStream_t st);
hipError_t launch_sh_bwd(gs_workspace* ws, const gs_params* p,
                         const gs_camera* cams, gs_params* grad,
                         hipStream_t st);
hipError_t launch_iota_u32(uint32_t* ptr, size_t count, hipStream_t st);
hipError_t launch_fill_u32(void* ptr, uint32_t value, size_t count,
                           hipStream_t st);
hipError_t launch_loss_l1(const float* rgb, const float* target, int V, int H,
                          int W, float lambda, float* dL, double* loss,
                          double* sqerr, hipStream_t st);
hipError_t launch_planar_reg(const gs_params* p, float lambda, float floor_,
                             gs_params* grad, double* loss, hipStream_t st);
// step_bias is added to *step_dev (the window graph advances the count
// before its Adam step).
hipError_t launch_adam(gs_params* p, const gs_params* g, gs_params* m,
                       gs_params* v, const float* lr, float b1, float b2,
                       float eps, int step, const int32_t* step_dev,
                       hipStream_t st, int step_bias = 0);
// gs_render_bwd_l1 with its argument checks, the planar regulariser's
// workgroups appended (or null) and the tile-loss reduction optionally left
// to the caller.
int render_bwd_l1_checked(gs_workspace* ws, const gs_params* params,
                         const gs_settings* s, const float* out_rgb,
                         const float* target, float lambda,
                         const float* T_final, const int32_t* n_last,
                         gs_params* grad, double* loss_dev, double* sqerr_dev,
                         void* stream, const PlanarJob* planar,
                         bool defer_reduce);
// gs_project_bwd with its argument checks and an optional tile-loss
// reduction workgroup; cam_table: the camera constants come from ws->camd
// (formed from cams earlier in the same launch sequence).
int project_bwd_checked(gs_workspace* ws, const gs_params* params,
                        const gs_camera* cams, gs_params* grad, void* stream,
                        const L1ReduceJob* l1, bool cam_table = false);
// gs_planar_reg's argument checks; on success *job holds its launch.
int planar_checked(const gs_params* params, float lambda, float floor_,
                   gs_params* grad, double* loss_dev, PlanarJob* job);
// gs_project_and_bin with its argument checks; shape_done: the per-Gaussian
// shapes are formed already (the window graph's clearing kernel does it).
int project_and_bin_checked(gs_workspace* ws, const gs_params* params,
                            const gs_camera* cams, const gs_settings* s,
                            void* stream, bool shape_done);
// gs_adam with its argument checks, the bias passed to launch_adam.
int adam_checked(gs_params* params, const gs_params* grad, gs_params* m,
                 gs_params* v, const float* lr, float beta1, float beta2,
                 float eps, int32_t step, const int32_t* step_dev,
                 int step_bias, void* stream);
hipError_t launch_insert(gs_params* p, gs_params* m, gs_params* v,
                         const gs_camera* cam, int W, int H,
                         const float* kf_rgb, const float* kf_T,
                         const float* pts, int n_pts, float alpha_skip,
                         int centre_only, const float* mlp_out,
                         int32_t* n_inserted, int32_t* status, hipStream_t st);

hipError_t launch_knn_features(const gs_params* p, const gs_camera* cam, int W,
                               int H, const float* kf_rgb, const float* pts,
                               int n_pts, int centre_only, float* feats,
                               int32_t* knn_idx, float* knn_dist,
                               hipStream_t st);
hipError_t launch_mlp_fwd(const float* w, const float* x, int M, float* y,
                          float* cache, hipStream_t st);
hipError_t launch_mlp_bwd(const float* w, const float* x, const float* cache,
                          const float* dy, int M, float* dw, hipStream_t st);
hipError_t launch_mlp_mse(const float* y, const float* t, int M, float* dy,
                          double* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v,
                           float lr, float b1, float b2, float eps, int step,
                           hipStream_t st);

}  // namespace gs
