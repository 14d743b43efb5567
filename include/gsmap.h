/*
 * gsmap: differentiable tile-based 3D Gaussian splatting rasterizer for
 * MI355X (gfx950), the data-parallel hot path of a Gaussian-splatting
 * mapping back end (MonoGS++, arXiv 2504.02437, Methodology: Scene
 * Representation and Map Optimization).
 *
 * C ABI.  Every pointer documented as "device" is a HIP device pointer the
 * caller owns; the library allocates no device memory.  Every call that takes
 * a stream only enqueues work on it (no host synchronisation) unless stated,
 * so a sequence of calls can be captured into a HIP graph.  Streams are
 * passed as void* (a hipStream_t; NULL is the null stream).  A workspace
 * holds the state that flows from one call to the next (records, sorted
 * lists, screen-space gradients, loss partials): the calls on one workspace
 * go on one stream, in the order of the method, and do not overlap; distinct
 * workspaces are independent.
 *
 * Return codes: GS_OK, or
 *   GS_E_INVALID   a host-side argument check failed; nothing was launched;
 *   GS_E_CAPACITY  a host-known size is too small; nothing was launched;
 *   GS_E_OVERFLOW  (gs_read_status only) a device-side capacity was exceeded;
 *   GS_E_HIP       a HIP runtime call failed; gs_last_error() has the text.
 * No call aborts or throws across the ABI.
 *
 * Conventions (shared with the rest of the method): pinhole camera with
 * OpenCV axes (x right, y down, z forward); a world point X maps to camera
 * space as R X + t; pixel (u, v) is sampled at integer coordinates;
 * quaternions are (w, x, y, z) and normalised inside the projection; scale is
 * exp(log_scale); opacity is sigmoid(opacity_logit); colour is raw RGB.
 */
#ifndef GSMAP_H
#define GSMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_API __attribute__((visibility("default")))

#define GS_OK 0
#define GS_E_INVALID 1
#define GS_E_CAPACITY 2
#define GS_E_OVERFLOW 3
#define GS_E_HIP 4

/* Device status word bits (gs_read_status). */
#define GS_STATUS_KEY_OVERFLOW 1      /* more (view, Gaussian, tile) keys than key_capacity */
#define GS_STATUS_GAUSSIAN_OVERFLOW 2 /* insertion wanted more than capacity */

/* gs_settings.flags bits. */
#define GS_FLAG_EMIT_KEYS 1 /* sort_tile_keys also writes the sorted 64-bit keys */
/* Bin and render every pixel of each Gaussian's integer box (the rule of the
 * method as stated).  Without this flag gs_project_and_bin narrows each
 * (view, Gaussian) box to a render box: the box intersected with a
 * conservative bound of the pixels whose alpha can reach alpha_min.  Every
 * pair outside it would be skipped for alpha < alpha_min, so images, T_final
 * and gradients do not change; the Gaussian is binned only into the tiles its
 * render box touches, so tile lists are shorter (and n_last, an index into
 * them, smaller) but hold the same contributing entries in the same order. */
#define GS_FLAG_FULL_BOX 2

/* Gaussian parameters (Eq. 1 and the parameter list after it: mean,
 * rotation quaternion, scale, opacity, colour coefficients), planar
 * structure of arrays, FP32, all device pointers.  Each row holds
 * `capacity` floats; entries [0, *n_dev) are live.
 *   mean          [3][capacity]  x, y, z (world)
 *   log_scale     [3][capacity]  log of the per-axis standard deviation
 *   quat          [4][capacity]  w, x, y, z (any non-zero norm)
 *   opacity_logit [capacity]
 *   rgb           [3][capacity]  colour; with sh_degree > 0 the base colour
 *   sh_degree     0..GS_SH_MAX_DEGREE: degree D of the view-dependent colour
 *   sh            [GS_SH_ROWS(D)][capacity] view-dependent colour
 *                 coefficients (NULL when D = 0): row 3 (j - 1) + c holds
 *                 coefficient j = 1 .. (D+1)^2 - 1 of channel c
 * With D > 0 the colour of a Gaussian in a view is
 *   max(0, rgb_c + sum_j Y_j(d) sh_{j,c})
 * where d is the unit direction from the camera centre -R^T t to the mean
 * and Y_j the real spherical harmonics of degree 1..D in the order
 * l = 1..D, m = -l..l (Y_lm = sqrt(2) Re Y_l^m for m > 0, sqrt(2) Im
 * Y_l^|m| for m < 0, Y_l^0 for m = 0, Condon-Shortley phase included).
 * With D = 0 the colour is rgb in every view, unclamped.
 * n_dev is a device int32 holding the live count, so a captured graph stays
 * valid while insertion grows the map.  The same struct describes gradient
 * and optimiser-moment arrays of the same layout (their n_dev may be NULL;
 * their sh_degree must equal the parameters').  Parameter, gradient and
 * moment arrays passed to one call must not share memory: every call that
 * takes two of them returns GS_E_INVALID, before any launch, when their rows
 * overlap. */
#define GS_SH_MAX_DEGREE 3
#define GS_SH_ROWS(d) (3 * (((d) + 1) * ((d) + 1) - 1))
typedef struct gs_params {
  float* mean;
  float* log_scale;
  float* quat;
  float* opacity_logit;
  float* rgb;
  int32_t* n_dev;
  int32_t capacity;
  int32_t sh_degree;
  float* sh;
} gs_params;

/* One view: world-to-camera rotation R (row-major) and translation t,
 * intrinsics in pixels, near-plane depth and image size.  80 bytes.  Arrays of
 * cameras passed to the library live in device memory. */
typedef struct gs_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float near_z;
  int32_t width, height;
  int32_t pad_;
} gs_camera;

/* Rasterizer settings, passed by host pointer and copied at each call.
 *   tile        screen tile edge in pixels: 8, 16 or 32
 *   lds_batch   Gaussians staged in LDS per batch: 128, 256 or 512
 *   block_threads  threads per tile workgroup (0 = default); each thread
 *               owns a vertical strip of tile*tile/block_threads pixels:
 *               tile 8: 64; tile 16: 64, 128 or 256 (default 64);
 *               tile 32: 128 or 256 (default 256)
 *   bg          background colour added with weight T_final
 *   alpha_min   entries with alpha below this are skipped (1/255)
 *   T_min       a pixel stops before the entry that would take its
 *               transmittance below this (1e-4)
 *   alpha_max   alpha clamp (0.99)
 *   flags       GS_FLAG_* bits */
typedef struct gs_settings {
  int32_t tile;
  int32_t lds_batch;
  float bg[3];
  float alpha_min;
  float T_min;
  float alpha_max;
  int32_t flags;
  int32_t block_threads;
} gs_settings;

/* Fixed sizes of one rasterization problem; all views share width, height
 * and tile. */
typedef struct gs_geometry {
  int32_t n_views;
  int32_t width;
  int32_t height;
  int32_t tile;
  int32_t capacity;      /* Gaussian capacity (matches gs_params.capacity) */
  int32_t pad_;
  int64_t key_capacity;  /* max number of (view, Gaussian, tile) keys */
} gs_geometry;

/* Opaque host-side handle over a caller-provided device buffer. */
typedef struct gs_workspace gs_workspace;

/* Device pointers inside a workspace (for inspection and tests).
 *   records        [n_views][capacity] 48-byte records, three float4:
 *                  (px, py, A, B), (C, opacity, r, g),
 *                  (b, depth, u_lo | u_hi << 16, v_lo | v_hi << 16)
 *                  where (A, B, C) is the conic (inverse screen covariance)
 *                  and the last two words are integer bit patterns
 *   tiles_touched  [n_views][capacity] int32 (0 = culled)
 *   render_box     [n_views][capacity] two int32: (u_lo | u_hi << 16,
 *                  v_lo | v_hi << 16) of the render box; an empty box has
 *                  u_lo = v_lo = 0xffff and u_hi = v_hi = 0
 *   ranges         [n_views * tiles_y * tiles_x][2] uint32 [start, end)
 *   vals_sorted    [key_capacity] uint32 Gaussian index per sorted key
 *   keys_sorted    [key_capacity] uint64 (tile << 32 | depth bits), written
 *                  only with GS_FLAG_EMIT_KEYS
 *   grad2d         [n_views][5][capacity] dL/d(px, py, A, B, C)
 *   n_keys         device int64 key count of the last project_and_bin
 *   status         device int32 GS_STATUS_* bits (sticky until cleared)
 *   grad_opacity   [capacity] dL/d opacity, summed over the views
 *   grad_colour    [n_views][3][capacity] dL/d colour per view (only with
 *                  view-dependent colour)
 * The three gradient buffers hold what the last compositing backward added
 * until gs_project_bwd consumes and clears them. */
typedef struct gs_workspace_view {
  void* records;
  int32_t* tiles_touched;
  int32_t* render_box;
  uint32_t* ranges;
  uint32_t* vals_sorted;
  uint64_t* keys_sorted;
  float* grad2d;
  int64_t* n_keys;
  int32_t* status;
  int32_t tiles_x;
  int32_t tiles_y;
  float* grad_opacity;
  float* grad_colour;
} gs_workspace_view;

/* Host only.  Bytes of device memory a workspace for `geo` needs. */
GS_API int gs_workspace_size(const gs_geometry* geo, size_t* bytes);

/* Host only.  Creates a handle over `device_buffer` (at least
 * gs_workspace_size bytes, 256-byte aligned, owned by the caller and kept
 * alive while the handle is used).  The handle itself is host memory freed by
 * gs_workspace_destroy.  Clears the status word on `stream`. */
GS_API int gs_workspace_create(const gs_geometry* geo, void* device_buffer,
                        size_t bytes, void* stream, gs_workspace** out);
GS_API int gs_workspace_destroy(gs_workspace* ws);
GS_API int gs_workspace_get_view(const gs_workspace* ws, gs_workspace_view* out);

/* Projection and tile binning (Eq. 1-2).  For every view k and live
 * Gaussian g: transform the mean to camera space, cull when not in front of
 * the near plane or non-finite, form Sigma = R S S^T R^T, the EWA screen
 * covariance J W Sigma W^T J^T plus a 0.3 px^2 dilation, its conic, a radius
 * of ceil(3 sqrt(lambda_max)), the integer pixel box clipped to the image,
 * the render box (see GS_FLAG_FULL_BOX) and the number of screen tiles the
 * render box touches.  This front end runs in FP64 and publishes FP32
 * records (the render box bound in FP32 with slack).  The record's colour is
 * the Gaussian's colour in that view (gs_params: view-dependent when
 * sh_degree > 0, evaluated in FP32 from an FP64 direction).  Then counts the keys
 * per tile, derives
 * the ranges by an exclusive scan (n_keys stays on the device; more keys than
 * key_capacity set GS_STATUS_KEY_OVERFLOW and no key is written past the
 * capacity), and scatters every Gaussian index into each of its tiles'
 * segments (order within a segment unspecified until sort_tile_keys).
 *   cams  device gs_camera[n_views] */
GS_API int gs_project_and_bin(gs_workspace* ws, const gs_params* params,
                       const gs_camera* cams, const gs_settings* s,
                       void* stream);

/* Sorts every tile's segment by (depth, Gaussian index) ascending, so each
 * tile's list is front to back with ties in index order (vals_sorted); with
 * GS_FLAG_EMIT_KEYS also writes keys_sorted.  The result equals a stable sort
 * of the keys (tile << 32 | depth bits) emitted in (view, Gaussian, tile row,
 * tile column) order. */
GS_API int gs_sort_tile_keys(gs_workspace* ws, const gs_settings* s, void* stream);

/* Forward render (Eq. 3): per pixel, front to back over its tile's list,
 * evaluate only entries whose pixel box contains the pixel, alpha =
 * min(alpha_max, opacity * exp(-1/2 d^T conic d)) with d = mean2D - pixel,
 * skip alpha < alpha_min, stop before an entry that would take T below T_min,
 * C += colour * alpha * T.  Outputs (device, caller-owned):
 *   out_rgb   [n_views][3][H][W]  C + T_final * bg
 *   out_T     [n_views][H][W]     final transmittance
 *   out_nlast [n_views][H][W]     index in the tile list of the last
 *                                 contributing entry plus one (0 if none) */
GS_API int gs_render_fwd(gs_workspace* ws, const gs_params* params,
                  const gs_settings* s, float* out_rgb, float* out_T,
                  int32_t* out_nlast, void* stream);

/* gs_render_fwd that also writes, per pixel, the dominant Gaussian of
 * Eq. 8: the Gaussian with the largest blend weight alpha * T among the
 * contributing ones (the front-most on exact ties), or -1 when nothing
 * contributes.
 *   out_dom [n_views][H][W] device int32 */
GS_API int gs_render_dominant(gs_workspace* ws, const gs_params* params,
                              const gs_settings* s, float* out_rgb,
                              float* out_T, int32_t* out_nlast,
                              int32_t* out_dom, void* stream);

/* Clarity-enhancing densification (Eq. 9): counts the pixels of dom (from
 * gs_render_dominant) each Gaussian dominates and splits every live
 * Gaussian that dominates more than sigma of them into two children with
 * means mu + R(q) (s * xi[g][c]) (s = exp(log_scale), xi [capacity][2][3]
 * device standard-normal draws supplied by the caller), log-scales reduced
 * by log(1.6), rotation, opacity, colour and view-dependent colour
 * coefficients copied.  Child 0 takes the
 * parent's slot; child 1 is appended at the live count, in ascending parent
 * order.  Parents whose appended child would not fit in the capacity stay
 * unsplit and GS_STATUS_GAUSSIAN_OVERFLOW is set in *status_dev (may be
 * NULL).  Zeroes the Adam moments of every child (adam_m, adam_v may be
 * NULL); updates *params->n_dev; writes the number split to *n_split_dev
 * (may be NULL).
 *   dom      device int32 [n_pixels]
 *   scratch  device int32 [capacity + ceil(capacity / 1024) + 4], caller-owned */
GS_API int gs_densify(gs_params* params, gs_params* adam_m, gs_params* adam_v,
                      const int32_t* dom, int64_t n_pixels, int32_t sigma,
                      const float* xi, int32_t* scratch, int32_t* n_split_dev,
                      int32_t* status_dev, void* stream);

/* Work counters of the forward walk (same decisions as gs_render_fwd, no
 * image written), for roofline accounting.  ADDS to counts_dev[4] (device
 * uint64):
 *   [0] (pixel, entry) pairs examined: from the start of the pixel's tile
 *       list up to and including the entry at which the pixel stops
 *   [1] those of them whose pixel lies in the entry's render box (the
 *       integer box with GS_FLAG_FULL_BOX)
 *   [2] contributing (admitted and blended) pairs
 *   [3] in-box pairs at positions before the pixel's n_last (the pairs a
 *       backward pass revisits) */
GS_API int gs_count_pairs(gs_workspace* ws, const gs_params* params,
                          const gs_settings* s, uint64_t* counts_dev,
                          void* stream);

/* Backward of the compositing (exact derivative of Eq. 3 with the forward's
 * decisions): given dL/d(out_rgb) [n_views][3][H][W] and the forward's out_T
 * and out_nlast, walks each tile's list back to front recomputing every
 * entry's transmittance from T_final (no per-entry state is stored), ADDS
 * dL/d(colour) into grad->rgb (with params->sh_degree > 0: accumulates it per
 * view into the workspace instead) and accumulates dL/d(mean2D, conic) per
 * view and dL/d(opacity) into the workspace, where gs_project_bwd consumes
 * them.  grad->sh_degree must equal params->sh_degree.
 * Clamped alphas pass no gradient to opacity or shape.  Call
 * gs_project_bwd afterwards, on the same stream, to finish the backward. */
GS_API int gs_render_bwd(gs_workspace* ws, const gs_params* params,
                         const gs_settings* s, const float* dL_drgb,
                         const float* T_final, const int32_t* n_last,
                         gs_params* grad, void* stream);

/* gs_render_bwd with the L1 photometric term of the map-optimisation loss
 * (Eq. 10-11, L1 part) fused in: instead of reading a dL/d(out_rgb) buffer,
 * every pixel forms dL/dC = lambda * sign(out_rgb - target) / (3HW)
 * (sign(0) = 0) from the forward's image, exactly as gs_loss_l1 writes it,
 * and the call ADDS lambda * mean over 3HW of |out_rgb - target|, summed
 * over views, to *loss_dev (device double) and each view's squared-error sum
 * to sqerr_dev[n_views] (device double, may be NULL).  The gradient then
 * flows as in gs_render_bwd.  Equivalent to gs_loss_l1 followed by
 * gs_render_bwd without the dL buffer's write and read.  The sums are taken
 * per tile, then over tiles in a fixed order, so repeated calls add the same
 * bits.  The workspace holds the per-tile partials: calls that share a
 * workspace must not overlap.
 *   out_rgb, target  device float [n_views][3][H][W] */
GS_API int gs_render_bwd_l1(gs_workspace* ws, const gs_params* params,
                            const gs_settings* s, const float* out_rgb,
                            const float* target, float lambda,
                            const float* T_final, const int32_t* n_last,
                            gs_params* grad, double* loss_dev,
                            double* sqerr_dev, void* stream);

/* Backward of the projection (Eq. 1-2, FP64): chains the screen-space
 * gradients that gs_render_bwd left in the workspace, summed over the views,
 * through the conic, the EWA covariance, the Jacobian and the view transform
 * to the mean, log-scale and quaternion, and the opacity gradient through the
 * sigmoid; with sh_degree > 0 also the per-view colour gradients through
 * the clamp and the harmonics to rgb, sh and (through the viewing direction)
 * the mean.  ADDS them into `grad` (same layout as gs_params; the caller
 * zeroes it) and clears the workspace's screen-space and colour gradients
 * for the next backward.  cams as in gs_project_and_bin. */
GS_API int gs_project_bwd(gs_workspace* ws, const gs_params* params,
                          const gs_camera* cams, gs_params* grad,
                          void* stream);

/* Photometric term of the map-optimisation loss (Eq. 10-11, L1 part):
 * per view lambda * mean over 3HW of |rgb - target|; writes dL/drgb =
 * lambda * sign(rgb - target) / (3HW) (sign(0) = 0) and ADDS the loss summed
 * over views to *loss_dev (device double) and the per-view squared error sum
 * to sqerr_dev[n_views] (device double, may be NULL) for PSNR. */
GS_API int gs_loss_l1(const float* rgb, const float* target, int32_t n_views,
               int32_t height, int32_t width, float lambda, float* dL_drgb,
               double* loss_dev, double* sqerr_dev, void* stream);

/* Structural-similarity term of the colour loss (Eq. 10, the term weighted
 * by lambda_photo): per view and channel, SSIM over an 11 x 11 Gaussian
 * window (sigma 1.5, normalised; samples outside the image are 0) with
 * C1 = 0.01^2, C2 = 0.03^2.  ADDS lambda * sum over views of (1 - mean SSIM
 * over 3HW) to *loss_dev (device double), ADDS its gradient into dL_drgb
 * (call after gs_loss_l1, which writes it), and ADDS each view's mean SSIM
 * into ssim_dev[n_views] (device double, may be NULL).
 *   rgb, target, dL_drgb  device float [n_views][3][height][width]
 *   scratch               device float [3][n_views][3][height][width],
 *                         caller-owned, overwritten */
GS_API int gs_loss_ssim(const float* rgb, const float* target, int32_t n_views,
                        int32_t height, int32_t width, float lambda,
                        float* dL_drgb, double* loss_dev, double* ssim_dev,
                        float* scratch, void* stream);

/* The whole colour loss of Eq. 10 in the two passes of gs_loss_ssim:
 * lambda_l1 * (L1 term of gs_loss_l1) + lambda_ssim * (SSIM term of
 * gs_loss_ssim), i.e. lambda_color (1 - lambda_photo) and lambda_color
 * lambda_photo.  WRITES dL_drgb (the sum of both gradients), ADDS both terms
 * to *loss_dev, the per-view squared-error sums to sqerr_dev[n_views] and the
 * per-view mean SSIM to ssim_dev[n_views] (both may be NULL).  Equivalent to
 * gs_loss_l1 then gs_loss_ssim, without the L1 pass over the images.
 *   rgb, target, dL_drgb, scratch  as in gs_loss_ssim */
GS_API int gs_loss_colour(const float* rgb, const float* target,
                          int32_t n_views, int32_t height, int32_t width,
                          float lambda_l1, float lambda_ssim, float* dL_drgb,
                          double* loss_dev, double* sqerr_dev,
                          double* ssim_dev, float* scratch, void* stream);

/* Planar regulariser of Eq. 10-11: lambda * mean over live Gaussians of
 * max(floor, min_j exp(log_scale_j)).  ADDS its gradient into
 * grad->log_scale (smallest axis only, lowest index on ties, only where the
 * smallest scale exceeds the floor) and the term to *loss_dev. */
GS_API int gs_planar_reg(const gs_params* params, float lambda, float floor_,
                  gs_params* grad, double* loss_dev, void* stream);

/* Adam step (the optimiser is not fixed by the paper) over the live entries
 * of the 14 parameter rows and the GS_SH_ROWS(sh_degree) coefficient rows.
 * lr[5] = learning rates of mean, log_scale, quat, opacity_logit, rgb; with
 * sh_degree > 0, lr[6], lr[5] being the coefficients'.  m and v are moment
 * arrays of the params layout (same sh_degree).
 * The bias-correction step count is *step_dev (device int32) when step_dev
 * is not NULL - so a captured graph can advance it on the device - and
 * `step` otherwise; it must be >= 1. */
GS_API int gs_adam(gs_params* params, const gs_params* grad, gs_params* m,
                   gs_params* v, const float* lr, float beta1, float beta2,
                   float eps, int32_t step, const int32_t* step_dev,
                   void* stream);

/* Keyframe insertion (Eq. 6 with an accumulated-alpha mask).  Candidates are
 * the 3x3 pixel patch around each of the n_pts centres pts_uvd [n][3] =
 * (u, v, inverse depth) (device), visited patch by patch, pixels row-major
 * (or only the centre pixel when centre_only != 0); candidate c is patch
 * c / 9, pixel c % 9 (c = patch with centre_only).  A candidate inside the
 * image is kept when 1 - kf_T_final(u, v) <= alpha_skip.  Kept candidates,
 * in visiting order, are appended at the live count: mean = R^T(K^-1
 * [u v 1]^T / d - t), colour = kf_rgb [3][H][W] at the pixel, opacity logit
 * 0, identity rotation and log-scale log(z / fx) on every axis - or, when
 * mlp_out is not NULL, log-scale, opacity logit and colour from row c of
 * mlp_out [candidates][7] (log-scale 3, opacity logit, RGB 3).  The
 * view-dependent colour coefficients of new entries are zero.  Zeroes the
 * Adam moments of the new entries (m, v may be NULL), updates
 * *params->n_dev, and sets GS_STATUS_GAUSSIAN_OVERFLOW in *status_dev when
 * capacity would be exceeded (nothing past capacity is written).  At most
 * 9 * n_pts <= 65536 candidates.  n_inserted_dev: device int32 receiving the
 * number kept before the capacity check (may be NULL).
 *   cam  device gs_camera (the keyframe's) */
GS_API int gs_insert_gaussians(gs_params* params, gs_params* adam_m,
                               gs_params* adam_v, const gs_camera* cam,
                               int32_t width, int32_t height,
                               const float* kf_rgb, const float* kf_T_final,
                               const float* pts_uvd, int32_t n_pts,
                               float alpha_skip, int32_t centre_only,
                               const float* mlp_out, int32_t* n_inserted_dev,
                               int32_t* status_dev, void* stream);

/* The paper's own insertion test (Eq. 7): same candidates, candidate order,
 * back-projection, initialisation, capacity handling and outputs as
 * gs_insert_gaussians, but a candidate inside the image (d > 0) is kept when
 * the distance from its back-projected point to the nearest live Gaussian
 * mean exceeds tau (strict; the equation's "<" is read as ">", as its text
 * states; every candidate is kept when the map is empty).  Distances are
 * FP64 from the FP32 means, against the map as it was before the call.
 *   scratch  device uint64 [candidates], caller-owned: receives the FP64
 *            bit pattern of each candidate's nearest squared distance (all
 *            ones for an empty map or a candidate that was not tested) */
GS_API int gs_insert_distance(gs_params* params, gs_params* adam_m,
                              gs_params* adam_v, const gs_camera* cam,
                              int32_t width, int32_t height,
                              const float* kf_rgb, const float* pts_uvd,
                              int32_t n_pts, float tau, int32_t centre_only,
                              const float* mlp_out, uint64_t* scratch,
                              int32_t* n_inserted_dev, int32_t* status_dev,
                              void* stream);

/* gs_insert_distance for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results without `scratch`.
 * The per-candidate scratch is a file-scope device array of the library,
 * 65536 candidates (512 KiB) per GPU, held until the process ends; more
 * candidates (9 n_pts, or n_pts with centre_only) return GS_E_CAPACITY
 * before any launch.  The call allocates nothing.  All calls on one GPU
 * share that GPU's array: calls that overlap on one GPU race. */
GS_API int gs_insert_distance_noalloc(gs_params* params, gs_params* adam_m,
                                      gs_params* adam_v, const gs_camera* cam,
                                      int32_t width, int32_t height,
                                      const float* kf_rgb,
                                      const float* pts_uvd, int32_t n_pts,
                                      float tau, int32_t centre_only,
                                      const float* mlp_out,
                                      int32_t* n_inserted_dev,
                                      int32_t* status_dev, void* stream);

/* Learned initialisation: the parameter vector of the network
 * (32 -> 64 -> 64 -> 7, GELU) holds GS_MLP_PARAMS FP32 master weights,
 * W1 [32][64], b1 [64], W2 [64][64], b2 [64], W3 [64][7], b3 [7], each layer
 * computing z = x W + b.  Weights, inputs and hidden activations are rounded
 * to BF16 where they enter a product (BF16 MFMA, FP32 accumulate). */
#define GS_MLP_PARAMS 6727
#define GS_MLP_IN 32
#define GS_MLP_OUT 7

/* Features of every insertion candidate (same candidate order as
 * gs_insert_gaussians), feats [candidates][32] (device FP32): the 3x3 RGB
 * neighbourhood of the candidate pixel in kf_rgb (27, neighbours row-major,
 * channels interleaved, 0 outside the image), the inverse depth, the mean
 * log-distance (m, floor 1e-6) from the back-projected point to its 8
 * nearest existing Gaussian means (exact search, FP64 distances, ties to the
 * lower index) and their inverse-distance-weighted mean colour (0 when the
 * map is empty).  knn_idx / knn_dist [candidates][8] (may be NULL) receive
 * the neighbours (-1 / 0 past the live count). */
GS_API int gs_knn_features(const gs_params* params, const gs_camera* cam,
                           int32_t width, int32_t height, const float* kf_rgb,
                           const float* pts_uvd, int32_t n_pts,
                           int32_t centre_only, float* feats, int32_t* knn_idx,
                           float* knn_dist, void* stream);

/* Forward pass: x [m][32] -> y [m][7].  cache [m][128] (may be NULL)
 * receives the two hidden pre-activations for gs_mlp_bwd. */
GS_API int gs_mlp_fwd(const float* weights, const float* x, int32_t m,
                      float* y, float* cache, void* stream);

/* Mean squared error over the m x 7 outputs: dy = 2 (y - target) / (7 m);
 * ADDS the loss to *loss_dev (device double, may be NULL). */
GS_API int gs_mlp_mse(const float* y, const float* target, int32_t m,
                      float* dy, double* loss_dev, void* stream);

/* Backward pass from dy [m][7]: ACCUMULATES (+=) the gradient of the
 * parameter vector into dweights [GS_MLP_PARAMS] (caller zeroes it). */
GS_API int gs_mlp_bwd(const float* weights, const float* x,
                      const float* cache, const float* dy, int32_t m,
                      float* dweights, void* stream);

/* Adam step on the parameter vector (step >= 1 for bias correction). */
GS_API int gs_mlp_adam(float* weights, const float* dweights, float* adam_m,
                       float* adam_v, float lr, float beta1, float beta2,
                       float eps, int32_t step, void* stream);

/* ---- One mapping iteration of a keyframe window as a HIP graph ----
 *
 * The map optimisation (Methodology: Map Optimization with Planar
 * Regularization, Eq. 10-11) runs the same iteration over the keyframe
 * window many times.  gs_window_build captures one iteration, on the
 * caller's stream, into a HIP graph the handle owns (the executable graph
 * only: the handle holds no device memory; every buffer below is borrowed
 * and must outlive it), gs_window_run replays it, gs_window_destroy frees
 * it.  The iteration, in order:
 *   clear grad (every row, the live and the spare capacity), *loss_dev and
 *   sqerr_dev[n_views] to zero;
 *   gs_project_and_bin, gs_sort_tile_keys, gs_render_fwd into out_rgb,
 *   out_T, out_nlast;
 *   with GS_WINDOW_PLANAR_REG, gs_planar_reg(lambda_reg, reg_floor);
 *   gs_render_bwd_l1 against target with lambda_l1;
 *   gs_project_bwd;
 *   with GS_WINDOW_ADAM, gs_adam(lr, beta1, beta2, eps, step_dev) and then
 *   *step_dev += 1, so the next run uses the next bias correction (the
 *   graph advances the count in its clearing kernel and has the Adam step
 *   read the count minus one: the same values, one launch fewer).
 * Each call is checked on the host at build time as the call itself checks
 * its arguments (GS_E_INVALID / GS_E_CAPACITY, nothing captured); the graph
 * keeps the pointers, sizes and settings of the build: rebuild after the
 * workspace, a buffer or a setting changes.  The live Gaussian count is read
 * on the device (params.n_dev), so insertion between runs needs no rebuild.
 * The stream must not be the null stream and must not be capturing.  Runs,
 * like the calls they replay, do not overlap other work on the same
 * workspace or buffers.  Device-side overflows are reported by
 * gs_read_status as usual.
 *   out_rgb [V][3][H][W], out_T [V][H][W], out_nlast [V][H][W], target
 *   [V][3][H][W] device; loss_dev device double; sqerr_dev device double
 *   [V] or NULL; grad, adam_m, adam_v of the params layout; lr as in
 *   gs_adam. */
#define GS_WINDOW_PLANAR_REG 1
#define GS_WINDOW_ADAM 2
typedef struct gs_window gs_window;
typedef struct gs_window_desc {
  gs_workspace* ws;
  gs_params params;
  const gs_camera* cams;
  gs_settings settings;
  float* out_rgb;
  float* out_T;
  int32_t* out_nlast;
  const float* target;
  float lambda_l1;
  float lambda_reg;
  float reg_floor;
  int32_t flags;
  double* loss_dev;
  double* sqerr_dev;
  gs_params grad;
  gs_params adam_m;
  gs_params adam_v;
  float lr[6];
  float beta1;
  float beta2;
  float eps;
  int32_t pad_;
  int32_t* step_dev;
} gs_window_desc;

GS_API int gs_window_build(const gs_window_desc* desc, void* stream,
                           gs_window** out);
GS_API int gs_window_run(gs_window* window, void* stream);
GS_API int gs_window_destroy(gs_window* window);

/* Synchronises `stream`, then reads the workspace's status bits and key
 * count (either output may be NULL).  Returns GS_E_OVERFLOW when any status
 * bit is set, GS_OK otherwise.  clear != 0 resets the status word. */
GS_API int gs_read_status(gs_workspace* ws, void* stream, int32_t* flags,
                   int64_t* n_keys, int32_t clear);

/* Text of the last error on the calling host thread ("" if none). */
GS_API const char* gs_last_error(void);

/* Library version string. */
GS_API const char* gs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GSMAP_H */
