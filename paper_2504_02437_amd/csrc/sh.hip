// View-dependent colour: the Gaussians' colour coefficients (the parameter
// list after Eq. 1) as real spherical harmonics of degree 1..3 of the
// viewing direction, added to the base colour and clamped at zero (the form
// of 3D Gaussian Splatting, which the method builds on).
//
// k_sh_colour runs after the projection and overwrites the colour of every
// binned (view, Gaussian) record with the Gaussian's colour in that view.
// The record already carries a colour per view, so the compositing kernels
// are unchanged: view-dependent colour adds no bytes per (pixel, Gaussian)
// pair.  k_sh_bwd chains the per-view colour gradients that the compositing
// backward accumulated in the workspace through the clamp and the harmonics
// to the base colour, the coefficients and, through the direction, the mean.
//
// One thread per Gaussian loops over the views, so the coefficients are read
// from HBM once per call (coalesced planar rows) and stay in registers.  The
// direction is formed in FP64 (the mean minus the camera centre -R^T t,
// normalised), the harmonics and sums in FP32.  This unit is compiled with
// -ffp-contract=off, so the forward and the backward evaluate the same
// roundings and take the same clamp decision.

#include <math.h>

#include "gs_internal.h"

namespace gs {
namespace {

// Normalisation constants of the real harmonics.
constexpr float kY1 = 0.4886025119029199f;    // sqrt(3 / (4 pi))
constexpr float kY2a = 1.0925484305920792f;   // sqrt(15 / pi) / 2
constexpr float kY2b = 0.31539156525252005f;  // sqrt(5 / pi) / 4
constexpr float kY2c = 0.5462742152960396f;   // sqrt(15 / pi) / 4
constexpr float kY3a = 0.5900435899266435f;   // sqrt(35 / (2 pi)) / 4
constexpr float kY3b = 2.890611442640554f;    // sqrt(105 / pi) / 2
constexpr float kY3c = 0.4570457994644658f;   // sqrt(21 / (2 pi)) / 4
constexpr float kY3d = 0.3731763325901154f;   // sqrt(7 / pi) / 4
constexpr float kY3e = 1.445305721320277f;    // sqrt(105 / pi) / 4

// Y[j - 1] = Y_j(x, y, z) for j = 1 .. (D+1)^2 - 1, order l = 1..D,
// m = -l..l; (x, y, z) is a unit vector.
template <int D>
__device__ inline void basis(float x, float y, float z, float* Y) {
  Y[0] = -kY1 * y;
  Y[1] = kY1 * z;
  Y[2] = -kY1 * x;
  if (D >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[3] = kY2a * (x * y);
    Y[4] = -kY2a * (y * z);
    Y[5] = kY2b * ((2.f * zz - xx) - yy);
    Y[6] = -kY2a * (x * z);
    Y[7] = kY2c * (xx - yy);
    if (D >= 3) {
      Y[8] = -kY3a * (y * (3.f * xx - yy));
      Y[9] = kY3b * ((x * y) * z);
      Y[10] = -kY3c * (y * ((4.f * zz - xx) - yy));
      Y[11] = kY3d * (z * ((2.f * zz - 3.f * xx) - 3.f * yy));
      Y[12] = -kY3c * (x * ((4.f * zz - xx) - yy));
      Y[13] = kY3e * (z * (xx - yy));
      Y[14] = -kY3a * (x * (xx - 3.f * yy));
    }
  }
}

// Gradient of sum_j w[j - 1] Y_j with respect to (x, y, z), each Y_j taken
// as the polynomial written in basis() (the radial part is projected out by
// the caller).
template <int D>
__device__ inline void basis_vjp(float x, float y, float z, const float* w,
                                 float& gx, float& gy, float& gz) {
  gx = -kY1 * w[2];
  gy = -kY1 * w[0];
  gz = kY1 * w[1];
  if (D >= 2) {
    gx += kY2a * (y * w[3] - z * w[6]) + 2.f * x * (kY2c * w[7] - kY2b * w[5]);
    gy += kY2a * (x * w[3] - z * w[4]) - 2.f * y * (kY2b * w[5] + kY2c * w[7]);
    gz += -kY2a * (y * w[4] + x * w[6]) + 4.f * kY2b * z * w[5];
    if (D >= 3) {
      const float xx = x * x, yy = y * y, zz = z * z;
      const float xy = x * y, xz = x * z, yz = y * z;
      gx += -6.f * kY3a * xy * w[8] + kY3b * yz * w[9] +
            2.f * kY3c * xy * w[10] - 6.f * kY3d * xz * w[11] -
            kY3c * ((4.f * zz - 3.f * xx) - yy) * w[12] +
            2.f * kY3e * xz * w[13] - 3.f * kY3a * (xx - yy) * w[14];
      gy += -3.f * kY3a * (xx - yy) * w[8] + kY3b * xz * w[9] -
            kY3c * ((4.f * zz - xx) - 3.f * yy) * w[10] -
            6.f * kY3d * yz * w[11] + 2.f * kY3c * xy * w[12] -
            2.f * kY3e * yz * w[13] + 6.f * kY3a * xy * w[14];
      gz += kY3b * xy * w[9] - 8.f * kY3c * yz * w[10] +
            kY3d * ((6.f * zz - 3.f * xx) - 3.f * yy) * w[11] -
            8.f * kY3c * xz * w[12] + kY3e * (xx - yy) * w[13];
    }
  }
}

// Unit direction from the camera centre to the mean and 1 / distance; a mean
// at the centre (culled in that view: before the near plane) gets zeros.
__device__ inline void view_dir(const gs_camera& c, double mx, double my,
                                double mz, float& x, float& y, float& z,
                                float& inv_r) {
  const double t0 = c.t[0], t1 = c.t[1], t2 = c.t[2];
  const double ox = -(((double)c.R[0] * t0 + (double)c.R[3] * t1) + (double)c.R[6] * t2);
  const double oy = -(((double)c.R[1] * t0 + (double)c.R[4] * t1) + (double)c.R[7] * t2);
  const double oz = -(((double)c.R[2] * t0 + (double)c.R[5] * t1) + (double)c.R[8] * t2);
  const double vx = mx - ox, vy = my - oy, vz = mz - oz;
  const double r2 = (vx * vx + vy * vy) + vz * vz;
  if (!(r2 > 0.0)) {
    x = y = z = inv_r = 0.f;
    return;
  }
  const double ir = 1.0 / sqrt(r2);
  x = (float)(vx * ir);
  y = (float)(vy * ir);
  z = (float)(vz * ir);
  inv_r = (float)ir;
}

struct ShArgs {
  const float* mean;
  const float* rgb;
  const float* sh;
  const int32_t* n_dev;
  int cap;
  const gs_camera* cams;
  int V;
  const int32_t* tiles;
  Record* rec;      // forward: colours overwritten
  float* gcol;      // backward: [V][3][cap], zeroed after reading
  float* d_mean;
  float* d_rgb;
  float* d_sh;
};

template <int D>
__device__ inline void raw_colour(const float (*f)[3], const float* base,
                                  const float* Y, float* raw) {
  constexpr int NR = (D + 1) * (D + 1) - 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float acc = base[c];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc = fmaf(Y[j], f[j][c], acc);
    raw[c] = acc;
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_sh_colour(ShArgs a) {
  constexpr int NR = (D + 1) * (D + 1) - 1;
  const int g = blockIdx.x * 256 + threadIdx.x;
  const int n = min(*a.n_dev, a.cap);
  if (g >= n) return;
  const int cap = a.cap;
  float f[NR][3];
#pragma unroll
  for (int j = 0; j < NR; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) f[j][c] = a.sh[(size_t)(3 * j + c) * cap + g];
  const float base[3] = {a.rgb[g], a.rgb[cap + g], a.rgb[2 * (size_t)cap + g]};
  const double mx = a.mean[g], my = a.mean[cap + g], mz = a.mean[2 * (size_t)cap + g];
  for (int k = 0; k < a.V; ++k) {
    const size_t slot = (size_t)k * cap + g;
    if (a.tiles[slot] == 0) continue;
    float x, y, z, ir;
    view_dir(a.cams[k], mx, my, mz, x, y, z, ir);
    float Y[NR], raw[3];
    basis<D>(x, y, z, Y);
    raw_colour<D>(f, base, Y, raw);
    Record* R = a.rec + slot;
    R->q1.z = raw[0] >= 0.f ? raw[0] : 0.f;
    R->q1.w = raw[1] >= 0.f ? raw[1] : 0.f;
    R->q2.x = raw[2] >= 0.f ? raw[2] : 0.f;
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_sh_bwd(ShArgs a) {
  constexpr int NR = (D + 1) * (D + 1) - 1;
  const int g = blockIdx.x * 256 + threadIdx.x;
  const int n = min(*a.n_dev, a.cap);
  if (g >= n) return;
  const int cap = a.cap;
  float f[NR][3], dsh[NR][3];
#pragma unroll
  for (int j = 0; j < NR; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      f[j][c] = a.sh[(size_t)(3 * j + c) * cap + g];
      dsh[j][c] = 0.f;
    }
  const float base[3] = {a.rgb[g], a.rgb[cap + g], a.rgb[2 * (size_t)cap + g]};
  const double mx = a.mean[g], my = a.mean[cap + g], mz = a.mean[2 * (size_t)cap + g];
  float drgb[3] = {0.f, 0.f, 0.f}, dm[3] = {0.f, 0.f, 0.f};
  bool any = false;
  for (int k = 0; k < a.V; ++k) {
    const size_t slot = (size_t)k * cap + g;
    if (a.tiles[slot] == 0) continue;
    float* gk = a.gcol + (size_t)k * 3 * cap + g;
    float gc[3] = {gk[0], gk[cap], gk[2 * (size_t)cap]};
    if (gc[0] == 0.f && gc[1] == 0.f && gc[2] == 0.f) continue;
    gk[0] = 0.f;
    gk[cap] = 0.f;
    gk[2 * (size_t)cap] = 0.f;
    any = true;
    float x, y, z, ir;
    view_dir(a.cams[k], mx, my, mz, x, y, z, ir);
    float Y[NR], raw[3];
    basis<D>(x, y, z, Y);
    raw_colour<D>(f, base, Y, raw);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      gc[c] = raw[c] >= 0.f ? gc[c] : 0.f;
      drgb[c] += gc[c];
    }
    float w[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
#pragma unroll
      for (int c = 0; c < 3; ++c) dsh[j][c] = fmaf(Y[j], gc[c], dsh[j][c]);
      w[j] = (f[j][0] * gc[0] + f[j][1] * gc[1]) + f[j][2] * gc[2];
    }
    float gx, gy, gz;
    basis_vjp<D>(x, y, z, w, gx, gy, gz);
    // Through the normalisation d = v / |v|: (I - d d^T) / |v|.
    const float dot = (gx * x + gy * y) + gz * z;
    dm[0] += (gx - x * dot) * ir;
    dm[1] += (gy - y * dot) * ir;
    dm[2] += (gz - z * dot) * ir;
  }
  if (!any) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a.d_rgb[(size_t)c * cap + g] += drgb[c];
    a.d_mean[(size_t)c * cap + g] += dm[c];
  }
#pragma unroll
  for (int j = 0; j < NR; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) a.d_sh[(size_t)(3 * j + c) * cap + g] += dsh[j][c];
}

ShArgs make_args(gs_workspace* ws, const gs_params* p, const gs_camera* cams) {
  ShArgs a;
  a.mean = p->mean; a.rgb = p->rgb; a.sh = p->sh; a.n_dev = p->n_dev;
  a.cap = p->capacity; a.cams = cams; a.V = ws->geo.n_views;
  a.tiles = ws->tiles_touched; a.rec = ws->records; a.gcol = ws->gcol;
  a.d_mean = a.d_rgb = a.d_sh = nullptr;
  return a;
}

}  // namespace

hipError_t launch_sh_colour(gs_workspace* ws, const gs_params* p,
                            const gs_camera* cams, hipStream_t st) {
  const ShArgs a = make_args(ws, p, cams);
  const dim3 grid((p->capacity + 255) / 256), block(256);
  if (p->capacity <= 0 || p->sh_degree <= 0) return hipSuccess;
  switch (p->sh_degree) {
    case 1: hipLaunchKernelGGL(k_sh_colour<1>, grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_sh_colour<2>, grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL(k_sh_colour<3>, grid, block, 0, st, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_sh_bwd(gs_workspace* ws, const gs_params* p,
                         const gs_camera* cams, gs_params* grad,
                         hipStream_t st) {
  ShArgs a = make_args(ws, p, cams);
  a.d_mean = grad->mean; a.d_rgb = grad->rgb; a.d_sh = grad->sh;
  const dim3 grid((p->capacity + 255) / 256), block(256);
  if (p->capacity <= 0 || p->sh_degree <= 0) return hipSuccess;
  switch (p->sh_degree) {
    case 1: hipLaunchKernelGGL(k_sh_bwd<1>, grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_sh_bwd<2>, grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL(k_sh_bwd<3>, grid, block, 0, st, a); break;
  }
  return hipGetLastError();
}

}  // namespace gs
