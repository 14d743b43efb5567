// The view-independent part of the projection (Eq. 1), per Gaussian: the
// 3D covariance from the log-scales and the normalised quaternion, and the
// opacity with its base-2 logarithm; and per view the FP64 camera constants
// of the projection backward.  Formed once per Gaussian before the
// per-view projection reads it: by k_shape, or, in the window graph, by the
// first workgroups of the kernel that clears the iteration.
#pragma once

#include <math.h>

#include "gs_internal.h"

namespace gs {

// View-independent part of Eq. 1: s = exp(l), R(q / |q|), M = R diag(s),
// Sigma = M M^T.
struct Shape {
  double s[3];
  double qn[4];
  double qnorm;
  double R[9];
  double M[9];
  double Sig[9];
  bool ok;
};

__device__ inline void make_shape(const float* lsc, const float* quat, int cap,
                                  int g, Shape& S) {
  for (int j = 0; j < 3; ++j) S.s[j] = exp((double)lsc[j * cap + g]);
  double q[4];
  for (int j = 0; j < 4; ++j) q[j] = (double)quat[j * cap + g];
  const double qq = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  S.qnorm = sqrt(qq);
  S.ok = S.qnorm > 0.0 && isfinite(S.qnorm) && isfinite(S.s[0]) &&
         isfinite(S.s[1]) && isfinite(S.s[2]);
  for (int j = 0; j < 4; ++j) S.qn[j] = q[j] / S.qnorm;
  const double w = S.qn[0], x = S.qn[1], y = S.qn[2], z = S.qn[3];
  double* R = S.R;
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) S.M[3 * i + j] = R[3 * i + j] * S.s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      S.Sig[3 * i + j] = (S.M[3 * i] * S.M[3 * j] + S.M[3 * i + 1] * S.M[3 * j + 1]) +
                         S.M[3 * i + 2] * S.M[3 * j + 2];
}

// Upper-triangle entries of the symmetric 3x3 covariance.
constexpr int kSigIdx[6] = {0, 1, 2, 4, 5, 8};

// Where the per-Gaussian shape goes: Sigma's upper triangle [6][cap] (FP64),
// the opacity and its base-2 logarithm [cap] each.
struct ShapeJob {
  const float* lsc;
  const float* quat;
  const float* opl;
  const int32_t* n_dev;
  int cap;
  double* sig;   // sig[0][g] = NaN: a failed shape
  float* op;
  float* lop;
};

ShapeJob shape_job(const gs_workspace* ws, const gs_params* p);

// Gaussian g (any g: those past the live count do nothing).
__device__ inline void shape_one(const ShapeJob& j, int g) {
  const int n = min(*j.n_dev, j.cap);
  if (g >= n) return;
  const int cap = j.cap;
  Shape S;
  make_shape(j.lsc, j.quat, cap, g, S);
  for (int i = 0; i < 6; ++i) j.sig[(size_t)i * cap + g] = S.Sig[kSigIdx[i]];
  // A failed shape (zero or non-finite quaternion, non-finite scale) is
  // culled in every view; a valid one has a finite, non-negative Sigma_00.
  if (!S.ok) j.sig[g] = NAN;
  const float op = (float)(1.0 / (1.0 + exp(-(double)j.opl[g])));
  j.op[g] = op;
  j.lop[g] = (float)log2((double)op);
}

// FP64 camera constants of the projection and its backward, kCamDoubles
// per view: the rotation (row-major), the translation, fx, fy, the
// backward's clamp limits of the projected position, the near-plane depth,
// cx, cy and the projection's clamp limits, each formed exactly as the
// per-lane code formed it from the camera record.  Written, from the
// cameras of the call, by the launch before the projection (k_shape, or the
// window graph's clearing launch, so they follow camera updates between
// replays); the kernels read them by scalar loads and hold them in scalar
// registers instead of converting them in every lane.
constexpr int kCamDoubles = 21;

struct CamD {
  double W[9], t[3], fx, fy, limx, limy, near_z, cx, cy, flimx, flimy;
};

__device__ inline CamD cam_d(const gs_camera& c) {
  CamD d;
  for (int i = 0; i < 9; ++i) d.W[i] = (double)c.R[i];
  for (int i = 0; i < 3; ++i) d.t[i] = (double)c.t[i];
  d.fx = (double)c.fx;
  d.fy = (double)c.fy;
  d.limx = 0.65 * (double)c.width / d.fx;
  d.limy = 0.65 * (double)c.height / d.fy;
  d.near_z = (double)c.near_z;
  d.cx = (double)c.cx;
  d.cy = (double)c.cy;
  d.flimx = 1.3 * ((double)c.width / (2.0 * d.fx));
  d.flimy = 1.3 * ((double)c.height / (2.0 * d.fy));
  return d;
}

// Entry i of a view's constants, in CamD's field order.
__device__ inline double cam_d_entry(const gs_camera& c, int i) {
  const CamD d = cam_d(c);
  if (i < 9) return d.W[i];
  if (i < 12) return d.t[i - 9];
  switch (i) {
    case 12: return d.fx;
    case 13: return d.fy;
    case 14: return d.limx;
    case 15: return d.limy;
    case 16: return d.near_z;
    case 17: return d.cx;
    case 18: return d.cy;
    case 19: return d.flimx;
    default: return d.flimy;
  }
}

using ConstDouble = const __attribute__((address_space(4))) double;

// A view's constants from the table (uniform: scalar loads).
__device__ inline CamD cam_d_table(ConstDouble* t) {
  CamD d;
  for (int i = 0; i < 9; ++i) d.W[i] = t[i];
  for (int i = 0; i < 3; ++i) d.t[i] = t[9 + i];
  d.fx = t[12]; d.fy = t[13]; d.limx = t[14]; d.limy = t[15];
  d.near_z = t[16];
  d.cx = t[17]; d.cy = t[18]; d.flimx = t[19]; d.flimy = t[20];
  return d;
}

// Workgroup 0 of a launch writes the V views' constants.
__device__ inline void cam_d_fill(const gs_camera* cams, int V, double* out) {
  if (blockIdx.x != 0) return;
  for (int i = threadIdx.x; i < kCamDoubles * V; i += blockDim.x)
    out[i] = cam_d_entry(cams[i / kCamDoubles], i % kCamDoubles);
}

}  // namespace gs
