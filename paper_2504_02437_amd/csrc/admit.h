// Conservative bounds on where the compositing kernels can admit a Gaussian.
//
// The kernels admit a (pixel, entry) pair only when their FP32 alpha =
// min(alpha_max, exp2(e2)) reaches alpha_min, with e2 the FP32 evaluation of
// log2(o) - log2(e)/2 * q(d), q(d) = A dx^2 + 2 B dx dy + C dy^2 over the
// published record (d = mean2D - pixel).  The rounding error of e2 is below
// u (8 S + 4 |log2 o|) (u = 2^-24, S the sum of the magnitudes of the three
// quadratic terms, log2(o) rounded once), and exp2 adds less than 2^-20
// relative.  So an admitted pixel of the integer box satisfies
//   q(d) <= 2 ln(o / alpha_min) + 2 ln(2) (u (16 S_max + 4 |log2 o|) + 2^-19)
//        =: L,
// with S_max bounding S over the box.  L is formed in FP32 with relative and
// absolute slack well above its own rounding.
#pragma once

#include "gs_internal.h"

namespace gs {

constexpr float kNoPixel = -1.f;   // admit_level: no pixel can be admitted

// L for record R and its integer box [iu0, iu1] x [iv0, iv1]; kNoPixel when
// o is below alpha_min (then o * G < alpha_min for every G <= 1), +inf when
// the conic is not positive definite (no bound).
__device__ inline float admit_level(const Record& R, int iu0, int iu1, int iv0,
                                    int iv1, float amin) {
  const float px = R.q0.x, py = R.q0.y, A = R.q0.z, B = R.q0.w;
  const float C = R.q1.x, o = R.q1.y;
  if (!(o >= amin * (1.f - 0x1p-19f))) return kNoPixel;
  const double det = (double)A * (double)C - (double)B * (double)B;
  if (!(det > 0.0) || !(A > 0.f) || !(C > 0.f)) return INFINITY;
  const float dxm = fmaxf(fabsf(px - (float)iu0), fabsf((float)iu1 - px)) + 1.f;
  const float dym = fmaxf(fabsf(py - (float)iv0), fabsf((float)iv1 - py)) + 1.f;
  const float smax = 0.7213475f * ((A * dxm * dxm + 2.f * fabsf(B) * dxm * dym) +
                                   C * dym * dym) * 1.0001f;
  const float marg = 0x1p-24f * (16.f * smax + 4.f * fabsf(log2f(o))) +
                     0x1p-19f;
  return 2.f * logf(o / amin) + 1.3862944f * marg + 1e-5f;
}

// Minimum of q(d) over the rectangle [dx0, dx1] x [dy0, dy1] (A, C > 0 and a
// positive definite form): 0 if the rectangle holds the origin, else the
// smallest of the four edge minima (each a clamped 1D quadratic).  FP64.
__device__ inline double qmin_rect(double A, double B, double C, double dx0,
                                   double dx1, double dy0, double dy1) {
  if (dx0 <= 0.0 && 0.0 <= dx1 && dy0 <= 0.0 && 0.0 <= dy1) return 0.0;
  double best = INFINITY;
  const double xs[2] = {dx0, dx1}, ys[2] = {dy0, dy1};
  for (int i = 0; i < 2; ++i) {
    const double dx = xs[i];
    const double dy = fmin(fmax(-B * dx / C, dy0), dy1);
    best = fmin(best, (A * dx + 2.0 * B * dy) * dx + C * dy * dy);
  }
  for (int i = 0; i < 2; ++i) {
    const double dy = ys[i];
    const double dx = fmin(fmax(-B * dy / A, dx0), dx1);
    best = fmin(best, (A * dx + 2.0 * B * dy) * dx + C * dy * dy);
  }
  return best;
}

// Whether the ellipse q(d) <= L can hold a pixel of the pixel rectangle
// [u0, u1] x [v0, v1] of record R.
__device__ inline bool ellipse_meets(const Record& R, float L, int u0, int u1,
                                     int v0, int v1) {
  if (u0 > u1 || v0 > v1 || L < 0.f) return false;
  if (!(L < INFINITY)) return true;
  const double px = R.q0.x, py = R.q0.y;
  const double q = qmin_rect(R.q0.z, R.q0.w, R.q1.x, px - u1, px - u0,
                             py - v1, py - v0);
  return q <= (double)L * (1.0 + 1e-9) + 1e-6;
}

}  // namespace gs
