// Pieces shared by the forward and backward compositing kernels.  Both
// kernels stage records into LDS with stage() and evaluate a (pixel, entry)
// pair with eval_alpha(); compiled without FMA contraction, both therefore
// take bit-identical admit / clamp / stop decisions.
#pragma once

#include "gs_internal.h"

namespace gs {

// One staged Gaussian in LDS (64 bytes).  The exponent coefficients are
// pre-scaled so that exp(-1/2 d^T Q d) = exp2(A2 dx^2 + C2 dy^2 + B2 dx dy).
struct __align__(16) Entry {
  float4 a;   // px, py, A2, B2
  float4 b;   // C2, opacity, r, g
  float4 c;   // b, A, B, C (unscaled conic, for the backward)
  int4 box;   // u_lo, u_hi, v_lo, v_hi
};

constexpr float kHalfLog2e = -0.72134752044448170368f;  // -log2(e) / 2
constexpr float kLog2e = -1.44269504088896340736f;      // -log2(e)

__device__ __forceinline__ void stage(Entry& E, const Record& R) {
  const float A = R.q0.z, B = R.q0.w, C = R.q1.x;
  E.a = make_float4(R.q0.x, R.q0.y, A * kHalfLog2e, B * kLog2e);
  E.b = make_float4(C * kHalfLog2e, R.q1.y, R.q1.z, R.q1.w);
  E.c = make_float4(R.q2.x, A, B, C);
  const int bu = __float_as_int(R.q2.z), bv = __float_as_int(R.q2.w);
  E.box = make_int4(bu & 0xffff, bu >> 16, bv & 0xffff, bv >> 16);
}

__device__ __forceinline__ bool in_box(const int4& b, int u, int v) {
  return u >= b.x && u <= b.y && v >= b.z && v <= b.w;
}

// alpha = min(alpha_max, opacity * exp2(e2)); e2 > 0 only by rounding and
// the entry is then skipped by the caller.  Returns o * G in oG.
__device__ __forceinline__ float eval_alpha(const Entry& E, float fu, float fv,
                                            float alpha_max, float& dx,
                                            float& dy, float& G, float& e2,
                                            float& oG) {
  dx = E.a.x - fu;
  dy = E.a.y - fv;
  e2 = fmaf(E.a.z * dx, dx, fmaf(E.b.x * dy, dy, (E.a.w * dx) * dy));
  G = __builtin_amdgcn_exp2f(e2);
  oG = E.b.y * G;
  return fminf(alpha_max, oG);
}

struct RasterArgs {
  const Record* rec;
  const uint32_t* vals;
  const uint32_t* ranges;
  long long key_cap;
  int cap, V, W, H, Tx, Ty;
  float bg0, bg1, bg2;
  float alpha_min, T_min, alpha_max;
};

RasterArgs make_raster_args(gs_workspace* ws, const gs_settings* s);

__device__ __forceinline__ void tile_range(const RasterArgs& a, int t,
                                           long long& s, long long& e) {
  s = min((long long)a.ranges[2 * t], a.key_cap);
  e = min((long long)a.ranges[2 * t + 1], a.key_cap);
}

}  // namespace gs
