// Pieces shared by the forward and backward compositing kernels.
//
// Both kernels stage records into LDS with stage() and evaluate (pixel,
// entry) pairs with lane_prep() + pixel_alpha(); compiled without FMA
// contraction (FMAs are written explicitly), both therefore take
// bit-identical admit / clamp / stop decisions.
//
// Pixel ownership: a tile of TILE x TILE pixels is served by NT threads laid
// out as TILE columns x (NT / TILE) row groups; each thread owns a vertical
// strip of PPT = TILE * TILE / NT consecutive pixels of one column.  The
// pixels of a strip share their column, so the x-offset terms of the
// exponent are formed once per (entry, thread).
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

// Column part of the exponent for one (entry, thread): dx and the terms that
// depend on dx only.
struct Lane {
  float dx, a0, b0;
  bool in_u;
};

__device__ __forceinline__ Lane lane_prep(const Entry& E, int u) {
  Lane L;
  L.in_u = u >= E.box.x && u <= E.box.y;
  L.dx = E.a.x - (float)u;
  L.a0 = (E.a.z * L.dx) * L.dx;   // A2 dx^2
  L.b0 = E.a.w * L.dx;            // B2 dx
  return L;
}

__device__ __forceinline__ bool in_v(const Entry& E, int v) {
  return v >= E.box.z && v <= E.box.w;
}

// alpha = min(alpha_max, opacity * exp2(e2)) for the pixel in row v of the
// thread's column; e2 > 0 happens only by rounding and the caller skips it.
__device__ __forceinline__ float pixel_alpha(const Entry& E, const Lane& L,
                                             int v, float alpha_max, float& dy,
                                             float& G, float& e2, float& oG) {
  dy = E.a.y - (float)v;
  e2 = fmaf(E.b.x * dy, dy, fmaf(L.b0, dy, L.a0));
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

inline int default_threads(int tile) { return tile == 32 ? 256 : 64; }

// Calls launcher.template go<TILE, BATCH, NT>() for a supported shape.
template <typename Launcher>
void dispatch_shape(int tile, int batch, int nt, const Launcher& l) {
  if (nt == 0) nt = default_threads(tile);
#define GS_BATCHES(T, N)                                  \
  do {                                                    \
    if (batch == 128) l.template go<T, 128, N>();         \
    else if (batch == 256) l.template go<T, 256, N>();    \
    else l.template go<T, 512, N>();                      \
  } while (0)
  if (tile == 8) {
    GS_BATCHES(8, 64);
  } else if (tile == 16) {
    if (nt == 64) GS_BATCHES(16, 64);
    else if (nt == 128) GS_BATCHES(16, 128);
    else GS_BATCHES(16, 256);
  } else {
    if (nt == 128) GS_BATCHES(32, 128);
    else GS_BATCHES(32, 256);
  }
#undef GS_BATCHES
}

}  // namespace gs
