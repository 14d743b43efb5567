// Pieces shared by the forward and backward compositing kernels.
//
// Both kernels stage records into LDS with stage() and evaluate (pixel,
// entry) pairs with column() + exponent2(); compiled without FMA contraction
// (FMAs are written explicitly), both therefore take bit-identical admit /
// clamp / stop decisions.
//
// Pixel ownership: each of the NT threads of a tile owns a vertical strip of
// PPT = TILE * TILE / NT consecutive pixels of one column.  The pixels of a
// strip share their column, so the x-offset terms of the exponent are formed
// once per (entry, thread).  The 64 lanes of a wave cover a footprint of WC
// columns x FH rows that is as square as the tile allows (16 x 16 for PPT 4),
// which keeps a Gaussian's box test coherent across the wave.
#pragma once

#include "admit.h"
#include "gs_internal.h"

namespace gs {

// One staged Gaussian in LDS (64 bytes).  The exponent coefficients are
// pre-scaled so that o exp(-1/2 d^T Q d) = exp2(log2(o) + A2 dx^2 + C2 dy^2
// + B2 dx dy).
struct __align__(16) Entry {
  float4 a;   // px, py, A2, B2
  float4 b;   // C2, log2(opacity), r, g
  float4 c;   // b, A, B, C (unscaled conic, for the backward)
  int4 box;   // u_lo, u_hi, v_lo, v_hi
};

template <int TILE, int NT>
struct PixLayout {
  static constexpr int PPT = TILE * TILE / NT;
  static constexpr int WC = PPT == 1 ? 8 : (TILE < 16 ? TILE : 16);
  static constexpr int FH = (64 / WC) * PPT;  // footprint rows of one wave
  static constexpr int WPR = TILE / WC;       // waves side by side
  static_assert(NT % 64 == 0 && WPR * (TILE / FH) == NT / 64 &&
                    TILE % FH == 0,
                "wave footprints must tile the tile");
  // Column and first row of thread tid's strip, relative to the tile.
  __device__ static void of(int tid, int& cu, int& cv0) {
    const int w = tid >> 6, l = tid & 63;
    cu = (w % WPR) * WC + l % WC;
    cv0 = (w / WPR) * FH + (l / WC) * PPT;
  }
  // Top-left pixel of the footprint of wave w, relative to the tile.
  __device__ static void wave_origin(int w, int& wu, int& wv) {
    wu = (w % WPR) * WC;
    wv = (w / WPR) * FH;
  }
};

constexpr float kHalfLog2e = -0.72134752044448170368f;  // -log2(e) / 2
constexpr float kLog2e = -1.44269504088896340736f;      // -log2(e)

// Unpacks a (lo | hi << 16, lo | hi << 16) box.
__device__ __forceinline__ int4 unpack_box(int2 b) {
  return make_int4(b.x & 0xffff, b.x >> 16, b.y & 0xffff, b.y >> 16);
}

// lo: log2 of the opacity, formed in FP64 by the projection and rounded
// once (relative error below u = 2^-24).
__device__ __forceinline__ void stage(Entry& E, const Record& R,
                                      const int4& box, float lo) {
  const float A = R.q0.z, B = R.q0.w, C = R.q1.x;
  E.a = make_float4(R.q0.x, R.q0.y, A * kHalfLog2e, B * kLog2e);
  E.b = make_float4(C * kHalfLog2e, lo, R.q1.z, R.q1.w);
  E.c = make_float4(R.q2.x, A, B, C);
  E.box = box;
}

// Bit w is set when wave w of a tile whose top-left pixel is (tu0, tv0) has
// to evaluate the staged entry: its footprint meets the render box rb and,
// with the ellipse test, the ellipse q(d) <= L outside which no pixel is
// admitted (admit.h).  Computed once per staged entry.
template <int TILE, int NT>
__device__ inline int wave_mask(const Record& R, const int4& rb, int tu0,
                                int tv0, float amin, bool ellipse) {
  using Lay = PixLayout<TILE, NT>;
  float L = INFINITY;
  if (ellipse) {
    const int bu = __float_as_int(R.q2.z), bv = __float_as_int(R.q2.w);
    L = admit_level(R, bu & 0xffff, bu >> 16, bv & 0xffff, bv >> 16, amin);
  }
  int m = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    int wu, wv;
    Lay::wave_origin(w, wu, wv);
    const int u0 = max(rb.x, tu0 + wu), u1 = min(rb.y, tu0 + wu + Lay::WC - 1);
    const int v0 = max(rb.z, tv0 + wv), v1 = min(rb.w, tv0 + wv + Lay::FH - 1);
    if (ellipse_meets(R, L, u0, u1, v0, v1)) m |= 1 << w;
  }
  return m;
}

// A float the compiler keeps in a register: a plain copy it cannot see
// through, so it does not re-derive the value (an int-to-float conversion
// per use) inside the compositing loops.
__device__ __forceinline__ float pinned(float x) {
  float y;
  asm("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
  return y;
}

// Column part of the exponent for one (entry, thread): dx and the terms that
// depend on dx only, with log2(o) added to the dx^2 term.
struct Column {
  float dx, a0, b0;
};

__device__ __forceinline__ Column column(const float4& ea, float lo,
                                         float uf) {
  Column c;
  c.dx = ea.x - uf;
  c.a0 = fmaf(ea.z * c.dx, c.dx, lo);   // log2(o) + A2 dx^2
  c.b0 = ea.w * c.dx;                   // B2 dx
  return c;
}

// Base-2 exponent of alpha at the pixel in row vf of the thread's column,
// e2 = log2(o) + A2 dx^2 + B2 dx dy + C2 dy^2 = a0 + dy (b0 + C2 dy) in
// Horner form (two FMAs; with the column terms its rounding error stays
// below u (3 S + 3 |log2 o|), S the sum of the three quadratic terms'
// magnitudes).
__device__ __forceinline__ float exponent2(const Column& c, float py, float C2,
                                           float vf, float& dy) {
  dy = py - vf;
  return fmaf(fmaf(C2, dy, c.b0), dy, c.a0);
}

// The unclamped alpha o G = exp2(e2), clamped to [0, 1] (the exponential's
// output clamp, no extra instruction): the quadratic form is negative
// semi-definite, so only rounding next to the centre of a very elongated
// footprint could take e2 above log2(o); alpha stays at most 1 there.
__device__ __forceinline__ float alpha2(float e2) {
  return __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(e2), 0.f, 1.f);
}

// Per staged entry and wave, two bits: bit 2w set when wave w evaluates the
// entry at all (wave_mask), bit 2w + 1 when it may take the fast path: the
// render box holds every pixel of the wave's footprint that lies in the
// image, and opacity <= alpha_max (so alpha = o G needs no clamp).
template <int TILE, int NT>
__device__ inline int wave_bits(const Record& R, const int4& rb, int tu0,
                                int tv0, int W, int H, float amin, float amax,
                                bool ellipse) {
  using Lay = PixLayout<TILE, NT>;
  const int m = wave_mask<TILE, NT>(R, rb, tu0, tv0, amin, ellipse);
  const bool no_clamp = R.q1.y <= amax;
  int bits = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    if (!((m >> w) & 1)) continue;
    int wu, wv;
    Lay::wave_origin(w, wu, wv);
    const int u0 = tu0 + wu, u1 = min(W - 1, tu0 + wu + Lay::WC - 1);
    const int v0 = tv0 + wv, v1 = min(H - 1, tv0 + wv + Lay::FH - 1);
    const bool full = rb.x <= u0 && rb.y >= u1 && rb.z <= v0 && rb.w >= v1;
    bits |= (no_clamp && full ? 3 : 1) << (2 * w);
  }
  return bits;
}

// Per staged batch and wave w: bit j of eval[w] is set when wave w has to
// evaluate staged entry j (wave_bits, bit 2w), bit j of fast[w] when it may
// take the fast path (bit 2w + 1).  A wave walks the set bits of its own
// words in scalar registers, so skipped entries cost nothing.
template <int BATCH, int NT>
struct alignas(8) WaveMasks {
  uint32_t eval[NT / 64][BATCH / 32];
  uint32_t fast[NT / 64][BATCH / 32];
};

// Called by every thread of the workgroup in converged control flow, after
// it staged entry i0 + tid (bits: its wave_bits, 0 past the batch's end):
// each wave turns its 64 entries' bits into two 64-bit ballots per target
// wave, stored by its first lane.  Every word that holds an entry below the
// batch's count is written by the round that stages it.
template <int BATCH, int NT>
__device__ inline void publish_masks(WaveMasks<BATCH, NT>& m, int i0,
                                     int bits, int wave, int lane) {
  if (i0 + 64 * wave >= BATCH) return;   // uniform over the wave
  const int dw = (i0 >> 5) + 2 * wave;   // even: 8-byte aligned
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint64_t e = __builtin_amdgcn_ballot_w64((bits >> (2 * w)) & 1);
    const uint64_t f = __builtin_amdgcn_ballot_w64((bits >> (2 * w + 1)) & 1);
    if (lane == 0) {
      *reinterpret_cast<uint64_t*>(&m.eval[w][dw]) = e;
      *reinterpret_cast<uint64_t*>(&m.fast[w][dw]) = f;
    }
  }
}

struct RasterArgs {
  const Record* rec;
  const int2* rbox;
  const float* lop;   // [capacity] log2(opacity)
  int ellipse_test;   // 0 with GS_FLAG_FULL_BOX
  const uint32_t* vals;
  const uint32_t* ranges;
  const uint32_t* order;   // block b renders tile order[b]
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
