// Projection front end (Eq. 1-2) and its backward, in FP64 on the GPU.
//
// This translation unit is compiled with -ffp-contract=off: every FP64
// operation below is one IEEE-754 rounding in the order written, so the
// published FP32 record and the integer pixel box are reproducible bit for
// bit by any FP64 implementation that follows the same order.
//
// Layout: the view-independent part (scale, rotation, 3D covariance,
// opacity and its base-2 logarithm) is formed once per Gaussian by k_shape
// and kept in the workspace (56 bytes per Gaussian); k_project then runs one thread per (view,
// Gaussian), ten times the parallelism of a per-Gaussian loop over the
// views, which the long FP64 division and square-root chains need to hide
// their latency.  Its blocks are ordered so that the views of one chunk of
// Gaussians run on the same XCD (blocks are dealt to the eight XCDs round
// robin), where the chunk's parameters stay in that XCD's L2.  The backward
// keeps one thread per Gaussian looping over the views: it accumulates the
// shape gradient over them.

#include <math.h>

#include "admit.h"
#include "gs_internal.h"
#include "shape.h"
#include "tails.h"

namespace gs {
namespace {

struct ProjArgs {
  const float* mean;
  const float* lsc;
  const float* quat;
  const float* opl;
  const float* rgb;
  const int32_t* n_dev;
  int cap;
  double* sig;    // [6][cap] Sigma upper triangle; sig[0] = NaN: bad shape
  float* op;      // [cap] opacity
  float* lop;     // [cap] log2(opacity) of the FP32 opacity, rounded once
  int chunks;     // ceil(cap / 256)
  const gs_camera* cams;
  const double* camd;   // [V][kCamDoubles], written by k_shape (workgroup 0)
  int V, W, H, tile, Tx, Ty;
  Record* rec;
  int32_t* tiles;
  int32_t* diff;
  int2* rbox;
  float* depth;
  float amin;     // alpha_min the render boxes are formed for
  int full_box;   // 1: render boxes equal the boxes
  int diff_atomics;   // 1: fill the coverage difference grid (large grids)
};

constexpr int kEmptyPair = 0xffff;   // u_lo = 0xffff, u_hi = 0

// Render box: the integer box narrowed to the bounding box of the ellipse
// q(d) <= L (admit.h) outside which no pixel is admitted: |dx| <=
// sqrt(L C / det), |dy| <= sqrt(L A / det) with det = A C - B^2 (the inverse
// conic's diagonal).  det is formed in FP64 (exact products of FP32 values),
// the root in FP32 with slack, the final bounds in FP64.
__device__ inline void render_box(const Record& R, int iu0, int iu1, int iv0,
                                  int iv1, float amin, int& ru0, int& ru1,
                                  int& rv0, int& rv1) {
  ru0 = iu0; ru1 = iu1; rv0 = iv0; rv1 = iv1;
  const float L = admit_level(R, iu0, iu1, iv0, iv1, amin);
  if (L == kNoPixel) {
    ru0 = rv0 = kEmptyPair;
    ru1 = rv1 = 0;
    return;
  }
  if (!(L < INFINITY)) return;
  const float px = R.q0.x, py = R.q0.y, A = R.q0.z, B = R.q0.w, C = R.q1.x;
  const double det = (double)A * (double)C - (double)B * (double)B;
  const float idet = (float)(1.0 / det);
  const float hx = sqrtf(L * C * idet * 1.0001f) * 1.0001f + 1e-3f;
  const float hy = sqrtf(L * A * idet * 1.0001f) * 1.0001f + 1e-3f;
  if (!isfinite(hx) || !isfinite(hy)) return;
  ru0 = (int)fmax((double)iu0, ceil((double)px - (double)hx));
  ru1 = (int)fmin((double)iu1, floor((double)px + (double)hx));
  rv0 = (int)fmax((double)iv0, ceil((double)py - (double)hy));
  rv1 = (int)fmin((double)iv1, floor((double)py + (double)hy));
  if (ru0 > ru1 || rv0 > rv1) {
    ru0 = rv0 = kEmptyPair;
    ru1 = rv1 = 0;
  }
}

// View-dependent part of Eq. 2 for one camera.
struct View {
  double W[9];
  double fx, fy, cx, cy;
  double t[3];
  double limx, limy, xc, yc;
  int clampx, clampy;
  double J00, J02, J11, J12;
  double T[6];
  double a, b, c, det, A, B, C;
  double px, py;
  bool ok;
};

// A camera record in the constant address space (read-only for the whole
// launch), copied field by field.
using ConstCamera = const __attribute__((address_space(4))) gs_camera;
__device__ inline gs_camera load_camera(ConstCamera* c) {
  gs_camera r;
  for (int i = 0; i < 9; ++i) r.R[i] = c->R[i];
  for (int i = 0; i < 3; ++i) r.t[i] = c->t[i];
  r.fx = c->fx; r.fy = c->fy; r.cx = c->cx; r.cy = c->cy;
  r.near_z = c->near_z;
  r.width = c->width; r.height = c->height; r.pad_ = 0;
  return r;
}

__device__ inline double T_dot(const double* Trow, const double* Sig, int j) {
  return Trow[0] * Sig[j] + Trow[1] * Sig[3 + j] + Trow[2] * Sig[6 + j];
}

__device__ inline void make_view(const CamD& cam, double mx, double my,
                                 double mz, const Shape& S, View& P) {
  for (int i = 0; i < 9; ++i) P.W[i] = cam.W[i];
  P.fx = cam.fx;
  P.fy = cam.fy;
  P.cx = cam.cx;
  P.cy = cam.cy;
  const double* W = P.W;
  P.t[0] = ((W[0] * mx + W[1] * my) + W[2] * mz) + cam.t[0];
  P.t[1] = ((W[3] * mx + W[4] * my) + W[5] * mz) + cam.t[1];
  P.t[2] = ((W[6] * mx + W[7] * my) + W[8] * mz) + cam.t[2];
  const double tx = P.t[0], ty = P.t[1], tz = P.t[2];
  P.ok = isfinite(tx) && isfinite(ty) && isfinite(tz) && tz > cam.near_z &&
         S.ok;
  if (!P.ok) return;
  P.limx = cam.flimx;
  P.limy = cam.flimy;
  double rx = tx / tz, ry = ty / tz;
  P.clampx = 0;
  P.clampy = 0;
  if (rx > P.limx) { rx = P.limx; P.clampx = 1; }
  if (rx < -P.limx) { rx = -P.limx; P.clampx = -1; }
  if (ry > P.limy) { ry = P.limy; P.clampy = 1; }
  if (ry < -P.limy) { ry = -P.limy; P.clampy = -1; }
  P.xc = rx * tz;
  P.yc = ry * tz;
  const double tz2 = tz * tz;
  P.J00 = P.fx / tz;
  P.J02 = -(P.fx * P.xc) / tz2;
  P.J11 = P.fy / tz;
  P.J12 = -(P.fy * P.yc) / tz2;
  for (int j = 0; j < 3; ++j) {
    P.T[j] = P.J00 * W[j] + P.J02 * W[6 + j];
    P.T[3 + j] = P.J11 * W[3 + j] + P.J12 * W[6 + j];
  }
  double U[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      U[3 * i + j] = (P.T[3 * i] * S.Sig[j] + P.T[3 * i + 1] * S.Sig[3 + j]) +
                     P.T[3 * i + 2] * S.Sig[6 + j];
  P.a = ((U[0] * P.T[0] + U[1] * P.T[1]) + U[2] * P.T[2]) + 0.3;
  P.b = (U[0] * P.T[3] + U[1] * P.T[4]) + U[2] * P.T[5];
  P.c = ((U[3] * P.T[3] + U[4] * P.T[4]) + U[5] * P.T[5]) + 0.3;
  P.det = P.a * P.c - P.b * P.b;
  P.ok = P.det > 0.0 && isfinite(P.det);
  if (!P.ok) return;
  P.A = P.c / P.det;
  P.B = -P.b / P.det;
  P.C = P.a / P.det;
  P.px = (P.fx * tx) / tz + P.cx;
  P.py = (P.fy * ty) / tz + P.cy;
}

// The view quantities the backward needs, formed with two reciprocals in
// place of the forward's correctly rounded divisions: the backward only has
// to be accurate, not reproducible bit for bit.
__device__ inline void make_view_grad(const CamD& cam, double mx, double my,
                                      double mz, const double* Sig,
                                      bool shape_ok, View& P) {
  for (int i = 0; i < 9; ++i) P.W[i] = cam.W[i];
  P.fx = cam.fx;
  P.fy = cam.fy;
  const double* W = P.W;
  P.t[0] = ((W[0] * mx + W[1] * my) + W[2] * mz) + cam.t[0];
  P.t[1] = ((W[3] * mx + W[4] * my) + W[5] * mz) + cam.t[1];
  P.t[2] = ((W[6] * mx + W[7] * my) + W[8] * mz) + cam.t[2];
  const double tx = P.t[0], ty = P.t[1], tz = P.t[2];
  P.ok = isfinite(tx) && isfinite(ty) && isfinite(tz) && tz > cam.near_z &&
         shape_ok;
  if (!P.ok) return;
  const double itz = 1.0 / tz;
  P.limx = cam.limx;
  P.limy = cam.limy;
  double rx = tx * itz, ry = ty * itz;
  P.clampx = rx > P.limx ? 1 : rx < -P.limx ? -1 : 0;
  P.clampy = ry > P.limy ? 1 : ry < -P.limy ? -1 : 0;
  if (P.clampx) rx = P.clampx * P.limx;
  if (P.clampy) ry = P.clampy * P.limy;
  P.xc = rx * tz;
  P.yc = ry * tz;
  P.J00 = P.fx * itz;
  P.J02 = -P.fx * rx * itz;
  P.J11 = P.fy * itz;
  P.J12 = -P.fy * ry * itz;
  for (int j = 0; j < 3; ++j) {
    P.T[j] = P.J00 * W[j] + P.J02 * W[6 + j];
    P.T[3 + j] = P.J11 * W[3 + j] + P.J12 * W[6 + j];
  }
  double U[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      U[3 * i + j] = T_dot(P.T + 3 * i, Sig, j);
  P.a = U[0] * P.T[0] + U[1] * P.T[1] + U[2] * P.T[2] + 0.3;
  P.b = U[0] * P.T[3] + U[1] * P.T[4] + U[2] * P.T[5];
  P.c = U[3] * P.T[3] + U[4] * P.T[4] + U[5] * P.T[5] + 0.3;
  P.det = P.a * P.c - P.b * P.b;
  P.ok = P.det > 0.0 && isfinite(P.det);
  if (!P.ok) return;
  const double idet = 1.0 / P.det;
  P.A = P.c * idet;
  P.B = -P.b * idet;
  P.C = P.a * idet;
}

__global__ __launch_bounds__(256) void k_shape(ShapeJob j,
                                               const gs_camera* cams, int V,
                                               double* camd) {
  cam_d_fill(cams, V, camd);
  shape_one(j, blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_project(ProjArgs a) {
  // Block b runs on XCD b % 8: chunk c of 256 Gaussians and view k with
  // b = ((c / 8) V + k) 8 + c % 8 keep every view of a chunk on one XCD.
  const int b = blockIdx.x;
  const int rest = b >> 3;
  const int k = rest % a.V;
  const int c = (rest / a.V) * 8 + (b & 7);
  if (c >= a.chunks) return;
  const int g = c * 256 + threadIdx.x;
  const int n = min(*a.n_dev, a.cap);
  if (g >= n) return;
  const int cap = a.cap;
  Shape S;
  for (int j = 0; j < 6; ++j) {
    const double v = a.sig[(size_t)j * cap + g];
    const int i = kSigIdx[j], r = i / 3, q = i % 3;
    S.Sig[3 * r + q] = v;
    S.Sig[3 * q + r] = v;
  }
  S.ok = !isnan(S.Sig[0]);
  const double mx = a.mean[g], my = a.mean[cap + g], mz = a.mean[2 * cap + g];
  const float op = a.op[g];
  const float r = a.rgb[g], gg = a.rgb[cap + g], bb = a.rgb[2 * cap + g];
  {
    const size_t slot = (size_t)k * cap + g;
    View P;
    make_view(cam_d_table((ConstDouble*)a.camd + kCamDoubles * k), mx, my, mz,
              S, P);
    bool ok = P.ok;
    double ulo = 0, uhi = -1, vlo = 0, vhi = -1;
    if (ok) {
      const double mid = 0.5 * (P.a + P.c);
      const double lam = mid + sqrt(fmax(0.1, mid * mid - P.det));
      const double rad = ceil(3.0 * sqrt(lam));
      ok = isfinite(P.px) && isfinite(P.py) && isfinite(rad);
      if (ok) {
        ulo = fmax(0.0, ceil(P.px - rad));
        uhi = fmin((double)(a.W - 1), floor(P.px + rad));
        vlo = fmax(0.0, ceil(P.py - rad));
        vhi = fmin((double)(a.H - 1), floor(P.py + rad));
        ok = ulo <= uhi && vlo <= vhi;
      }
    }
    if (!ok) {
      a.tiles[slot] = 0;
      return;
    }
    const int iu0 = (int)ulo, iu1 = (int)uhi, iv0 = (int)vlo, iv1 = (int)vhi;
    Record R;
    R.q0 = make_float4((float)P.px, (float)P.py, (float)P.A, (float)P.B);
    R.q1 = make_float4((float)P.C, op, r, gg);
    R.q2 = make_float4(bb, (float)P.t[2],
                       __int_as_float(iu0 | (iu1 << 16)),
                       __int_as_float(iv0 | (iv1 << 16)));
    a.rec[slot] = R;
    a.depth[slot] = R.q2.y;
    int ru0 = iu0, ru1 = iu1, rv0 = iv0, rv1 = iv1;
    if (!a.full_box) render_box(R, iu0, iu1, iv0, iv1, a.amin, ru0, ru1, rv0, rv1);
    a.rbox[slot] = make_int2(ru0 | (ru1 << 16), rv0 | (rv1 << 16));
    if (ru0 > ru1) {   // empty render box: nothing to bin
      a.tiles[slot] = 0;
      return;
    }
    // The Gaussian is binned into the tiles its render box touches.
    const int tx0 = ru0 / a.tile, tx1 = ru1 / a.tile;
    const int ty0 = rv0 / a.tile, ty1 = rv1 / a.tile;
    a.tiles[slot] = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
    if (!a.diff_atomics) return;
    // Tile-coverage difference grid: +1/-1 at the four corners of the box of
    // tiles; a 2D prefix sum then yields the key count of every tile.
    int32_t* d = a.diff + (size_t)k * (a.Ty + 1) * (a.Tx + 1);
    const int stride = a.Tx + 1;
    atomicAdd(&d[ty0 * stride + tx0], 1);
    atomicAdd(&d[ty0 * stride + tx1 + 1], -1);
    atomicAdd(&d[(ty1 + 1) * stride + tx0], -1);
    atomicAdd(&d[(ty1 + 1) * stride + tx1 + 1], 1);
  }
}

struct ProjBwdArgs {
  const float* mean;
  const float* lsc;
  const float* quat;
  const float* opl;
  const int32_t* n_dev;
  int cap;
  const gs_camera* cams;
  int V;
  const int32_t* tiles;
  float* grad2d;  // [V][5][cap], zeroed after reading
  float* gop;     // [cap], zeroed after reading
  float* d_mean;
  float* d_lsc;
  float* d_quat;
  float* d_opl;
  const double* camd;   // [V][kCamDoubles] (k_project_bwd<true>)
  // Workgroups past main_blocks reduce the fused L1 term's tile losses.
  int main_blocks;
  L1ReduceJob l1;
};

// Chain rule from dL/d(px, py, A, B, C) of every view back to the mean,
// log-scale and quaternion, and from dL/d(opacity) to the logit.  Written in
// matrix form: for the conic Q = Sigma2D^-1 the symmetric gradient is
// G2 = -Q dQ Q; for Sigma2D = T Sigma T^T, dSigma = T^T G2 T and
// dT = 2 G2 T Sigma; Sigma = M M^T gives dM = 2 dSigma M (summed over views).
// TABLE: the views' FP64 camera constants come from a table formed earlier
// in the launch sequence (scalar registers, no per-lane conversions).
template <bool TABLE>
__global__ __launch_bounds__(256) void k_project_bwd(ProjBwdArgs a) {
  __shared__ double part[4];
  if ((int)blockIdx.x >= a.main_blocks) {   // dispatched last: the tail
    l1_reduce_part(a.l1, part);
    return;
  }
  const int g = blockIdx.x * 256 + threadIdx.x;
  const int n = min(*a.n_dev, a.cap);
  if (g >= n) return;
  const int cap = a.cap;
  // Only Sigma stays live through the loop over the views; the rest of the
  // shape chain is formed again after it.  Fewer registers per thread (about
  // 150 instead of about 190) let three waves per SIMD instead of two hide
  // the latency of the per-view FP64 chain.
  double Sig[9];
  bool shape_ok;
  {
    Shape S;
    make_shape(a.lsc, a.quat, cap, g, S);
    for (int i = 0; i < 9; ++i) Sig[i] = S.Sig[i];
    shape_ok = S.ok;
  }
  const double mx = a.mean[g], my = a.mean[cap + g], mz = a.mean[2 * cap + g];
  double dmu[3] = {0, 0, 0};
  double dS[6] = {0, 0, 0, 0, 0, 0};   // dSigma + dSigma^T, upper triangle
  // The camera records are read through the constant address space: the
  // view index is uniform, so they arrive by scalar loads (a generic pointer
  // would take vector loads, the loop's stores keeping the compiler from
  // proving them read-only).
  ConstCamera* cams = (ConstCamera*)a.cams;
  // Each view's tile count and five gradients are loaded one view ahead,
  // so their latency overlaps the previous view's chain.
  int nx_binned = 0;
  float nx[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (a.V > 0) {
    nx_binned = a.tiles[g];
    for (int i = 0; i < 5; ++i) nx[i] = a.grad2d[(size_t)i * cap + g];
  }
  for (int k = 0; k < a.V; ++k) {
    const int binned = nx_binned;
    const float f0 = nx[0], f1 = nx[1], f2 = nx[2], f3 = nx[3], f4 = nx[4];
    if (k + 1 < a.V) {
      nx_binned = a.tiles[(size_t)(k + 1) * cap + g];
      const float* gn = a.grad2d + (size_t)(k + 1) * 5 * cap + g;
      for (int i = 0; i < 5; ++i) nx[i] = gn[(size_t)i * cap];
    }
    float* gk = a.grad2d + (size_t)k * 5 * cap + g;
    const CamD cam = TABLE ? cam_d_table((ConstDouble*)a.camd + kCamDoubles * k)
                           : cam_d(load_camera(cams + k));
    // One test: a slot with no tiles or an all-zero gradient has nothing to
    // add (and nothing to clear).  (Bitwise, not short-circuit: the loads
    // must not wait on one another.)
    if ((binned == 0) | ((f0 == 0.f) & (f1 == 0.f) & (f2 == 0.f) &
                         (f3 == 0.f) & (f4 == 0.f)))
      continue;
    gk[0] = 0.f; gk[cap] = 0.f; gk[2 * (size_t)cap] = 0.f;
    gk[3 * (size_t)cap] = 0.f; gk[4 * (size_t)cap] = 0.f;
    const double dpx = f0, dpy = f1, dA = f2, dB = f3, dC = f4;
    View P;
    make_view_grad(cam, mx, my, mz, Sig, shape_ok, P);
    if (!P.ok) continue;
    // Conic -> dilated screen covariance (symmetric matrix gradient).
    const double Q[4] = {P.A, P.B, P.B, P.C};
    const double GQ[4] = {dA, 0.5 * dB, 0.5 * dB, dC};
    double X[4];  // GQ Q
    X[0] = GQ[0] * Q[0] + GQ[1] * Q[2];
    X[1] = GQ[0] * Q[1] + GQ[1] * Q[3];
    X[2] = GQ[2] * Q[0] + GQ[3] * Q[2];
    X[3] = GQ[2] * Q[1] + GQ[3] * Q[3];
    double G2[4];  // -Q X
    G2[0] = -(Q[0] * X[0] + Q[1] * X[2]);
    G2[1] = -(Q[0] * X[1] + Q[1] * X[3]);
    G2[2] = -(Q[2] * X[0] + Q[3] * X[2]);
    G2[3] = -(Q[2] * X[1] + Q[3] * X[3]);
    const double* T = P.T;
    // dSigma += T^T G2 T, kept symmetrised: N + N^T with N = T^T G2 T.
    double GT[6];   // G2 T
    for (int j = 0; j < 3; ++j) {
      GT[j] = G2[0] * T[j] + G2[1] * T[3 + j];
      GT[3 + j] = G2[2] * T[j] + G2[3] * T[3 + j];
    }
    for (int u = 0; u < 6; ++u) {
      const int i = kSigIdx[u] / 3, j = kSigIdx[u] % 3;
      dS[u] += (T[i] * GT[j] + T[3 + i] * GT[3 + j]) +
               (T[j] * GT[i] + T[3 + j] * GT[3 + i]);
    }
    // dT = (G2 + G2^T) T Sigma
    double TS[6];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j)
        TS[3 * i + j] = T[3 * i] * Sig[j] + T[3 * i + 1] * Sig[3 + j] +
                        T[3 * i + 2] * Sig[6 + j];
    double dT[6];
    for (int j = 0; j < 3; ++j) {
      dT[j] = (2.0 * G2[0]) * TS[j] + (G2[1] + G2[2]) * TS[3 + j];
      dT[3 + j] = (G2[1] + G2[2]) * TS[j] + (2.0 * G2[3]) * TS[3 + j];
    }
    // T = J W with J = [[J00, 0, J02], [0, J11, J12]]
    const double* W = P.W;
    double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
    for (int j = 0; j < 3; ++j) {
      dJ00 += dT[j] * W[j];
      dJ02 += dT[j] * W[6 + j];
      dJ11 += dT[3 + j] * W[3 + j];
      dJ12 += dT[3 + j] * W[6 + j];
    }
    const double tx = P.t[0], ty = P.t[1], tz = P.t[2];
    const double itz = 1.0 / tz, itz2 = itz * itz, itz3 = itz2 * itz;
    double dt[3];
    // J02 = -fx xc / tz^2 with xc = tx, or xc = +-limx tz when clamped.
    const double dJ02_dxc = -P.fx * itz2, dJ12_dyc = -P.fy * itz2;
    dt[0] = (P.clampx ? 0.0 : dJ02 * dJ02_dxc) + dpx * P.fx * itz;
    dt[1] = (P.clampy ? 0.0 : dJ12 * dJ12_dyc) + dpy * P.fy * itz;
    dt[2] = -dJ00 * P.fx * itz2 - dJ11 * P.fy * itz2 +
            dJ02 * (2.0 * P.fx * P.xc * itz3 +
                    (P.clampx ? dJ02_dxc * P.clampx * P.limx : 0.0)) +
            dJ12 * (2.0 * P.fy * P.yc * itz3 +
                    (P.clampy ? dJ12_dyc * P.clampy * P.limy : 0.0)) -
            dpx * P.fx * tx * itz2 - dpy * P.fy * ty * itz2;
    for (int j = 0; j < 3; ++j)
      dmu[j] += W[j] * dt[0] + W[3 + j] * dt[1] + W[6 + j] * dt[2];
  }
  // Shared shape chain: dM = (dSigma + dSigma^T) M.
  Shape S;
  make_shape(a.lsc, a.quat, cap, g, S);
  constexpr int kSym[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};   // (i, m) -> dS slot
  double dM[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int m = 0; m < 3; ++m) acc += dS[kSym[3 * i + m]] * S.M[3 * m + j];
      dM[3 * i + j] = acc;
    }
  double dR[9], ds[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      dR[3 * i + j] = dM[3 * i + j] * S.s[j];
      ds[j] += dM[3 * i + j] * S.R[3 * i + j];
    }
  const double w = S.qn[0], x = S.qn[1], y = S.qn[2], z = S.qn[3];
  // Partial derivatives of R(w, x, y, z) contracted with dR.
  double dq[4];
  dq[0] = 2.0 * (z * (dR[3] - dR[1]) + y * (dR[2] - dR[6]) + x * (dR[7] - dR[5]));
  dq[1] = 2.0 * (y * (dR[1] + dR[3]) + z * (dR[2] + dR[6]) + w * (dR[7] - dR[5])) -
          4.0 * x * (dR[4] + dR[8]);
  dq[2] = 2.0 * (x * (dR[1] + dR[3]) + w * (dR[2] - dR[6]) + z * (dR[5] + dR[7])) -
          4.0 * y * (dR[0] + dR[8]);
  dq[3] = 2.0 * (w * (dR[3] - dR[1]) + x * (dR[2] + dR[6]) + y * (dR[5] + dR[7])) -
          4.0 * z * (dR[0] + dR[4]);
  const double dot = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
  const bool any = S.ok;
  for (int j = 0; j < 3; ++j) {
    a.d_mean[j * cap + g] += (float)dmu[j];
    if (any) a.d_lsc[j * cap + g] += (float)(ds[j] * S.s[j]);
  }
  if (any)
    for (int j = 0; j < 4; ++j)
      a.d_quat[j * cap + g] += (float)((dq[j] - S.qn[j] * dot) / S.qnorm);
  const double gop = a.gop[g];
  a.gop[g] = 0.f;
  const double o = 1.0 / (1.0 + exp(-(double)a.opl[g]));
  a.d_opl[g] += (float)(gop * o * (1.0 - o));
}

}  // namespace

ShapeJob shape_job(const gs_workspace* ws, const gs_params* p) {
  ShapeJob j;
  j.lsc = p->log_scale; j.quat = p->quat; j.opl = p->opacity_logit;
  j.n_dev = p->n_dev; j.cap = p->capacity;
  j.sig = ws->shape;
  j.op = (float*)(ws->shape + 6 * (size_t)p->capacity);
  j.lop = j.op + p->capacity;
  return j;
}

hipError_t launch_project(gs_workspace* ws, const gs_params* p,
                          const gs_camera* cams, const gs_settings* s,
                          hipStream_t st, bool shape_done) {
  ProjArgs a;
  a.mean = p->mean; a.lsc = p->log_scale; a.quat = p->quat;
  a.opl = p->opacity_logit; a.rgb = p->rgb; a.n_dev = p->n_dev;
  a.cap = p->capacity; a.cams = cams; a.V = ws->geo.n_views;
  a.W = ws->geo.width; a.H = ws->geo.height; a.tile = ws->geo.tile;
  a.Tx = ws->tiles_x; a.Ty = ws->tiles_y;
  a.rec = ws->records; a.tiles = ws->tiles_touched; a.diff = ws->diff;
  a.rbox = ws->rbox; a.depth = ws->depth; a.amin = s->alpha_min;
  a.full_box = (s->flags & GS_FLAG_FULL_BOX) ? 1 : 0;
  a.diff_atomics = bin_chunk(ws->tiles_x, ws->tiles_y) == 0;
  a.sig = ws->shape;
  a.op = (float*)(ws->shape + 6 * (size_t)p->capacity);
  a.lop = a.op + p->capacity;
  a.chunks = (p->capacity + 255) / 256;
  if (a.chunks <= 0) return hipSuccess;
  a.camd = ws->camd;
  if (!shape_done)   // else the window graph's clearing launch did both
    hipLaunchKernelGGL(k_shape, dim3(a.chunks), dim3(256), 0, st,
                       shape_job(ws, p), cams, a.V, ws->camd);
  const long long blocks = (long long)((a.chunks + 7) / 8) * 8 * a.V;
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_project, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_project_bwd(gs_workspace* ws, const gs_params* p,
                              const gs_camera* cams, gs_params* grad,
                              hipStream_t st, const L1ReduceJob* l1,
                              bool cam_table) {
  ProjBwdArgs a;
  a.mean = p->mean; a.lsc = p->log_scale; a.quat = p->quat;
  a.opl = p->opacity_logit; a.n_dev = p->n_dev; a.cap = p->capacity;
  a.cams = cams; a.V = ws->geo.n_views; a.tiles = ws->tiles_touched;
  a.grad2d = ws->grad2d; a.gop = ws->gop;
  a.d_mean = grad->mean; a.d_lsc = grad->log_scale; a.d_quat = grad->quat;
  a.d_opl = grad->opacity_logit;
  const int blocks = (p->capacity + 255) / 256;
  a.main_blocks = blocks;
  a.l1 = l1 ? *l1 : L1ReduceJob{};
  a.camd = ws->camd;
  const int nb = blocks + (l1 ? 1 : 0);
  if (nb > 0) {
    if (cam_table)
      hipLaunchKernelGGL(k_project_bwd<true>, dim3(nb), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL(k_project_bwd<false>, dim3(nb), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace gs
