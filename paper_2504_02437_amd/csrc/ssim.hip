// Structural-similarity term of the colour loss (Eq. 10) and its gradient.
//
// Per channel and pixel: window sums over an 11 x 11 Gaussian window
// (sigma 1.5, normalised, zero padding outside the image) of x, y, x^2, y^2
// and x y give mu_x, mu_y, var_x, var_y and cov; SSIM = A1 A2 / (B1 B2) with
// A1 = 2 mu_x mu_y + C1, A2 = 2 cov + C2, B1 = mu_x^2 + mu_y^2 + C1,
// B2 = var_x + var_y + C2 (C1 = 0.01^2, C2 = 0.03^2).  The loss adds
// lam * sum over views of (1 - mean SSIM over 3HW).
//
// Two passes, both LDS-tiled and separable (a horizontal then a vertical
// 11-tap pass over a tile plus its 5-pixel halo):
//   k_ssim_stats: the five window sums, SSIM, its sum per view, and the
//     three per-pixel derivatives dS/dmu_x, dS/dm_xx, dS/dm_xy (pre-scaled
//     by -lam / 3HW) into the caller's scratch;
//   k_ssim_grad: window sums of those three maps (the window is symmetric,
//     so the adjoint of a window sum is a window sum), combined as
//     dL/dx(p) += D1(p) + 2 x(p) D2(p) + y(p) D3(p).

#include <math.h>

#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kR = 5;                     // window radius (11 taps)
constexpr int kTW = 64, kTH = 16;         // output tile
constexpr int kIW = kTW + 2 * kR, kIH = kTH + 2 * kR;
// LDS row strides padded so that the lanes of a half-wave in the horizontal
// pass spread over the banks (hitem below).
constexpr int kSW = kIW + 7;    // 81
constexpr int kHW = kTW + 1;    // 65
constexpr int kNT = 256;
constexpr int kRunX = 8;                  // horizontal outputs per item
constexpr int kRunY = kTH * kTW / kNT;    // vertical outputs per thread (4)
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;
static_assert(kTW * (kTH / kRunY) == kNT, "vertical pass layout");

struct SsimArgs {
  float w[2 * kR + 1];  // normalised 1D window
  const float* x;       // rendered [V][3][H][W]
  const float* y;       // target
  float* dL;            // [V][3][H][W], accumulated
  float* scratch;       // [3][V*3][H][W]
  double* loss;
  double* ssim;         // [V] mean SSIM, accumulated (may be null)
  int V, H, W;
  float lam;
  // L1 term fused in (l1 != 0): the statistics pass adds lam_l1 mean |x - y|
  // to the loss and the squared errors to sqerr; the gradient pass WRITES
  // dL = lam_l1 sign(x - y) / (3HW) + the SSIM gradient instead of adding
  // to dL.
  int l1;
  float l1_scale;      // lam_l1 / (3HW)
  double l1_lam_inv;   // lam_l1 / (3HW) in FP64
  double* sqerr;       // [V], may be null
};

// Work item it of a horizontal pass -> (halo row r, first output column
// c0).  The 32 lanes of a half-wave take 8 rows x 4 runs: with row strides
// of 17 and 1 modulo 32 (kSW, kHW) their LDS reads and writes fall in 32
// distinct banks.  Items with r >= kIH have no row.
constexpr int kHItems = 64 * ((kIH + 7) / 8);
static_assert(kTW / kRunX == 8 && kSW % 32 == 17 && kHW % 32 == 1,
              "horizontal-pass lane layout");
__device__ inline void hitem(int it, int& r, int& c0) {
  const int g = it >> 6, l = it & 63;
  r = ((l & 31) >> 2) + 8 * g;
  c0 = ((l & 3) + 4 * (l >> 5)) * kRunX;
}

__device__ inline float block_sum(float v, float* part) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0)
    for (int i = 0; i < kNT / 64; ++i) s += part[i];
  return s;
}

// Both passes: one plane per grid row; each workgroup takes every
// gridDim.x-th tile of its plane, with the next tile's inputs loaded while
// the current one is computed.  In the statistics pass the loss and the
// per-view SSIM then take one FP64 atomic per workgroup rather than per tile
// (atomics on one address serialise).
__global__ __launch_bounds__(kNT) void k_ssim_stats(SsimArgs a) {
  __shared__ float sx[kIH][kSW], sy[kIH][kSW];
  __shared__ float hs[5][kIH][kHW];
  __shared__ float part[kNT / 64];
  const int tid = threadIdx.x;
  const int plane = blockIdx.y;                 // view * 3 + channel
  const int H = a.H, W = a.W;
  const size_t HW = (size_t)H * W;
  const float* X = a.x + (size_t)plane * HW;
  const float* Y = a.y + (size_t)plane * HW;
  const int tiles_x = (W + kTW - 1) / kTW;
  const int tiles = tiles_x * ((H + kTH - 1) / kTH);
  float w[2 * kR + 1];
#pragma unroll
  for (int i = 0; i < 2 * kR + 1; ++i) w[i] = a.w[i];
  const float n_inv = 1.f / (3.f * (float)HW);
  const float scale = -a.lam * n_inv;
  float ssum = 0.f, l1sum = 0.f;
  double sqsum = 0.0;
  // The halo region of a tile is loaded into registers one tile ahead: the
  // loads of the next tile are in flight while this one is computed.
  constexpr int kLoads = (kIH * kIW + kNT - 1) / kNT;
  float lx[kLoads], ly[kLoads];
  auto fetch = [&](int tile) {
    const int ou = (tile % tiles_x) * kTW, ov = (tile / tiles_x) * kTH;
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const int i = tid + j * kNT;
      const int r = i / kIW, c = i - r * kIW;
      const int u = ou - kR + c, v = ov - kR + r;
      const bool in = i < kIH * kIW && u >= 0 && u < W && v >= 0 && v < H;
      lx[j] = in ? X[(size_t)v * W + u] : 0.f;
      ly[j] = in ? Y[(size_t)v * W + u] : 0.f;
    }
  };
  if ((int)blockIdx.x < tiles) fetch(blockIdx.x);
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int ou = (tile % tiles_x) * kTW, ov = (tile / tiles_x) * kTH;
    __syncthreads();   // the previous tile's LDS reads are done
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const int i = tid + j * kNT;
      if (i < kIH * kIW) {
        const int r = i / kIW, c = i - r * kIW;
        sx[r][c] = lx[j];
        sy[r][c] = ly[j];
      }
    }
    __syncthreads();
    if (tile + (int)gridDim.x < tiles) fetch(tile + gridDim.x);
    // Horizontal pass: five sums for every row of the halo region.
    for (int it = tid; it < kHItems; it += kNT) {
      int r, c0;
      hitem(it, r, c0);
      if (r >= kIH) continue;
      float px[kRunX + 2 * kR], py[kRunX + 2 * kR];
      float pxx[kRunX + 2 * kR], pyy[kRunX + 2 * kR], pxy[kRunX + 2 * kR];
#pragma unroll
      for (int i = 0; i < kRunX + 2 * kR; ++i) {
        px[i] = sx[r][c0 + i];
        py[i] = sy[r][c0 + i];
        pxx[i] = px[i] * px[i];
        pyy[i] = py[i] * py[i];
        pxy[i] = px[i] * py[i];
      }
#pragma unroll
      for (int o = 0; o < kRunX; ++o) {
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
        for (int b = 0; b < 2 * kR + 1; ++b) {
          const float wb = w[b];
          s0 = fmaf(wb, px[o + b], s0);
          s1 = fmaf(wb, py[o + b], s1);
          s2 = fmaf(wb, pxx[o + b], s2);
          s3 = fmaf(wb, pyy[o + b], s3);
          s4 = fmaf(wb, pxy[o + b], s4);
        }
        hs[0][r][c0 + o] = s0; hs[1][r][c0 + o] = s1; hs[2][r][c0 + o] = s2;
        hs[3][r][c0 + o] = s3; hs[4][r][c0 + o] = s4;
      }
    }
    __syncthreads();
    // Vertical pass: each thread finishes kRunY pixels of one column.
    const int c = tid % kTW, r0 = (tid / kTW) * kRunY;
    float* D1 = a.scratch + (size_t)plane * HW;
    float* D2 = D1 + (size_t)a.V * 3 * HW;
    float* D3 = D2 + (size_t)a.V * 3 * HW;
    float col[5][kRunY + 2 * kR];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int i = 0; i < kRunY + 2 * kR; ++i) col[q][i] = hs[q][r0 + i][c];
    const int u = ou + c;
#pragma unroll
    for (int o = 0; o < kRunY; ++o) {
      float m[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        float s = 0.f;
#pragma unroll
        for (int b = 0; b < 2 * kR + 1; ++b) s = fmaf(w[b], col[q][o + b], s);
        m[q] = s;
      }
      const int v = ov + r0 + o;
      if (u >= W || v >= H) continue;
      if (a.l1) {
        const float d = sx[kR + r0 + o][kR + c] - sy[kR + r0 + o][kR + c];
        l1sum += fabsf(d);
        sqsum += (double)d * (double)d;
      }
      const float mx = m[0], my = m[1];
      const float A1 = 2.f * mx * my + kC1;
      const float A2 = 2.f * (m[4] - mx * my) + kC2;
      const float B1 = mx * mx + my * my + kC1;
      const float B2 = (m[2] - mx * mx) + (m[3] - my * my) + kC2;
      // Reciprocals are enough here (the term is compared at 1e-5 / 1e-3).
      const float iA1 = __builtin_amdgcn_rcpf(A1), iA2 = __builtin_amdgcn_rcpf(A2);
      const float iB1 = __builtin_amdgcn_rcpf(B1), iB2 = __builtin_amdgcn_rcpf(B2);
      const float S = (A1 * A2) * (iB1 * iB2);
      ssum += S;
      const float d_mu = 2.f * S * (my * (iA1 - iA2) + mx * (iB2 - iB1));
      const size_t p = (size_t)v * W + u;
      D1[p] = scale * d_mu;
      D2[p] = scale * (-S * iB2);
      D3[p] = scale * (2.f * S * iA2);
    }
  }
  const float tot = block_sum(ssum, part);
  float l1tot = 0.f;
  double sqtot = 0.0;
  if (a.l1) {
    __syncthreads();
    l1tot = block_sum(l1sum, part);
    __shared__ double dpart[kNT / 64];
    for (int off = 32; off > 0; off >>= 1) sqsum += __shfl_down(sqsum, off, 64);
    if ((tid & 63) == 0) dpart[tid >> 6] = sqsum;
    __syncthreads();
    if (tid == 0)
      for (int i = 0; i < kNT / 64; ++i) sqtot += dpart[i];
  }
  if (tid == 0) {
    const int k = plane / 3;
    atomicAdd(a.loss, -(double)a.lam * (double)tot * (double)n_inv +
                          (double)l1tot * a.l1_lam_inv);
    if (a.l1 && a.sqerr) atomicAdd(&a.sqerr[k], sqtot);
    if (a.ssim) atomicAdd(&a.ssim[k], (double)tot * (double)n_inv);
    if (plane == 0 && blockIdx.x == 0)
      atomicAdd(a.loss, (double)a.lam * a.V);
  }
}

__global__ __launch_bounds__(kNT) void k_ssim_grad(SsimArgs a) {
  __shared__ float sd[3][kIH][kSW];
  __shared__ float hs[3][kIH][kHW];
  const int tid = threadIdx.x;
  const int plane = blockIdx.y;
  const int H = a.H, W = a.W;
  const size_t HW = (size_t)H * W;
  const size_t PL = (size_t)a.V * 3 * HW;
  const float* D = a.scratch + (size_t)plane * HW;
  const int tiles_x = (W + kTW - 1) / kTW;
  const int tiles = tiles_x * ((H + kTH - 1) / kTH);
  float w[2 * kR + 1];
#pragma unroll
  for (int i = 0; i < 2 * kR + 1; ++i) w[i] = a.w[i];
  // This thread's output pixels: column c, rows r0 .. r0 + kRunY - 1.
  const int c = tid % kTW, r0 = (tid / kTW) * kRunY;
  const float* X = a.x + (size_t)plane * HW;
  const float* Y = a.y + (size_t)plane * HW;
  float* G = a.dL + (size_t)plane * HW;
  // A tile's inputs (the derivative maps over the halo region, and x, y and
  // dL at this thread's pixels) are loaded into registers one tile ahead.
  constexpr int kLoads = (kIH * kIW + kNT - 1) / kNT;
  float ld[3][kLoads];
  float xo[kRunY], yo[kRunY], go[kRunY];
  auto fetch = [&](int tile) {
    const int ou = (tile % tiles_x) * kTW, ov = (tile / tiles_x) * kTH;
    const int u = ou + c;
#pragma unroll
    for (int o = 0; o < kRunY; ++o) {
      const int v = ov + r0 + o;
      const bool in = u < W && v < H;
      const size_t p = (size_t)v * W + u;
      xo[o] = in ? X[p] : 0.f;
      yo[o] = in ? Y[p] : 0.f;
      go[o] = (in && !a.l1) ? G[p] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const int i = tid + j * kNT;
      const int r = i / kIW, cc = i - r * kIW;
      const int uu = ou - kR + cc, vv = ov - kR + r;
      const bool in = i < kIH * kIW && uu >= 0 && uu < W && vv >= 0 && vv < H;
      const size_t p = (size_t)vv * W + uu;
#pragma unroll
      for (int q = 0; q < 3; ++q) ld[q][j] = in ? D[q * PL + p] : 0.f;
    }
  };
  if ((int)blockIdx.x < tiles) fetch(blockIdx.x);
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int ou = (tile % tiles_x) * kTW, ov = (tile / tiles_x) * kTH;
    const int u = ou + c;
    float x0[kRunY], y0[kRunY], g0[kRunY];
#pragma unroll
    for (int o = 0; o < kRunY; ++o) {
      x0[o] = xo[o];
      y0[o] = yo[o];
      if (a.l1) {
        const float d = xo[o] - yo[o];
        g0[o] = d > 0.f ? a.l1_scale : (d < 0.f ? -a.l1_scale : 0.f);
      } else {
        g0[o] = go[o];
      }
    }
    __syncthreads();   // the previous tile's LDS reads are done
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const int i = tid + j * kNT;
      if (i < kIH * kIW) {
        const int r = i / kIW, cc = i - r * kIW;
#pragma unroll
        for (int q = 0; q < 3; ++q) sd[q][r][cc] = ld[q][j];
      }
    }
    __syncthreads();
    if (tile + (int)gridDim.x < tiles) fetch(tile + gridDim.x);
    for (int it = tid; it < kHItems; it += kNT) {
      int r, c0;
      hitem(it, r, c0);
      if (r >= kIH) continue;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        float pv[kRunX + 2 * kR];
#pragma unroll
        for (int i = 0; i < kRunX + 2 * kR; ++i) pv[i] = sd[q][r][c0 + i];
#pragma unroll
        for (int o = 0; o < kRunX; ++o) {
          float s = 0.f;
#pragma unroll
          for (int b = 0; b < 2 * kR + 1; ++b) s = fmaf(w[b], pv[o + b], s);
          hs[q][r][c0 + o] = s;
        }
      }
    }
    __syncthreads();
    float col[3][kRunY + 2 * kR];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int i = 0; i < kRunY + 2 * kR; ++i) col[q][i] = hs[q][r0 + i][c];
#pragma unroll
    for (int o = 0; o < kRunY; ++o) {
      float m[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        float s = 0.f;
#pragma unroll
        for (int b = 0; b < 2 * kR + 1; ++b) s = fmaf(w[b], col[q][o + b], s);
        m[q] = s;
      }
      const int v = ov + r0 + o;
      if (u >= W || v >= H) continue;
      G[(size_t)v * W + u] = g0[o] + (m[0] + 2.f * x0[o] * m[1] + y0[o] * m[2]);
    }
  }
}

}  // namespace

hipError_t launch_loss_colour(const float* rgb, const float* target, int V,
                              int H, int W, float lam_l1, float lam,
                              int fuse_l1, float* dL, double* loss,
                              double* sqerr, double* ssim, float* scratch,
                              hipStream_t st);

hipError_t launch_loss_ssim(const float* rgb, const float* target, int V,
                            int H, int W, float lam, float* dL, double* loss,
                            double* ssim, float* scratch, hipStream_t st) {
  return launch_loss_colour(rgb, target, V, H, W, 0.f, lam, 0, dL, loss,
                            nullptr, ssim, scratch, st);
}

hipError_t launch_loss_colour(const float* rgb, const float* target, int V,
                              int H, int W, float lam_l1, float lam,
                              int fuse_l1, float* dL, double* loss,
                              double* sqerr, double* ssim, float* scratch,
                              hipStream_t st) {
  SsimArgs a;
  {
    double g[2 * kR + 1], sum = 0.0;
    for (int i = 0; i < 2 * kR + 1; ++i) {
      const double d = i - kR;
      g[i] = exp(-d * d / (2.0 * 1.5 * 1.5));
      sum += g[i];
    }
    for (int i = 0; i < 2 * kR + 1; ++i) a.w[i] = (float)(g[i] / sum);
  }
  a.x = rgb; a.y = target; a.dL = dL; a.scratch = scratch; a.loss = loss;
  a.ssim = ssim; a.V = V; a.H = H; a.W = W; a.lam = lam;
  const size_t per = (size_t)3 * H * W;
  a.l1 = fuse_l1;
  a.l1_scale = (float)((double)lam_l1 / (double)per);
  a.l1_lam_inv = (double)lam_l1 / (double)per;
  a.sqerr = sqerr;
  const dim3 grid((W + kTW - 1) / kTW, (H + kTH - 1) / kTH, V * 3);
  const int tiles = (int)(grid.x * grid.y);
  hipLaunchKernelGGL(k_ssim_stats, dim3(min(tiles, 64), V * 3), dim3(kNT), 0,
                     st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ssim_grad, dim3(min(tiles, 64), V * 3), dim3(kNT), 0,
                     st, a);
  return hipGetLastError();
}

}  // namespace gs
