// Learned initialisation of inserted Gaussians: kNN features and a small
// MLP (32 -> 64 -> 64 -> 7, GELU) on BF16 MFMA with FP32 accumulation.
//
// Parameters: one FP32 vector of 6727 master weights, W1 [32][64], b1 [64],
// W2 [64][64], b2 [64], W3 [64][7], b3 [7] (z = x W + b).  Weights, the
// features and each hidden activation are rounded to BF16 (nearest, ties to
// even) where they enter a product; biases, pre-activations and GELU are
// FP32.  Backward: every gradient entering a product is rounded to BF16,
// bias gradients are not, and the rounding of weights and activations
// passes gradients unchanged.
//
// MFMA: v_mfma_f32_16x16x16_bf16 (one wave computes a 16x16 FP32 tile);
// lane l holds A[l % 16][4 (l / 16) + i], B[4 (l / 16) + i][l % 16] and
// D[4 (l / 16) + i][l % 16] for i = 0..3.  A workgroup of four waves takes
// 64 rows (one 16-row block per wave) through all three layers with the
// weights staged in LDS as BF16.

#include <math.h>

#include "gs_internal.h"

namespace gs {
namespace {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kIn = 32, kHid = 64, kOut = 7, kOutPad = 16;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kIn * kHid;
constexpr int kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid * kOut;
constexpr int kParams = kOffB3 + kOut;
static_assert(kParams == 6727, "parameter count");

__device__ __forceinline__ unsigned short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float from_bf16(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ f4v mfma(s4v a, s4v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Weights staged in LDS as BF16: W1 [32][64], W2 [64][64], W3 [64][16]
// (output columns 7..15 zero), biases FP32.
struct SharedWeights {
  unsigned short w1[kIn * kHid];
  unsigned short w2[kHid * kHid];
  unsigned short w3[kHid * kOutPad];
  float b1[kHid], b2[kHid], b3[kOutPad];
};

__device__ void stage_weights(SharedWeights& S, const float* w, int tid,
                              int nthr) {
  for (int i = tid; i < kIn * kHid; i += nthr) S.w1[i] = to_bf16(w[kOffW1 + i]);
  for (int i = tid; i < kHid * kHid; i += nthr) S.w2[i] = to_bf16(w[kOffW2 + i]);
  for (int i = tid; i < kHid * kOutPad; i += nthr) {
    const int r = i / kOutPad, c = i % kOutPad;
    S.w3[i] = c < kOut ? to_bf16(w[kOffW3 + r * kOut + c]) : 0;
  }
  for (int i = tid; i < kHid; i += nthr) {
    S.b1[i] = w[kOffB1 + i];
    S.b2[i] = w[kOffB2 + i];
  }
  for (int i = tid; i < kOutPad; i += nthr) S.b3[i] = i < kOut ? w[kOffB3 + i] : 0.f;
}

// One 16x16 output tile: rows of A from a row-major [.][lda] BF16 array
// starting at row r0, columns of B from a row-major [K][ldb] array starting
// at column c0 (or, with BT, B[k][n] = src[(c0 + n) * ldb + k]).
template <int K, bool BT>
__device__ __forceinline__ f4v tile(const unsigned short* A, int lda, int r0,
                                    const unsigned short* B, int ldb, int c0,
                                    int lane) {
  f4v acc = {0.f, 0.f, 0.f, 0.f};
  const int m = lane & 15, kq = 4 * (lane >> 4);
#pragma unroll
  for (int kb = 0; kb < K; kb += 16) {
    s4v a, b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = (short)A[(r0 + m) * lda + kb + kq + i];
      b[i] = BT ? (short)B[(c0 + m) * ldb + kb + kq + i]
                : (short)B[(kb + kq + i) * ldb + c0 + m];
    }
    acc = mfma(a, b, acc);
  }
  return acc;
}

// Tile of A^T B where both operands are row-major over the batch (K) axis:
// C[m][n] = sum_k A[k][r0 + m] B[k][c0 + n].
template <int K>
__device__ __forceinline__ f4v tile_tn(const unsigned short* A, int lda,
                                       int r0, const unsigned short* B, int ldb,
                                       int c0, int lane) {
  f4v acc = {0.f, 0.f, 0.f, 0.f};
  const int m = lane & 15, kq = 4 * (lane >> 4);
#pragma unroll
  for (int kb = 0; kb < K; kb += 16) {
    s4v a, b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = (short)A[(kb + kq + i) * lda + r0 + m];
      b[i] = (short)B[(kb + kq + i) * ldb + c0 + m];
    }
    acc = mfma(a, b, acc);
  }
  return acc;
}

struct MlpFwdShared {
  SharedWeights W;
  unsigned short x[64 * kIn];
  unsigned short h1[64 * kHid];
  unsigned short h2[64 * kHid];
};

__global__ __launch_bounds__(256) void k_mlp_fwd(const float* w, const float* x,
                                                 int M, float* y, float* cache) {
  __shared__ MlpFwdShared S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row0 = blockIdx.x * 64;
  stage_weights(S.W, w, tid, 256);
  for (int i = tid; i < 64 * kIn; i += 256) {
    const int r = row0 + i / kIn;
    S.x[i] = r < M ? to_bf16(x[(size_t)r * kIn + i % kIn]) : 0;
  }
  __syncthreads();
  const int r0 = wv * 16;
  const int rq = 4 * (lane >> 4), cc = lane & 15;
  // Layer 1.
  for (int nb = 0; nb < kHid; nb += 16) {
    const f4v acc = tile<kIn, false>(S.x, kIn, r0, S.W.w1, kHid, nb, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + rq + i, c = nb + cc;
      const float z = acc[i] + S.W.b1[c];
      if (cache && row0 + r < M) cache[(size_t)(row0 + r) * 128 + c] = z;
      S.h1[r * kHid + c] = to_bf16(gelu(z));
    }
  }
  __syncthreads();
  // Layer 2.
  for (int nb = 0; nb < kHid; nb += 16) {
    const f4v acc = tile<kHid, false>(S.h1, kHid, r0, S.W.w2, kHid, nb, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + rq + i, c = nb + cc;
      const float z = acc[i] + S.W.b2[c];
      if (cache && row0 + r < M) cache[(size_t)(row0 + r) * 128 + 64 + c] = z;
      S.h2[r * kHid + c] = to_bf16(gelu(z));
    }
  }
  __syncthreads();
  // Layer 3 (7 outputs padded to 16).
  const f4v acc = tile<kHid, false>(S.h2, kHid, r0, S.W.w3, kOutPad, 0, lane);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = r0 + rq + i, c = cc;
    if (c < kOut && row0 + r < M) y[(size_t)(row0 + r) * kOut + c] = acc[i] + S.W.b3[c];
  }
}

struct MlpBwdShared {
  SharedWeights W;
  unsigned short x[64 * kIn];
  unsigned short h1[64 * kHid];
  unsigned short h2[64 * kHid];
  unsigned short dy[64 * kOutPad];
  unsigned short dz2[64 * kHid];
  unsigned short dz1[64 * kHid];
  float db[kHid + kHid + kOutPad];
};

__global__ __launch_bounds__(256) void k_mlp_bwd(const float* w, const float* x,
                                                 const float* cache,
                                                 const float* dy, int M,
                                                 float* dw) {
  __shared__ MlpBwdShared S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row0 = blockIdx.x * 64;
  stage_weights(S.W, w, tid, 256);
  for (int i = tid; i < 64 * kIn; i += 256) {
    const int r = row0 + i / kIn;
    S.x[i] = r < M ? to_bf16(x[(size_t)r * kIn + i % kIn]) : 0;
  }
  for (int i = tid; i < 64 * kHid; i += 256) {
    const int r = row0 + i / kHid, c = i % kHid;
    const bool ok = r < M;
    S.h1[i] = ok ? to_bf16(gelu(cache[(size_t)r * 128 + c])) : 0;
    S.h2[i] = ok ? to_bf16(gelu(cache[(size_t)r * 128 + 64 + c])) : 0;
  }
  for (int i = tid; i < 64 * kOutPad; i += 256) {
    const int r = row0 + i / kOutPad, c = i % kOutPad;
    S.dy[i] = (r < M && c < kOut) ? to_bf16(dy[(size_t)r * kOut + c]) : 0;
  }
  for (int i = tid; i < 2 * kHid + kOutPad; i += 256) S.db[i] = 0.f;
  __syncthreads();
  // db3 = column sums of dy (unrounded).
  if (tid < kOut) {
    float s = 0.f;
    for (int r = 0; r < 64 && row0 + r < M; ++r) s += dy[(size_t)(row0 + r) * kOut + tid];
    S.db[2 * kHid + tid] = s;
  }
  const int r0 = wv * 16;
  const int rq = 4 * (lane >> 4), cc = lane & 15;
  // dZ2 = (dY W3^T) * gelu'(Z2).
  for (int nb = 0; nb < kHid; nb += 16) {
    const f4v acc = tile<kOutPad, true>(S.dy, kOutPad, r0, S.W.w3, kOutPad, nb, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + rq + i, c = nb + cc;
      float dz = 0.f;
      if (row0 + r < M) dz = acc[i] * gelu_grad(cache[(size_t)(row0 + r) * 128 + 64 + c]);
      S.dz2[r * kHid + c] = to_bf16(dz);
      atomicAdd(&S.db[kHid + c], dz);
    }
  }
  __syncthreads();
  // dZ1 = (dZ2 W2^T) * gelu'(Z1).
  for (int nb = 0; nb < kHid; nb += 16) {
    const f4v acc = tile<kHid, true>(S.dz2, kHid, r0, S.W.w2, kHid, nb, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + rq + i, c = nb + cc;
      float dz = 0.f;
      if (row0 + r < M) dz = acc[i] * gelu_grad(cache[(size_t)(row0 + r) * 128 + c]);
      S.dz1[r * kHid + c] = to_bf16(dz);
      atomicAdd(&S.db[c], dz);
    }
  }
  __syncthreads();
  // Weight gradients over this block's 64 rows, then one atomic per weight.
  {  // dW3 [64][7]: wave wv takes input rows 16 wv ..
    const f4v acc = tile_tn<64>(S.h2, kHid, r0, S.dy, kOutPad, 0, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + rq + i, c = cc;
      if (c < kOut) atomicAdd(&dw[kOffW3 + r * kOut + c], acc[i]);
    }
  }
  for (int nb = 0; nb < kHid; nb += 16) {  // dW2 [64][64]
    const f4v acc = tile_tn<64>(S.h1, kHid, r0, S.dz2, kHid, nb, lane);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      atomicAdd(&dw[kOffW2 + (r0 + rq + i) * kHid + nb + cc], acc[i]);
  }
  {  // dW1 [32][64]: 8 tiles, two per wave
    const int mb = (wv >> 1) * 16;
    for (int nb = (wv & 1) * 32; nb < (wv & 1) * 32 + 32; nb += 16) {
      const f4v acc = tile_tn<64>(S.x, kIn, mb, S.dz1, kHid, nb, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        atomicAdd(&dw[kOffW1 + (mb + rq + i) * kHid + nb + cc], acc[i]);
    }
  }
  __syncthreads();
  for (int i = tid; i < kHid; i += 256) {
    atomicAdd(&dw[kOffB1 + i], S.db[i]);
    atomicAdd(&dw[kOffB2 + i], S.db[kHid + i]);
  }
  if (tid < kOut) atomicAdd(&dw[kOffB3 + tid], S.db[2 * kHid + tid]);
}

__global__ __launch_bounds__(256) void k_mlp_mse(const float* y, const float* t,
                                                 int n, float scale, float* dy,
                                                 double* loss) {
  __shared__ double part[4];
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float d = y[i] - t[i];
    dy[i] = scale * d;
    s += (double)d * (double)d;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0 && loss)
    atomicAdd(loss, (part[0] + part[1] + part[2] + part[3]) / (double)n);
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* w, const float* g,
                                                  float* m, float* v, float lr,
                                                  float b1, float b2, float eps,
                                                  float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kParams) return;
  const float gr = g[i];
  const float mm = b1 * m[i] + (1.f - b1) * gr;
  const float vv = b2 * v[i] + (1.f - b2) * gr * gr;
  m[i] = mm;
  v[i] = vv;
  w[i] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ---- kNN features ----------------------------------------------------------

struct KnnArgs {
  const float* mean;   // [3][cap]
  const float* rgb;    // [3][cap]
  const int32_t* n_dev;
  int cap;
  const gs_camera* cam;
  int W, H;
  const float* kf_rgb;
  const float* pts;
  int n_pts, per;
  float* feats;        // [C][32]
  int32_t* knn_idx;    // [C][8] or null
  float* knn_dist;     // [C][8] or null
};

struct Nb {
  double d2;
  int idx;
};

__device__ __forceinline__ bool nb_less(const Nb& a, const Nb& b) {
  return a.d2 < b.d2 || (a.d2 == b.d2 && (unsigned)a.idx < (unsigned)b.idx);
}

// One workgroup per candidate: every thread keeps the 8 nearest of its
// stride of Gaussians (FP64 squared distances), then the lists are merged
// pairwise in LDS.
__global__ __launch_bounds__(256) void k_knn_features(KnnArgs a) {
  __shared__ Nb lists[256][8];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int patch = c / a.per;
  const int pix = a.per == 1 ? 4 : c - patch * a.per;
  const int u = (int)a.pts[3 * patch] + pix % 3 - 1;
  const int v = (int)a.pts[3 * patch + 1] + pix / 3 - 1;
  const float d = a.pts[3 * patch + 2];
  const gs_camera cam = *a.cam;
  const double z = d > 0.f ? 1.0 / (double)d : 0.0;
  const double xc[3] = {((double)u - (double)cam.cx) / (double)cam.fx * z,
                        ((double)v - (double)cam.cy) / (double)cam.fy * z, z};
  double X[3];
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int j = 0; j < 3; ++j) s += (double)cam.R[3 * j + i] * (xc[j] - (double)cam.t[j]);
    X[i] = s;
  }
  Nb best[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) best[j] = Nb{INFINITY, -1};
  const int n = min(*a.n_dev, a.cap);
  for (int g = tid; g < n; g += 256) {
    const double dx = (double)a.mean[g] - X[0];
    const double dy = (double)a.mean[a.cap + g] - X[1];
    const double dz = (double)a.mean[2 * a.cap + g] - X[2];
    Nb cand{dx * dx + dy * dy + dz * dz, g};
    if (!nb_less(cand, best[7])) continue;
#pragma unroll
    for (int j = 7; j >= 0; --j) {
      if (j > 0 && nb_less(cand, best[j - 1])) {
        best[j] = best[j - 1];
      } else {
        best[j] = cand;
        break;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) lists[tid][j] = best[j];
  __syncthreads();
  for (int step = 1; step < 256; step <<= 1) {
    if ((tid & (2 * step - 1)) == 0) {
      Nb m[8];
      int ia = 0, ib = 0;
      for (int j = 0; j < 8; ++j) {
        const Nb& A = lists[tid][ia];
        const Nb& B = lists[tid + step][ib];
        if (nb_less(B, A)) { m[j] = B; ++ib; } else { m[j] = A; ++ia; }
      }
      for (int j = 0; j < 8; ++j) lists[tid][j] = m[j];
    }
    __syncthreads();
  }
  float* f = a.feats + (size_t)c * 32;
  if (tid < 27) {
    const int q = tid / 3, ch = tid % 3;
    const int uu = u + q % 3 - 1, vv = v + q / 3 - 1;
    f[tid] = (uu >= 0 && uu < a.W && vv >= 0 && vv < a.H)
                 ? a.kf_rgb[((size_t)ch * a.H + vv) * a.W + uu] : 0.f;
  } else if (tid == 27) {
    f[27] = d;
  } else if (tid == 28) {
    double sl = 0.0, sw = 0.0, sc[3] = {0, 0, 0};
    int cnt = 0;
    for (int j = 0; j < 8; ++j) {
      const Nb& b = lists[0][j];
      if (b.idx < 0) break;
      const double dist = fmax(sqrt(b.d2), 1e-6);
      sl += log(dist);
      const double wgt = 1.0 / dist;
      sw += wgt;
      for (int ch = 0; ch < 3; ++ch) sc[ch] += wgt * (double)a.rgb[(size_t)ch * a.cap + b.idx];
      if (a.knn_idx) a.knn_idx[(size_t)c * 8 + j] = b.idx;
      if (a.knn_dist) a.knn_dist[(size_t)c * 8 + j] = (float)sqrt(b.d2);
      ++cnt;
    }
    for (int j = cnt; j < 8; ++j) {
      if (a.knn_idx) a.knn_idx[(size_t)c * 8 + j] = -1;
      if (a.knn_dist) a.knn_dist[(size_t)c * 8 + j] = 0.f;
    }
    f[28] = cnt ? (float)(sl / cnt) : 0.f;
    for (int ch = 0; ch < 3; ++ch) f[29 + ch] = cnt ? (float)(sc[ch] / sw) : 0.f;
  }
}

}  // namespace

hipError_t launch_knn_features(const gs_params* p, const gs_camera* cam, int W,
                               int H, const float* kf_rgb, const float* pts,
                               int n_pts, int centre_only, float* feats,
                               int32_t* knn_idx, float* knn_dist,
                               hipStream_t st) {
  KnnArgs a;
  a.mean = p->mean; a.rgb = p->rgb; a.n_dev = p->n_dev; a.cap = p->capacity;
  a.cam = cam; a.W = W; a.H = H; a.kf_rgb = kf_rgb; a.pts = pts;
  a.n_pts = n_pts; a.per = centre_only ? 1 : 9; a.feats = feats;
  a.knn_idx = knn_idx; a.knn_dist = knn_dist;
  const int C = n_pts * a.per;
  if (C > 0) hipLaunchKernelGGL(k_knn_features, dim3(C), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_mlp_fwd(const float* w, const float* x, int M, float* y,
                          float* cache, hipStream_t st) {
  if (M > 0)
    hipLaunchKernelGGL(k_mlp_fwd, dim3((M + 63) / 64), dim3(256), 0, st, w, x,
                       M, y, cache);
  return hipGetLastError();
}

hipError_t launch_mlp_bwd(const float* w, const float* x, const float* cache,
                          const float* dy, int M, float* dw, hipStream_t st) {
  if (M > 0)
    hipLaunchKernelGGL(k_mlp_bwd, dim3((M + 63) / 64), dim3(256), 0, st, w, x,
                       cache, dy, M, dw);
  return hipGetLastError();
}

hipError_t launch_mlp_mse(const float* y, const float* t, int M, float* dy,
                          double* loss, hipStream_t st) {
  const int n = M * kOut;
  if (n <= 0) return hipSuccess;
  int blocks = (n + 255) / 256;
  if (blocks > 120) blocks = 120;
  hipLaunchKernelGGL(k_mlp_mse, dim3(blocks), dim3(256), 0, st, y, t, n,
                     2.f / (float)n, dy, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v,
                           float lr, float b1, float b2, float eps, int step,
                           hipStream_t st) {
  const float c1 = (float)(1.0 - pow((double)b1, step));
  const float c2 = (float)(1.0 - pow((double)b2, step));
  hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, st,
                     w, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace gs
