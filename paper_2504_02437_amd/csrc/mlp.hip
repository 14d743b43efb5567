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

// kNN features.  A workgroup serves kKnnCpb candidates with kKnnWpc waves
// each.  The means pass through LDS a chunk at a time (read once per
// workgroup), the next chunk's loads in flight while the current one is
// scanned; every lane keeps the 8 nearest of its share in registers (FP64
// squared distances in (distance, index) order).  The lists of a wave are
// then merged with a bitonic network over lane shuffles, and the waves of a
// candidate through LDS.  Each distance is formed from the same FP32 means
// in the same order, so the result does not depend on the partition.
constexpr int kKnnWpc = 4;      // waves per candidate
constexpr int kKnnCpb = 4;      // candidates per workgroup
constexpr int kKnnThreads = 64 * kKnnWpc * kKnnCpb;
constexpr int kKnnChunk = 4096;  // means staged per round
constexpr int kKnnPer = kKnnChunk / kKnnThreads;   // staged per thread
constexpr int kKnnIt = kKnnChunk / (64 * kKnnWpc);   // scanned per lane
static_assert(kKnnChunk % kKnnThreads == 0, "whole staging rounds");

// Sorted insertion as a chain of compare-swaps (no dynamic index, so the
// list stays in registers).
__device__ __forceinline__ void nb_insert(Nb (&best)[8], Nb x) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const bool lt = nb_less(x, best[j]);
    const double td = best[j].d2;
    const int ti = best[j].idx;
    best[j].d2 = lt ? x.d2 : td;
    best[j].idx = lt ? x.idx : ti;
    x.d2 = lt ? td : x.d2;
    x.idx = lt ? ti : x.idx;
  }
}

__device__ __forceinline__ void nb_cswap(Nb& lo, Nb& hi) {
  const bool sw = nb_less(hi, lo);
  const double d = lo.d2;
  const int i = lo.idx;
  lo.d2 = sw ? hi.d2 : d;
  lo.idx = sw ? hi.idx : i;
  hi.d2 = sw ? d : hi.d2;
  hi.idx = sw ? i : hi.idx;
}

// 64-bit value of lane (lane ^ m).
__device__ __forceinline__ unsigned long long xor_lane64(unsigned long long v, int m) {
  const int src = ((int)__lane_id() ^ m) << 2;
  const unsigned lo = __builtin_amdgcn_ds_bpermute(src, (int)v);
  const unsigned hi = __builtin_amdgcn_ds_bpermute(src, (int)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// The 8 smallest of the union of this lane's sorted list and that of lane
// (lane ^ m), for m = 1, 2, .. < span: every lane of an aligned group of
// span lanes ends with the group's 8 smallest, sorted.  (Elementwise minima
// of one ascending and one descending list are the lower half of their
// union and form a bitonic sequence; three half-cleaner stages sort it.)
__device__ __forceinline__ void nb_wave_merge(Nb (&best)[8], int span) {
  for (int m = 1; m < span; m <<= 1) {
    Nb o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      o[j].d2 = __longlong_as_double(
          (long long)xor_lane64((unsigned long long)__double_as_longlong(best[j].d2), m));
      o[j].idx = __builtin_amdgcn_ds_bpermute(((int)__lane_id() ^ m) << 2, best[j].idx);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const bool tb = nb_less(o[7 - j], best[j]);
      best[j].d2 = tb ? o[7 - j].d2 : best[j].d2;
      best[j].idx = tb ? o[7 - j].idx : best[j].idx;
    }
#pragma unroll
    for (int s = 4; s >= 1; s >>= 1)
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if ((j & s) == 0) nb_cswap(best[j], best[j + s]);
  }
}

// Squared distances compare as their bit patterns (they are >= 0 or NaN,
// and NaN orders last); a full key for "no entry".
__device__ __forceinline__ unsigned long long d2_key(double d2) {
  return (unsigned long long)__double_as_longlong(d2);
}

// The 8th smallest key over the wave's 64 lanes (bitonic sort across lanes),
// in every lane.
__device__ __forceinline__ unsigned long long wave_eighth(unsigned long long v) {
  const int lane = (int)__lane_id();
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const unsigned long long o = xor_lane64(v, j);
      const bool take_min = ((lane & j) == 0) == ((lane & k) == 0);
      const bool ol = o < v;
      v = take_min == ol ? o : v;
    }
  const unsigned lo = __builtin_amdgcn_readlane((int)v, 7);
  const unsigned hi = __builtin_amdgcn_readlane((int)(v >> 32), 7);
  return ((unsigned long long)hi << 32) | lo;
}

// Chunks after which the waves refresh the shared rejection threshold: 1, 2,
// 3, 4, 6, 8, 12, 16, .. (it falls roughly as the inverse of the count
// scanned, so a geometric schedule keeps it close).
__device__ __forceinline__ bool knn_refresh(int m) {
  const int q = m % 3 == 0 ? m / 3 : 0;
  return (m & (m - 1)) == 0 || (q && (q & (q - 1)) == 0);
}

__global__ __launch_bounds__(kKnnThreads) void k_knn_features(KnnArgs a) {
  __shared__ float sm[2][3][kKnnChunk];   // double-buffered chunks
  __shared__ double ld[kKnnCpb][kKnnWpc][8];
  __shared__ int li[kKnnCpb][kKnnWpc][8];
  __shared__ unsigned long long tau_sh[2][kKnnCpb][kKnnWpc];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int cw = wave / kKnnWpc, ww = wave % kKnnWpc;
  const int C = a.n_pts * a.per;
  const int c = blockIdx.x * kKnnCpb + cw;
  const bool live = c < C;   // uniform over the wave
  const int cc = live ? c : 0;
  const int patch = cc / a.per;
  const int pix = a.per == 1 ? 4 : cc - patch * a.per;
  const int u = (int)a.pts[3 * patch] + pix % 3 - 1;
  const int v = (int)a.pts[3 * patch + 1] + pix / 3 - 1;
  const float d = a.pts[3 * patch + 2];
  const gs_camera cam = *a.cam;
  const double z = d > 0.f ? 1.0 / (double)d : 0.0;
  const double xc[3] = {((double)u - (double)cam.cx) / (double)cam.fx * z,
                        ((double)v - (double)cam.cy) / (double)cam.fy * z, z};
  double X[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) s += (double)cam.R[3 * j + i] * (xc[j] - (double)cam.t[j]);
    X[i] = s;
  }
  Nb best[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) best[j] = Nb{INFINITY, -1};
  const int n = min(*a.n_dev, a.cap);
  float pf[3][kKnnPer];
  auto fetch = [&](int g0) {
    if (g0 + kKnnChunk <= n) {
#pragma unroll
      for (int p = 0; p < kKnnPer; ++p)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          pf[k][p] = a.mean[(size_t)k * a.cap + g0 + tid + p * kKnnThreads];
    } else {
#pragma unroll
      for (int p = 0; p < kKnnPer; ++p) {
        const int g = g0 + tid + p * kKnnThreads;
#pragma unroll
        for (int k = 0; k < 3; ++k) pf[k][p] = g < n ? a.mean[(size_t)k * a.cap + g] : 0.f;
      }
    }
  };
  auto put = [&](int b) {
#pragma unroll
    for (int p = 0; p < kKnnPer; ++p)
#pragma unroll
      for (int k = 0; k < 3; ++k) sm[b][k][tid + p * kKnnThreads] = pf[k][p];
  };
  // Workgroups start at chunks spread over the map and wrap around, so that
  // they do not all read the same lines at once.  The lists are ordered by
  // (distance, index), so the scan order does not change them.
  //
  // Rejection threshold: when 8 lanes of the candidate each hold an entry at
  // squared distance <= tau, a Gaussian farther than tau cannot be among the
  // 8 nearest, so tau = the 8th smallest of the lanes' nearest entries lets
  // a lane skip it even while its own list is not full.  Equal distances
  // still reach the insertion, which settles them by index.
  const int nch = (n + kKnnChunk - 1) / kKnnChunk;
  int ch = (int)(((long long)blockIdx.x * nch) / gridDim.x);
  if (nch) {
    fetch(ch * kKnnChunk);
    put(0);
  }
  __syncthreads();
  const int sub = ww * 64 + lane;
  unsigned long long tau = ~0ull, thr = d2_key(INFINITY);
  auto scan = [&](const float* mx, const float* my, const float* mz, int i, int g) {
    const double dx = (double)mx[i] - X[0];
    const double dy = (double)my[i] - X[1];
    const double dz = (double)mz[i] - X[2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    if (d2_key(d2) <= thr) {
      nb_insert(best, Nb{d2, g});
      thr = min(d2_key(best[7].d2), tau);
    }
  };
  for (int t = 0, b = 0; t < nch; ++t, b ^= 1) {
    // Chunk t is in buffer b; the loads of chunk t + 1 fly meanwhile.
    const int g0 = ch * kKnnChunk;
    const int cnt = min(kKnnChunk, n - g0);
    ch = ch + 1 == nch ? 0 : ch + 1;
    if (t + 1 < nch) fetch(ch * kKnnChunk);
    const bool refresh = knn_refresh(t + 1);
    if (live) {
      const float* mx = sm[b][0];
      const float* my = sm[b][1];
      const float* mz = sm[b][2];
      if (cnt == kKnnChunk) {
#pragma unroll
        for (int u = 0; u < kKnnIt; ++u) scan(mx, my, mz, sub + u * 64 * kKnnWpc, g0 + sub + u * 64 * kKnnWpc);
      } else {
        for (int i = sub; i < cnt; i += 64 * kKnnWpc) scan(mx, my, mz, i, g0 + i);
      }
      if (refresh) {
        const unsigned long long tw = wave_eighth(d2_key(best[0].d2));
        if (lane == 0) tau_sh[b][cw][ww] = tw;
      }
    }
    // Buffer b ^ 1 was released by the barrier that ended chunk t - 1.
    if (t + 1 < nch) put(b ^ 1);
    __syncthreads();
    if (live && refresh) {
#pragma unroll
      for (int w = 0; w < kKnnWpc; ++w) tau = min(tau, tau_sh[b][cw][w]);
      thr = min(d2_key(best[7].d2), tau);
    }
  }
  nb_wave_merge(best, 64);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ld[cw][ww][j] = best[j].d2;
      li[cw][ww][j] = best[j].idx;
    }
  }
  __syncthreads();
  if (!live || ww != 0) return;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    best[j].d2 = lane < kKnnWpc ? ld[cw][lane % kKnnWpc][j] : INFINITY;
    best[j].idx = lane < kKnnWpc ? li[cw][lane % kKnnWpc][j] : -1;
  }
  nb_wave_merge(best, 64);
  float* f = a.feats + (size_t)c * 32;
  if (lane < 27) {
    const int q = lane / 3, ch = lane % 3;
    const int uu = u + q % 3 - 1, vv = v + q / 3 - 1;
    f[lane] = (uu >= 0 && uu < a.W && vv >= 0 && vv < a.H)
                  ? a.kf_rgb[((size_t)ch * a.H + vv) * a.W + uu] : 0.f;
  } else if (lane == 27) {
    f[27] = d;
  } else if (lane == 28) {
    double sl = 0.0, sw = 0.0, sc[3] = {0, 0, 0};
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const Nb& b = best[j];
      if (b.idx < 0) continue;
      const double dist = fmax(sqrt(b.d2), 1e-6);
      sl += log(dist);
      const double wgt = 1.0 / dist;
      sw += wgt;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) sc[ch] += wgt * (double)a.rgb[(size_t)ch * a.cap + b.idx];
      ++cnt;
    }
    f[28] = cnt ? (float)(sl / cnt) : 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) f[29 + ch] = cnt ? (float)(sc[ch] / sw) : 0.f;
  }
  if (lane < 8) {
    // Lane j writes neighbour j (the lists are identical on every lane).
    Nb b = best[0];
#pragma unroll
    for (int j = 1; j < 8; ++j)
      if (lane == j) b = best[j];
    if (a.knn_idx) a.knn_idx[(size_t)c * 8 + lane] = b.idx;
    if (a.knn_dist) a.knn_dist[(size_t)c * 8 + lane] = b.idx < 0 ? 0.f : (float)sqrt(b.d2);
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
  if (C > 0)
    hipLaunchKernelGGL(k_knn_features, dim3((C + kKnnCpb - 1) / kKnnCpb),
                       dim3(kKnnThreads), 0, st, a);
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
