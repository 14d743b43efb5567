// Loss terms of the map optimisation (Eq. 10-11), the Adam step and keyframe
// insertion (Eq. 6), plus a fill kernel used instead of memset so every call
// stays safe to capture in a HIP graph.

#include <math.h>

#include "gs_internal.h"
#include "tails.h"

namespace gs {
namespace {

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
__device__ inline T block_sum(T x, T* sh) {
  // 256 threads, wave64.
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = x;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < 4; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// L1 photometric term: per view lambda * mean |rgb - target| over 3HW.
// A few hundred blocks per view stream the images with 16-byte loads (the
// per-view image starts 16-byte aligned when 3HW is a multiple of 4; other
// sizes take the scalar path), so only a few hundred FP64 atomics land on
// the loss accumulator.
__global__ __launch_bounds__(256) void k_loss_l1(const float* rgb,
                                                 const float* tgt, size_t per,
                                                 float scale, float* dL,
                                                 double* loss, double* sqerr,
                                                 double lam_inv) {
  __shared__ double sh[4];
  const int k = blockIdx.y;
  const float* x = rgb + (size_t)k * per;
  const float* y = tgt + (size_t)k * per;
  float* d = dL + (size_t)k * per;
  float sa = 0.f;
  double sq = 0.0;
  const size_t stride = (size_t)gridDim.x * 256;
  const size_t first = blockIdx.x * 256 + threadIdx.x;
  auto one = [&](float a, float b) -> float {
    const float r = a - b;
    sa += fabsf(r);
    sq += (double)r * (double)r;
    return r > 0.f ? scale : (r < 0.f ? -scale : 0.f);
  };
  if ((per & 3) == 0) {
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const float4* y4 = reinterpret_cast<const float4*>(y);
    float4* d4 = reinterpret_cast<float4*>(d);
    for (size_t i = first; i < per / 4; i += stride) {
      const float4 a = x4[i], b = y4[i];
      float4 o;
      o.x = one(a.x, b.x);
      o.y = one(a.y, b.y);
      o.z = one(a.z, b.z);
      o.w = one(a.w, b.w);
      d4[i] = o;
    }
  } else {
    for (size_t i = first; i < per; i += stride) d[i] = one(x[i], y[i]);
  }
  const double ta = block_sum((double)sa, sh);
  const double tq = block_sum(sq, sh);
  if (threadIdx.x == 0) {
    atomicAdd(loss, ta * lam_inv);
    if (sqerr) atomicAdd(&sqerr[k], tq);
  }
}

// Planar regulariser: lambda * mean_g max(floor, min_j exp(l_gj)).  A grid
// stride over the Gaussians with a few hundred workgroups: the loss takes
// one FP64 atomic per workgroup, and atomics on one address serialise.
__global__ __launch_bounds__(256) void k_planar_reg(PlanarJob j) {
  __shared__ double sh[4];
  planar_part(j, blockIdx.x, gridDim.x, sh);
}

struct AdamArgs {
  float* p[14];
  const float* g[14];
  float* m[14];
  float* v[14];
  float lr[14];
  // View-dependent colour coefficient rows (row 14 + r at offset r cap).
  float* psh;
  const float* gsh;
  float* msh;
  float* vsh;
  float lr_sh;
  const int32_t* n_dev;
  const int32_t* step_dev;
  int cap, step;
  int step_bias;   // added to *step_dev
  float b1, b2, eps;
};

// Elements per thread: the bias corrections (two FP64 powers by one thread
// of the workgroup) are formed once per kAdamPer * 256 elements.
constexpr int kAdamPer = 4;

__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
  __shared__ float corr[2];
  const int g0 = blockIdx.x * 256 * kAdamPer + threadIdx.x;
  const int row = blockIdx.y;
  const int n = min(*a.n_dev, a.cap);
  if (blockIdx.x * 256 * kAdamPer >= n) return;
  float *P, *M, *Vv;
  const float* G;
  float lr;
  if (row < 14) {
    P = a.p[row]; G = a.g[row]; M = a.m[row]; Vv = a.v[row]; lr = a.lr[row];
  } else {
    const size_t o = (size_t)(row - 14) * a.cap;
    P = a.psh + o; G = a.gsh + o; M = a.msh + o; Vv = a.vsh + o; lr = a.lr_sh;
  }
  // All loads first, so their latencies overlap each other and the bias
  // corrections' powers below.
  float gr[kAdamPer], mo[kAdamPer], vo[kAdamPer], po[kAdamPer];
#pragma unroll
  for (int i = 0; i < kAdamPer; ++i) {
    const int g = g0 + i * 256;
    const bool in = g < n;
    gr[i] = in ? G[g] : 0.f;
    mo[i] = in ? M[g] : 0.f;
    vo[i] = in ? Vv[g] : 0.f;
    po[i] = in ? P[g] : 0.f;
  }
  if (threadIdx.x == 0) {
    const int step = a.step_dev ? max(1, *a.step_dev + a.step_bias) : a.step;
    corr[0] = (float)(1.0 - pow((double)a.b1, (double)step));
    corr[1] = (float)(1.0 - pow((double)a.b2, (double)step));
  }
  __syncthreads();
  const float c1 = corr[0], c2 = corr[1];
#pragma unroll
  for (int i = 0; i < kAdamPer; ++i) {
    const int g = g0 + i * 256;
    if (g >= n) break;
    const float m = a.b1 * mo[i] + (1.f - a.b1) * gr[i];
    const float v = a.b2 * vo[i] + (1.f - a.b2) * gr[i] * gr[i];
    M[g] = m;
    Vv[g] = v;
    P[g] = po[i] - lr * (m / c1) / (sqrtf(v / c2) + a.eps);
  }
}

struct InsertArgs {
  float* rows[14];   // mean 0-2, log_scale 3-5, quat 6-9, opacity 10, rgb 11-13
  float* mrows[14];  // may be null
  float* vrows[14];
  int32_t* n_dev;
  int cap;
  const gs_camera* cam;
  int W, H;
  const float* kf_rgb;
  const float* kf_T;
  const float* pts;
  int n_pts;
  float alpha_skip;
  int centre_only;
  const float* mlp_out;
  int32_t* n_inserted;
  int32_t* status;
  // Distance test (Eq. 7) instead of the alpha mask when not null: FP64
  // bits of each candidate's nearest squared distance (all ones: no mean).
  const unsigned long long* d2bits;
  double tau2;
  // View-dependent colour coefficient rows, zeroed for new entries (the
  // moments' may be null).
  float* sh;
  float* msh;
  float* vsh;
  int n_sh_rows;
};

// Back-projection of candidate pixel (u, v) with inverse depth d (Eq. 6),
// FP64 without contraction so the distance test reproduces exactly.
__device__ inline void back_project(const gs_camera& cam, int u, int v,
                                    double d, double* X) {
#pragma clang fp contract(off)
  const double z = 1.0 / d;
  const double xc[3] = {((double)u - (double)cam.cx) / (double)cam.fx * z,
                        ((double)v - (double)cam.cy) / (double)cam.fy * z, z};
  for (int i = 0; i < 3; ++i) {
    double sacc = 0.0;
    for (int j = 0; j < 3; ++j)
      sacc += (double)cam.R[3 * j + i] * (xc[j] - (double)cam.t[j]);
    X[i] = sacc;
  }
}

constexpr int kInsThreads = 1024;

__global__ __launch_bounds__(kInsThreads) void k_insert(InsertArgs a) {
  __shared__ int scan[kInsThreads];
  const int tid = threadIdx.x;
  const int n0 = min(*a.n_dev, a.cap);
  const gs_camera cam = *a.cam;
  const int per = a.centre_only ? 1 : 9;
  const int total = a.n_pts * per;
  int running = 0;
  for (int base = 0; base < total; base += kInsThreads) {
    const int c = base + tid;
    int keep = 0, u = 0, v = 0, patch = 0;
    if (c < total) {
      patch = c / per;
      const int pix = a.centre_only ? 4 : c - patch * per;
      u = (int)a.pts[3 * patch] + pix % 3 - 1;
      v = (int)a.pts[3 * patch + 1] + pix / 3 - 1;
      const float d = a.pts[3 * patch + 2];
      if (u >= 0 && u < a.W && v >= 0 && v < a.H && d > 0.f) {
        if (a.d2bits) {
          const unsigned long long b = a.d2bits[c];
          keep = b == ~0ull || __longlong_as_double((long long)b) > a.tau2;
        } else {
          const double accum = 1.0 - (double)a.kf_T[(size_t)v * a.W + u];
          keep = accum <= (double)a.alpha_skip;
        }
      }
    }
    scan[tid] = keep;
    __syncthreads();
    for (int off = 1; off < kInsThreads; off <<= 1) {
      const int x = tid >= off ? scan[tid - off] : 0;
      __syncthreads();
      scan[tid] += x;
      __syncthreads();
    }
    const int incl = scan[tid];
    const int count = scan[kInsThreads - 1];
    if (keep) {
      const int dst = n0 + running + incl - 1;
      if (dst < a.cap) {
        const double z = 1.0 / (double)a.pts[3 * patch + 2];
        double X[3];
        back_project(cam, u, v, (double)a.pts[3 * patch + 2], X);
        for (int i = 0; i < 3; ++i) a.rows[i][dst] = (float)X[i];
        if (a.mlp_out) {
          const float* o = a.mlp_out + 7 * (size_t)c;
          for (int i = 0; i < 3; ++i) a.rows[3 + i][dst] = o[i];
          a.rows[10][dst] = o[3];
          for (int i = 0; i < 3; ++i) a.rows[11 + i][dst] = o[4 + i];
        } else {
          const float ls = (float)log(z / (double)cam.fx);
          for (int i = 0; i < 3; ++i) a.rows[3 + i][dst] = ls;
          a.rows[10][dst] = 0.f;
          for (int i = 0; i < 3; ++i)
            a.rows[11 + i][dst] =
                a.kf_rgb[((size_t)i * a.H + v) * a.W + u];
        }
        a.rows[6][dst] = 1.f;
        a.rows[7][dst] = 0.f;
        a.rows[8][dst] = 0.f;
        a.rows[9][dst] = 0.f;
        for (int r = 0; r < 14; ++r) {
          if (a.mrows[r]) a.mrows[r][dst] = 0.f;
          if (a.vrows[r]) a.vrows[r][dst] = 0.f;
        }
        for (int r = 0; r < a.n_sh_rows; ++r) {
          const size_t o = (size_t)r * a.cap + dst;
          a.sh[o] = 0.f;
          if (a.msh) a.msh[o] = 0.f;
          if (a.vsh) a.vsh[o] = 0.f;
        }
      }
    }
    running += count;
    __syncthreads();
  }
  if (tid == 0) {
    if (a.n_inserted) *a.n_inserted = running;
    const long long want = (long long)n0 + running;
    *a.n_dev = (int)min(want, (long long)a.cap);
    if (want > a.cap && a.status) atomicOr(a.status, GS_STATUS_GAUSSIAN_OVERFLOW);
  }
}

// Distance test of Eq. 7: the squared distance from each candidate's
// back-projected point to the nearest live mean, as the FP64 bit pattern
// (non-negative doubles order like their bits) min-combined over blocks that
// each scan a slice of the means.  A block stages its slice in LDS (FP64)
// and each thread holds kNearPer candidates (threads tid, tid + 256, ...),
// so one LDS broadcast read of a mean serves kNearPer distances.  The
// distance is formed exactly as before in the same order, so the minimum
// does not depend on the partition.
constexpr int kNearPer = 4;      // candidates per thread
constexpr int kNearSlice = 256;  // means per block

struct NearestArgs {
  const float* mean;   // [3][cap]
  const int32_t* n_dev;
  int cap;
  const gs_camera* cam;
  int W, H;
  const float* pts;
  int n_pts, centre_only;
  unsigned long long* d2bits;
};

__global__ __launch_bounds__(256) void k_nearest(NearestArgs a) {
#pragma clang fp contract(off)
  __shared__ double sm[3][kNearSlice];
  const int per = a.centre_only ? 1 : 9;
  const int C = a.n_pts * per;
  const int n = min(*a.n_dev, a.cap);
  const int g0 = blockIdx.y * kNearSlice;
  if (g0 >= n) return;   // uniform over the block
  const int cnt = min(kNearSlice, n - g0);
  const int tid = threadIdx.x;
  for (int i = tid; i < cnt; i += 256) {
    sm[0][i] = (double)a.mean[g0 + i];
    sm[1][i] = (double)a.mean[a.cap + g0 + i];
    sm[2][i] = (double)a.mean[2 * a.cap + g0 + i];
  }
  const gs_camera cam = *a.cam;
  double X[kNearPer][3];
  bool live[kNearPer];
  int cid[kNearPer];
#pragma unroll
  for (int q = 0; q < kNearPer; ++q) {
    const int c = (blockIdx.x * kNearPer + q) * 256 + tid;
    cid[q] = c;
    live[q] = false;
    X[q][0] = X[q][1] = X[q][2] = 0.0;
    if (c >= C) continue;
    const int patch = c / per;
    const int pix = a.centre_only ? 4 : c - patch * per;
    const int u = (int)a.pts[3 * patch] + pix % 3 - 1;
    const int v = (int)a.pts[3 * patch + 1] + pix / 3 - 1;
    const float d = a.pts[3 * patch + 2];
    if (!(u >= 0 && u < a.W && v >= 0 && v < a.H && d > 0.f)) continue;
    back_project(cam, u, v, (double)d, X[q]);
    live[q] = true;
  }
  __syncthreads();
  double best[kNearPer];
#pragma unroll
  for (int q = 0; q < kNearPer; ++q) best[q] = INFINITY;
  for (int i = 0; i < cnt; ++i) {
    const double mx = sm[0][i], my = sm[1][i], mz = sm[2][i];
#pragma unroll
    for (int q = 0; q < kNearPer; ++q) {
      const double e0 = X[q][0] - mx;
      const double e1 = X[q][1] - my;
      const double e2 = X[q][2] - mz;
      const double d2 = (e0 * e0 + e1 * e1) + e2 * e2;
      best[q] = fmin(best[q], d2);
    }
  }
#pragma unroll
  for (int q = 0; q < kNearPer; ++q)
    if (live[q])
      atomicMin(&a.d2bits[cid[q]], (unsigned long long)__double_as_longlong(best[q]));
}

void rows_of(const gs_params* p, float** rows) {
  const int cap = p->capacity;
  for (int i = 0; i < 3; ++i) rows[i] = p->mean ? p->mean + (size_t)i * cap : nullptr;
  for (int i = 0; i < 3; ++i)
    rows[3 + i] = p->log_scale ? p->log_scale + (size_t)i * cap : nullptr;
  for (int i = 0; i < 4; ++i) rows[6 + i] = p->quat ? p->quat + (size_t)i * cap : nullptr;
  rows[10] = p->opacity_logit;
  for (int i = 0; i < 3; ++i) rows[11 + i] = p->rgb ? p->rgb + (size_t)i * cap : nullptr;
}

// Row pointers of the parameters and (optional) moments for k_insert.
void insert_rows(gs_params* p, gs_params* m, gs_params* v, InsertArgs& a) {
  rows_of(p, a.rows);
  if (m) rows_of(m, a.mrows); else for (int i = 0; i < 14; ++i) a.mrows[i] = nullptr;
  if (v) rows_of(v, a.vrows); else for (int i = 0; i < 14; ++i) a.vrows[i] = nullptr;
  a.n_sh_rows = p->sh_degree > 0 ? GS_SH_ROWS(p->sh_degree) : 0;
  a.sh = p->sh;
  a.msh = m ? m->sh : nullptr;
  a.vsh = v ? v->sh : nullptr;
}

}  // namespace

hipError_t launch_fill_u32(void* ptr, uint32_t value, size_t count,
                           hipStream_t st) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st,
                     (uint32_t*)ptr, value, count);
  return hipGetLastError();
}

hipError_t launch_loss_l1(const float* rgb, const float* target, int V, int H,
                          int W, float lambda, float* dL, double* loss,
                          double* sqerr, hipStream_t st) {
  const size_t per = (size_t)3 * H * W;
  const float scale = (float)((double)lambda / (double)per);
  size_t bx = (per + 256 * 16 - 1) / (256 * 16);
  if (bx > 160) bx = 160;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_loss_l1, dim3((unsigned)bx, V), dim3(256), 0, st, rgb,
                     target, per, scale, dL, loss, sqerr,
                     (double)lambda / (double)per);
  return hipGetLastError();
}

PlanarJob planar_job(const gs_params* p, float lambda, float floor_,
                     gs_params* grad, double* loss) {
  return PlanarJob{p->log_scale, p->n_dev, p->capacity, lambda,
                   (double)floor_, grad->log_scale, loss};
}

hipError_t launch_planar_job(const PlanarJob& j, hipStream_t st) {
  const int blocks = min(256, (j.cap + 255) / 256);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_planar_reg, dim3(blocks), dim3(256), 0, st, j);
  return hipGetLastError();
}

hipError_t launch_planar_reg(const gs_params* p, float lambda, float floor_,
                             gs_params* grad, double* loss, hipStream_t st) {
  return launch_planar_job(planar_job(p, lambda, floor_, grad, loss), st);
}

hipError_t launch_adam(gs_params* p, const gs_params* g, gs_params* m,
                       gs_params* v, const float* lr, float b1, float b2,
                       float eps, int step, const int32_t* step_dev,
                       hipStream_t st, int step_bias) {
  AdamArgs a;
  float* tmp[14];
  rows_of(p, a.p);
  rows_of(g, tmp);
  for (int i = 0; i < 14; ++i) a.g[i] = tmp[i];
  rows_of(m, a.m);
  rows_of(v, a.v);
  const int grp[14] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 2, 3, 4, 4, 4};
  for (int i = 0; i < 14; ++i) a.lr[i] = lr[grp[i]];
  const int nsh = p->sh_degree > 0 ? GS_SH_ROWS(p->sh_degree) : 0;
  a.psh = p->sh; a.gsh = g->sh; a.msh = m->sh; a.vsh = v->sh;
  a.lr_sh = nsh ? lr[5] : 0.f;
  a.n_dev = p->n_dev; a.cap = p->capacity;
  a.b1 = b1; a.b2 = b2; a.eps = eps;
  a.step = step; a.step_dev = step_dev; a.step_bias = step_bias;
  const int blocks = (p->capacity + 256 * kAdamPer - 1) / (256 * kAdamPer);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3(blocks, 14 + nsh), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_insert(gs_params* p, gs_params* m, gs_params* v,
                         const gs_camera* cam, int W, int H,
                         const float* kf_rgb, const float* kf_T,
                         const float* pts, int n_pts, float alpha_skip,
                         int centre_only, const float* mlp_out,
                         int32_t* n_inserted, int32_t* status, hipStream_t st) {
  InsertArgs a;
  insert_rows(p, m, v, a);
  a.n_dev = p->n_dev; a.cap = p->capacity; a.cam = cam; a.W = W; a.H = H;
  a.kf_rgb = kf_rgb; a.kf_T = kf_T; a.pts = pts; a.n_pts = n_pts;
  a.alpha_skip = alpha_skip; a.centre_only = centre_only; a.mlp_out = mlp_out;
  a.n_inserted = n_inserted; a.status = status;
  a.d2bits = nullptr; a.tau2 = 0.0;
  hipLaunchKernelGGL(k_insert, dim3(1), dim3(kInsThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_insert_distance(gs_params* p, gs_params* m, gs_params* v,
                                  const gs_camera* cam, int W, int H,
                                  const float* kf_rgb, const float* pts,
                                  int n_pts, float tau, int centre_only,
                                  const float* mlp_out,
                                  unsigned long long* d2bits,
                                  int32_t* n_inserted, int32_t* status,
                                  hipStream_t st) {
  const int per = centre_only ? 1 : 9;
  const int C = n_pts * per;
  if (C > 0) {
    hipError_t e = launch_fill_u32(d2bits, 0xffffffffu, 2 * (size_t)C, st);
    if (e != hipSuccess) return e;
    NearestArgs na;
    na.mean = p->mean; na.n_dev = p->n_dev; na.cap = p->capacity; na.cam = cam;
    na.W = W; na.H = H; na.pts = pts; na.n_pts = n_pts;
    na.centre_only = centre_only; na.d2bits = d2bits;
    const int bc = (C + 256 * kNearPer - 1) / (256 * kNearPer);
    const int slices = (p->capacity + kNearSlice - 1) / kNearSlice;
    if (slices > 0)
      hipLaunchKernelGGL(k_nearest, dim3(bc, slices), dim3(256), 0, st, na);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  InsertArgs a;
  insert_rows(p, m, v, a);
  a.n_dev = p->n_dev; a.cap = p->capacity; a.cam = cam; a.W = W; a.H = H;
  a.kf_rgb = kf_rgb; a.kf_T = nullptr; a.pts = pts; a.n_pts = n_pts;
  a.alpha_skip = 0.f; a.centre_only = centre_only; a.mlp_out = mlp_out;
  a.n_inserted = n_inserted; a.status = status;
  a.d2bits = d2bits;
  a.tau2 = (double)tau * (double)tau;
  hipLaunchKernelGGL(k_insert, dim3(1), dim3(kInsThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
