// Clarity-enhancing densification (Eq. 8-9) after the dominant-Gaussian
// forward (render_fwd.hip, kDominant variant).
//
// k_dom_count counts, per Gaussian, the pixels it dominates.  A Gaussian that
// dominates more than sigma pixels is split into two children (the split of
// 3D Gaussian Splatting: means mu + R(q) (s * xi_c) with caller-drawn
// standard-normal xi, log-scales reduced by log 1.6, rotation, opacity,
// colour and view-dependent colour coefficients copied; child 0 in the
// parent's slot, child 1 appended).  The
// appended slots follow ascending parent index through a two-level
// exclusive scan (per-block counts, one scan block, per-block ranks), so the
// result is deterministic; parents whose appended child would not fit in
// the capacity are left unsplit and the overflow is reported.

#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kBlk = 1024;
constexpr float kLogSplit = 0.47000362924573558f;   // log(1.6)

struct DensifyArgs {
  gs_params p, m, v;
  const int32_t* dom;
  long long n_pix;
  int sigma;
  const float* xi;       // [cap][2][3]
  int32_t* counts;       // [cap]
  int32_t* bsum;         // [nb] block counts, then exclusive offsets
  int32_t* info;         // [4]: n before, appended, eligible
  int32_t* n_split;      // may be null
  int32_t* status;       // may be null
  int nb;
};

// Neighbouring pixels are mostly dominated by the same Gaussian, so each wave
// adds runs of equal indices (consecutive lanes) with one atomic per run.
__global__ __launch_bounds__(256) void k_dom_count(DensifyArgs a) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int g = i < a.n_pix ? a.dom[i] : -1;
  const int prev = __shfl_up(g, 1, 64);
  const bool head = lane == 0 || g != prev;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto =
      lane == 63 ? ~0ull : ((2ull << lane) - 1ull);   // lanes <= this one
  const unsigned long long after = heads & ~upto;
  const int next = after ? __ffsll((long long)after) - 1 : 64;
  if (head && g >= 0 && g < a.p.capacity) atomicAdd(&a.counts[g], next - lane);
}

__device__ inline bool eligible(const DensifyArgs& a, int g, int n) {
  return g < n && a.counts[g] > a.sigma;
}

// Inclusive scan over a block of kBlk threads (wave scans, then the wave
// totals); returns this thread's inclusive prefix and the block total.
__device__ inline int block_scan(int x, int* wsum, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  if (threadIdx.x < 64) {
    int s = threadIdx.x < kBlk / 64 ? wsum[threadIdx.x] : 0;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(s, off, 64);
      if (lane >= off) s += y;
    }
    if (threadIdx.x < kBlk / 64) wsum[threadIdx.x] = s;
  }
  __syncthreads();
  total = wsum[kBlk / 64 - 1];
  const int before = w ? wsum[w - 1] : 0;
  __syncthreads();
  return x + before;
}

__global__ __launch_bounds__(kBlk) void k_split_count(DensifyArgs a) {
  __shared__ int wsum[kBlk / 64];
  const int n = min(*a.p.n_dev, a.p.capacity);
  const int g = blockIdx.x * kBlk + threadIdx.x;
  int total;
  block_scan(eligible(a, g, n) ? 1 : 0, wsum, total);
  if (threadIdx.x == 0) a.bsum[blockIdx.x] = total;
}

// One block: exclusive offsets of the block counts, the number appended and
// the new live count.
__global__ __launch_bounds__(kBlk) void k_split_scan(DensifyArgs a) {
  __shared__ int wsum[kBlk / 64];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < a.nb; b0 += kBlk) {
    const int b = b0 + threadIdx.x;
    const int x = b < a.nb ? a.bsum[b] : 0;
    int total;
    const int incl = block_scan(x, wsum, total);
    const int c = carry;
    if (b < a.nb) a.bsum[b] = c + incl - x;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + total;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int n = min(*a.p.n_dev, a.p.capacity);
    const int want = carry;
    const int k = min(want, a.p.capacity - n);
    a.info[0] = n;
    a.info[1] = k;
    a.info[2] = want;
    *a.p.n_dev = n + k;
    if (a.n_split) *a.n_split = k;
    if (k < want && a.status) atomicOr(a.status, GS_STATUS_GAUSSIAN_OVERFLOW);
  }
}

__device__ inline void zero_slot(const gs_params& q, int cap, int s) {
  if (!q.mean) return;
  for (int j = 0; j < 3; ++j) {
    q.mean[j * cap + s] = 0.f;
    q.log_scale[j * cap + s] = 0.f;
    q.rgb[j * cap + s] = 0.f;
  }
  for (int j = 0; j < 4; ++j) q.quat[j * cap + s] = 0.f;
  q.opacity_logit[s] = 0.f;
  const int nsh = q.sh_degree > 0 ? GS_SH_ROWS(q.sh_degree) : 0;
  for (int r = 0; r < nsh; ++r) q.sh[(size_t)r * cap + s] = 0.f;
}

__global__ __launch_bounds__(kBlk) void k_split_write(DensifyArgs a) {
  __shared__ int wsum[kBlk / 64];
  const int n = a.info[0], k = a.info[1];
  const int cap = a.p.capacity;
  const int g = blockIdx.x * kBlk + threadIdx.x;
  const bool e = eligible(a, g, n);
  int total;
  const int rank = a.bsum[blockIdx.x] + block_scan(e ? 1 : 0, wsum, total) - 1;
  if (!e || rank >= k) return;
  const gs_params& P = a.p;
  float mu[3], ls[3], q[4], rgb[3];
  for (int j = 0; j < 3; ++j) {
    mu[j] = P.mean[j * cap + g];
    ls[j] = P.log_scale[j * cap + g];
    rgb[j] = P.rgb[j * cap + g];
  }
  for (int j = 0; j < 4; ++j) q[j] = P.quat[j * cap + g];
  const float op = P.opacity_logit[g];
  const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
  const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z),
                      2.f * (x * z + w * y),       2.f * (x * y + w * z),
                      1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                      2.f * (x * z - w * y),       2.f * (y * z + w * x),
                      1.f - 2.f * (x * x + y * y)};
  const float s[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
  const int slots[2] = {g, n + rank};
  for (int c = 0; c < 2; ++c) {
    const float* xi = a.xi + ((size_t)g * 2 + c) * 3;
    const float d0 = s[0] * xi[0], d1 = s[1] * xi[1], d2 = s[2] * xi[2];
    const int t = slots[c];
    for (int j = 0; j < 3; ++j) {
      P.mean[j * cap + t] = mu[j] + (R[3 * j] * d0 + R[3 * j + 1] * d1 +
                                     R[3 * j + 2] * d2);
      P.log_scale[j * cap + t] = ls[j] - kLogSplit;
      P.rgb[j * cap + t] = rgb[j];
    }
    for (int j = 0; j < 4; ++j) P.quat[j * cap + t] = q[j];
    P.opacity_logit[t] = op;
    zero_slot(a.m, cap, t);
    zero_slot(a.v, cap, t);
  }
  // View-dependent colour coefficients: child 0 keeps the parent's.
  const int nsh = P.sh_degree > 0 ? GS_SH_ROWS(P.sh_degree) : 0;
  for (int r = 0; r < nsh; ++r)
    P.sh[(size_t)r * cap + slots[1]] = P.sh[(size_t)r * cap + g];
}

}  // namespace

hipError_t launch_densify(gs_params* p, gs_params* m, gs_params* v,
                          const int32_t* dom, long long n_pix, int sigma,
                          const float* xi, int32_t* scratch, int32_t* n_split,
                          int32_t* status, hipStream_t st) {
  DensifyArgs a;
  a.p = *p;
  gs_params none{};
  a.m = m ? *m : none;
  a.v = v ? *v : none;
  a.dom = dom; a.n_pix = n_pix; a.sigma = sigma; a.xi = xi;
  const int cap = p->capacity;
  a.nb = (cap + kBlk - 1) / kBlk;
  a.counts = scratch;
  a.bsum = scratch + cap;
  a.info = a.bsum + a.nb;
  a.n_split = n_split; a.status = status;
  if (cap <= 0) return hipSuccess;
  hipError_t e = launch_fill_u32(a.counts, 0u, (size_t)cap, st);
  if (e != hipSuccess) return e;
  if (n_pix > 0)
    hipLaunchKernelGGL(k_dom_count, dim3((unsigned)((n_pix + 255) / 256)),
                       dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_split_count, dim3(a.nb), dim3(kBlk), 0, st, a);
  hipLaunchKernelGGL(k_split_scan, dim3(1), dim3(kBlk), 0, st, a);
  hipLaunchKernelGGL(k_split_write, dim3(a.nb), dim3(kBlk), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
