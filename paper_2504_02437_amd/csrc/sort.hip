// Per-tile sort of the binned keys.
//
// After the scatter every tile owns a contiguous segment of 64-bit keys
// (FP32 depth bits << 32 | Gaussian index) in unspecified order.  One
// workgroup per (view, tile) sorts its segment ascending.  Depths are
// positive, so their IEEE bit patterns order like the values; the index in
// the low half makes every key unique and breaks depth ties in index order,
// which is exactly the order of a stable sort of (tile << 32 | depth bits)
// keys emitted Gaussian by Gaussian.
//
// Sorting network: bitonic, in the form whose first comparator of every
// merge stage pairs mirrored positions, so every comparator is ascending and
// positions past the segment end act as +infinity without being stored.
// Segments up to kCap keys sort in LDS; longer ones sort in place in the
// unsorted key buffer (rare: a tile covered by more than kCap Gaussians).

#include "gs_internal.h"

namespace gs {
namespace {

struct SortArgs {
  const uint32_t* ranges;
  unsigned long long* keys_in;   // sorted in place when a segment is long
  uint32_t* vals_out;
  unsigned long long* keys_out;  // may be null
  long long key_cap;
};

template <typename P>
__device__ inline void cmp_swap(P a, int lo, int hi) {
  const unsigned long long x = a[lo], y = a[hi];
  if (y < x) {
    a[lo] = y;
    a[hi] = x;
  }
}

template <typename P>
__device__ void bitonic_sort(P a, int L, int tid, int nthr) {
  int P2 = 1;
  while (P2 < L) P2 <<= 1;
  const int pairs = P2 >> 1;
  for (int k = 2; k <= P2; k <<= 1) {
    const int half = k >> 1;
    const int hshift = __builtin_ctz(half);
    for (int i = tid; i < pairs; i += nthr) {
      const int blk = i >> hshift, off = i & (half - 1);
      const int lo = blk * k + off, hi = blk * k + k - 1 - off;
      if (hi < L) cmp_swap(a, lo, hi);
    }
    __syncthreads();
    for (int j = half >> 1; j > 0; j >>= 1) {
      const int jshift = __builtin_ctz(j);
      for (int i = tid; i < pairs; i += nthr) {
        const int lo = ((i >> jshift) << (jshift + 1)) + (i & (j - 1));
        const int hi = lo + j;
        if (hi < L) cmp_swap(a, lo, hi);
      }
      __syncthreads();
    }
  }
}

template <int kCap>
__global__ __launch_bounds__(256) void k_sort_tiles(SortArgs a) {
  __shared__ unsigned long long buf[kCap];
  const int t = blockIdx.x;
  const int tid = threadIdx.x;
  const long long s = min((long long)a.ranges[2 * t], a.key_cap);
  const long long e = min((long long)a.ranges[2 * t + 1], a.key_cap);
  const int L = (int)(e - s);
  if (L <= 0) return;
  auto store = [&](int i, unsigned long long v) {
    a.vals_out[s + i] = (uint32_t)v;
    if (a.keys_out)
      a.keys_out[s + i] = ((unsigned long long)(uint32_t)t << 32) | (v >> 32);
  };
  if (L <= kCap) {
    for (int i = tid; i < L; i += 256) buf[i] = a.keys_in[s + i];
    __syncthreads();
    bitonic_sort(buf, L, tid, 256);
    for (int i = tid; i < L; i += 256) store(i, buf[i]);
  } else {
    unsigned long long* g = a.keys_in + s;
    bitonic_sort(g, L, tid, 256);
    for (int i = tid; i < L; i += 256) store(i, g[i]);
  }
}

}  // namespace

hipError_t launch_sort(gs_workspace* ws, const gs_settings* s, hipStream_t st) {
  SortArgs a;
  a.ranges = ws->ranges; a.keys_in = ws->keys_unsorted;
  a.vals_out = ws->vals_sorted;
  a.keys_out = (s->flags & GS_FLAG_EMIT_KEYS) ? ws->keys_sorted : nullptr;
  a.key_cap = ws->geo.key_capacity;
  const int blocks = ws->geo.n_views * ws->tiles_x * ws->tiles_y;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_tiles<4096>, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
