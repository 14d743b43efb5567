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
// Sorting network: bitonic over the segment padded to a power of two P2
// with all-ones keys (larger than any real key).  Segments up to kCap keys
// sort in registers: lane l of wave w holds the E consecutive positions
// (64 w + l) E .. + E - 1 (one wave with E = 1 up to 64 keys, else four waves
// with E = P2 / 256), so a compare-exchange at distance j < E stays inside a
// lane, one at E <= j < 64 E pairs lane l with lane l ^ (j / E) of the same
// wave (DPP for 1 and 2, swizzles for 4, 8 and 16, a lane permute for
// 32), and only j >= 64 E - at most three stages per segment - goes through
// LDS with barriers.  Longer segments (rare: a tile covered by more than kCap
// Gaussians) sort in place in the unsorted key buffer, with a global-memory
// bitonic network whose first comparator of every merge stage pairs mirrored
// positions, so positions past the end act as +infinity without being
// stored.

#include "gs_internal.h"

namespace gs {
namespace {

struct SortArgs {
  const uint32_t* ranges;
  const uint32_t* order;         // block b sorts tile order[b]
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

// 32-bit value of lane (lane ^ M): a DPP quad permutation for M = 1, 2 (one
// VALU instruction), a swizzle in bit-mask mode for 4, 8 and 16 (the LDS
// unit's crossbar, no LDS memory; a DPP form would take two row shifts and a
// select), a lane permute for 32.  Every lane of the wave is active here.
template <int M>
__device__ __forceinline__ int xor_lane32(int v, int lane) {
  if constexpr (M == 1) {
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, true);  // quad_perm 1,0,3,2
  } else if constexpr (M == 2) {
    return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, true);  // quad_perm 2,3,0,1
  } else if constexpr (M == 4 || M == 8 || M == 16) {
    return __builtin_amdgcn_ds_swizzle(v, 0x1f | (M << 10));  // and 31, xor M
  } else {
    return __shfl_xor(v, M, 64);
  }
}

template <int M>
__device__ __forceinline__ unsigned long long xor_lane(unsigned long long v,
                                                       int lane) {
  const uint32_t lo = (uint32_t)xor_lane32<M>((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)xor_lane32<M>((int)(uint32_t)(v >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

// Stage (k, J) with J < E: pairs inside the lane.
template <int E, int J>
__device__ __forceinline__ void stage_in_lane(unsigned long long (&x)[E],
                                              int base, int k) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e & J) continue;
    const bool asc = ((base + e) & k) == 0;
    const unsigned long long a = x[e], b = x[e + J];
    const bool swap = (b < a) == asc;
    x[e] = swap ? b : a;
    x[e + J] = swap ? a : b;
  }
}

// Stage (k, j) with E <= j < 64 E: lane l pairs with lane l ^ M, M = j / E.
template <int E, int M>
__device__ __forceinline__ void stage_across_lanes(unsigned long long (&x)[E],
                                                   int base, int k, int lane) {
  const bool asc = (base & k) == 0;
  const bool keep_min = ((lane & M) == 0) == asc;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const unsigned long long y = xor_lane<M>(x[e], lane);
    x[e] = ((y < x[e]) == keep_min) ? y : x[e];
  }
}

// Bitonic sort of P2 <= 64 E * nw keys held E per lane by the first nw waves
// of the workgroup (all waves reach the barriers of cross-wave stages).
template <int E>
__device__ void sort_in_registers(unsigned long long (&x)[E], int P2, int nw,
                                  unsigned long long* buf) {
  const int tid = threadIdx.x, lane = tid & 63;
  const bool active = (tid >> 6) < nw;
  const int base = tid * E;
  for (int k = 2; k <= P2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64 * E) {
        __syncthreads();
        if (active) {
#pragma unroll
          for (int e = 0; e < E; ++e) buf[base + e] = x[e];
        }
        __syncthreads();
        if (active) {
          const bool asc = (base & k) == 0;
          const bool keep_min = ((base & j) == 0) == asc;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const unsigned long long y = buf[(base + e) ^ j];
            x[e] = ((y < x[e]) == keep_min) ? y : x[e];
          }
        }
      } else if (j >= E) {
        if (!active) continue;
        switch (j / E) {
          case 1: stage_across_lanes<E, 1>(x, base, k, lane); break;
          case 2: stage_across_lanes<E, 2>(x, base, k, lane); break;
          case 4: stage_across_lanes<E, 4>(x, base, k, lane); break;
          case 8: stage_across_lanes<E, 8>(x, base, k, lane); break;
          case 16: stage_across_lanes<E, 16>(x, base, k, lane); break;
          default: stage_across_lanes<E, 32>(x, base, k, lane); break;
        }
      } else {
        if (!active) continue;
        if constexpr (E > 8) { if (j == 8) { stage_in_lane<E, 8>(x, base, k); continue; } }
        if constexpr (E > 4) { if (j == 4) { stage_in_lane<E, 4>(x, base, k); continue; } }
        if constexpr (E > 2) { if (j == 2) { stage_in_lane<E, 2>(x, base, k); continue; } }
        if constexpr (E > 1) { if (j == 1) { stage_in_lane<E, 1>(x, base, k); continue; } }
      }
    }
  }
}

template <int E>
__device__ void sort_tile(const SortArgs& a, int t, long long s, int L, int P2,
                          int nw, unsigned long long* buf) {
  const int tid = threadIdx.x;
  const bool active = (tid >> 6) < nw;
  if (nw == 1 && !active) return;   // no cross-wave stage: no barrier
  unsigned long long x[E];
  const int base = tid * E;
#pragma unroll
  for (int e = 0; e < E; ++e)
    x[e] = (active && base + e < L) ? a.keys_in[s + base + e] : ~0ull;
  sort_in_registers<E>(x, P2, nw, buf);
  if (!active) return;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = base + e;
    if (p < L) {
      a.vals_out[s + p] = (uint32_t)x[e];
      if (a.keys_out)
        a.keys_out[s + p] = ((unsigned long long)(uint32_t)t << 32) | (x[e] >> 32);
    }
  }
}

template <int kCap>
__global__ __launch_bounds__(256) void k_sort_tiles(SortArgs a) {
  static_assert(kCap == 4 * 64 * 16, "four waves of 16 keys per lane");
  __shared__ unsigned long long buf[kCap];
  const int t = (int)a.order[blockIdx.x];
  const int tid = threadIdx.x;
  const long long s = min((long long)a.ranges[2 * t], a.key_cap);
  const long long e = min((long long)a.ranges[2 * t + 1], a.key_cap);
  const int L = (int)(e - s);
  if (L <= 0) return;
  if (L <= kCap) {
    int P2 = 1;
    while (P2 < L) P2 <<= 1;
    // One wave for up to 64 keys, else all four waves (E = P2 / 256 keys
    // per lane, at least one), so enough waves per CU hide the latency of
    // the dependent compare-exchange stages.
    if (P2 <= 64) sort_tile<1>(a, t, s, L, P2, 1, buf);
    else if (P2 <= 256) sort_tile<1>(a, t, s, L, P2, 4, buf);
    else if (P2 <= 512) sort_tile<2>(a, t, s, L, P2, 4, buf);
    else if (P2 <= 1024) sort_tile<4>(a, t, s, L, P2, 4, buf);
    else if (P2 <= 2048) sort_tile<8>(a, t, s, L, P2, 4, buf);
    else sort_tile<16>(a, t, s, L, P2, 4, buf);
  } else {
    unsigned long long* g = a.keys_in + s;
    bitonic_sort(g, L, tid, 256);
    for (int i = tid; i < L; i += 256) {
      const unsigned long long v = g[i];
      a.vals_out[s + i] = (uint32_t)v;
      if (a.keys_out)
        a.keys_out[s + i] = ((unsigned long long)(uint32_t)t << 32) | (v >> 32);
    }
  }
}

}  // namespace

hipError_t launch_sort(gs_workspace* ws, const gs_settings* s, hipStream_t st) {
  SortArgs a;
  a.ranges = ws->ranges; a.order = ws->tile_order; a.keys_in = ws->keys_unsorted;
  a.vals_out = ws->vals_sorted;
  a.keys_out = (s->flags & GS_FLAG_EMIT_KEYS) ? ws->keys_sorted : nullptr;
  a.key_cap = ws->geo.key_capacity;
  const int blocks = ws->geo.n_views * ws->tiles_x * ws->tiles_y;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_tiles<4096>, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
