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
// Segments up to kCap keys sort in registers on 32-bit keys standing for
// the 64-bit ones (see sort_tile: exact offsets when the segment's depth
// and index ranges allow, else its depth bits quantised to 20 bits and
// tagged with the key's position, equal quanta put in order afterwards), so
// that a compare-exchange is a min and a max rather than a 64-bit compare
// and four selects.
//
// Sorting network: bitonic, in its all-ascending form, over the segment
// padded to a power of two P2 with all-ones keys (larger than any real key),
// unrolled at compile time for each P2.  In registers, lane l of wave w
// holds the E consecutive positions (64 w + l) E .. + E - 1 (one wave with
// E = 1 up to 64 keys, else four waves with E = P2 / 256), so a comparator
// whose positions differ only below bit log2 E stays inside a lane, one that
// differs below bit log2 64E pairs two lanes of the same wave (DPP,
// swizzles, lane permutes or swaps), and only the others - at most three
// merge steps per segment - go through LDS with barriers.  Padding never
// moves in the all-ascending form, so waves that hold only padding skip the
// compare-exchanges.  Longer segments (rare: a tile covered by more than
// kCap Gaussians) sort in place in the unsorted key buffer, with a
// global-memory bitonic network on the 64-bit keys in the same
// all-ascending form, so positions past the end act as +infinity without
// being stored.

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

// 32-bit value of lane (lane ^ M), every lane of the wave active:
//   M = 1, 3      DPP quad permutation (one VALU instruction)
//   M = 2         DPP quad permutation
//   M = 7, 15     DPP half-row and row mirror
//   M = 8         DPP row rotation by 8 (lane l of a 16-lane row reads l ^ 8)
//   M = 4, 16, 31 swizzle in bit-mask mode (the LDS unit's crossbar, no
//                 LDS memory)
//   M = 32, 63    lane permute.
// (The compare-exchanges at distance 16 and 32 use swap_halves below
// instead.)
template <int M>
__device__ __forceinline__ int xor_lane32(int v) {
  if constexpr (M == 1) {
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, true);  // quad_perm 1,0,3,2
  } else if constexpr (M == 2) {
    return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, true);  // quad_perm 2,3,0,1
  } else if constexpr (M == 3) {
    return __builtin_amdgcn_update_dpp(0, v, 0x1B, 0xf, 0xf, true);  // quad_perm 3,2,1,0
  } else if constexpr (M == 7) {
    return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, true); // row_half_mirror
  } else if constexpr (M == 15) {
    return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, true); // row_mirror
  } else if constexpr (M == 8) {
    return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, true); // row_ror:8
  } else if constexpr (M == 4 || M == 16 || M == 31) {
    return __builtin_amdgcn_ds_swizzle(v, 0x1f | (M << 10));  // and 31, xor M
  } else {
    static_assert(M == 32 || M == 63, "unsupported lane mask");
    return __shfl_xor(v, M, 64);
  }
}

template <int M>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  return (uint32_t)xor_lane32<M>((int)v);
}

__device__ __forceinline__ void keep(uint32_t& x, uint32_t y, bool keep_min) {
  x = ((y < x) == keep_min) ? y : x;
}

// The network is the all-ascending ("mirror") form of bitonic sort: merge
// step k first compares position p with p ^ (k - 1), the mirror image of p in
// its block of k, then p with p ^ j for j = k/4 .. 1; every comparator puts
// the smaller key at the lower position.  Padding keys (all ones) at the
// positions >= L therefore never move, so a wave whose positions all lie at
// or past L has nothing to do but its part of the barriers.  It runs on the
// 32-bit keys of sort_tile: a compare-exchange within a lane is one min and
// one max.
//
// In-lane stages: mirror step k <= E, or distance j < E.
template <int E, int K>
__device__ __forceinline__ void mirror_in_lane(uint32_t (&x)[E]) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e & (K >> 1)) continue;
    const int h = e ^ (K - 1);
    const uint32_t a = x[e], b = x[h];
    x[e] = min(a, b);
    x[h] = max(a, b);
  }
}

template <int E, int J>
__device__ __forceinline__ void stage_in_lane(uint32_t (&x)[E]) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e & J) continue;
    const uint32_t a = x[e], b = x[e + J];
    x[e] = min(a, b);
    x[e + J] = max(a, b);
  }
}

// Mirror step E < k <= 64 E: position (lane, e) pairs with (lane ^ M,
// E - 1 - e), M = k / E - 1.
template <int E, int M>
__device__ __forceinline__ void mirror_across_lanes(uint32_t (&x)[E], int lane) {
  const bool keep_min = (lane & ((M + 1) >> 1)) == 0;
  if constexpr (E == 1) {
    keep(x[0], xor_lane<M>(x[0]), keep_min);
  } else {
    // Mirrored pairs (e, E - 1 - e) together: two temporaries live at once.
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
      const uint32_t ya = xor_lane<M>(x[E - 1 - e]);
      const uint32_t yb = xor_lane<M>(x[e]);
      keep(x[e], ya, keep_min);
      keep(x[E - 1 - e], yb, keep_min);
    }
  }
}

// Both halves of the pair (l, l ^ M) for M = 16 or 32 without an LDS-unit
// round trip: v_permlane16_swap / v_permlane32_swap of a value with itself
// leave, in every lane, its own key in t0 and its partner's in t1 when
// (l & M) == 0, and the other way round otherwise.
template <int M>
__device__ __forceinline__ void swap_halves(uint32_t v, uint32_t& t0,
                                            uint32_t& t1) {
  if constexpr (M == 32) {
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    t0 = p[0];
    t1 = p[1];
  } else {
    static_assert(M == 16, "row or half-wave exchange only");
    const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    t0 = p[0];
    t1 = p[1];
  }
}

// Distance E <= j < 64 E: lane l pairs with lane l ^ M, M = j / E.
template <int E, int M>
__device__ __forceinline__ void stage_across_lanes(uint32_t (&x)[E], int lane) {
  const bool keep_min = (lane & M) == 0;
  if constexpr (M == 16 || M == 32) {
    // The lower lane of a pair keeps min(t0, t1), the upper max(t0, t1):
    // with t0 its own key in the lower lane and its partner's in the upper,
    // both take t1 exactly when (t1 < t0) equals being the lower.
#pragma unroll
    for (int e = 0; e < E; ++e) {
      uint32_t t0, t1;
      swap_halves<M>(x[e], t0, t1);
      x[e] = ((t1 < t0) == keep_min) ? t1 : t0;
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) keep(x[e], xor_lane<M>(x[e]), keep_min);
  }
}

// A stage whose partner lies in another wave (position p ^ m with m >= 64 E),
// through LDS.  The buffer is element-major (element e of thread t at
// buf[e * 256 + t]), so every store and every load of a wave touches 64
// consecutive slots in some lane order and no two lanes share a bank.
// m = ml E + ex with ex = 0 (distance j) or E - 1 (mirror step): the partner
// of element e of thread t is element e ^ ex of thread t ^ ml.  half is the
// bit of p that decides which side keeps the minimum.
template <int E>
__device__ __forceinline__ void stage_lds(uint32_t (&x)[E], int m, int half,
                                          bool active, bool work,
                                          uint32_t* buf) {
  const int tid = threadIdx.x;
  const int ml = m / E, ex = m % E;
  __syncthreads();
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) buf[e * 256 + tid] = x[e];
  }
  __syncthreads();
  if (work) {
    const bool keep_min = ((tid * E) & half) == 0;
    const uint32_t* src = buf + (tid ^ ml);
#pragma unroll
    for (int e = 0; e < E; ++e) keep(x[e], src[(e ^ ex) * 256], keep_min);
  }
}

// The network for a padded size P2 known at compile time, as a recursion
// over the merge steps k = 2 .. P2 and their distances j = k/4 .. 1, so that
// every stage's kind, partner mask and LDS offsets are constants (no loop or
// switch left to the scalar unit).  Sorts the first L of P2 <= 64 E nw keys
// held E per lane by the first nw waves of the workgroup (all waves reach
// the barriers of cross-wave stages); positions >= L hold all-ones keys.
template <int E, int J>
__device__ __forceinline__ void distance_stages(uint32_t (&x)[E], bool active,
                                                bool work, int lane,
                                                uint32_t* buf) {
  if constexpr (J >= 64 * E) {
    stage_lds<E>(x, J, J, active, work, buf);
  } else if (work) {
    if constexpr (J >= E) stage_across_lanes<E, J / E>(x, lane);
    else stage_in_lane<E, J>(x);
  }
  if constexpr (J > 1) distance_stages<E, J / 2>(x, active, work, lane, buf);
}

template <int E, int P2, int K>
__device__ __forceinline__ void merge_steps(uint32_t (&x)[E], bool active,
                                            bool work, int lane,
                                            uint32_t* buf) {
  if constexpr (K > 64 * E) {
    stage_lds<E>(x, K - 1, K >> 1, active, work, buf);
  } else if (work) {
    if constexpr (K <= E) mirror_in_lane<E, K>(x);
    else mirror_across_lanes<E, K / E - 1>(x, lane);
  }
  if constexpr (K >= 4) distance_stages<E, K / 4>(x, active, work, lane, buf);
  if constexpr (K < P2) merge_steps<E, P2, 2 * K>(x, active, work, lane, buf);
}

template <int E, int P2>
__device__ __forceinline__ void sort_in_registers(uint32_t (&x)[E], int L,
                                                  int nw, uint32_t* buf) {
  const int tid = threadIdx.x, lane = tid & 63;
  const bool active = (tid >> 6) < nw;
  const bool work = active && (tid >> 6) * 64 * E < L;
  if constexpr (P2 >= 2) merge_steps<E, P2, 2>(x, active, work, lane, buf);
}

// Orders one wave's LDS accesses before and after this point (the one-wave
// segments have no other wave to wait for).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr int kIdxBits = 12;   // position in a segment of at most 4096 keys
constexpr int kQBits = 32 - kIdxBits;

// One segment of L <= 4096 keys, sorted by the network on 32-bit keys that
// stand for the 64-bit ones.  With d the depth bits and g the index less
// the segment's smallest of each:
//  - exact, when the ranges of d and g fit 31 bits together (a segment of
//    one depth, or nearly): d << gbits | g, the 64-bit order itself;
//  - quantised otherwise: q << 12 | i, q = d >> shift with the least shift
//    that fits d's range in 20 bits, i the key's position in the unsorted
//    segment.  Integer shifts keep the order of the depth bits (a smaller q
//    means a smaller depth); i makes every key unique and names its 64-bit
//    key.  After the network each run of equal q - in practice a single key,
//    or the few Gaussians of an inserted patch - is put in (depth, index)
//    order by ranking its members' 64-bit keys, so the result is exactly
//    the sorted 64-bit segment.
// The all-ones padding stays above every real key (exact keys are below
// 2^31; i = 4095 only when L = 4096, with no padding).
template <int E, int P2>
__device__ void sort_tile(const SortArgs& a, int t, long long s, int L, int nw,
                          uint32_t* buf, uint32_t* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool active = wave < nw;
  if (nw == 1 && !active) return;   // no cross-wave stage: no barrier
  const int base = tid * E;
  uint32_t dhi[E], glo[E];
  uint32_t dmin = 0xffffffffu, dmax = 0u, gmin = 0xffffffffu, gmax = 0u;
  // Positions clamped into the segment (L >= 1), so every load is valid
  // and a lane's E loads are issued together instead of one guarded load
  // and wait after another; padding then takes 0.
  unsigned long long kin[E];
#pragma unroll
  for (int e = 0; e < E; ++e) kin[e] = a.keys_in[s + min(base + e, L - 1)];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = base + e;
    const bool real = active && p < L;
    const unsigned long long k = real ? kin[e] : 0ull;
    dhi[e] = (uint32_t)(k >> 32);
    glo[e] = (uint32_t)k;
    if (real) {
      dmin = min(dmin, dhi[e]);
      dmax = max(dmax, dhi[e]);
      gmin = min(gmin, glo[e]);
      gmax = max(gmax, glo[e]);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    dmin = min(dmin, (uint32_t)__shfl_xor((int)dmin, off, 64));
    dmax = max(dmax, (uint32_t)__shfl_xor((int)dmax, off, 64));
    gmin = min(gmin, (uint32_t)__shfl_xor((int)gmin, off, 64));
    gmax = max(gmax, (uint32_t)__shfl_xor((int)gmax, off, 64));
  }
  if (nw > 1) {
    if (lane == 0) {
      red[4 * wave] = dmin;
      red[4 * wave + 1] = dmax;
      red[4 * wave + 2] = gmin;
      red[4 * wave + 3] = gmax;
    }
    __syncthreads();
    for (int w = 0; w < nw; ++w) {
      dmin = min(dmin, red[4 * w]);
      dmax = max(dmax, red[4 * w + 1]);
      gmin = min(gmin, red[4 * w + 2]);
      gmax = max(gmax, red[4 * w + 3]);
    }
  }
  // dmax >= dmin and gmax >= gmin for L >= 1.
  const uint32_t drange = dmax - dmin, grange = gmax - gmin;
  const int dbits = drange ? 32 - __clz((int)drange) : 0;
  const int gbits = grange ? 32 - __clz((int)grange) : 0;
  const bool exact = dbits + gbits <= 31;
  const int shift = dbits > kQBits ? dbits - kQBits : 0;
  uint32_t x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = base + e;
    const uint32_t d = dhi[e] - dmin;
    x[e] = !(active && p < L) ? 0xffffffffu
           : exact ? (d << gbits) | (glo[e] - gmin)
                   : ((d >> shift) << kIdxBits) | (uint32_t)p;
  }
  sort_in_registers<E, P2>(x, L, nw, buf);
  if (exact) {   // the keys are the 64-bit order: write them out
    if (!active) return;
    const uint32_t gmask = gbits ? 0xffffffffu >> (32 - gbits) : 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = base + e;
      if (p >= L) continue;
      a.vals_out[s + p] = (x[e] & gmask) + gmin;
      if (a.keys_out)
        a.keys_out[s + p] = ((unsigned long long)(uint32_t)t << 32) |
                            ((x[e] >> gbits) + dmin);
    }
    return;
  }
  // Publish the sorted 32-bit keys position-major for the run tests.
  if (nw > 1) __syncthreads(); else wave_sync();
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (base + e < L) buf[base + e] = x[e];
  }
  if (nw > 1) __syncthreads(); else wave_sync();
  if (!active || base >= L) return;
  // The lane's E positions are consecutive, so the runs they fall in cover
  // one range [A, B): one scan to the left of the first position and one to
  // the right of the last.  Inside it a smaller quantum means a smaller
  // 64-bit key, so each key's final position is A plus the number of keys
  // of the range below it; the range's keys are loaded once for all E.
  // (Quadratic in the length of a run: fine for the runs of real scenes, a
  // few keys; a segment of many Gaussians at a few exact depths is correct
  // but slow.)
  constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1;
  const int ne = min(E, L - base);
  unsigned long long full[E];
  bool multi = false;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    full[e] = e < ne ? a.keys_in[s + (x[e] & kIdxMask)] : 0ull;
    if (e + 1 < ne) multi |= (x[e] >> kIdxBits) == (x[e + 1] >> kIdxBits);
  }
  const uint32_t q0 = x[0] >> kIdxBits;
  uint32_t ql = q0;
#pragma unroll
  for (int e = 1; e < E; ++e)
    if (e < ne) ql = x[e] >> kIdxBits;
  int A = base;
  while (A > 0 && (buf[A - 1] >> kIdxBits) == q0) --A;
  int B = base + ne;
  while (B < L && (buf[B] >> kIdxBits) == ql) ++B;
  multi |= A < base || B > base + ne;
  int r[E];
#pragma unroll
  for (int e = 0; e < E; ++e) r[e] = e;
  if (multi) {
#pragma unroll
    for (int e = 0; e < E; ++e) r[e] = A - base;
    for (int i = A; i < B; ++i) {
      const unsigned long long fi = a.keys_in[s + (buf[i] & kIdxMask)];
#pragma unroll
      for (int e = 0; e < E; ++e) r[e] += fi < full[e] ? 1 : 0;
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e >= ne) continue;
    const int pos = base + r[e];
    a.vals_out[s + pos] = (uint32_t)full[e];
    if (a.keys_out)
      a.keys_out[s + pos] =
          ((unsigned long long)(uint32_t)t << 32) | (full[e] >> 32);
  }
}

// At most 96 VGPRs (five waves per SIMD); the 16 KB LDS buffer allows more
// workgroups per CU than the registers do.
template <int kCap>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
void k_sort_tiles(SortArgs a) {
  static_assert(kCap == 4 * 64 * 16, "four waves of 16 keys per lane");
  static_assert(kCap <= (1 << kIdxBits), "positions fit the key's index bits");
  __shared__ uint32_t buf[kCap];
  __shared__ uint32_t red[16];
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
    switch (P2) {   // padded sizes: 1 .. 64 in one wave, then 256 E
      case 1: sort_tile<1, 1>(a, t, s, L, 1, buf, red); break;
      case 2: sort_tile<1, 2>(a, t, s, L, 1, buf, red); break;
      case 4: sort_tile<1, 4>(a, t, s, L, 1, buf, red); break;
      case 8: sort_tile<1, 8>(a, t, s, L, 1, buf, red); break;
      case 16: sort_tile<1, 16>(a, t, s, L, 1, buf, red); break;
      case 32: sort_tile<1, 32>(a, t, s, L, 1, buf, red); break;
      case 64: sort_tile<1, 64>(a, t, s, L, 1, buf, red); break;
      case 128: sort_tile<1, 128>(a, t, s, L, 4, buf, red); break;
      case 256: sort_tile<1, 256>(a, t, s, L, 4, buf, red); break;
      case 512: sort_tile<2, 512>(a, t, s, L, 4, buf, red); break;
      case 1024: sort_tile<4, 1024>(a, t, s, L, 4, buf, red); break;
      case 2048: sort_tile<8, 2048>(a, t, s, L, 4, buf, red); break;
      default: sort_tile<16, 4096>(a, t, s, L, 4, buf, red); break;
    }
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
