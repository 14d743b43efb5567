// Tile binning: per-tile key counts, ranges, and the scatter of the
// (depth, index) keys into their tiles' segments, without global atomics.
//
// Each workgroup owns a chunk of Gaussians of one view (1024 or 2048) and
// counts the chunk's keys per tile in LDS, walking the keys with wave-level
// load balancing (one lane per key); the counts go to a [view][chunk][tile]
// matrix.  A column scan over the chunks turns every entry into the chunk's
// offset inside the tile's segment and gives the tile totals; one exclusive
// scan per view (plus the totals of the preceding views) gives every tile's
// [start, end) range, so n_keys never leaves the device.  The scatter then
// walks the same keys again and claims positions with LDS atomics from
// start + offset.  Each key is written as (depth bits << 32 | index), so the
// per-tile sort needs no gather.
//
// Tile grids too large for LDS counters bin the old way: the projection adds
// the four corners of each box of tiles into a coverage difference grid,
// whose 2D prefix sum is the count of every tile, and the scatter takes one
// global atomic per key.

#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kScanThreads = 1024;
constexpr int kMaxGridCells = 16384;  // LDS difference grid (64 KB)

struct CountArgs {
  int32_t* diff;        // [V][Ty + 1][Tx + 1], consumed and cleared
  uint32_t* counts;     // [V][Ty][Tx] key count per tile (the cursor array)
  int Tx, Ty;
};

// One workgroup per view: counts = 2D inclusive prefix of the difference
// grid.  Grids larger than kMaxGridCells are scanned in global memory.
__global__ __launch_bounds__(kScanThreads) void k_tile_count(CountArgs a) {
  __shared__ int32_t grid[kMaxGridCells];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int stride = a.Tx + 1, rows = a.Ty + 1;
  const int cells = stride * rows;
  int32_t* d = a.diff + (size_t)k * cells;
  const bool in_lds = cells <= kMaxGridCells;
  int32_t* G = in_lds ? grid : d;
  if (in_lds)
    for (int i = tid; i < cells; i += kScanThreads) grid[i] = d[i];
  __syncthreads();
  for (int y = tid; y < rows; y += kScanThreads) {
    int acc = 0;
    for (int x = 0; x < stride; ++x) { acc += G[y * stride + x]; G[y * stride + x] = acc; }
  }
  __syncthreads();
  for (int x = tid; x < stride; x += kScanThreads) {
    int acc = 0;
    for (int y = 0; y < rows; ++y) { acc += G[y * stride + x]; G[y * stride + x] = acc; }
  }
  __syncthreads();
  const int tiles = a.Tx * a.Ty;
  uint32_t* c = a.counts + (size_t)k * tiles;
  for (int t = tid; t < tiles; t += kScanThreads) {
    const int ty = t / a.Tx, tx = t - ty * a.Tx;
    c[t] = (uint32_t)G[ty * stride + tx];
  }
  for (int i = tid; i < cells; i += kScanThreads) d[i] = 0;
}

struct RangeArgs {
  uint32_t* counts;   // tile counts (read only)
  uint32_t* ranges;
  Counters* ctr;
  int V, Tx, Ty;
  long long key_cap;
};

// One workgroup per view: exclusive scan of the view's tile counts, offset by
// the totals of the preceding views (summed here from their counts), into
// the ranges.  The counts are left as they are: the other views' workgroups
// read them too.  The totals take four loads in flight per thread; the scan
// is a shuffle scan per wave plus the preceding waves' totals, so the
// workgroup meets at one barrier.
__global__ __launch_bounds__(kScanThreads) void k_tile_ranges(RangeArgs a) {
  constexpr int kWaves = kScanThreads / 64;
  __shared__ long long red[2][kWaves];
  __shared__ long long wsum[kWaves];
  const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int tiles = a.Tx * a.Ty;
  const long long all = (long long)a.V * tiles, before = (long long)k * tiles;
  long long base = 0, total = 0;
  for (long long i0 = tid; i0 < all; i0 += 4LL * kScanThreads) {
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long i = i0 + (long long)u * kScanThreads;
      v[u] = i < all ? a.counts[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      total += v[u];
      if (i0 + (long long)u * kScanThreads < before) base += v[u];
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    base += __shfl_down(base, off, 64);
    total += __shfl_down(total, off, 64);
  }
  // This thread's run of the view's tiles, scanned within the wave.
  const int per = (tiles + kScanThreads - 1) / kScanThreads;
  const int t0 = tid * per, t1 = min(tiles, t0 + per);
  uint32_t* c = a.counts + (size_t)k * tiles;
  long long local = 0;
  for (int t = t0; t < t1; ++t) local += c[t];
  long long incl = local;
  for (int off = 1; off < 64; off <<= 1) {
    const long long y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 0) {
    red[0][w] = base;
    red[1][w] = total;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  base = 0;
  total = 0;
  long long before_w = 0;
  for (int i = 0; i < kWaves; ++i) {
    base += red[0][i];
    total += red[1][i];
    if (i < w) before_w += wsum[i];
  }
  long long run = base + before_w + incl - local;
  uint32_t* r = a.ranges + 2 * (size_t)k * tiles;
  for (int t = t0; t < t1; ++t) {
    r[2 * t] = (uint32_t)run;
    run += c[t];
    r[2 * t + 1] = (uint32_t)run;
  }
  if (k == 0 && tid == 0) {
    a.ctr->n_keys = total;
    if (total > a.key_cap) atomicOr(&a.ctr->status, GS_STATUS_KEY_OVERFLOW);
  }
}

struct ScatterArgs {
  const float* depth;
  const int2* rbox;
  const int32_t* tiles;
  const int32_t* n_dev;
  int cap, tile, Tx, Ty;
  uint32_t* cursor;              // tile counts (the per-key-atomic scatter
                                 // counts them down)
  uint32_t* chunk_counts;        // [V][chunks][tiles]
  unsigned long long* keys;
  long long key_cap;
  int nch;                       // chunks per view (chunked scatter)
  const uint32_t* ranges;        // final ranges: the tiles' starts, and the
                                 // tile order
  uint32_t* order;
  int order_n;                   // tiles to order in the scatter (0: none)
};

// Per-wave key enumeration: lane l owns one Gaussian with cnt keys (the tiles
// of its render box, row-major); f(tile_in_view, g, depth_bits) runs once per key,
// 64 keys per step, each lane locating its key's owner by binary search over
// the wave's inclusive prefix of counts.
struct WaveOwners {
  int incl[64], x0[64], y0[64], w[64];
  uint32_t g[64], d[64];
};

// The binned tile box of (view k, Gaussian g) among the n live ones: its
// tile count (0 when g is not live or not binned), tile columns [tx0, tx1],
// rows [ty0, ty1] and depth bits.  The three loads are issued together from
// an index clamped into the arrays and the result selected afterwards, so a
// thread's owners cost one memory round trip, not a chain of two (tile count,
// then box and depth); tile is 8, 16 or 32, a shift.
struct OwnerBox {
  int cnt, tx0, tx1, ty0, ty1;
  uint32_t dbits;
};

__device__ inline OwnerBox load_box(const ScatterArgs& a, int n, int k, int g,
                                    int tsh) {
  const bool live = g < n;
  const size_t slot = (size_t)k * a.cap + (live ? g : 0);
  const int c = a.tiles[slot];
  const int2 rb = a.rbox[slot];
  const uint32_t d = __float_as_uint(a.depth[slot]);
  const bool any = live && c > 0;
  OwnerBox o;
  o.cnt = any ? c : 0;
  o.tx0 = any ? (rb.x & 0xffff) >> tsh : 0;
  o.tx1 = any ? (rb.x >> 16) >> tsh : 0;
  o.ty0 = any ? (rb.y & 0xffff) >> tsh : 0;
  o.ty1 = any ? (rb.y >> 16) >> tsh : 0;
  o.dbits = any ? d : 0u;
  return o;
}

__device__ inline void load_owner(const ScatterArgs& a, int n, int k, int g,
                                  int tsh, int& cnt, int& x0, int& y0, int& w,
                                  uint32_t& dbits) {
  const OwnerBox o = load_box(a, n, k, g, tsh);
  cnt = o.cnt; x0 = o.tx0; y0 = o.ty0; w = o.tx1 - o.tx0 + 1;
  dbits = o.dbits;
}

// Orders one wave's LDS accesses before and after this point.  The owner
// table below is private to a wave: its lanes only need to see each other's
// writes, not the other waves' (a block barrier would make the waves of a
// workgroup wait for the slowest one).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename F>
__device__ inline void wave_enumerate(WaveOwners& O, int lane, int cnt, int x0,
                                      int y0, int w, uint32_t g, uint32_t dbits,
                                      int Tx, F&& f) {
  int s = cnt;
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(s, off, 64);
    if (lane >= off) s += v;
  }
  O.incl[lane] = s; O.x0[lane] = x0; O.y0[lane] = y0; O.w[lane] = w;
  O.g[lane] = g; O.d[lane] = dbits;
  wave_sync();
  const int total = __shfl(s, 63, 64);
  for (int b = 0; b < total; b += 64) {
    const int j = b + lane;
    if (j < total) {
      int lo = 0, hi = 63;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (O.incl[mid] > j) hi = mid; else lo = mid + 1;
      }
      const int local = j - (lo ? O.incl[lo - 1] : 0);
      const int ww = O.w[lo];
      const int ty = O.y0[lo] + local / ww;
      const int tx = O.x0[lo] + local % ww;
      f(ty * Tx + tx, O.g[lo], O.d[lo]);
    }
  }
  wave_sync();   // the table is rewritten by the wave's next call
}

// Keys of one chunk (GPT Gaussians per thread, one view per block) per tile,
// to row [view][chunk] of the chunk-count matrix: each Gaussian adds the
// four corners of its box of tiles into an LDS coverage difference grid,
// whose 2D prefix sum (rows, then columns) is the count of every tile.
template <int MAXBINS, int GPT>
__global__ __launch_bounds__(256) void k_chunk_count(ScatterArgs a) {
  constexpr int kCells = MAXBINS + kGridSlack;
  __shared__ int grid[kCells];
  const int tid = threadIdx.x;
  const int k = blockIdx.y;
  const int nb = a.Tx * a.Ty;
  const int stride = a.Tx + 1, cells = stride * (a.Ty + 1);
  for (int i = tid; i < cells; i += 256) grid[i] = 0;
  __syncthreads();
  const int g0 = blockIdx.x * 256 * GPT;
  const int n = min(*a.n_dev, a.cap);
  const int tsh = __builtin_ctz(a.tile);
  // Every sub-chunk's loads first (their latencies overlap), then the adds.
  OwnerBox o[GPT];
#pragma unroll
  for (int sub = 0; sub < GPT; ++sub)
    o[sub] = load_box(a, n, k, g0 + sub * 256 + tid, tsh);
#pragma unroll
  for (int sub = 0; sub < GPT; ++sub) {
    if (o[sub].cnt <= 0) continue;
    const int tx0 = o[sub].tx0, tx1 = o[sub].tx1;
    const int ty0 = o[sub].ty0, ty1 = o[sub].ty1;
    atomicAdd(&grid[ty0 * stride + tx0], 1);
    atomicAdd(&grid[ty0 * stride + tx1 + 1], -1);
    atomicAdd(&grid[(ty1 + 1) * stride + tx0], -1);
    atomicAdd(&grid[(ty1 + 1) * stride + tx1 + 1], 1);
  }
  __syncthreads();
  for (int y = tid; y < a.Ty; y += 256) {
    int acc = 0;
    for (int x = 0; x < a.Tx; ++x) { acc += grid[y * stride + x]; grid[y * stride + x] = acc; }
  }
  __syncthreads();
  for (int x = tid; x < a.Tx; x += 256) {
    int acc = 0;
    for (int y = 0; y < a.Ty; ++y) { acc += grid[y * stride + x]; grid[y * stride + x] = acc; }
  }
  __syncthreads();
  uint32_t* C = a.chunk_counts + ((size_t)k * gridDim.x + blockIdx.x) * nb;
  for (int i = tid; i < nb; i += 256) {
    const int ty = i / a.Tx, tx = i - ty * a.Tx;
    C[i] = (uint32_t)grid[ty * stride + tx];
  }
}

struct ChunkScanArgs {
  uint32_t* chunk_counts;   // in: counts; out: offsets inside the tile
  uint32_t* counts;         // out: [V][tiles] tile totals
  int tiles, chunks;
};

// Column scan of the chunk-count matrix: 64 tiles per workgroup, the chunks
// split in 16 segments (one wave each), one view per grid row.
__global__ __launch_bounds__(1024) void k_chunk_scan(ChunkScanArgs a) {
  __shared__ uint32_t part[16][64];
  const int tl = threadIdx.x & 63, seg = threadIdx.x >> 6;
  const int k = blockIdx.y;
  const int t = blockIdx.x * 64 + tl;
  const int nb = a.tiles, nch = a.chunks;
  const int sl = (nch + 15) / 16;
  const int c0 = min(nch, seg * sl), c1 = min(nch, c0 + sl);
  uint32_t* C = a.chunk_counts + (size_t)k * nch * nb;
  // The first kReg counts of the segment stay in registers between the two
  // passes, so the offsets are stored without a load before each store.
  constexpr int kReg = 32;
  uint32_t v[kReg];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kReg; ++j) {
    const int c = c0 + j;
    v[j] = (t < nb && c < c1) ? C[(size_t)c * nb + t] : 0u;
    sum += v[j];
  }
  if (t < nb)
    for (int c = c0 + kReg; c < c1; ++c) sum += C[(size_t)c * nb + t];
  part[seg][tl] = sum;
  __syncthreads();
  uint32_t run = 0;
  for (int s2 = 0; s2 < seg; ++s2) run += part[s2][tl];
  if (t >= nb) return;
  if (seg == 15) a.counts[(size_t)k * nb + t] = run + sum;
#pragma unroll
  for (int j = 0; j < kReg; ++j) {
    const int c = c0 + j;
    if (c < c1) C[(size_t)c * nb + t] = run;
    run += v[j];
  }
  for (int c = c0 + kReg; c < c1; ++c) {
    const size_t i = (size_t)c * nb + t;
    const uint32_t x = C[i];
    C[i] = run;
    run += x;
  }
}

template <int NT>
__device__ void order_tiles(const uint32_t* ranges, uint32_t* order, int n,
                            uint32_t* cnt, uint32_t* wsum, uint32_t* mm);

// Workgroup i of a launch goes to XCD i mod 8.  This renumbering of n
// workgroups gives every XCD a contiguous run of logical ids (a bijection on
// [0, n)), so neighbouring logical workgroups share an L2.
__device__ __forceinline__ int xcd_contiguous(int i, int n) {
  const int q = n >> 3, r = n & 7, x = i & 7, j = i >> 3;
  return x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

// The scatter: the chunk's keys claim positions start + offset + (LDS
// counter) in their tiles' segments.  Logical grid (1 + chunks) x views,
// numbered so that consecutive chunks run on one XCD: their keys fill
// neighbouring slots of every tile's segment (a few keys per chunk and
// tile), so the partial-line writes combine in that XCD's L2.  Workgroup
// (0, 0) orders the tiles by list length meanwhile (the ranges are final);
// the other workgroups of column 0 have nothing to do.
template <int MAXBINS, int GPT>
__global__ __launch_bounds__(256) void k_scatter_chunks(ScatterArgs a) {
  static_assert(MAXBINS >= 1024, "the tile order counts in the bins");
  __shared__ uint32_t bins[MAXBINS];
  __shared__ WaveOwners owners[4];
  const int lid = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
  const int bx = lid % (1 + a.nch), k = lid / (1 + a.nch);
  if (bx == 0) {
    if (k == 0 && a.order_n > 0)
      order_tiles<256>(a.ranges, a.order, a.order_n, bins,
                       (uint32_t*)owners[0].incl, (uint32_t*)owners[0].x0);
    return;
  }
  const int chunk = bx - 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nb = a.Tx * a.Ty;
  const uint32_t* C = a.chunk_counts + ((size_t)k * a.nch + chunk) * nb;
  const uint32_t* range = a.ranges + 2 * (size_t)k * nb;   // [start, end)
  const int g0 = chunk * 256 * GPT;
  const int n = min(*a.n_dev, a.cap);
  const int tsh = __builtin_ctz(a.tile);
  // The owners of all GPT sub-chunks are loaded up front, so their latencies
  // overlap each other and the bins' set-up.
  int cnt[GPT], x0[GPT], y0[GPT], w[GPT];
  uint32_t d[GPT];
#pragma unroll
  for (int sub = 0; sub < GPT; ++sub)
    load_owner(a, n, k, g0 + sub * 256 + tid, tsh, cnt[sub], x0[sub], y0[sub],
               w[sub], d[sub]);
  // The bins in groups of four per thread, each group's loads issued before
  // the first is used (clamped indices keep them in bounds).
  for (int i0 = tid; i0 < nb; i0 += 4 * 256) {
    uint32_t sv[4], cv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = min(i0 + u * 256, nb - 1);
      sv[u] = range[2 * i];
      cv[u] = C[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u * 256 < nb) bins[i0 + u * 256] = sv[u] + cv[u];
  }
  __syncthreads();
#pragma unroll
  for (int sub = 0; sub < GPT; ++sub) {
    const int g = g0 + sub * 256 + tid;
    wave_enumerate(owners[wv], lane, cnt[sub], x0[sub], y0[sub], w[sub],
                   (uint32_t)g, d[sub], a.Tx,
                   [&](int t, uint32_t gg, uint32_t dd) {
                     const uint32_t pos = atomicAdd(&bins[t], 1u);
                     if ((long long)pos < a.key_cap)
                       a.keys[pos] = ((unsigned long long)dd << 32) | gg;
                   });
  }
}

// Fallback for tile grids larger than the LDS bins: one global atomic per key.
__global__ __launch_bounds__(256) void k_scatter_global(ScatterArgs a) {
  __shared__ WaveOwners owners[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int k = blockIdx.y;
  const int g = blockIdx.x * 256 + tid;
  int cnt, x0, y0, w;
  uint32_t d;
  load_owner(a, min(*a.n_dev, a.cap), k, g, __builtin_ctz(a.tile), cnt, x0, y0,
             w, d);
  // Each tile's count, taken down by one per key, numbers its keys within
  // the tile's range.
  uint32_t* cur = a.cursor + (size_t)k * a.Tx * a.Ty;
  const uint32_t* range = a.ranges + 2 * (size_t)k * a.Tx * a.Ty;
  wave_enumerate(owners[wv], lane, cnt, x0, y0, w, (uint32_t)g, d, a.Tx,
                 [&](int t, uint32_t gg, uint32_t dd) {
                   const uint32_t pos =
                       range[2 * t] + atomicSub(&cur[t], 1u) - 1u;
                   if ((long long)pos < a.key_cap)
                     a.keys[pos] = ((unsigned long long)dd << 32) | gg;
                 });
}

// LDS per chunk-scatter workgroup, static and padding: three workgroups per
// CU (160 KB).  Each XCD then has about 96 chunks in flight, whose key runs
// share each tile's segment: the partly written lines of that frontier stay
// in the XCD's 4 MB L2 until they fill and leave as whole lines.  With the
// eight workgroups per CU that the registers allow, the frontier of about
// 256 chunks outgrows the L2 and partial lines are written back (the
// scatter of the 10-view 1200x680 window: 0.178 -> 0.166 ms for projection
// and binning; two workgroups per CU, 0.186 ms, hide too little latency).
constexpr size_t kScatterLds = 48 * 1024;

constexpr int kOrderBuckets = 1024;
constexpr int kOrderMaxTiles = 1 << 18;   // larger grids keep index order

__global__ void k_iota(uint32_t* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = (uint32_t)i;
}

template <int NT>
__device__ void order_tiles(const uint32_t* ranges, uint32_t* order, int n,
                            uint32_t* cnt, uint32_t* wsum, uint32_t* mm) {
  constexpr int PER = kOrderBuckets / NT;   // buckets per thread in the scan
  static_assert(PER * NT == kOrderBuckets && NT % 64 == 0, "order layout");
  const int tid = threadIdx.x;
  for (int b = tid; b < kOrderBuckets; b += NT) cnt[b] = 0;
  if (tid == 0) { mm[0] = 0xffffffffu; mm[1] = 0; }
  __syncthreads();
  // The buckets span [shortest, longest], so few tiles share a bucket (and
  // its LDS counter).
  uint32_t mn = 0xffffffffu, mx = 0;
  for (int t = tid; t < n; t += NT) {
    const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
    mn = min(mn, len);
    mx = max(mx, len);
  }
  for (int off = 32; off > 0; off >>= 1) {
    mn = min(mn, (uint32_t)__shfl_down((int)mn, off, 64));
    mx = max(mx, (uint32_t)__shfl_down((int)mx, off, 64));
  }
  if ((tid & 63) == 0) { atomicMin(&mm[0], mn); atomicMax(&mm[1], mx); }
  __syncthreads();
  const uint32_t base = mm[0], width = (mm[1] - mm[0]) / kOrderBuckets + 1;
  for (int t = tid; t < n; t += NT) {
    const uint32_t b = (ranges[2 * t + 1] - ranges[2 * t] - base) / width;
    atomicAdd(&cnt[kOrderBuckets - 1 - b], 1u);
  }
  __syncthreads();
  // Exclusive scan of the bucket counts (longest bucket first): each thread
  // owns PER consecutive buckets.
  const int lane = tid & 63, w = tid >> 6;
  uint32_t c[PER], own = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    c[q] = cnt[tid * PER + q];
    own += c[q];
  }
  uint32_t x = own;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t run = x - own;
  for (int i = 0; i < w; ++i) run += wsum[i];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    cnt[tid * PER + q] = run;
    run += c[q];
  }
  __syncthreads();
  for (int t = tid; t < n; t += NT) {
    const uint32_t b = (ranges[2 * t + 1] - ranges[2 * t] - base) / width;
    order[atomicAdd(&cnt[kOrderBuckets - 1 - b], 1u)] = (uint32_t)t;
  }
}

// Tiles by descending key count (a counting sort over 1024 length buckets)
// for the per-tile kernels, whose block b takes tile order[b]: the dispatcher
// hands out the long lists first and the short ones fill the tail.  One
// workgroup; the order within a bucket is unspecified (the tiles are
// independent).  The chunked scatter forms the same order in its first
// workgroup instead.
__global__ __launch_bounds__(1024) void k_tile_order(const uint32_t* ranges,
                                                     uint32_t* order, int n) {
  __shared__ uint32_t cnt[kOrderBuckets];
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t mm[2];
  order_tiles<1024>(ranges, order, n, cnt, wsum, mm);
}

hipError_t launch_order(const gs_workspace* ws, hipStream_t st) {
  const int n = ws->geo.n_views * ws->tiles_x * ws->tiles_y;
  if (n <= 0 || n > kOrderMaxTiles) return hipSuccess;   // index order kept
  hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, st, ws->ranges,
                     ws->tile_order, n);
  return hipGetLastError();
}

template <int MAXBINS, int GPT>
hipError_t launch_chunked(const ScatterArgs& c, const RangeArgs& ra,
                          uint32_t* counts, int V, hipStream_t st) {
  const int nch = (c.cap + 256 * GPT - 1) / (256 * GPT);
  const int nb = c.Tx * c.Ty;
  hipLaunchKernelGGL((k_chunk_count<MAXBINS, GPT>), dim3(nch, V), dim3(256), 0,
                     st, c);
  ChunkScanArgs sa;
  sa.chunk_counts = c.chunk_counts; sa.counts = counts;
  sa.tiles = nb; sa.chunks = nch;
  hipLaunchKernelGGL(k_chunk_scan, dim3((nb + 63) / 64, V), dim3(1024), 0, st,
                     sa);
  hipLaunchKernelGGL(k_tile_ranges, dim3(V), dim3(kScanThreads), 0, st, ra);
  ScatterArgs cs = c;
  cs.nch = nch;
  const int n = V * nb;
  cs.order_n = n <= kOrderMaxTiles ? n : 0;   // larger grids keep index order
  // Padding LDS (unused) holds the scatter at three workgroups per CU.
  constexpr size_t kStatic = MAXBINS * sizeof(uint32_t) + 4 * sizeof(WaveOwners);
  const size_t pad = kStatic < kScatterLds ? kScatterLds - kStatic : 0;
  hipLaunchKernelGGL((k_scatter_chunks<MAXBINS, GPT>), dim3((1 + nch) * V),
                     dim3(256), pad, st, cs);
  return hipGetLastError();
}

// Ranges are final: order the tiles for the per-tile kernels.
hipError_t finish_bin(const gs_workspace* ws, hipError_t e, hipStream_t st) {
  if (e != hipSuccess) return e;
  return launch_order(ws, st);
}

}  // namespace

hipError_t launch_bin(gs_workspace* ws, const gs_params* p, hipStream_t st) {
  const int V = ws->geo.n_views;
  const int nb = ws->tiles_x * ws->tiles_y;
  RangeArgs ra;
  ra.counts = ws->cursor; ra.ranges = ws->ranges;
  ra.ctr = ws->counters; ra.V = V; ra.Tx = ws->tiles_x; ra.Ty = ws->tiles_y;
  ra.key_cap = ws->geo.key_capacity;
  ScatterArgs c;
  c.depth = ws->depth; c.rbox = ws->rbox; c.tiles = ws->tiles_touched;
  c.n_dev = p->n_dev;
  c.cap = p->capacity; c.tile = ws->geo.tile; c.Tx = ws->tiles_x;
  c.Ty = ws->tiles_y; c.cursor = ws->cursor; c.chunk_counts = ws->chunk_counts;
  c.keys = ws->keys_unsorted;
  c.key_cap = ws->geo.key_capacity;
  c.nch = 0; c.ranges = nullptr; c.order = nullptr; c.order_n = 0;
  const int ch = bin_chunk(ws->tiles_x, ws->tiles_y);
  const int cells = (ws->tiles_x + 1) * (ws->tiles_y + 1);
  if (ch && p->capacity <= 0) {
    // No Gaussians: every range is empty.
    hipError_t e = launch_fill_u32(ws->cursor, 0u, (size_t)V * nb, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_ranges, dim3(V), dim3(kScanThreads), 0, st, ra);
    return finish_bin(ws, hipGetLastError(), st);
  }
  // The chunked scatter also orders the tiles.
  c.ranges = ws->ranges; c.order = ws->tile_order;
  if (ch == 1024)
    return launch_chunked<1024, 4>(c, ra, ws->cursor, V, st);
  if (ch == 2048 && nb <= 4096 && cells <= 4096 + kGridSlack)
    return launch_chunked<4096, 8>(c, ra, ws->cursor, V, st);
  if (ch == 2048)
    return launch_chunked<16384, 8>(c, ra, ws->cursor, V, st);
  CountArgs ca;
  ca.diff = ws->diff; ca.counts = ws->cursor;
  ca.Tx = ws->tiles_x; ca.Ty = ws->tiles_y;
  hipLaunchKernelGGL(k_tile_count, dim3(V), dim3(kScanThreads), 0, st, ca);
  hipLaunchKernelGGL(k_tile_ranges, dim3(V), dim3(kScanThreads), 0, st, ra);
  if (p->capacity > 0)
    hipLaunchKernelGGL(k_scatter_global, dim3((c.cap + 255) / 256, V),
                       dim3(256), 0, st, c);
  return finish_bin(ws, hipGetLastError(), st);
}

hipError_t launch_iota_u32(uint32_t* ptr, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)blocks), dim3(256), 0, st, ptr,
                     count);
  return hipGetLastError();
}

}  // namespace gs
