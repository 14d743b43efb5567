// Tile binning: per-tile key counts, ranges, and the scatter of Gaussian
// indices into their tiles' segments.
//
// Counts come from the tile-coverage difference grid the projection kernel
// fills (four corner increments per box of tiles); a 2D prefix sum turns it
// into the number of boxes covering each tile.  One exclusive scan over all
// (view, tile) cells then gives every tile's [start, end) range in the key
// buffer, so n_keys never leaves the device.  The scatter walks each box of
// tiles with wave-level load balancing (one lane per emitted key) and claims
// slots with one atomic per key; sort_tile_keys makes the order inside each
// segment deterministic.

#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kScanThreads = 1024;

struct ScanArgs {
  int32_t* diff;  // [V][Ty + 1][Tx + 1], consumed and cleared
  uint32_t* ranges;
  uint32_t* cursor;
  Counters* ctr;
  int V, Tx, Ty;
  long long key_cap;
};

__global__ __launch_bounds__(kScanThreads) void k_tile_scan(ScanArgs a) {
  const int tid = threadIdx.x;
  const int stride = a.Tx + 1;
  const int rows = a.Ty + 1;
  // 1. Prefix along x of every row of every view.
  for (int r = tid; r < a.V * rows; r += kScanThreads) {
    int32_t* row = a.diff + (size_t)r * stride;
    int acc = 0;
    for (int x = 0; x < stride; ++x) {
      acc += row[x];
      row[x] = acc;
    }
  }
  __syncthreads();
  // 2. Prefix along y of every column of every view.
  for (int c = tid; c < a.V * stride; c += kScanThreads) {
    const int k = c / stride, x = c % stride;
    int32_t* col = a.diff + (size_t)k * rows * stride + x;
    int acc = 0;
    for (int y = 0; y < rows; ++y) {
      acc += col[(size_t)y * stride];
      col[(size_t)y * stride] = acc;
    }
  }
  __syncthreads();
  // 3. Exclusive scan of the counts over (view, ty, tx), chunked per thread.
  const long long total_tiles = (long long)a.V * a.Ty * a.Tx;
  const long long per = (total_tiles + kScanThreads - 1) / kScanThreads;
  const long long t0 = tid * per;
  const long long t1 = min(total_tiles, t0 + per);
  auto count_of = [&](long long t) -> long long {
    const int k = (int)(t / ((long long)a.Tx * a.Ty));
    const int rem = (int)(t % ((long long)a.Tx * a.Ty));
    const int ty = rem / a.Tx, tx = rem % a.Tx;
    return a.diff[((size_t)k * rows + ty) * stride + tx];
  };
  long long local = 0;
  for (long long t = t0; t < t1; ++t) local += count_of(t);
  __shared__ long long part[kScanThreads];
  part[tid] = local;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    long long v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  long long run = part[tid] - local;
  for (long long t = t0; t < t1; ++t) {
    const long long c = count_of(t);
    a.ranges[2 * t] = (uint32_t)run;
    a.cursor[t] = (uint32_t)run;
    run += c;
    a.ranges[2 * t + 1] = (uint32_t)run;
  }
  if (tid == kScanThreads - 1) {
    a.ctr->n_keys = part[tid];
    if (part[tid] > a.key_cap) atomicOr(&a.ctr->status, GS_STATUS_KEY_OVERFLOW);
  }
  __syncthreads();
  // 4. Clear the difference grid for the next call.
  const size_t cells = (size_t)a.V * rows * stride;
  for (size_t i = tid; i < cells; i += kScanThreads) a.diff[i] = 0;
}

struct ScatterArgs {
  const Record* rec;
  const int32_t* tiles;
  const int32_t* n_dev;
  int cap, tile, Tx, Ty;
  uint32_t* cursor;
  uint32_t* vals;
  long long key_cap;
};

// One thread per (view, Gaussian); the keys of a wave's 64 Gaussians are
// emitted 64 at a time, each lane locating its owner by binary search over
// the wave's inclusive prefix of key counts.
__global__ __launch_bounds__(256) void k_scatter(ScatterArgs a) {
  __shared__ int incl[4][64];
  __shared__ int own_x0[4][64], own_y0[4][64], own_w[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.y;
  const int g = blockIdx.x * 256 + threadIdx.x;
  const int n = min(*a.n_dev, a.cap);
  int cnt = 0, x0 = 0, y0 = 0, w = 1;
  if (g < n) {
    const size_t slot = (size_t)k * a.cap + g;
    cnt = a.tiles[slot];
    if (cnt > 0) {
      const float4 q2 = a.rec[slot].q2;
      const int bu = __float_as_int(q2.z), bv = __float_as_int(q2.w);
      x0 = (bu & 0xffff) / a.tile;
      const int x1 = (bu >> 16) / a.tile;
      y0 = (bv & 0xffff) / a.tile;
      w = x1 - x0 + 1;
    }
  }
  // Inclusive prefix of counts across the wave.
  int s = cnt;
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(s, off, 64);
    if (lane >= off) s += v;
  }
  incl[wv][lane] = s;
  own_x0[wv][lane] = x0;
  own_y0[wv][lane] = y0;
  own_w[wv][lane] = w;
  __syncthreads();
  const int total = __shfl(s, 63, 64);
  const uint32_t tile_base = (uint32_t)k * a.Tx * a.Ty;
  for (int base = 0; base < total; base += 64) {
    const int j = base + lane;
    if (j < total) {
      // First owner o with incl[o] > j.
      int lo = 0, hi = 63;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (incl[wv][mid] > j) hi = mid; else lo = mid + 1;
      }
      const int o = lo;
      const int local = j - (o ? incl[wv][o - 1] : 0);
      const int ww = own_w[wv][o];
      const int ty = own_y0[wv][o] + local / ww;
      const int tx = own_x0[wv][o] + local % ww;
      const uint32_t t = tile_base + (uint32_t)(ty * a.Tx + tx);
      const uint32_t pos = atomicAdd(&a.cursor[t], 1u);
      if ((long long)pos < a.key_cap)
        a.vals[pos] = (uint32_t)(blockIdx.x * 256 + wv * 64 + o);
    }
  }
}

}  // namespace

hipError_t launch_bin(gs_workspace* ws, const gs_params* p, hipStream_t st) {
  ScanArgs s;
  s.diff = ws->diff; s.ranges = ws->ranges; s.cursor = ws->cursor;
  s.ctr = ws->counters; s.V = ws->geo.n_views; s.Tx = ws->tiles_x;
  s.Ty = ws->tiles_y; s.key_cap = ws->geo.key_capacity;
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kScanThreads), 0, st, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  ScatterArgs c;
  c.rec = ws->records; c.tiles = ws->tiles_touched; c.n_dev = p->n_dev;
  c.cap = p->capacity; c.tile = ws->geo.tile; c.Tx = ws->tiles_x;
  c.Ty = ws->tiles_y; c.cursor = ws->cursor; c.vals = ws->vals_unsorted;
  c.key_cap = ws->geo.key_capacity;
  const int bx = (p->capacity + 255) / 256;
  if (bx > 0)
    hipLaunchKernelGGL(k_scatter, dim3(bx, ws->geo.n_views), dim3(256), 0, st,
                       c);
  return hipGetLastError();
}

}  // namespace gs
