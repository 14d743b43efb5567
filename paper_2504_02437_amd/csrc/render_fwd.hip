// Forward compositing (Eq. 3) over screen tiles.
//
// One workgroup per (view, tile).  Threads own pixels (one per thread for
// 8x8 and 16x16 tiles, four per thread for 32x32).  The tile's sorted list is
// walked front to back in batches: the workgroup stages a batch of records
// into LDS (one coalesced gather per thread), then every thread blends its
// pixels against the batch, reading each entry by an LDS broadcast.  A pixel
// stops before the entry that would take its transmittance below T_min; a
// wave leaves the batch once all its pixels stopped, and the workgroup stops
// fetching batches once every pixel has.

#include "raster_common.h"

namespace gs {
namespace {

struct FwdArgs {
  RasterArgs r;
  float* rgb;
  float* T;
  int32_t* nlast;
  unsigned long long* counts;  // counting variant only
};

// COUNT = true is the work-counting variant: the same walk and decisions,
// adding up examined / in-box / contributing / revisited pairs instead of
// writing the image.
template <int TILE, int BATCH, bool COUNT>
__global__ __launch_bounds__(TILE * TILE > 256 ? 256 : TILE * TILE) void
k_render_fwd(FwdArgs a) {
  constexpr int NT = TILE * TILE > 256 ? 256 : TILE * TILE;
  constexpr int PPT = TILE * TILE / NT;
  __shared__ Entry ent[BATCH];
  const RasterArgs& r = a.r;
  const int t = blockIdx.x;
  const int tpv = r.Tx * r.Ty;
  const int k = t / tpv;
  const int rem = t - k * tpv;
  const int ty = rem / r.Tx, tx = rem - ty * r.Tx;
  const int tid = threadIdx.x;
  long long s, e;
  tile_range(r, t, s, e);

  int u[PPT], v[PPT], last[PPT];
  float T[PPT], C0[PPT], C1[PPT], C2[PPT];
  bool done[PPT];
  unsigned n_exam = 0, n_inbox = 0, n_contrib = 0;
  unsigned ib[PPT], ib_last[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int l = tid + p * NT;
    u[p] = tx * TILE + (l % TILE);
    v[p] = ty * TILE + (l / TILE);
    done[p] = !(u[p] < r.W && v[p] < r.H);
    T[p] = 1.f;
    C0[p] = C1[p] = C2[p] = 0.f;
    last[p] = 0;
    ib[p] = ib_last[p] = 0;
  }
  const Record* rv = r.rec + (size_t)k * r.cap;
  for (long long b0 = s; b0 < e; b0 += BATCH) {
    int alive = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) alive |= !done[p];
    if (__syncthreads_or(alive) == 0) break;
    const int cnt = (int)min((long long)BATCH, e - b0);
    for (int i = tid; i < cnt; i += NT) stage(ent[i], rv[r.vals[b0 + i]]);
    __syncthreads();
    const int base = (int)(b0 - s);
    for (int j = 0; j < cnt; ++j) {
      bool any = false;
#pragma unroll
      for (int p = 0; p < PPT; ++p) any |= !done[p];
      if (!__any(any)) break;
      const Entry& E = ent[j];
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        if (COUNT && !done[p]) ++n_exam;
        if (done[p] || !in_box(E.box, u[p], v[p])) continue;
        if (COUNT) { ++n_inbox; ++ib[p]; }
        float dx, dy, G, e2, oG;
        const float al = eval_alpha(E, (float)u[p], (float)v[p], r.alpha_max,
                                    dx, dy, G, e2, oG);
        if (e2 > 0.f || al < r.alpha_min) continue;
        const float Tn = T[p] * (1.f - al);
        if (Tn < r.T_min) {
          done[p] = true;
          continue;
        }
        const float w = al * T[p];
        C0[p] = fmaf(E.b.z, w, C0[p]);
        C1[p] = fmaf(E.b.w, w, C1[p]);
        C2[p] = fmaf(E.c.x, w, C2[p]);
        T[p] = Tn;
        last[p] = base + j + 1;
        if (COUNT) { ++n_contrib; ib_last[p] = ib[p]; }
      }
    }
  }
  if (COUNT) {
    unsigned long long c[4] = {n_exam, n_inbox, n_contrib, 0};
#pragma unroll
    for (int p = 0; p < PPT; ++p) c[3] += ib_last[p];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      unsigned long long x = c[q];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if ((tid & 63) == 0 && x) atomicAdd(&a.counts[q], x);
    }
    return;
  }
  const size_t HW = (size_t)r.H * r.W;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    if (!(u[p] < r.W && v[p] < r.H)) continue;
    const size_t pix = (size_t)v[p] * r.W + u[p];
    a.rgb[((size_t)k * 3 + 0) * HW + pix] = fmaf(T[p], r.bg0, C0[p]);
    a.rgb[((size_t)k * 3 + 1) * HW + pix] = fmaf(T[p], r.bg1, C1[p]);
    a.rgb[((size_t)k * 3 + 2) * HW + pix] = fmaf(T[p], r.bg2, C2[p]);
    a.T[(size_t)k * HW + pix] = T[p];
    a.nlast[(size_t)k * HW + pix] = last[p];
  }
}

template <int TILE, int BATCH, bool COUNT>
void launch_t(const FwdArgs& a, int blocks, hipStream_t st) {
  constexpr int NT = TILE * TILE > 256 ? 256 : TILE * TILE;
  hipLaunchKernelGGL((k_render_fwd<TILE, BATCH, COUNT>), dim3(blocks), dim3(NT),
                     0, st, a);
}

template <int TILE, bool COUNT>
void launch_b(const FwdArgs& a, int batch, int blocks, hipStream_t st) {
  if (batch == 128) launch_t<TILE, 128, COUNT>(a, blocks, st);
  else if (batch == 256) launch_t<TILE, 256, COUNT>(a, blocks, st);
  else launch_t<TILE, 512, COUNT>(a, blocks, st);
}

template <bool COUNT>
void launch_tile(const FwdArgs& a, int tile, int batch, int blocks,
                 hipStream_t st) {
  switch (tile) {
    case 8: launch_b<8, COUNT>(a, batch, blocks, st); break;
    case 16: launch_b<16, COUNT>(a, batch, blocks, st); break;
    default: launch_b<32, COUNT>(a, batch, blocks, st); break;
  }
}

}  // namespace

RasterArgs make_raster_args(gs_workspace* ws, const gs_settings* s) {
  RasterArgs r;
  r.rec = ws->records; r.vals = ws->vals_sorted; r.ranges = ws->ranges;
  r.key_cap = ws->geo.key_capacity; r.cap = ws->geo.capacity;
  r.V = ws->geo.n_views; r.W = ws->geo.width; r.H = ws->geo.height;
  r.Tx = ws->tiles_x; r.Ty = ws->tiles_y;
  r.bg0 = s->bg[0]; r.bg1 = s->bg[1]; r.bg2 = s->bg[2];
  r.alpha_min = s->alpha_min; r.T_min = s->T_min; r.alpha_max = s->alpha_max;
  return r;
}

hipError_t launch_render_fwd(gs_workspace* ws, const gs_settings* s,
                             float* rgb, float* T, int32_t* nlast,
                             hipStream_t st) {
  FwdArgs a;
  a.r = make_raster_args(ws, s);
  a.rgb = rgb; a.T = T; a.nlast = nlast; a.counts = nullptr;
  const int blocks = ws->geo.n_views * ws->tiles_x * ws->tiles_y;
  if (blocks <= 0) return hipSuccess;
  launch_tile<false>(a, ws->geo.tile, s->lds_batch, blocks, st);
  return hipGetLastError();
}

hipError_t launch_count_pairs(gs_workspace* ws, const gs_settings* s,
                              unsigned long long* counts, hipStream_t st) {
  FwdArgs a;
  a.r = make_raster_args(ws, s);
  a.rgb = nullptr; a.T = nullptr; a.nlast = nullptr; a.counts = counts;
  const int blocks = ws->geo.n_views * ws->tiles_x * ws->tiles_y;
  if (blocks <= 0) return hipSuccess;
  launch_tile<true>(a, ws->geo.tile, s->lds_batch, blocks, st);
  return hipGetLastError();
}

}  // namespace gs
