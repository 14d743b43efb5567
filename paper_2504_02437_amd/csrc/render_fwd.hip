// Forward compositing (Eq. 3) over screen tiles.
//
// One workgroup per (view, tile); each thread owns a vertical strip of the
// tile's pixels (see raster_common.h).  The tile's sorted list is walked
// front to back in batches: the workgroup stages a batch of records into LDS
// (one gather per entry), then every thread blends its pixels against the
// batch, reading each entry by an LDS broadcast.  A pixel stops before the
// entry that would take its transmittance below T_min; a wave leaves the
// batch once all its pixels stopped, and the workgroup stops fetching
// batches once every pixel has.

#include "raster_common.h"

namespace gs {
namespace {

struct FwdArgs {
  RasterArgs r;
  float* rgb;
  float* T;
  int32_t* nlast;
  int32_t* dom;                // dominant variant only
  unsigned long long* counts;  // counting variant only
};

// MODE kRender writes the image; kCount is the work-counting variant: the
// same walk and decisions, adding up examined / in-box / contributing /
// revisited pairs instead of writing the image; kDominant also writes each
// pixel's dominant Gaussian (Eq. 8): the one with the largest blend weight
// alpha T, the first one on exact ties, -1 when nothing contributes.
//
// A pixel's transmittance is kept with its sign as the liveness flag: a
// pixel that stopped holds -T, so "still compositing" is one compare and the
// output is |T|.  T >= T_min > 0 holds for every accepted step, so a live
// pixel's T is never zero, and a stopped pixel needs no test of its own: its
// candidate T (1 - alpha) is negative, below T_min, so it never contributes,
// and stopping it again (T = -|T|) leaves it as it is.  The per-pixel work is
// predicated rather than branched: every lane evaluates alpha for each of
// its pixels and the decisions select what is accumulated.  A wave skips an
// entry outright when no pixel of its footprint can admit it (wave_mask).
// The candidate transmittance is formed as fma(-alpha, T, T), one rounding.
enum { kRender = 0, kCount = 1, kDominant = 2 };

template <int TILE, int BATCH, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_render_fwd(FwdArgs a) {
  constexpr bool COUNT = MODE == kCount;
  constexpr bool DOM = MODE == kDominant;
  using Lay = PixLayout<TILE, NT>;
  constexpr int PPT = Lay::PPT;
  __shared__ Entry ent[BATCH];
  const RasterArgs& r = a.r;
  const int t = (int)r.order[blockIdx.x];
  const int tpv = r.Tx * r.Ty;
  const int k = t / tpv;
  const int rem = t - k * tpv;
  const int ty = rem / r.Tx, tx = rem - ty * r.Tx;
  const int tid = threadIdx.x;
  long long s, e;
  tile_range(r, t, s, e);

  int cu, cv0;
  Lay::of(tid, cu, cv0);
  const int u = tx * TILE + cu;
  const int v0 = ty * TILE + cv0;
  const int wave = tid >> 6;
  __shared__ int wmask[BATCH];   // per staged entry: waves that evaluate it
  __shared__ uint32_t egid[DOM ? BATCH : 1];   // Gaussian index per entry
  const float uf = (float)u;
  const float amax = __builtin_canonicalizef(r.alpha_max);
  const float amin = r.alpha_min, tmin = r.T_min;
  int last[PPT];
  float T[PPT], C0[PPT], C1[PPT], C2[PPT], vf[PPT];
  unsigned n_exam = 0, n_inbox = 0, n_contrib = 0;
  unsigned ib[PPT], ib_last[PPT];
  float wbest[PPT];
  int32_t best[PPT];
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    wbest[p] = 0.f;
    best[p] = -1;
    T[p] = (u < r.W && v0 + p < r.H) ? 1.f : -1.f;
    C0[p] = C1[p] = C2[p] = 0.f;
    last[p] = 0;
    vf[p] = pinned((float)(v0 + p));
    ib[p] = ib_last[p] = 0;
  }
  const Record* rv = r.rec + (size_t)k * r.cap;
  const int2* rbv = r.rbox + (size_t)k * r.cap;
  for (long long b0 = s; b0 < e; b0 += BATCH) {
    int alive = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) alive |= T[p] > 0.f;
    if (__syncthreads_or(alive) == 0) break;
    const int cnt = (int)min((long long)BATCH, e - b0);
    for (int i = tid; i < cnt; i += NT) {
      const uint32_t g = r.vals[b0 + i];
      const Record R = rv[g];
      const int4 box = unpack_box(rbv[g]);
      stage(ent[i], R, box);
      wmask[i] = wave_mask<TILE, NT>(R, box, tx * TILE, ty * TILE, amin,
                                     r.ellipse_test);
      if (DOM) egid[i] = g;
    }
    __syncthreads();
    const int base = (int)(b0 - s) + 1;
    for (int j = 0; j < cnt; ++j) {
      if ((j & 7) == 0) {
        bool any = false;
#pragma unroll
        for (int p = 0; p < PPT; ++p) any |= T[p] > 0.f;
        if (!__any(any)) break;
      }
      const int4 box = ent[j].box;
      const bool evaluate = (wmask[j] >> wave) & 1;
      if (COUNT) {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
          if (!(T[p] > 0.f)) continue;
          ++n_exam;
          if (evaluate && u >= box.x && u <= box.y && v0 + p >= box.z &&
              v0 + p <= box.w) {
            ++n_inbox;
            ++ib[p];
          }
        }
      }
      if (!evaluate) continue;
      const float4 ea = ent[j].a;
      const float4 eb = ent[j].b;
      const float ecb = ent[j].c.x;
      const bool in_u = u >= box.x && u <= box.y;
      const int lo = box.z - v0, hi = box.w - v0;
      const Column col = column(ea, uf);
      const int idx = base + j;
      const int32_t gj = DOM ? (int32_t)egid[j] : 0;
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        float dy;
        const float e2 = exponent2(col, ea.y, eb.x, vf[p], dy);
        const float G = __builtin_amdgcn_exp2f(e2);
        const float al = fminf(amax, eb.y * G);
        const bool ok = in_u && lo <= p && p <= hi && !(e2 > 0.f) &&
                        al >= amin;
        const float Tn = fmaf(-al, T[p], T[p]);
        const bool con = ok && Tn >= tmin;
        const float w = con ? al * T[p] : 0.f;
        C0[p] = fmaf(eb.z, w, C0[p]);
        C1[p] = fmaf(eb.w, w, C1[p]);
        C2[p] = fmaf(ecb, w, C2[p]);
        T[p] = con ? Tn : (ok ? -fabsf(T[p]) : T[p]);
        last[p] = con ? idx : last[p];
        if (DOM) {
          const bool better = con && w > wbest[p];
          wbest[p] = better ? w : wbest[p];
          best[p] = better ? gj : best[p];
        }
        if (COUNT) {
          n_contrib += con;
          ib_last[p] = con ? ib[p] : ib_last[p];
        }
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
    const int v = v0 + p;
    if (!(u < r.W && v < r.H)) continue;
    const float Tf = fabsf(T[p]);
    const size_t pix = (size_t)v * r.W + u;
    a.rgb[((size_t)k * 3 + 0) * HW + pix] = fmaf(Tf, r.bg0, C0[p]);
    a.rgb[((size_t)k * 3 + 1) * HW + pix] = fmaf(Tf, r.bg1, C1[p]);
    a.rgb[((size_t)k * 3 + 2) * HW + pix] = fmaf(Tf, r.bg2, C2[p]);
    a.T[(size_t)k * HW + pix] = Tf;
    a.nlast[(size_t)k * HW + pix] = last[p];
    if (DOM) a.dom[(size_t)k * HW + pix] = best[p];
  }
}

template <int MODE>
struct FwdLauncher {
  const FwdArgs& a;
  int blocks;
  hipStream_t st;
  template <int T, int B, int N>
  void go() const {
    hipLaunchKernelGGL((k_render_fwd<T, B, N, MODE>), dim3(blocks), dim3(N),
                       0, st, a);
  }
};

}  // namespace

RasterArgs make_raster_args(gs_workspace* ws, const gs_settings* s) {
  RasterArgs r;
  r.rec = ws->records; r.rbox = ws->rbox;
  r.ellipse_test = (s->flags & GS_FLAG_FULL_BOX) ? 0 : 1;
  r.vals = ws->vals_sorted; r.ranges = ws->ranges; r.order = ws->tile_order;
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
  a.rgb = rgb; a.T = T; a.nlast = nlast; a.dom = nullptr; a.counts = nullptr;
  const int blocks = ws->geo.n_views * ws->tiles_x * ws->tiles_y;
  if (blocks <= 0) return hipSuccess;
  dispatch_shape(ws->geo.tile, s->lds_batch, s->block_threads,
                 FwdLauncher<kRender>{a, blocks, st});
  return hipGetLastError();
}

hipError_t launch_render_dominant(gs_workspace* ws, const gs_settings* s,
                                  float* rgb, float* T, int32_t* nlast,
                                  int32_t* dom, hipStream_t st) {
  FwdArgs a;
  a.r = make_raster_args(ws, s);
  a.rgb = rgb; a.T = T; a.nlast = nlast; a.dom = dom; a.counts = nullptr;
  const int blocks = ws->geo.n_views * ws->tiles_x * ws->tiles_y;
  if (blocks <= 0) return hipSuccess;
  dispatch_shape(ws->geo.tile, s->lds_batch, s->block_threads,
                 FwdLauncher<kDominant>{a, blocks, st});
  return hipGetLastError();
}

hipError_t launch_count_pairs(gs_workspace* ws, const gs_settings* s,
                              unsigned long long* counts, hipStream_t st) {
  FwdArgs a;
  a.r = make_raster_args(ws, s);
  a.rgb = nullptr; a.T = nullptr; a.nlast = nullptr; a.dom = nullptr;
  a.counts = counts;
  const int blocks = ws->geo.n_views * ws->tiles_x * ws->tiles_y;
  if (blocks <= 0) return hipSuccess;
  dispatch_shape(ws->geo.tile, s->lds_batch, s->block_threads,
                 FwdLauncher<kCount>{a, blocks, st});
  return hipGetLastError();
}

}  // namespace gs
