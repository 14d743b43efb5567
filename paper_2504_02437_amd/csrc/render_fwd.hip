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
// and stopping it again (T = -|T|) leaves it as it is.  Pixels outside the
// image start stopped.  The per-pixel work is predicated rather than
// branched: every lane evaluates alpha for each of its pixels and the
// decisions select what is accumulated.  A wave skips an entry outright
// when no pixel of its footprint can admit it (its eval mask bit), and
// takes a fast path without the per-pixel box tests and the alpha clamp
// when the entry's render box holds the whole footprint and its opacity is
// at most alpha_max (its fast mask bit); the choice is uniform over the
// wave, made in scalar registers.  The candidate transmittance is formed as
// fma(-alpha, T, T), one rounding.
enum { kRender = 0, kCount = 1, kDominant = 2 };

template <int PPT, int MODE>
struct PixState {
  float T[PPT], C0[PPT], C1[PPT], C2[PPT], vf[PPT];
  int last[PPT];
  float wbest[MODE == kDominant ? PPT : 1];
  int32_t best[MODE == kDominant ? PPT : 1];
  unsigned ib[MODE == kCount ? PPT : 1], ib_last[MODE == kCount ? PPT : 1];
  unsigned n_contrib;
};

// Blends one staged entry into the thread's strip.  inb[p]: the pixel lies
// in the entry's render box (all true on the fast path).  CLAMP: some entry
// of the batch has opacity above alpha_max, so alpha is clamped; batches
// without such an entry (nearly all) run the version without the clamp.
template <bool CLAMP, int PPT, int MODE>
__device__ __forceinline__ void blend_entry(PixState<PPT, MODE>& st,
                                            const Column& col, float py,
                                            float C2, float cr, float cg,
                                            float cb, float amin, float amax,
                                            float tmin, const bool* inb,
                                            int idx, int32_t gj) {
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    float dy;
    const float e2 = exponent2(col, py, C2, st.vf[p], dy);
    const float oG = alpha2(e2);
    const float al = CLAMP ? fminf(amax, oG) : oG;
    const bool ok = inb[p] && al >= amin;
    const float Tn = fmaf(-al, st.T[p], st.T[p]);
    const bool con = ok && Tn >= tmin;
    const float w = con ? al * st.T[p] : 0.f;
    st.C0[p] = fmaf(cr, w, st.C0[p]);
    st.C1[p] = fmaf(cg, w, st.C1[p]);
    st.C2[p] = fmaf(cb, w, st.C2[p]);
    st.T[p] = con ? Tn : (ok ? -fabsf(st.T[p]) : st.T[p]);
    st.last[p] = con ? idx : st.last[p];
    if (MODE == kDominant) {
      const bool better = con && w > st.wbest[p];
      st.wbest[p] = better ? w : st.wbest[p];
      st.best[p] = better ? gj : st.best[p];
    }
    if (MODE == kCount) {
      st.n_contrib += con;
      st.ib_last[p] = con ? st.ib[p] : st.ib_last[p];
    }
  }
}

// Staged entry j for one thread's strip; fast: the wave's fast-path bit.
template <bool CLAMP, int TILE, int NT, int MODE>
__device__ __forceinline__ void walk_entry(
    PixState<PixLayout<TILE, NT>::PPT, MODE>& st, const Entry* ent,
    const uint32_t* egid, int j, bool fast, int base, int u, int v0,
    float uf, float amin, float amax, float tmin) {
  constexpr int PPT = PixLayout<TILE, NT>::PPT;
  const float4 ea = ent[j].a;
  const float4 eb = ent[j].b;
  const float ecb = ent[j].c.x;
  const Column col = column(ea, eb.y, uf);
  const int32_t gj = MODE == kDominant ? (int32_t)egid[j] : 0;
  // Only the box masks differ between the fast and the general path, chosen
  // in scalar registers, so the pixels' running state is updated by one
  // common body.
  bool inb[PPT];
  if (fast) {
#pragma unroll
    for (int p = 0; p < PPT; ++p) inb[p] = true;
  } else {
    const int4 box = ent[j].box;
    const bool in_u = u >= box.x && u <= box.y;
    const int lo = box.z - v0, hi = box.w - v0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) inb[p] = in_u && lo <= p && p <= hi;
  }
  blend_entry<CLAMP>(st, col, ea.y, eb.x, eb.z, eb.w, ecb, amin, amax, tmin,
                     inb, base + j, gj);
}

template <int PPT, int MODE>
__device__ __forceinline__ bool any_alive(const PixState<PPT, MODE>& st) {
  bool any = false;
#pragma unroll
  for (int p = 0; p < PPT; ++p) any |= st.T[p] > 0.f;
  return __builtin_amdgcn_ballot_w64(any) != 0;
}

// The staged batch front to back for one thread's strip: the set bits of
// the wave's eval mask, in order; the wave leaves the batch once all its
// pixels stopped (checked every eight evaluated entries).
template <bool CLAMP, int TILE, int BATCH, int NT, int MODE>
__device__ __forceinline__ void walk_batch(
    PixState<PixLayout<TILE, NT>::PPT, MODE>& st, const Entry* ent,
    const WaveMasks<BATCH, NT>& masks, const uint32_t* egid, int cnt,
    int base, int wave, int u, int v0, float uf, float amin, float amax,
    float tmin) {
  const int nw = (cnt + 31) >> 5;
  int seen = 0;
  for (int k = 0; k < nw; ++k) {
    uint32_t e = __builtin_amdgcn_readfirstlane(masks.eval[wave][k]);
    const uint32_t f = __builtin_amdgcn_readfirstlane(masks.fast[wave][k]);
    while (e) {
      const int b = __builtin_ctz(e);
      e &= e - 1;
      if ((seen++ & 7) == 0 && !any_alive(st)) return;
      walk_entry<CLAMP, TILE, NT, MODE>(st, ent, egid, 32 * k + b,
                                        (f >> b) & 1, base, u, v0, uf, amin,
                                        amax, tmin);
    }
  }
}

// The counting variant walks every staged entry, adding the examined and
// in-box pairs of the pixels still compositing, and blends the evaluated
// ones as walk_batch does.
template <bool CLAMP, int TILE, int BATCH, int NT, int MODE>
__device__ __forceinline__ void count_batch(
    PixState<PixLayout<TILE, NT>::PPT, MODE>& st, const Entry* ent,
    const WaveMasks<BATCH, NT>& masks, const uint32_t* egid, int cnt,
    int base, int wave, int u, int v0, float uf, float amin, float amax,
    float tmin, unsigned& n_exam, unsigned& n_inbox) {
  constexpr int PPT = PixLayout<TILE, NT>::PPT;
  for (int j = 0; j < cnt; ++j) {
    if ((j & 7) == 0 && !any_alive(st)) break;
    const uint32_t e = __builtin_amdgcn_readfirstlane(masks.eval[wave][j >> 5]);
    const uint32_t f = __builtin_amdgcn_readfirstlane(masks.fast[wave][j >> 5]);
    const bool evaluate = (e >> (j & 31)) & 1;
    const int4 box = ent[j].box;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      if (!(st.T[p] > 0.f)) continue;
      ++n_exam;
      if (evaluate && u >= box.x && u <= box.y && v0 + p >= box.z &&
          v0 + p <= box.w) {
        ++n_inbox;
        ++st.ib[p];
      }
    }
    if (!evaluate) continue;
    walk_entry<CLAMP, TILE, NT, MODE>(st, ent, egid, j, (f >> (j & 31)) & 1,
                                      base, u, v0, uf, amin, amax, tmin);
  }
}

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
  // The wave index, uniform over the wave, in a scalar register.
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  __shared__ WaveMasks<BATCH, NT> masks;
  __shared__ uint32_t egid[DOM ? BATCH : 1];   // Gaussian index per entry
  const float uf = pinned((float)u);
  const float amax = r.alpha_max;
  const float amin = r.alpha_min, tmin = r.T_min;
  PixState<PPT, MODE> st;
  unsigned n_exam = 0, n_inbox = 0;
  st.n_contrib = 0;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    if (DOM) {
      st.wbest[p] = 0.f;
      st.best[p] = -1;
    }
    st.T[p] = (u < r.W && v0 + p < r.H) ? 1.f : -1.f;
    st.C0[p] = st.C1[p] = st.C2[p] = 0.f;
    st.last[p] = 0;
    st.vf[p] = pinned((float)(v0 + p));
    if (COUNT) st.ib[p] = st.ib_last[p] = 0;
  }
  const Record* rv = r.rec + (size_t)k * r.cap;
  const int2* rbv = r.rbox + (size_t)k * r.cap;
  for (long long b0 = s; b0 < e; b0 += BATCH) {
    int alive = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) alive |= st.T[p] > 0.f;
    if (__syncthreads_or(alive) == 0) break;
    const int cnt = (int)min((long long)BATCH, e - b0);
    int clampable = 0;
#pragma unroll
    for (int i0 = 0; i0 < BATCH; i0 += NT) {
      const int i = i0 + tid;
      int bits = 0;
      if (i < cnt) {
        const uint32_t g = r.vals[b0 + i];
        const Record R = rv[g];
        const int4 box = unpack_box(rbv[g]);
        stage(ent[i], R, box, r.lop[g]);
        bits = wave_bits<TILE, NT>(R, box, tx * TILE, ty * TILE, r.W, r.H,
                                   amin, amax, r.ellipse_test);
        clampable |= R.q1.y > amax;
        if (DOM) egid[i] = g;
      }
      publish_masks(masks, i0, bits, wave, lane);
    }
    const int base = (int)(b0 - s) + 1;
    if (COUNT) {
      if (__syncthreads_or(clampable))
        count_batch<true, TILE>(st, ent, masks, egid, cnt, base, wave, u, v0,
                                uf, amin, amax, tmin, n_exam, n_inbox);
      else
        count_batch<false, TILE>(st, ent, masks, egid, cnt, base, wave, u, v0,
                                 uf, amin, amax, tmin, n_exam, n_inbox);
    } else if (__syncthreads_or(clampable)) {
      walk_batch<true, TILE>(st, ent, masks, egid, cnt, base, wave, u, v0, uf,
                             amin, amax, tmin);
    } else {
      walk_batch<false, TILE>(st, ent, masks, egid, cnt, base, wave, u, v0,
                              uf, amin, amax, tmin);
    }
  }
  if (COUNT) {
    unsigned long long c[4] = {n_exam, n_inbox, st.n_contrib, 0};
#pragma unroll
    for (int p = 0; p < PPT; ++p) c[3] += st.ib_last[p];
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
    const float Tf = fabsf(st.T[p]);
    const size_t pix = (size_t)v * r.W + u;
    a.rgb[((size_t)k * 3 + 0) * HW + pix] = fmaf(Tf, r.bg0, st.C0[p]);
    a.rgb[((size_t)k * 3 + 1) * HW + pix] = fmaf(Tf, r.bg1, st.C1[p]);
    a.rgb[((size_t)k * 3 + 2) * HW + pix] = fmaf(Tf, r.bg2, st.C2[p]);
    a.T[(size_t)k * HW + pix] = Tf;
    a.nlast[(size_t)k * HW + pix] = st.last[p];
    if (DOM) a.dom[(size_t)k * HW + pix] = st.best[p];
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
  r.lop = (const float*)(ws->shape + 6 * (size_t)ws->geo.capacity) +
          ws->geo.capacity;
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
