// Backward of the compositing (exact derivative of Eq. 3 with the forward's
// decisions), per screen tile.
//
// One workgroup per (view, tile), the same pixel ownership as the forward.
// Only per-pixel state is kept from the forward (T_final and n_last); the
// list is walked back to front from the tile's largest n_last, and each
// admitted entry's transmittance is recovered as T_i = T_{i+1} / (1 - a_i).
// The colour accumulated behind entry i, dotted with g = dL/dC, follows
// S_{i-1} = a_i (c_i . g) + (1 - a_i) S_i, so
//   dL/dc_i     = a_i T_i g
//   dL/da_i     = T_i (c_i . g - S_i) - T_final (bg . g) / (1 - a_i)
//   dL/dpi_i    = a_i dL/da_i                 (a = o exp(pi), unclamped)
//   dL/do_i     = G_i dL/da_i = (dL/dpi_i) / o   (summed per entry, then / o)
// with pi = -(A dx^2 + C dy^2) / 2 - B dx dy.  A thread's pixels share dx, so
// it accumulates only sum(dL/dpi), sum(dL/dpi dy) and sum(dL/dpi dy^2) over
// its strip and forms the mean and conic gradients once per entry.  The nine
// per-entry sums are reduced over each 16-lane row with DPP (a transposed
// reduction that packs four quantities into one register), merged across
// rows and waves by LDS adds, and added to global memory with one atomic per
// (entry, quantity).

#include "raster_common.h"

namespace gs {
namespace {

struct BwdArgs {
  RasterArgs r;
  const float* dL;
  const float* Tfin;
  const int32_t* nlast;
  float* grad2d;   // [V][5][cap]
  float* gop;      // [cap]
  float* grgb;     // [3][cap] (caller's gradient rows, accumulated), or
                   // [V][3][cap] per view (view-dependent colour)
  size_t grgb_vstride;   // 0, or 3 cap for per-view colour gradients
  // L1 photometric term fused in (target not null): dL/dC is formed per
  // pixel from the forward's image instead of read from dL.
  const float* rgb;
  const float* target;
  float l1_scale;        // lambda / (3HW), the gradient's magnitude
  double l1_lam_inv;     // lambda / (3HW) in FP64, for the loss
  double* tile_loss;     // [tiles][2]: this tile's loss and squared error
};

// Sign of r times scale (sign(0) = 0): the L1 term's gradient.
__device__ __forceinline__ float l1_grad(float r, float scale) {
  return r > 0.f ? scale : (r < 0.f ? -scale : 0.f);
}

// x plus the DPP-permuted y.  Lanes whose source lies outside their row read
// 0; the reductions below only keep lanes whose source is inside the row.
template <int CTRL>
__device__ __forceinline__ float add_dpp(float x, float y) {
  const int t = __builtin_amdgcn_update_dpp(0, __float_as_int(y), CTRL, 0xf,
                                            0xf, true);
  return x + __int_as_float(t);
}

// Transposed row reduction of four per-lane values: returns, in each lane,
// the sum over the lane's 16-lane row of value number (lane >> 2) & 3.
// Two bank-masked exchange levels halve the number of registers each time
// (shift 4: banks 0, 2 keep a / c and banks 1, 3 keep b / d; shift 8: banks
// 0, 1 keep the first pair), then a quad reduction finishes each bank.
__device__ __forceinline__ float row_sum4(float a, float b, float c, float d,
                                          bool bank02, bool bank01) {
  // The DPP reads of neighbouring lanes run in converged control flow; only
  // the selects depend on the lane.
  const float a1 = add_dpp<0x104>(a, a);   // row_shl:4
  const float b1 = add_dpp<0x114>(b, b);   // row_shr:4
  const float c1 = add_dpp<0x104>(c, c);
  const float d1 = add_dpp<0x114>(d, d);
  const float ab = bank02 ? a1 : b1;
  const float cd = bank02 ? c1 : d1;
  const float ab1 = add_dpp<0x108>(ab, ab);  // row_shl:8
  const float cd1 = add_dpp<0x118>(cd, cd);  // row_shr:8
  float x = bank01 ? ab1 : cd1;
  x = add_dpp<0xb1>(x, x);   // quad_perm [1,0,3,2]
  x = add_dpp<0x4e>(x, x);   // quad_perm [2,3,0,1]
  return x;
}

// Sum over the lane's 16-lane row, in every lane of the row.
__device__ __forceinline__ float row_sum(float x) {
  x = add_dpp<0xb1>(x, x);   // quad_perm [1,0,3,2]
  x = add_dpp<0x4e>(x, x);   // quad_perm [2,3,0,1]
  x = add_dpp<0x141>(x, x);  // row_half_mirror
  x = add_dpp<0x140>(x, x);  // row_mirror
  return x;
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off, 64));
  return x;
}

template <int PPT>
struct BwdPix {
  float T[PPT], g0[PPT], g1[PPT], g2[PPT], Tb[PPT], Sg[PPT], vf[PPT];
  int last[PPT];
};

// Per-lane sums of one entry over the thread's strip.
struct EntrySums {
  float S0, S1, S2, d_r, d_g, d_b;
  bool hit;
};

// The backward of one entry over the thread's strip, back to front: T is
// recovered as T_{i+1} / (1 - alpha_i) (a pair that is not admitted takes
// alpha 0: 1 / (1 - 0) is exactly 1, so T, the weight and the running colour
// sum come out unchanged without a select each).  inb[p]: the pixel lies in
// the entry's render box and before its n_last (all true on the fast path).
// CLAMP: some entry of the batch has opacity above alpha_max, so alpha is
// clamped and a clamped pair passes no shape or opacity gradient; batches
// without such an entry (nearly all) run the version without the clamp.
// BG: a non-zero background, whose term enters dL/dalpha.  The opacity
// gradient is formed once per entry from S0 = sum of dL/dpi: with
// alpha = o G unclamped, dL/dpi = alpha dL/dalpha and dL/do = G dL/dalpha =
// S0 / o (clamped pairs add 0 to both).
template <bool CLAMP, bool BG, int PPT>
__device__ __forceinline__ EntrySums entry_bwd(BwdPix<PPT>& px,
                                               const Column& col, float py,
                                               float C2, float o, float cr,
                                               float cgc, float cbc, float amin,
                                               float amax, const bool* inb) {
  EntrySums r = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, false};
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    float dy;
    const float e2 = exponent2(col, py, C2, px.vf[p], dy);
    const float G = gauss2(e2);
    const float oG = o * G;
    const float al = CLAMP ? fminf(amax, oG) : oG;
    const bool ok = inb[p] && al >= amin;
    r.hit |= ok;
    const float alo = ok ? al : 0.f;
    const float rom = __builtin_amdgcn_rcpf(1.f - alo);
    const float Ti = px.T[p] * rom;                 // T_i
    px.T[p] = Ti;
    const float w = alo * Ti;
    r.d_r = fmaf(w, px.g0[p], r.d_r);
    r.d_g = fmaf(w, px.g1[p], r.d_g);
    r.d_b = fmaf(w, px.g2[p], r.d_b);
    const float cgp = fmaf(cr, px.g0[p], fmaf(cgc, px.g1[p], cbc * px.g2[p]));
    const float diff = cgp - px.Sg[p];
    const float dal = BG ? fmaf(Ti, diff, -(px.Tb[p] * rom)) : Ti * diff;
    px.Sg[p] = fmaf(alo, diff, px.Sg[p]);
    const float dpw = (CLAMP && oG > amax) ? 0.f : dal * alo;
    const float tdy = dpw * dy;
    r.S0 += dpw;
    r.S1 += tdy;
    r.S2 = fmaf(tdy, dy, r.S2);
  }
  return r;
}

// The entries [0, jn) of the staged batch, back to front, for one wave.
template <bool CLAMP, bool BG, int TILE, int BATCH, int NT>
__device__ __forceinline__ void walk_batch(
    BwdPix<PixLayout<TILE, NT>::PPT>& px, const Entry* ent, const int* wbits,
    float (*acc)[9], int jn, int lo, int wave, int wfirst, int u, int v0,
    float uf, float amin, float amax, int lane, bool bank02, bool bank01) {
  constexpr int PPT = PixLayout<TILE, NT>::PPT;
  for (int j = jn - 1; j >= 0; --j) {
    const int pos = lo + j;
    const int wb = __builtin_amdgcn_readfirstlane(wbits[j]) >> (2 * wave);
    if (!(wb & 1)) continue;
    const float4 ea = ent[j].a;
    const float4 eb = ent[j].b;
    const float4 ec = ent[j].c;
    const Column col = column(ea, uf);
    // Only the box / position masks differ between the fast and the general
    // path, chosen in scalar registers, so the pixels' running state is
    // updated by one common body.
    bool inb[PPT];
    if ((wb & 2) && pos < wfirst) {
#pragma unroll
      for (int p = 0; p < PPT; ++p) inb[p] = true;
    } else {
      const int4 box = ent[j].box;
      const bool in_u = u >= box.x && u <= box.y;
      const int rlo = box.z - v0, rhi = box.w - v0;
#pragma unroll
      for (int p = 0; p < PPT; ++p)
        inb[p] = in_u && rlo <= p && p <= rhi && pos < px.last[p];
    }
    const EntrySums es = entry_bwd<CLAMP, BG>(px, col, ea.y, eb.x, eb.y, eb.z,
                                              eb.w, ec.x, amin, amax, inb);
    if (__any(es.hit)) {
      const float A = ec.y, B = ec.z, C = ec.w;
      const float dx = col.dx, dxS0 = dx * es.S0;
      const float d_px = -fmaf(A, dxS0, B * es.S1);
      const float d_py = -fmaf(C, es.S1, B * dxS0);
      const float d_A = -0.5f * dx * dxS0;
      const float d_B = -dx * es.S1;
      const float d_C = -0.5f * es.S2;
      const float d_o = es.S0 * __builtin_amdgcn_rcpf(eb.y);
      // Row sums of the nine quantities, added into the entry's LDS slot by
      // lanes 0, 4, 8, 12 of each row (the four rows of the wave and the
      // other waves of the tile meet in the LDS adds).
      const float x = row_sum4(d_px, d_py, d_A, d_B, bank02, bank01);
      const float y = row_sum4(d_C, d_o, es.d_r, es.d_g, bank02, bank01);
      const float z = row_sum(es.d_b);
      float* ac = acc[j];
      if ((lane & 3) == 0) {
        const int q = (lane >> 2) & 3;
        atomicAdd(&ac[q], x);
        atomicAdd(&ac[4 + q], y);
        if (q == 0) atomicAdd(&ac[8], z);
      }
    }
  }
}

// The per-pixel work is predicated like the forward's: every lane evaluates
// its pixels for each entry and the admit decision selects what is
// accumulated.  A wave starts its backward walk at the largest n_last of its
// own pixels, skips entries no pixel of its footprint can admit and takes
// the fast path (wave_bits, and the entry before every pixel's n_last) when
// it can; the choice is uniform over the wave.
template <int TILE, int BATCH, int NT, bool BG>
__global__ __launch_bounds__(NT) void k_render_bwd(BwdArgs a) {
  using Lay = PixLayout<TILE, NT>;
  constexpr int PPT = Lay::PPT;
  __shared__ Entry ent[BATCH];
  __shared__ float acc[BATCH][9];
  __shared__ uint32_t gid[BATCH];
  __shared__ int smax;
  const RasterArgs& r = a.r;
  const int t = (int)r.order[blockIdx.x];
  const int tpv = r.Tx * r.Ty;
  const int k = t / tpv;
  const int rem = t - k * tpv;
  const int ty = rem / r.Tx, tx = rem - ty * r.Tx;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const bool bank02 = ((lane >> 2) & 1) == 0;   // lane in bank 0 or 2 of its row
  const bool bank01 = ((lane >> 3) & 1) == 0;   // lane in bank 0 or 1
  long long s, e;
  tile_range(r, t, s, e);
  const size_t HW = (size_t)r.H * r.W;

  int cu, cv0;
  Lay::of(tid, cu, cv0);
  const int u = tx * TILE + cu;
  const int v0 = ty * TILE + cv0;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  __shared__ int wbits[BATCH];   // per staged entry: wave_bits
  const float uf = pinned((float)u);
  const float amax = r.alpha_max, amin = r.alpha_min;
  BwdPix<PPT> px;
  int mylast = 0, myfirst = 0x7fffffff;
  float l1_abs = 0.f;
  double l1_sq = 0.0;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    const int v = v0 + p;
    px.last[p] = 0;
    px.vf[p] = pinned((float)v);
    // Pixels outside the image keep T = 0 and a zero gradient: every term
    // they could add is zero.
    px.T[p] = 0.f; px.g0[p] = px.g1[p] = px.g2[p] = 0.f; px.Tb[p] = 0.f;
    px.Sg[p] = 0.f;
    if (u < r.W && v < r.H) {
      const size_t pix = (size_t)v * r.W + u;
      px.T[p] = a.Tfin[(size_t)k * HW + pix];
      px.last[p] = a.nlast[(size_t)k * HW + pix];
      if (a.target) {
        float gg[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          const size_t i = ((size_t)k * 3 + ch) * HW + pix;
          const float d = a.rgb[i] - a.target[i];
          l1_abs += fabsf(d);
          l1_sq += (double)d * (double)d;
          gg[ch] = l1_grad(d, a.l1_scale);
        }
        px.g0[p] = gg[0]; px.g1[p] = gg[1]; px.g2[p] = gg[2];
      } else {
        px.g0[p] = a.dL[((size_t)k * 3 + 0) * HW + pix];
        px.g1[p] = a.dL[((size_t)k * 3 + 1) * HW + pix];
        px.g2[p] = a.dL[((size_t)k * 3 + 2) * HW + pix];
      }
      px.Tb[p] = px.T[p] * (r.bg0 * px.g0[p] + r.bg1 * px.g1[p] + r.bg2 * px.g2[p]);
      mylast = max(mylast, px.last[p]);
      myfirst = min(myfirst, px.last[p]);
    }
  }
  // The tile's share of the fused L1 loss: wave sums, then one plain store
  // per workgroup (a second kernel sums the tiles: FP64 atomics on one
  // address would serialise).
  __shared__ double lpart[2][NT / 64];
  if (a.target) {
    double la = l1_abs, lq = l1_sq;
    for (int off = 32; off > 0; off >>= 1) {
      la += __shfl_down(la, off, 64);
      lq += __shfl_down(lq, off, 64);
    }
    if (lane == 0) {
      lpart[0][wave] = la;
      lpart[1][wave] = lq;
    }
  }
  if (tid == 0) smax = 0;
  __syncthreads();
  atomicMax(&smax, mylast);
  const int wlast = __builtin_amdgcn_readfirstlane(wave_max(mylast));
  // Entries before every pixel's n_last: no per-pixel position test.
  const int wfirst = __builtin_amdgcn_readfirstlane(wave_min(myfirst));
  __syncthreads();
  if (a.target && tid == 0) {
    double la = 0.0, lq = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      la += lpart[0][w];
      lq += lpart[1][w];
    }
    a.tile_loss[2 * (size_t)t] = la * a.l1_lam_inv;
    a.tile_loss[2 * (size_t)t + 1] = lq;
  }
  const int maxlast = (int)min((long long)smax, e - s);
  const Record* rv = r.rec + (size_t)k * r.cap;
  const int2* rbv = r.rbox + (size_t)k * r.cap;
  float* gk = a.grad2d + (size_t)k * 5 * r.cap;
  float* gc = a.grgb + (size_t)k * a.grgb_vstride;

  for (int hi = maxlast; hi > 0; hi -= BATCH) {
    const int lo = max(0, hi - BATCH);
    const int cnt = hi - lo;
    __syncthreads();   // the previous batch is flushed
    int clampable = 0;
    for (int i = tid; i < cnt; i += NT) {
      const uint32_t g = r.vals[s + lo + i];
      gid[i] = g;
      const Record R = rv[g];
      const int4 box = unpack_box(rbv[g]);
      stage(ent[i], R, box);
      wbits[i] = wave_bits<TILE, NT>(R, box, tx * TILE, ty * TILE, r.W, r.H,
                                     amin, amax, r.ellipse_test);
      clampable |= R.q1.y > amax;
    }
    for (int i = tid; i < cnt * 9; i += NT) (&acc[0][0])[i] = 0.f;
    const int jn = min(cnt, wlast - lo);
    if (__syncthreads_or(clampable)) {
      walk_batch<true, BG, TILE, BATCH, NT>(px, ent, wbits, acc, jn, lo, wave,
                                            wfirst, u, v0, uf, amin, amax,
                                            lane, bank02, bank01);
    } else {
      walk_batch<false, BG, TILE, BATCH, NT>(px, ent, wbits, acc, jn, lo, wave,
                                             wfirst, u, v0, uf, amin, amax,
                                             lane, bank02, bank01);
    }
    __syncthreads();
    for (int i = tid; i < cnt * 9; i += NT) {
      const float val = (&acc[0][0])[i];
      if (val == 0.f) continue;
      const int jj = i / 9, q = i - jj * 9;
      const uint32_t g = gid[jj];
      if (q < 5) atomicAdd(&gk[(size_t)q * r.cap + g], val);
      else if (q == 5) atomicAdd(&a.gop[g], val);
      else atomicAdd(&gc[(size_t)(q - 6) * r.cap + g], val);
    }
  }
}

// Sum of the tiles' fused L1 losses into *loss and of each view's squared
// errors into sqerr[view], in a fixed order (so the sums do not depend on
// scheduling): wave w of the one workgroup reduces view k0 + w, then thread 0
// adds the views in order.
__global__ __launch_bounds__(1024) void k_l1_reduce(const double2* tile_loss,
                                                    int V, int tpv,
                                                    double* loss,
                                                    double* sqerr) {
  __shared__ double part[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double total = 0.0;
  for (int k0 = 0; k0 < V; k0 += 16) {
    const int k = k0 + w;
    if (k < V) {
      double la = 0.0, lq = 0.0;
      for (int i = lane; i < tpv; i += 64) {
        const double2 q = tile_loss[(size_t)k * tpv + i];
        la += q.x;
        lq += q.y;
      }
      for (int off = 32; off > 0; off >>= 1) {
        la += __shfl_down(la, off, 64);
        lq += __shfl_down(lq, off, 64);
      }
      if (lane == 0) {
        part[w] = la;
        if (sqerr) atomicAdd(&sqerr[k], lq);
      }
    }
    __syncthreads();
    if (tid == 0)
      for (int i = 0; i < 16 && k0 + i < V; ++i) total += part[i];
    __syncthreads();
  }
  // One atomic add each: other calls (other workspaces, other streams) may
  // accumulate into the same buffers.
  if (tid == 0) atomicAdd(loss, total);
}

struct BwdLauncher {
  const BwdArgs& a;
  int blocks;
  bool bg;
  hipStream_t st;
  template <int T, int B, int N>
  void go() const {
    if (bg)
      hipLaunchKernelGGL((k_render_bwd<T, B, N, true>), dim3(blocks), dim3(N),
                         0, st, a);
    else
      hipLaunchKernelGGL((k_render_bwd<T, B, N, false>), dim3(blocks),
                         dim3(N), 0, st, a);
  }
};

}  // namespace

hipError_t launch_render_bwd(gs_workspace* ws, const gs_settings* s,
                             const float* dL, const float* T,
                             const int32_t* nlast, float* grad_rgb,
                             int per_view_colour, const L1Fused* l1,
                             hipStream_t st) {
  BwdArgs a;
  a.r = make_raster_args(ws, s);
  a.dL = dL; a.Tfin = T; a.nlast = nlast;
  a.rgb = nullptr; a.target = nullptr; a.l1_scale = 0.f; a.l1_lam_inv = 0.0;
  a.tile_loss = ws->tile_loss;
  if (l1) {
    const size_t per = (size_t)3 * ws->geo.height * ws->geo.width;
    a.rgb = l1->rgb; a.target = l1->target;
    a.l1_scale = (float)((double)l1->lambda / (double)per);
    a.l1_lam_inv = (double)l1->lambda / (double)per;
  }
  a.grad2d = ws->grad2d; a.gop = ws->gop;
  a.grgb = per_view_colour ? ws->gcol : grad_rgb;
  a.grgb_vstride = per_view_colour ? (size_t)3 * ws->geo.capacity : 0;
  const int blocks = ws->geo.n_views * ws->tiles_x * ws->tiles_y;
  if (blocks <= 0) return hipSuccess;
  const bool bg = s->bg[0] != 0.f || s->bg[1] != 0.f || s->bg[2] != 0.f;
  dispatch_shape(ws->geo.tile, s->lds_batch, s->block_threads,
                 BwdLauncher{a, blocks, bg, st});
  if (l1) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_l1_reduce, dim3(1), dim3(1024), 0, st,
                       (const double2*)ws->tile_loss,
                       ws->geo.n_views, ws->tiles_x * ws->tiles_y, l1->loss,
                       l1->sqerr);
  }
  return hipGetLastError();
}

}  // namespace gs
