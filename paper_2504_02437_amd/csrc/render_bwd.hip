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
// with pi = -(A dx^2 + C dy^2) / 2 - B dx dy.  A thread's pixels share dx,
// so per entry it needs only the moments sum(dL/dpi), sum(dL/dpi dy) and
// sum(dL/dpi dy^2) over its strip; the rows of a strip are consecutive
// (dy_p = dy_0 - p), so these follow from sums weighted by the constants p
// and p^2.  Nine per-lane sums per entry (the three moments, the first one
// times dx and dx^2, the second times dx, and the colour gradient) are
// reduced over each 16-lane row with DPP (a transposed reduction that packs
// four quantities into one register), merged across rows and waves by LDS
// adds, and turned into the mean, conic and opacity gradients once per
// entry and workgroup, which adds them to global memory with one atomic per
// (entry, quantity).

#include "raster_common.h"
#include "tails.h"

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
  // Workgroups past the tiles' (tile_blocks) run the planar regulariser.
  int tile_blocks;
  PlanarJob planar;
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

// a + b over the two halves of the wave: returns, in lanes 0-31, a's lanes
// l + (l + 32) and, in lanes 32-63, b's (v_permlane32_swap exchanges the
// upper half of its first operand with the lower half of its second).
__device__ __forceinline__ float fold32(float a, float b) {
  const auto t = __builtin_amdgcn_permlane32_swap(__float_as_uint(a),
                                                  __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(t[0]) + __uint_as_float(t[1]);
}

// The same over adjacent rows: rows 0 and 2 receive a's rows r + (r + 1)
// and rows 1 and 3 b's (v_permlane16_swap exchanges the odd rows of its
// first operand with the even rows of its second).
__device__ __forceinline__ float fold16(float a, float b) {
  const auto t = __builtin_amdgcn_permlane16_swap(__float_as_uint(a),
                                                  __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(t[0]) + __uint_as_float(t[1]);
}

// Sum over the wave of eight per-lane values: lane 8k receives the total of
// q[k].  A transposed reduction: the two half-wave folds and the two row
// folds leave two registers whose row r holds one value's 16 row partials
// (value r of the first four, in the order 0, 2, 4, 6 / 1, 3, 5, 7 below),
// a shift-8 exchange writing only banks 0-1 from the first register and
// banks 2-3 from the second (bank_mask: no select) merges them, and three
// shifts within each half-row finish the sums.  The DPP adds read
// registers written just before them, which needs two wait states after a
// VALU write (the s_nop 1 before each); lanes whose DPP source lies outside
// their row are not written and are not used.  Runs in converged control
// flow with every lane active.
__device__ __forceinline__ float wave_sum8(const float (&q)[8]) {
  const float r1 = fold16(fold32(q[0], q[4]), fold32(q[2], q[6]));
  const float r2 = fold16(fold32(q[1], q[5]), fold32(q[3], q[7]));
  float x;
  asm volatile(
      "s_nop 1\n\t"
      "v_add_f32_dpp %[x], %[r1], %[r1] row_shl:8 row_mask:0xf bank_mask:0x3\n\t"
      "v_add_f32_dpp %[x], %[r2], %[r2] row_shr:8 row_mask:0xf bank_mask:0xc\n\t"
      "s_nop 1\n\t"
      "v_add_f32_dpp %[x], %[x], %[x] row_shl:4 row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 1\n\t"
      "v_add_f32_dpp %[x], %[x], %[x] row_shl:2 row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 1\n\t"
      "v_add_f32_dpp %[x], %[x], %[x] row_shl:1 row_mask:0xf bank_mask:0xf"
      : [x] "=&v"(x)
      : [r1] "v"(r1), [r2] "v"(r2));
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

// Per-lane sums of one entry over the thread's strip: S0, S1, S2 are the
// moments sum(dL/dpi dy^k), k = 0, 1, 2.
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
// BG: a non-zero background, whose term enters dL/dalpha.  With the weight
// w = alpha T_i, dL/dpi = alpha dL/dalpha is w (c.g - S) without a
// background.  The moments are formed from P0 = sum(dL/dpi),
// P1 = sum(p dL/dpi) and P2 = sum(p^2 dL/dpi) over the strip's rows p:
// with dy_p = dy_0 - p, S1 = dy_0 P0 - P1 and
// S2 = dy_0^2 P0 - 2 dy_0 P1 + P2 = dy_0 (S1 - P1) + P2.
template <bool CLAMP, bool BG, int PPT>
__device__ __forceinline__ EntrySums entry_bwd(BwdPix<PPT>& px,
                                               const Column& col, float py,
                                               float C2, float cr, float cgc,
                                               float cbc, float amin,
                                               float amax, const bool* inb) {
  EntrySums r;
  r.hit = false;
  r.d_r = r.d_g = r.d_b = 0.f;
  float P0 = 0.f, P1 = 0.f, P2 = 0.f, dy0 = 0.f;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    float dy;
    const float e2 = exponent2(col, py, C2, px.vf[p], dy);
    if (p == 0) dy0 = dy;
    const float oG = alpha2(e2);
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
    px.Sg[p] = fmaf(alo, diff, px.Sg[p]);
    float dpw = BG ? alo * fmaf(Ti, diff, -(px.Tb[p] * rom)) : w * diff;
    if (CLAMP) dpw = oG > amax ? 0.f : dpw;
    if (p == 0) {
      P0 = dpw;
    } else {
      P0 += dpw;
      P1 = p == 1 ? dpw : fmaf((float)p, dpw, P1);
      P2 = p == 1 ? dpw : fmaf((float)(p * p), dpw, P2);
    }
  }
  r.S0 = P0;
  r.S1 = fmaf(dy0, P0, -P1);
  r.S2 = fmaf(dy0, r.S1 - P1, P2);
  return r;
}

// Staged entry j for one wave; fast: the wave's fast-path bit and the entry
// lies before every pixel's n_last.
template <bool CLAMP, bool BG, int TILE, int NT>
__device__ __forceinline__ void walk_entry(
    BwdPix<PixLayout<TILE, NT>::PPT>& px, const Entry* ent, float (*acc)[9],
    int j, int pos, bool fast, int u, int v0, float uf, float amin,
    float amax, int lane) {
  constexpr int PPT = PixLayout<TILE, NT>::PPT;
  const float4 ea = ent[j].a;
  const float4 eb = ent[j].b;
  const float ecb = ent[j].c.x;
  const Column col = column(ea, eb.y, uf);
  // Only the box / position masks differ between the fast and the general
  // path, chosen in scalar registers, so the pixels' running state is
  // updated by one common body.
  bool inb[PPT];
  if (fast) {
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
  const EntrySums es = entry_bwd<CLAMP, BG>(px, col, ea.y, eb.x, eb.z, eb.w,
                                            ecb, amin, amax, inb);
  if (__builtin_amdgcn_ballot_w64(es.hit) != 0) {
    // Wave totals of eight of the nine per-lane sums, added into the
    // entry's LDS slot by lanes 0, 8, ..., 56 (distinct addresses), and row
    // totals of the ninth by lane 0 of each row; the other waves of the
    // tile meet in the LDS adds.
    const float dx = col.dx, dxS0 = dx * es.S0;
    const float q[8] = {es.S0, dxS0, dx * dxS0, es.S1,
                        dx * es.S1, es.S2, es.d_r, es.d_g};
    const float x = wave_sum8(q);
    const float z = row_sum(es.d_b);
    float* ac = acc[j];
    if ((lane & 7) == 0) atomicAdd(&ac[lane >> 3], x);
    if ((lane & 15) == 0) atomicAdd(&ac[8], z);
  }
}

// The entries [0, jn) of the staged batch, back to front, for one wave: the
// set bits of its eval mask below jn, highest first.
template <bool CLAMP, bool BG, int TILE, int BATCH, int NT>
__device__ __forceinline__ void walk_batch(
    BwdPix<PixLayout<TILE, NT>::PPT>& px, const Entry* ent,
    const WaveMasks<BATCH, NT>& masks, float (*acc)[9], int jn, int lo,
    int wave, int wfirst, int u, int v0, float uf, float amin, float amax,
    int lane) {
  for (int k = (jn - 1) >> 5; k >= 0; --k) {
    uint32_t e = __builtin_amdgcn_readfirstlane(masks.eval[wave][k]);
    const uint32_t f = __builtin_amdgcn_readfirstlane(masks.fast[wave][k]);
    const int top = jn - 32 * k;   // entries of this word below jn
    if (top < 32) e &= (1u << top) - 1u;
    while (e) {
      const int b = 31 - __builtin_clz(e);
      e &= ~(1u << b);
      const int j = 32 * k + b;
      const int pos = lo + j;
      walk_entry<CLAMP, BG, TILE, NT>(px, ent, acc, j, pos,
                                      ((f >> b) & 1) && pos < wfirst, u, v0,
                                      uf, amin, amax, lane);
    }
  }
}

// The per-pixel work is predicated like the forward's: every lane evaluates
// its pixels for each entry and the admit decision selects what is
// accumulated.  A wave starts its backward walk at the largest n_last of its
// own pixels, skips entries no pixel of its footprint can admit and takes
// the fast path (its fast mask bit, and the entry before every pixel's
// n_last) when it can; the choice is uniform over the wave, made in scalar
// registers.
template <int TILE, int BATCH, int NT, bool BG>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(BG ? 1 : 5))) void k_render_bwd(BwdArgs a) {
  using Lay = PixLayout<TILE, NT>;
  constexpr int PPT = Lay::PPT;
  __shared__ Entry ent[BATCH];
  __shared__ float acc[BATCH][9];
  __shared__ uint32_t gid[BATCH];
  __shared__ float eop[BATCH];   // opacity per staged entry
  __shared__ int smax;
  __shared__ double psh[NT / 64];
  if ((int)blockIdx.x >= a.tile_blocks) {   // dispatched last: the tail
    planar_part(a.planar, (int)blockIdx.x - a.tile_blocks,
                (int)gridDim.x - a.tile_blocks, psh);
    return;
  }
  const RasterArgs& r = a.r;
  const int t = (int)r.order[blockIdx.x];
  const int tpv = r.Tx * r.Ty;
  const int k = t / tpv;
  const int rem = t - k * tpv;
  const int ty = rem / r.Tx, tx = rem - ty * r.Tx;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  long long s, e;
  tile_range(r, t, s, e);
  const size_t HW = (size_t)r.H * r.W;

  int cu, cv0;
  Lay::of(tid, cu, cv0);
  const int u = tx * TILE + cu;
  const int v0 = ty * TILE + cv0;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  __shared__ WaveMasks<BATCH, NT> masks;
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
#pragma unroll
    for (int i0 = 0; i0 < BATCH; i0 += NT) {
      const int i = i0 + tid;
      int bits = 0;
      if (i < cnt) {
        const uint32_t g = r.vals[s + lo + i];
        gid[i] = g;
        const Record R = rv[g];
        eop[i] = R.q1.y;
        const int4 box = unpack_box(rbv[g]);
        stage(ent[i], R, box, r.lop[g]);
        bits = wave_bits<TILE, NT>(R, box, tx * TILE, ty * TILE, r.W, r.H,
                                   amin, amax, r.ellipse_test);
        clampable |= R.q1.y > amax;
      }
      publish_masks(masks, i0, bits, wave, lane);
    }
    for (int i = tid; i < cnt * 9; i += NT) (&acc[0][0])[i] = 0.f;
    const int jn = min(cnt, wlast - lo);
    if (__syncthreads_or(clampable)) {
      walk_batch<true, BG, TILE, BATCH, NT>(px, ent, masks, acc, jn, lo, wave,
                                            wfirst, u, v0, uf, amin, amax,
                                            lane);
    } else {
      walk_batch<false, BG, TILE, BATCH, NT>(px, ent, masks, acc, jn, lo, wave,
                                             wfirst, u, v0, uf, amin, amax,
                                             lane);
    }
    __syncthreads();
    // Per entry: the mean, conic and opacity gradients from the nine sums
    // (A, B, C the unscaled conic, o the opacity), then one atomic each.
    for (int jj = tid; jj < cnt; jj += NT) {
      const float* ac = acc[jj];
      const float s0 = ac[0], xs0 = ac[1], x2s0 = ac[2], s1 = ac[3];
      const float xs1 = ac[4], s2 = ac[5];
      const float4 ec = ent[jj].c;
      const float A = ec.y, B = ec.z, C = ec.w;
      float val[9];
      val[0] = -fmaf(A, xs0, B * s1);   // dL/dpx
      val[1] = -fmaf(C, s1, B * xs0);   // dL/dpy
      val[2] = -0.5f * x2s0;            // dL/dA
      val[3] = -xs1;                    // dL/dB
      val[4] = -0.5f * s2;              // dL/dC
      val[5] = s0 / eop[jj];            // dL/do
      val[6] = ac[6];
      val[7] = ac[7];
      val[8] = ac[8];
      const uint32_t g = gid[jj];
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        if (val[q] == 0.f) continue;
        if (q < 5) atomicAdd(&gk[(size_t)q * r.cap + g], val[q]);
        else if (q == 5) atomicAdd(&a.gop[g], val[q]);
        else atomicAdd(&gc[(size_t)(q - 6) * r.cap + g], val[q]);
      }
    }
  }
}

// Sum of the tiles' fused L1 losses into *loss and of each view's squared
// errors into sqerr[view], in a fixed order (l1_reduce_part).
__global__ __launch_bounds__(1024) void k_l1_reduce(L1ReduceJob j) {
  __shared__ double part[16];
  l1_reduce_part(j, part);
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
                             hipStream_t st, const PlanarJob* planar) {
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
  const int tiles = ws->geo.n_views * ws->tiles_x * ws->tiles_y;
  a.tile_blocks = tiles;
  a.planar = planar ? *planar : PlanarJob{};
  if (tiles <= 0) {
    if (planar) {
      const hipError_t e = launch_planar_job(*planar, st);
      if (e != hipSuccess) return e;
    }
  } else {
    // The regulariser's workgroups (a grid stride over the Gaussians, as
    // many as its own launch would have) follow the tiles'.
    const int nt = s->block_threads ? s->block_threads
                                    : default_threads(ws->geo.tile);
    const int pb = planar ? min(256, (planar->cap + nt - 1) / nt) : 0;
    const bool bg = s->bg[0] != 0.f || s->bg[1] != 0.f || s->bg[2] != 0.f;
    dispatch_shape(ws->geo.tile, s->lds_batch, s->block_threads,
                   BwdLauncher{a, tiles + pb, bg, st});
  }
  if (l1 && !l1->defer_reduce) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_l1_reduce(ws, l1->loss, l1->sqerr, st);
  }
  return hipGetLastError();
}

L1ReduceJob l1_reduce_job(const gs_workspace* ws, double* loss, double* sqerr) {
  return L1ReduceJob{(const double2*)ws->tile_loss, ws->geo.n_views,
                     ws->tiles_x * ws->tiles_y, loss, sqerr};
}

hipError_t launch_l1_reduce(const gs_workspace* ws, double* loss,
                            double* sqerr, hipStream_t st) {
  hipLaunchKernelGGL(k_l1_reduce, dim3(1), dim3(1024), 0, st,
                     l1_reduce_job(ws, loss, sqerr));
  return hipGetLastError();
}

}  // namespace gs
