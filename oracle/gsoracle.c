/*
 * CPU FP64 oracle of the tile-based differentiable Gaussian rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * GPU library.
 *
 * What it follows:
 *   - Scene representation, Eq. 1: G(x) = exp(-1/2 (x-mu)^T Sigma^-1 (x-mu)),
 *     Sigma = R S S^T R^T, with quaternion orientation, scale vector s,
 *     opacity and colour per Gaussian.
 *   - Projection to the image plane, Eq. 2: Sigma2D = J W Sigma W^T J^T.
 *   - Alpha blending, Eq. 3: C(p) = sum_i c_i alpha_i prod_{j<i}(1 - alpha_j).
 *   - Map optimisation loss, Eq. 10-11: L1 photometric term and the planar
 *     regulariser |max(0.01, min(s))| on the smallest scale axis.
 *   - Map initialisation / insertion, Eq. 6: back-projection of patch centres
 *     T^-1 K^-1 [u, v, 1, d].
 *
 * Conventions where the paper is silent (the readings are listed in the
 * design document): OpenCV camera axes; world->camera t = R mu + t_k; pixels
 * sampled at integer coordinates; quaternion (w, x, y, z) normalised in the
 * forward pass; s = exp(log_scale); opacity = sigmoid(logit); raw RGB;
 * near plane 0.2; 1.3 x field-of-view clamp of the Jacobian; +0.3 screen
 * dilation; lambda floor 0.1; radius ceil(3 sqrt(lambda_max)); a pixel is
 * evaluated only inside the Gaussian's integer pixel box; alpha clamped to
 * alpha_max; entries with alpha < alpha_min skipped; a pixel stops (entry
 * excluded) when the transmittance would drop below T_min.
 *
 * Everything is FP64 and compiled without FMA contraction.  In "publish"
 * mode the projected record is rounded to FP32 (round-to-nearest-even) and
 * widened again, which is what the GPU path composites with.
 */
#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_EXPORT __attribute__((visibility("default")))

/* Camera as 19 doubles: R[9] (world->camera, row-major), t[3], fx, fy, cx,
 * cy, near, W, H. */
typedef struct {
  double R[9], t[3];
  double fx, fy, cx, cy, znear;
  int W, H;
} ocam;

static void cam_load(const double* c, ocam* o) {
  for (int i = 0; i < 9; ++i) o->R[i] = c[i];
  for (int i = 0; i < 3; ++i) o->t[i] = c[9 + i];
  o->fx = c[12]; o->fy = c[13]; o->cx = c[14]; o->cy = c[15];
  o->znear = c[16];
  o->W = (int)c[17]; o->H = (int)c[18];
}

#define REC_STRIDE 8   /* px py A B C opacity depth radius */

/* Everything the forward projection computes for one (view, Gaussian). */
typedef struct {
  int valid;
  double t[3];
  double s[3];
  double qraw[4], qn[4], qnorm;
  double Rq[9];
  double M[9];
  double Sig[9];       /* full symmetric 3x3 */
  double limx, limy, rx, ry, xc, yc;
  int clampx, clampy;  /* -1, 0, +1 */
  double J00, J02, J11, J12;
  double Tm[6];        /* T = J W, 2x3 row-major */
  double a, b, c;      /* dilated screen covariance */
  double det, A, B, C;
  double lam, radius;
  double px, py, opacity, depth;
  int box[4];
} proj_t;

static int finite3(double a, double b, double c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

/* Eq. 1 (covariance from quaternion and scale) and Eq. 2 (EWA projection),
 * evaluated in FP64 in a fixed operation order. */
static void project_one(const ocam* cam, double mx, double my, double mz,
                        const double l[3], const double q[4], double ologit,
                        proj_t* P) {
  const double* W = cam->R;
  memset(P, 0, sizeof(*P));
  P->valid = 1;
  P->t[0] = ((W[0] * mx + W[1] * my) + W[2] * mz) + cam->t[0];
  P->t[1] = ((W[3] * mx + W[4] * my) + W[5] * mz) + cam->t[1];
  P->t[2] = ((W[6] * mx + W[7] * my) + W[8] * mz) + cam->t[2];
  const double tx = P->t[0], ty = P->t[1], tz = P->t[2];
  if (!finite3(tx, ty, tz) || !(tz > cam->znear)) { P->valid = 0; return; }

  for (int j = 0; j < 3; ++j) P->s[j] = exp(l[j]);
  for (int j = 0; j < 4; ++j) P->qraw[j] = q[j];
  double qq = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  P->qnorm = sqrt(qq);
  if (!(P->qnorm > 0.0) || !isfinite(P->qnorm) || !finite3(P->s[0], P->s[1], P->s[2])) {
    P->valid = 0; return;
  }
  for (int j = 0; j < 4; ++j) P->qn[j] = q[j] / P->qnorm;
  const double w = P->qn[0], x = P->qn[1], y = P->qn[2], z = P->qn[3];
  double* R = P->Rq;
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P->M[3 * i + j] = R[3 * i + j] * P->s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double* Mi = &P->M[3 * i];
      const double* Mj = &P->M[3 * j];
      P->Sig[3 * i + j] = (Mi[0] * Mj[0] + Mi[1] * Mj[1]) + Mi[2] * Mj[2];
    }

  /* Perspective Jacobian at the (field-of-view clamped) mean. */
  P->limx = 1.3 * ((double)cam->W / (2.0 * cam->fx));
  P->limy = 1.3 * ((double)cam->H / (2.0 * cam->fy));
  P->rx = tx / tz;
  P->ry = ty / tz;
  double cxr = P->rx, cyr = P->ry;
  P->clampx = 0; P->clampy = 0;
  if (cxr > P->limx) { cxr = P->limx; P->clampx = 1; }
  if (cxr < -P->limx) { cxr = -P->limx; P->clampx = -1; }
  if (cyr > P->limy) { cyr = P->limy; P->clampy = 1; }
  if (cyr < -P->limy) { cyr = -P->limy; P->clampy = -1; }
  P->xc = cxr * tz;
  P->yc = cyr * tz;
  const double tz2 = tz * tz;
  P->J00 = cam->fx / tz;
  P->J02 = -(cam->fx * P->xc) / tz2;
  P->J11 = cam->fy / tz;
  P->J12 = -(cam->fy * P->yc) / tz2;
  /* T = J W (J01 = J10 = 0). */
  for (int j = 0; j < 3; ++j) {
    P->Tm[j] = P->J00 * W[j] + P->J02 * W[6 + j];
    P->Tm[3 + j] = P->J11 * W[3 + j] + P->J12 * W[6 + j];
  }
  /* U = T Sigma, then Sigma2D = U T^T, plus the 0.3 screen dilation. */
  double U[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      U[3 * i + j] = (P->Tm[3 * i + 0] * P->Sig[0 + j] +
                      P->Tm[3 * i + 1] * P->Sig[3 + j]) +
                     P->Tm[3 * i + 2] * P->Sig[6 + j];
  P->a = ((U[0] * P->Tm[0] + U[1] * P->Tm[1]) + U[2] * P->Tm[2]) + 0.3;
  P->b = (U[0] * P->Tm[3] + U[1] * P->Tm[4]) + U[2] * P->Tm[5];
  P->c = ((U[3] * P->Tm[3] + U[4] * P->Tm[4]) + U[5] * P->Tm[5]) + 0.3;
  P->det = P->a * P->c - P->b * P->b;
  if (!(P->det > 0.0) || !isfinite(P->det)) { P->valid = 0; return; }
  P->A = P->c / P->det;
  P->B = -P->b / P->det;
  P->C = P->a / P->det;
  const double mid = 0.5 * (P->a + P->c);
  P->lam = mid + sqrt(fmax(0.1, mid * mid - P->det));
  P->radius = ceil(3.0 * sqrt(P->lam));
  P->px = (cam->fx * tx) / tz + cam->cx;
  P->py = (cam->fy * ty) / tz + cam->cy;
  P->opacity = 1.0 / (1.0 + exp(-ologit));
  P->depth = tz;
  if (!isfinite(P->px) || !isfinite(P->py) || !isfinite(P->radius)) {
    P->valid = 0; return;
  }
  double ulo = fmax(0.0, ceil(P->px - P->radius));
  double uhi = fmin((double)(cam->W - 1), floor(P->px + P->radius));
  double vlo = fmax(0.0, ceil(P->py - P->radius));
  double vhi = fmin((double)(cam->H - 1), floor(P->py + P->radius));
  if (!(ulo <= uhi) || !(vlo <= vhi)) { P->valid = 0; return; }
  P->box[0] = (int)ulo; P->box[1] = (int)uhi;
  P->box[2] = (int)vlo; P->box[3] = (int)vhi;
}

static double r32(double x) { return (double)(float)x; }

/* Projects n Gaussians into one camera.  rec [n][8] receives px, py, A, B, C,
 * opacity, depth, radius (rounded to FP32 and widened when publish != 0);
 * cov [n][3] (optional) the dilated screen covariance a, b, c; box [n][4]
 * u_lo, u_hi, v_lo, v_hi; tiles [n] the number of tiles the box touches (0
 * when culled).  Returns the number of Gaussians kept. */
OR_EXPORT int or_project(int n, const double* mean, const double* lsc,
                         const double* quat, const double* opl,
                         const double* camd, int tile, int publish,
                         double* rec, double* cov, int32_t* box,
                         int32_t* tiles, int nthreads) {
  ocam cam;
  cam_load(camd, &cam);
  int kept = 0;
#ifdef _OPENMP
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) reduction(+ : kept) num_threads(nthreads)
#endif
  for (int g = 0; g < n; ++g) {
    double l[3] = {lsc[g], lsc[n + g], lsc[2 * n + g]};
    double q[4] = {quat[g], quat[n + g], quat[2 * n + g], quat[3 * n + g]};
    proj_t P;
    project_one(&cam, mean[g], mean[n + g], mean[2 * n + g], l, q, opl[g], &P);
    double* r = &rec[(size_t)g * REC_STRIDE];
    if (!P.valid) {
      for (int k = 0; k < REC_STRIDE; ++k) r[k] = 0.0;
      box[4 * g + 0] = 0; box[4 * g + 1] = -1;
      box[4 * g + 2] = 0; box[4 * g + 3] = -1;
      tiles[g] = 0;
      if (cov) { cov[3 * g] = cov[3 * g + 1] = cov[3 * g + 2] = 0.0; }
      continue;
    }
    kept += 1;
    double vals[REC_STRIDE] = {P.px, P.py, P.A, P.B, P.C, P.opacity, P.depth,
                               P.radius};
    for (int k = 0; k < REC_STRIDE; ++k)
      r[k] = (publish && k < 7) ? r32(vals[k]) : vals[k];
    if (cov) { cov[3 * g] = P.a; cov[3 * g + 1] = P.b; cov[3 * g + 2] = P.c; }
    for (int k = 0; k < 4; ++k) box[4 * g + k] = P.box[k];
    int tx0 = P.box[0] / tile, tx1 = P.box[1] / tile;
    int ty0 = P.box[2] / tile, ty1 = P.box[3] / tile;
    tiles[g] = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
  }
  return kept;
}

/* ---- Binning: duplicated (tile, depth) keys and a stable sort. ---- */

static uint32_t f32bits(double d) {
  float f = (float)d;
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

static void merge_sort_pairs(uint64_t* k, uint32_t* v, uint64_t* tk,
                             uint32_t* tv, int64_t n) {
  /* Bottom-up stable merge sort by key. */
  uint64_t *ks = k, *kd = tk;
  uint32_t *vs = v, *vd = tv;
  for (int64_t width = 1; width < n; width *= 2) {
    for (int64_t lo = 0; lo < n; lo += 2 * width) {
      int64_t mid = lo + width < n ? lo + width : n;
      int64_t hi = lo + 2 * width < n ? lo + 2 * width : n;
      int64_t i = lo, j = mid, o = lo;
      while (i < mid && j < hi) {
        if (ks[j] < ks[i]) { kd[o] = ks[j]; vd[o++] = vs[j++]; }
        else { kd[o] = ks[i]; vd[o++] = vs[i++]; }
      }
      while (i < mid) { kd[o] = ks[i]; vd[o++] = vs[i++]; }
      while (j < hi) { kd[o] = ks[j]; vd[o++] = vs[j++]; }
    }
    uint64_t* t = ks; ks = kd; kd = t;
    uint32_t* u = vs; vs = vd; vd = u;
  }
  if (ks != k) {
    memcpy(k, ks, sizeof(uint64_t) * (size_t)n);
    memcpy(v, vs, sizeof(uint32_t) * (size_t)n);
  }
}

/* Emits, for every view k, Gaussian g ascending and every tile of g's box
 * (rows ty ascending, then tx ascending), the key
 *   ((k * Ty + ty) * Tx + tx) << 32 | bits(float(depth))
 * with value g, sorts the pairs stably by key and derives each tile's
 * [start, end) range in the sorted list (start = number of keys in lower
 * tiles, so empty tiles have start == end).  keys_emit / vals_emit may be
 * NULL.  Returns the key count, or -1 when it exceeds cap.
 *
 * The keys of view k all lie in [k Ty Tx << 32, (k + 1) Ty Tx << 32) and are
 * emitted as one contiguous run after those of views < k, so the stable sort
 * of the whole array is the concatenation of the stable sorts of the views'
 * runs: each view is emitted and sorted on its own (over nthreads threads),
 * which yields exactly the array a single stable sort of all keys gives. */
OR_EXPORT int64_t or_bin_sort(int V, int n, const int32_t* box,
                              const int32_t* tiles, const double* rec,
                              int tile, int W, int H, uint64_t* keys_emit,
                              uint32_t* vals_emit, uint64_t* keys_sorted,
                              uint32_t* vals_sorted, int64_t cap,
                              uint32_t* ranges, int nthreads) {
  const int Tx = (W + tile - 1) / tile, Ty = (H + tile - 1) / tile;
  int64_t* voff = (int64_t*)calloc((size_t)V + 1, sizeof(int64_t));
  for (int k = 0; k < V; ++k) {
    int64_t t = 0;
    for (int g = 0; g < n; ++g) t += tiles[(size_t)k * n + g];
    voff[k + 1] = voff[k] + t;
  }
  const int64_t total = voff[V];
  if (total > cap) { free(voff); return -1; }
  if (nthreads < 1) nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int k = 0; k < V; ++k) {
    int64_t o = voff[k];
    for (int g = 0; g < n; ++g) {
      const int32_t* b = &box[((size_t)k * n + g) * 4];
      if (tiles[(size_t)k * n + g] == 0) continue;
      uint32_t dbits = f32bits(rec[((size_t)k * n + g) * REC_STRIDE + 6]);
      for (int ty = b[2] / tile; ty <= b[3] / tile; ++ty)
        for (int tx = b[0] / tile; tx <= b[1] / tile; ++tx) {
          uint64_t tid = (uint64_t)((int64_t)(k * Ty + ty) * Tx + tx);
          keys_sorted[o] = (tid << 32) | dbits;
          vals_sorted[o] = (uint32_t)g;
          ++o;
        }
    }
    const int64_t m = voff[k + 1] - voff[k];
    if (keys_emit)
      memcpy(keys_emit + voff[k], keys_sorted + voff[k], sizeof(uint64_t) * (size_t)m);
    if (vals_emit)
      memcpy(vals_emit + voff[k], vals_sorted + voff[k], sizeof(uint32_t) * (size_t)m);
    uint64_t* tk = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
    uint32_t* tv = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
    merge_sort_pairs(keys_sorted + voff[k], vals_sorted + voff[k], tk, tv, m);
    free(tk);
    free(tv);
  }
  free(voff);
  const int64_t nt = (int64_t)V * Tx * Ty;
  int64_t* cnt = (int64_t*)calloc((size_t)nt, sizeof(int64_t));
  for (int64_t i = 0; i < total; ++i) cnt[keys_sorted[i] >> 32] += 1;
  int64_t acc = 0;
  for (int64_t t = 0; t < nt; ++t) {
    ranges[2 * t] = (uint32_t)acc;
    acc += cnt[t];
    ranges[2 * t + 1] = (uint32_t)acc;
  }
  free(cnt);
  return total;
}

/* ---- Forward compositing (Eq. 3). ---- */

#define EPS32 5.9604644775390625e-08 /* 2^-24: unit roundoff of FP32 */

/* Decision codes used when recording / replaying the decision set. */
enum { DEC_SKIP = 0, DEC_ADMIT = 1, DEC_CLAMP = 2, DEC_STOP = 3 };

typedef struct {
  int W, H, tile, Tx, Ty, n;
  double alpha_min, T_min, alpha_max;
  double bg[3];
} fwdcfg;

/* Evaluates one (pixel, entry) pair.  Returns the decision code and fills
 * alpha, G, dx, dy; err (optional) receives a bound on the relative error an
 * FP32 evaluation of alpha can carry, and amb is set when a threshold
 * decision lies within that error. */
static int eval_pair(const fwdcfg* F, const double* r, const int32_t* b,
                     int u, int v, double T, double* alpha, double* G,
                     double* dxo, double* dyo, double* ea_out, int* amb,
                     double rT) {
  if (u < b[0] || u > b[1] || v < b[2] || v > b[3]) return DEC_SKIP;
  const double px = r[0], py = r[1], A = r[2], B = r[3], C = r[4], o = r[5];
  const double dx = px - (double)u, dy = py - (double)v;
  const double pw = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy;
  const double S = fabs(A) * dx * dx + 2.0 * fabs(B) * fabs(dx * dy) +
                   fabs(C) * dy * dy;
  /* First-order bound on the relative error of alpha evaluated in FP32 as
   * the exponential of log2(o) plus the scaled exponent: the exponent is a
   * sum of three products (about 2 eps S), its scaling and exponential add
   * about eps (|pi| + 2) <= eps (S / 2 + 2), and log2(o), rounded once and
   * added inside the sum, about 2 eps |ln o|; 4 S + 4 + 3 |ln o| keeps a
   * margin over 2.5 S + 2 + 2 |ln o|. */
  const double ea = EPS32 * (4.0 * S + 4.0 + 3.0 * fabs(log(o)));
  if (ea_out) *ea_out = ea;
  *dxo = dx; *dyo = dy;
  if (amb && pw != 0.0 && fabs(pw) <= 8.0 * EPS32 * S) *amb |= 8;
  if (pw > 0.0) return DEC_SKIP;
  const double g = exp(pw);
  const double og = o * g;
  const double a = og < F->alpha_max ? og : F->alpha_max;
  *G = g;
  const double band = fmax(1e-5, ea);
  if (amb && fabs(og - F->alpha_max) <= F->alpha_max * band) *amb |= 2;
  if (amb && fabs(a - F->alpha_min) <= F->alpha_min * band) *amb |= 1;
  if (a < F->alpha_min) return DEC_SKIP;
  *alpha = a;
  /* A clamped alpha is exactly alpha_max in any precision: no alpha error. */
  if (og > F->alpha_max && ea_out) *ea_out = 0.0;
  const double Tn = T * (1.0 - a);
  if (amb) {
    const double rTn = rT + (og > F->alpha_max ? 0.0 : ea * a / (1.0 - a)) +
                       2.0 * EPS32;
    if (fabs(Tn - F->T_min) <= F->T_min * fmax(1e-5, rTn)) *amb |= 4;
  }
  if (Tn < F->T_min) return DEC_STOP;
  return og > F->alpha_max ? DEC_CLAMP : DEC_ADMIT;
}

/* Per view: rec [V][n][8], box [V][n][4]; rgb [3][n], or [V][3][n] when
 * rgb_per_view is non-zero (the per-view colours c_i of Eq. 3 that
 * view-dependent colour gives); sorted values and
 * ranges from or_bin_sort.  Outputs image [V][3][H][W], T_final [V][H][W],
 * n_last [V][H][W] (index in the tile list of the last contributing entry,
 * plus one).  flags (optional): non-zero when a threshold decision of the
 * pixel lies within the error an FP32 evaluation can carry (bit 0: alpha vs
 * alpha_min, bit 1: the alpha clamp, bit 2: the transmittance stop, bit 3:
 * the sign of the exponent).  errb (optional): bound on the FP32 colour error of the
 * pixel; terr (optional): bound on the relative FP32 error of T_final.
 * counters (optional) [4]: examined pairs (up to and including the stop
 * entry), in-box pairs among them, contributing pairs, and in-box pairs at
 * positions before n_last (the ones a backward pass revisits).
 * dec (optional) [V][H][W][L]: decision codes recorded (dec_mode 1) or
 * replayed (dec_mode 2) per list position.
 * Dominant Gaussian (Eq. 8, optional): dom [V][H][W] receives the index of
 * the Gaussian with the largest blend weight w = alpha T of the pixel (the
 * first one on exact ties, -1 when nothing contributes), w1 that weight, w2
 * the largest weight of any other contributing Gaussian (0 if none) and werr
 * a bound on the relative FP32 error of the weights of the pixel. */
OR_EXPORT int or_forward(int V, int W, int H, int tile, int n,
                         const double* rec, const int32_t* box,
                         const double* rgb, int rgb_per_view,
                         const uint32_t* vals,
                         const uint32_t* ranges, const double* bg,
                         double alpha_min, double T_min, double alpha_max,
                         double* img, double* Tfin, int32_t* nlast,
                         uint8_t* flags, double* errb, double* terr,
                         int64_t* counters, uint8_t* dec, int L, int dec_mode,
                         int32_t* dom, double* w1, double* w2, double* werr,
                         int nthreads) {
  fwdcfg F = {W, H, tile, (W + tile - 1) / tile, (H + tile - 1) / tile, n,
              alpha_min, T_min, alpha_max, {bg[0], bg[1], bg[2]}};
  const int64_t ntiles = (int64_t)V * F.Tx * F.Ty;
  int64_t c_exam = 0, c_inbox = 0, c_contrib = 0, c_revisit = 0;
  int bad = 0;
#ifdef _OPENMP
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads) \
    reduction(+ : c_exam, c_inbox, c_contrib, c_revisit, bad)
#endif
  for (int64_t t = 0; t < ntiles; ++t) {
    const int k = (int)(t / ((int64_t)F.Tx * F.Ty));
    const int tt = (int)(t % ((int64_t)F.Tx * F.Ty));
    const int ty = tt / F.Tx, tx = tt % F.Tx;
    const uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
    const size_t cview = rgb_per_view ? (size_t)k * 3 * n : 0;
    for (int v = ty * tile; v < (ty + 1) * tile && v < H; ++v)
      for (int u = tx * tile; u < (tx + 1) * tile && u < W; ++u) {
        const size_t pix = ((size_t)k * H + v) * W + u;
        double T = 1.0, Cc[3] = {0, 0, 0}, err[3] = {0, 0, 0}, rT = 0.0;
        double wbest = 0.0, wnext = 0.0, wrel = 0.0;
        int32_t best = -1;
        int last = 0, amb = 0;
        int64_t ib = 0, ib_last = 0;
        for (uint32_t i = s; i < e; ++i) {
          const uint32_t g = vals[i];
          const double* r = &rec[((size_t)k * n + g) * REC_STRIDE];
          const int32_t* b = &box[((size_t)k * n + g) * 4];
          double alpha = 0, G = 0, dx = 0, dy = 0, ea = 0;
          int code;
          c_exam += 1;
          if (u >= b[0] && u <= b[1] && v >= b[2] && v <= b[3]) {
            c_inbox += 1;
            ib += 1;
          }
          if (dec_mode == 2) {
            if ((int)(i - s) >= L) { bad = 1; break; }
            code = dec[pix * L + (i - s)];
            if (code == DEC_STOP) break;
            if (code == DEC_SKIP) continue;
            const double ddx = r[0] - (double)u, ddy = r[1] - (double)v;
            const double pw = -0.5 * (r[2] * ddx * ddx + r[4] * ddy * ddy) -
                              r[3] * ddx * ddy;
            alpha = code == DEC_CLAMP ? alpha_max : r[5] * exp(pw);
          } else {
            code = eval_pair(&F, r, b, u, v, T, &alpha, &G, &dx, &dy, &ea,
                             &amb, rT);
            if (dec_mode == 1) {
              if ((int)(i - s) >= L) { bad = 1; break; }
              dec[pix * L + (i - s)] = (uint8_t)code;
            }
            if (code == DEC_STOP) break;
            if (code == DEC_SKIP) continue;
          }
          c_contrib += 1;
          {
            const double w = alpha * T;
            if (w > wbest) {
              wnext = wbest;
              wbest = w;
              best = (int32_t)g;
            } else if (w > wnext) {
              wnext = w;
            }
            const double we = ea + rT + 2.0 * EPS32;
            if (we > wrel) wrel = we;
          }
          for (int ch = 0; ch < 3; ++ch) {
            const double cc = rgb[cview + (size_t)ch * n + g];
            Cc[ch] += cc * alpha * T;
            err[ch] += fabs(cc) * alpha * T * (ea + rT + 4.0 * EPS32);
          }
          rT += ea * alpha / (1.0 - alpha) + 2.0 * EPS32;
          T = T * (1.0 - alpha);
          last = (int)(i - s) + 1;
          ib_last = ib;
        }
        c_revisit += ib_last;
        double eb = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
          img[(((size_t)k * 3 + ch) * H + v) * W + u] = Cc[ch] + T * F.bg[ch];
          double e = err[ch] + T * rT * fabs(F.bg[ch]) + 4.0 * EPS32 * fabs(Cc[ch]);
          if (e > eb) eb = e;
        }
        Tfin[pix] = T;
        nlast[pix] = last;
        if (flags) flags[pix] = (uint8_t)amb;
        if (errb) errb[pix] = eb;
        if (terr) terr[pix] = rT;
        if (dom) dom[pix] = best;
        if (w1) w1[pix] = wbest;
        if (w2) w2[pix] = wnext;
        if (werr) werr[pix] = wrel;
      }
  }
  if (counters) {
    counters[0] = c_exam; counters[1] = c_inbox; counters[2] = c_contrib;
    counters[3] = c_revisit;
  }
  return bad ? -1 : 0;
}

/* The front-to-back walk of or_forward at selected pixels only, listing the
 * walk: for each pixel pix[i] (flat index (k H + v) W + u), every entry of
 * its tile's list whose integer box holds the pixel, in list order, up to
 * and including the entry that stops the pixel: out_g [npix][maxw] the
 * Gaussian, out_w the blend weight alpha T it receives (0 when it does not
 * contribute), out_code the decision (DEC_SKIP, DEC_ADMIT, DEC_CLAMP,
 * DEC_STOP); out_cnt [npix] the number listed.  Returns -1 when a pixel
 * lists more than maxw entries. */
OR_EXPORT int or_pixel_walk(int V, int W, int H, int tile, int n,
                            const double* rec, const int32_t* box,
                            const uint32_t* vals, const uint32_t* ranges,
                            double alpha_min, double T_min, double alpha_max,
                            int npix, const int64_t* pix, int maxw,
                            int32_t* out_g, double* out_w, uint8_t* out_code,
                            int32_t* out_cnt) {
  fwdcfg F = {W, H, tile, (W + tile - 1) / tile, (H + tile - 1) / tile, n,
              alpha_min, T_min, alpha_max, {0.0, 0.0, 0.0}};
  int bad = 0;
  for (int q = 0; q < npix; ++q) {
    const int64_t p = pix[q];
    const int k = (int)(p / ((int64_t)W * H));
    const int rem = (int)(p % ((int64_t)W * H));
    const int v = rem / W, u = rem % W;
    if (p < 0 || k >= V) { bad = 1; out_cnt[q] = 0; continue; }
    const int64_t t = ((int64_t)k * F.Ty + v / tile) * F.Tx + u / tile;
    double T = 1.0;
    int m = 0;
    for (uint32_t i = ranges[2 * t]; i < ranges[2 * t + 1]; ++i) {
      const uint32_t g = vals[i];
      const double* r = &rec[((size_t)k * n + g) * REC_STRIDE];
      const int32_t* b = &box[((size_t)k * n + g) * 4];
      if (u < b[0] || u > b[1] || v < b[2] || v > b[3]) continue;
      double alpha = 0, G = 0, dx = 0, dy = 0;
      const int code = eval_pair(&F, r, b, u, v, T, &alpha, &G, &dx, &dy,
                                 NULL, NULL, 0.0);
      if (m >= maxw) { bad = 1; break; }
      const size_t o = (size_t)q * maxw + m;
      out_g[o] = (int32_t)g;
      out_code[o] = (uint8_t)code;
      out_w[o] = (code == DEC_ADMIT || code == DEC_CLAMP) ? alpha * T : 0.0;
      ++m;
      if (code == DEC_STOP) break;
      if (code == DEC_ADMIT || code == DEC_CLAMP) T = T * (1.0 - alpha);
    }
    out_cnt[q] = m;
  }
  return bad ? -1 : 0;
}

/* Where a Gaussian can be admitted at all: for every view k and Gaussian g
 * with a non-empty integer box, the smallest pixel rectangle holding every
 * pixel of the box at which an FP32 evaluation of alpha could reach
 * alpha_min, i.e. where o exp(pi) >= alpha_min (1 - max(1e-5, ea)) with the
 * FP32 error bound ea of the pair's alpha and pi <= 8 eps S (the exponent's
 * sign within its rounding).  rect [V][n][4] = (u_lo, u_hi, v_lo, v_hi), or
 * (0, -1, 0, -1) when no pixel qualifies.  Transmittance is ignored, so the
 * rectangle holds every pixel where the Gaussian might contribute. */
OR_EXPORT void or_admit_extent(int V, int n, const double* rec,
                               const int32_t* box, double alpha_min,
                               int32_t* rect, int nthreads) {
#ifdef _OPENMP
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
#endif
  for (int64_t kg = 0; kg < (int64_t)V * n; ++kg) {
    const double* r = &rec[(size_t)kg * REC_STRIDE];
    const int32_t* b = &box[(size_t)kg * 4];
    int32_t* o = &rect[(size_t)kg * 4];
    o[0] = 0; o[1] = -1; o[2] = 0; o[3] = -1;
    if (b[1] < b[0] || b[3] < b[2]) continue;
    const double px = r[0], py = r[1], A = r[2], B = r[3], C = r[4], op = r[5];
    int ulo = INT32_MAX, uhi = -1, vlo = INT32_MAX, vhi = -1;
    for (int v = b[2]; v <= b[3]; ++v)
      for (int u = b[0]; u <= b[1]; ++u) {
        const double dx = px - (double)u, dy = py - (double)v;
        const double pw = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy;
        const double S = fabs(A) * dx * dx + 2.0 * fabs(B) * fabs(dx * dy) +
                         fabs(C) * dy * dy;
        if (pw > 8.0 * EPS32 * S) continue;
        const double ea = EPS32 * (4.0 * S + 4.0 + 3.0 * fabs(log(op)));
        if (op * exp(pw) < alpha_min * (1.0 - fmax(1e-5, ea))) continue;
        if (u < ulo) ulo = u;
        if (u > uhi) uhi = u;
        if (v < vlo) vlo = v;
        if (v > vhi) vhi = v;
      }
    if (uhi >= 0) { o[0] = ulo; o[1] = uhi; o[2] = vlo; o[3] = vhi; }
  }
}

/* ---- Backward of the compositing (exact derivative of Eq. 3 with the
 * decision set fixed). ---- */

typedef struct {
  uint32_t g;
  double alpha, G, dx, dy, T;
  int clamped;
} admitted_t;

/* Inputs as or_forward plus dimg [V][3][H][W] = dL/dC.  Outputs (overwritten):
 * g2d [V][n][5] = dL/d(px, py, A, B, C) per view, gop [n] = dL/d opacity
 * summed over views, grgb = dL/d colour: [3][n] summed over views, or
 * [V][3][n] per view when rgb_per_view is non-zero.  The per-pair
 * transmittance is recomputed front to back (no division). */
OR_EXPORT int or_backward(int V, int W, int H, int tile, int n,
                          const double* rec, const int32_t* box,
                          const double* rgb, int rgb_per_view,
                          const uint32_t* vals,
                          const uint32_t* ranges, const double* bg,
                          double alpha_min, double T_min, double alpha_max,
                          const double* dimg, const uint8_t* dec, int L,
                          int dec_mode, double* g2d, double* gop,
                          double* grgb, int nthreads) {
  fwdcfg F = {W, H, tile, (W + tile - 1) / tile, (H + tile - 1) / tile, n,
              alpha_min, T_min, alpha_max, {bg[0], bg[1], bg[2]}};
  const int64_t ntiles = (int64_t)V * F.Tx * F.Ty;
  uint32_t maxlen = 1;
  for (int64_t t = 0; t < ntiles; ++t) {
    uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
    if (len > maxlen) maxlen = len;
  }
  if (nthreads < 1) nthreads = 1;
#ifndef _OPENMP
  nthreads = 1;
#endif
  const size_t per2d = (size_t)V * n * 5;
  double* acc2d = (double*)calloc((size_t)nthreads * per2d, sizeof(double));
  double* accop = (double*)calloc((size_t)nthreads * n, sizeof(double));
  const size_t perrgb = (size_t)3 * n * (rgb_per_view ? V : 1);
  double* accrgb = (double*)calloc((size_t)nthreads * perrgb, sizeof(double));
  int bad = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads) reduction(+ : bad)
#endif
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    admitted_t* list = (admitted_t*)malloc(sizeof(admitted_t) * maxlen);
    double* my2d = acc2d + (size_t)tid * per2d;
    double* myop = accop + (size_t)tid * n;
    double* myrgb = accrgb + (size_t)tid * perrgb;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t t = 0; t < ntiles; ++t) {
      const int k = (int)(t / ((int64_t)F.Tx * F.Ty));
      const int tt = (int)(t % ((int64_t)F.Tx * F.Ty));
      const int ty = tt / F.Tx, tx = tt % F.Tx;
      const uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
      const size_t cview = rgb_per_view ? (size_t)k * 3 * n : 0;
      for (int v = ty * tile; v < (ty + 1) * tile && v < H; ++v)
        for (int u = tx * tile; u < (tx + 1) * tile && u < W; ++u) {
          const size_t pix = ((size_t)k * H + v) * W + u;
          /* Forward again, keeping every admitted entry. */
          double T = 1.0;
          int m = 0;
          for (uint32_t i = s; i < e; ++i) {
            const uint32_t g = vals[i];
            const double* r = &rec[((size_t)k * n + g) * REC_STRIDE];
            const int32_t* b = &box[((size_t)k * n + g) * 4];
            double alpha = 0, G = 0, dx = 0, dy = 0;
            int code;
            if (dec_mode == 2) {
              if ((int)(i - s) >= L) { bad = 1; break; }
              code = dec[pix * L + (i - s)];
              if (code == DEC_STOP) break;
              if (code == DEC_SKIP) continue;
              dx = r[0] - (double)u; dy = r[1] - (double)v;
              const double pw = -0.5 * (r[2] * dx * dx + r[4] * dy * dy) -
                                r[3] * dx * dy;
              G = exp(pw);
              alpha = code == DEC_CLAMP ? alpha_max : r[5] * G;
            } else {
              code = eval_pair(&F, r, b, u, v, T, &alpha, &G, &dx, &dy, NULL,
                               NULL, 0.0);
              if (code == DEC_STOP) break;
              if (code == DEC_SKIP) continue;
            }
            list[m].g = g; list[m].alpha = alpha; list[m].G = G;
            list[m].dx = dx; list[m].dy = dy; list[m].T = T;
            list[m].clamped = code == DEC_CLAMP;
            ++m;
            T = T * (1.0 - alpha);
          }
          const double Tfinal = T;
          double gC[3];
          for (int ch = 0; ch < 3; ++ch)
            gC[ch] = dimg[(((size_t)k * 3 + ch) * H + v) * W + u];
          /* Back to front: S is the colour accumulated behind entry i,
           * normalised by the transmittance just behind it. */
          double S[3] = {0, 0, 0};
          for (int j = m - 1; j >= 0; --j) {
            const admitted_t* P = &list[j];
            const uint32_t g = P->g;
            const double* r = &rec[((size_t)k * n + g) * REC_STRIDE];
            double dalpha = 0.0;
            for (int ch = 0; ch < 3; ++ch) {
              const double cc = rgb[cview + (size_t)ch * n + g];
              myrgb[cview + (size_t)ch * n + g] += P->alpha * P->T * gC[ch];
              dalpha += P->T * (cc - S[ch]) * gC[ch];
              dalpha -= Tfinal / (1.0 - P->alpha) * F.bg[ch] * gC[ch];
              S[ch] = P->alpha * cc + (1.0 - P->alpha) * S[ch];
            }
            if (P->clamped) continue;
            /* alpha = o * G, G = exp(pw). */
            const double o = r[5], A = r[2], B = r[3], C = r[4];
            myop[g] += P->G * dalpha;
            const double dpw = dalpha * o * P->G;
            const double dx = P->dx, dy = P->dy;
            double* d = &my2d[((size_t)k * n + g) * 5];
            d[0] += dpw * (-(A * dx + B * dy));
            d[1] += dpw * (-(C * dy + B * dx));
            d[2] += dpw * (-0.5 * dx * dx);
            d[3] += dpw * (-dx * dy);
            d[4] += dpw * (-0.5 * dy * dy);
          }
        }
    }
    free(list);
  }
  memset(g2d, 0, sizeof(double) * per2d);
  memset(gop, 0, sizeof(double) * (size_t)n);
  memset(grgb, 0, sizeof(double) * perrgb);
  for (int th = 0; th < nthreads; ++th) {
    for (size_t i = 0; i < per2d; ++i) g2d[i] += acc2d[(size_t)th * per2d + i];
    for (int i = 0; i < n; ++i) gop[i] += accop[(size_t)th * n + i];
    for (size_t i = 0; i < perrgb; ++i)
      grgb[i] += accrgb[(size_t)th * perrgb + i];
  }
  free(acc2d); free(accop); free(accrgb);
  return bad ? -1 : 0;
}

/* ---- Backward of the projection (chain rule through Eq. 2 and Eq. 1). ---- */

/* Chain rule of one view: adds to dmu [3], dl [3], dq [4] the gradients that
 * the screen-space gradient d = dL/d(px, py, A, B, C) of view cam sends back
 * through Eq. 2 (conic -> screen covariance -> Jacobian, world-to-camera
 * rotation and camera-space mean) and Eq. 1 (covariance -> rotation and
 * scale -> quaternion and log-scale).  Linear in d. */
static void chain_view(const ocam* cam, const proj_t* P, const double* d,
                       double* dmu, double* dl, double* dq) {
  const double dpx = d[0], dpy = d[1], dA = d[2], dB = d[3], dC = d[4];
  if (dpx == 0.0 && dpy == 0.0 && dA == 0.0 && dB == 0.0 && dC == 0.0)
    return;
  const double a = P->a, b = P->b, c = P->c, det = P->det;
  const double det2 = det * det;
  /* conic (A, B, C) = (c, -b, a) / det  ->  (a, b, c) */
  const double da = dA * (-c * c / det2) + dB * (b * c / det2) +
                    dC * (1.0 / det - a * c / det2);
  const double db = dA * (2.0 * b * c / det2) +
                    dB * (-1.0 / det - 2.0 * b * b / det2) +
                    dC * (2.0 * a * b / det2);
  const double dc = dA * (1.0 / det - c * a / det2) + dB * (b * a / det2) +
                    dC * (-a * a / det2);
  /* a = T0 Sig T0^T + 0.3, b = T0 Sig T1^T, c = T1 Sig T1^T + 0.3 */
  const double* T0 = &P->Tm[0];
  const double* T1 = &P->Tm[3];
  double ST0[3], ST1[3];
  for (int i = 0; i < 3; ++i) {
    ST0[i] = P->Sig[3 * i] * T0[0] + P->Sig[3 * i + 1] * T0[1] +
             P->Sig[3 * i + 2] * T0[2];
    ST1[i] = P->Sig[3 * i] * T1[0] + P->Sig[3 * i + 1] * T1[1] +
             P->Sig[3 * i + 2] * T1[2];
  }
  double GS[9];  /* dL/dSig_mn treating all nine entries as free */
  for (int m = 0; m < 3; ++m)
    for (int nn = 0; nn < 3; ++nn)
      GS[3 * m + nn] = da * T0[m] * T0[nn] + db * T0[m] * T1[nn] +
                       dc * T1[m] * T1[nn];
  double dT0[3], dT1[3];
  for (int m = 0; m < 3; ++m) {
    dT0[m] = 2.0 * da * ST0[m] + db * ST1[m];
    dT1[m] = db * ST0[m] + 2.0 * dc * ST1[m];
  }
  /* T = J W */
  const double* Wm = cam->R;
  double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
  for (int j = 0; j < 3; ++j) {
    dJ00 += dT0[j] * Wm[j];
    dJ02 += dT0[j] * Wm[6 + j];
    dJ11 += dT1[j] * Wm[3 + j];
    dJ12 += dT1[j] * Wm[6 + j];
  }
  const double tx = P->t[0], ty = P->t[1], tz = P->t[2];
  const double tz2 = tz * tz, tz3 = tz2 * tz;
  double dt[3] = {0, 0, 0};
  /* J00 = fx/tz, J11 = fy/tz */
  dt[2] += dJ00 * (-cam->fx / tz2) + dJ11 * (-cam->fy / tz2);
  /* J02 = -fx xc / tz^2, xc = tx (unclamped) or +-limx tz (clamped) */
  const double dxc_dtx = P->clampx ? 0.0 : 1.0;
  const double dxc_dtz = P->clampx ? (double)P->clampx * P->limx : 0.0;
  const double dyc_dty = P->clampy ? 0.0 : 1.0;
  const double dyc_dtz = P->clampy ? (double)P->clampy * P->limy : 0.0;
  dt[0] += dJ02 * (-cam->fx / tz2) * dxc_dtx;
  dt[2] += dJ02 * (-cam->fx / tz2 * dxc_dtz + 2.0 * cam->fx * P->xc / tz3);
  dt[1] += dJ12 * (-cam->fy / tz2) * dyc_dty;
  dt[2] += dJ12 * (-cam->fy / tz2 * dyc_dtz + 2.0 * cam->fy * P->yc / tz3);
  /* px = fx tx / tz + cx, py = fy ty / tz + cy */
  dt[0] += dpx * cam->fx / tz;
  dt[2] += dpx * (-cam->fx * tx / tz2);
  dt[1] += dpy * cam->fy / tz;
  dt[2] += dpy * (-cam->fy * ty / tz2);
  /* t = W mu + t_k */
  for (int j = 0; j < 3; ++j)
    dmu[j] += Wm[j] * dt[0] + Wm[3 + j] * dt[1] + Wm[6 + j] * dt[2];
  /* Sig = M M^T: dM = (GS + GS^T) M */
  double dM[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int m = 0; m < 3; ++m)
        acc += (GS[3 * i + m] + GS[3 * m + i]) * P->M[3 * m + j];
      dM[3 * i + j] = acc;
    }
  /* M = R diag(s) */
  double dR[9], ds[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      dR[3 * i + j] = dM[3 * i + j] * P->s[j];
      ds[j] += dM[3 * i + j] * P->Rq[3 * i + j];
    }
  for (int j = 0; j < 3; ++j) dl[j] += ds[j] * P->s[j];
  /* R(w, x, y, z) of the normalised quaternion */
  const double w = P->qn[0], x = P->qn[1], y = P->qn[2], z = P->qn[3];
  double dqn[4];
  dqn[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] -
                  y * dR[6] + x * dR[7]);
  dqn[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - w * dR[5] +
                  z * dR[6] + w * dR[7]) -
           4.0 * x * (dR[4] + dR[8]);
  dqn[2] = 2.0 * (x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] -
                  w * dR[6] + z * dR[7]) -
           4.0 * y * (dR[0] + dR[8]);
  dqn[3] = 2.0 * (-w * dR[1] + x * dR[2] + w * dR[3] + y * dR[5] +
                  x * dR[6] + y * dR[7]) -
           4.0 * z * (dR[0] + dR[4]);
  /* qn = q / |q| */
  const double dot = dqn[0] * w + dqn[1] * x + dqn[2] * y + dqn[3] * z;
  for (int j = 0; j < 4; ++j)
    dq[j] += (dqn[j] - P->qn[j] * dot) / P->qnorm;
}

/* cams [V][19]; g2d [V][n][5]; gop [n]; grgb_in [3][n].  Outputs
 * (overwritten) in planar layout: gmean [3][n], glsc [3][n], gquat [4][n],
 * gopl [n], grgb [3][n]. */
OR_EXPORT int or_project_bwd(int V, int n, const double* mean,
                             const double* lsc, const double* quat,
                             const double* opl,
                             const double* cams, const double* g2d,
                             const double* gop, const double* grgb_in,
                             double* gmean, double* glsc, double* gquat,
                             double* gopl, double* grgb, int nthreads) {
#ifdef _OPENMP
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
  for (int g = 0; g < n; ++g) {
    double dmu[3] = {0, 0, 0}, dl[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0};
    const double l[3] = {lsc[g], lsc[n + g], lsc[2 * n + g]};
    const double q[4] = {quat[g], quat[n + g], quat[2 * n + g],
                         quat[3 * n + g]};
    for (int k = 0; k < V; ++k) {
      ocam cam;
      cam_load(&cams[(size_t)k * 19], &cam);
      proj_t P;
      project_one(&cam, mean[g], mean[n + g], mean[2 * n + g], l, q, opl[g],
                  &P);
      if (!P.valid) continue;
      chain_view(&cam, &P, &g2d[((size_t)k * n + g) * 5], dmu, dl, dq);
    }
    for (int j = 0; j < 3; ++j) {
      gmean[(size_t)j * n + g] = dmu[j];
      glsc[(size_t)j * n + g] = dl[j];
      grgb[(size_t)j * n + g] = grgb_in[(size_t)j * n + g];
    }
    for (int j = 0; j < 4; ++j) gquat[(size_t)j * n + g] = dq[j];
    const double o = 1.0 / (1.0 + exp(-opl[g]));
    gopl[g] = gop[g] * o * (1.0 - o);
  }
  return 0;
}

/* Magnitudes through the projection backward: for non-negative per-view
 * screen-space magnitudes x2d [V][n][5] (for instance |dL/d(px, py, A, B,
 * C)|), every output receives the sum over views k and screen quantities c
 * of |d output / d g2d[k][g][c]| x2d[k][g][c] -- the sum of the absolute
 * values of the chain-rule terms that the projection backward adds up (the
 * chain is linear in g2d, so each column is the chain of one unit input).
 * The opacity magnitude xop [n] is scaled by o (1 - o) and the colour
 * magnitude xrgb [3][n] passed through.  Outputs in the layout of
 * or_project_bwd. */
OR_EXPORT int or_project_bwd_abs(int V, int n, const double* mean,
                                 const double* lsc, const double* quat,
                                 const double* opl, const double* cams,
                                 const double* x2d, const double* xop,
                                 const double* xrgb_in, double* amean,
                                 double* alsc, double* aquat, double* aopl,
                                 double* argb, int nthreads) {
#ifdef _OPENMP
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
  for (int g = 0; g < n; ++g) {
    double amu[3] = {0, 0, 0}, al[3] = {0, 0, 0}, aq[4] = {0, 0, 0, 0};
    const double l[3] = {lsc[g], lsc[n + g], lsc[2 * n + g]};
    const double q[4] = {quat[g], quat[n + g], quat[2 * n + g],
                         quat[3 * n + g]};
    for (int k = 0; k < V; ++k) {
      const double* e = &x2d[((size_t)k * n + g) * 5];
      if (e[0] == 0.0 && e[1] == 0.0 && e[2] == 0.0 && e[3] == 0.0 &&
          e[4] == 0.0)
        continue;
      ocam cam;
      cam_load(&cams[(size_t)k * 19], &cam);
      proj_t P;
      project_one(&cam, mean[g], mean[n + g], mean[2 * n + g], l, q, opl[g],
                  &P);
      if (!P.valid) continue;
      for (int c = 0; c < 5; ++c) {
        if (e[c] == 0.0) continue;
        double d[5] = {0, 0, 0, 0, 0};
        d[c] = e[c];
        double dmu[3] = {0, 0, 0}, dl[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0};
        chain_view(&cam, &P, d, dmu, dl, dq);
        for (int j = 0; j < 3; ++j) {
          amu[j] += fabs(dmu[j]);
          al[j] += fabs(dl[j]);
        }
        for (int j = 0; j < 4; ++j) aq[j] += fabs(dq[j]);
      }
    }
    for (int j = 0; j < 3; ++j) {
      amean[(size_t)j * n + g] = amu[j];
      alsc[(size_t)j * n + g] = al[j];
      argb[(size_t)j * n + g] = xrgb_in[(size_t)j * n + g];
    }
    for (int j = 0; j < 4; ++j) aquat[(size_t)j * n + g] = aq[j];
    const double o = 1.0 / (1.0 + exp(-opl[g]));
    aopl[g] = xop[g] * o * (1.0 - o);
  }
  return 0;
}

/* ---- Loss terms (Eq. 10-11). ---- */

/* Sum over views of lambda * mean over 3HW of |img - target|; dimg receives
 * lambda * sign(img - target) / (3HW) with sign(0) = 0.  Returns the loss. */
OR_EXPORT double or_l1(int V, int H, int W, const double* img,
                       const double* target, double lam, double* dimg) {
  const double inv = 1.0 / (3.0 * (double)H * (double)W);
  double loss = 0.0;
  for (int k = 0; k < V; ++k) {
    double s = 0.0;
    for (size_t i = 0; i < (size_t)3 * H * W; ++i) {
      const size_t j = (size_t)k * 3 * H * W + i;
      const double d = img[j] - target[j];
      s += fabs(d);
      dimg[j] = d > 0 ? lam * inv : (d < 0 ? -lam * inv : 0.0);
    }
    loss += lam * s * inv;
  }
  return loss;
}

/* Planar regulariser: lambda * mean_g max(floor, min_j exp(l_gj)).  Adds its
 * gradient to glsc [3][n] (only on the smallest axis, lowest index on ties,
 * and only where that scale exceeds the floor).  Returns the term. */
OR_EXPORT double or_planar_reg(int n, const double* lsc, double lam,
                               double floor_, double* glsc) {
  if (n <= 0) return 0.0;
  double acc = 0.0;
  for (int g = 0; g < n; ++g) {
    int jm = 0;
    double sm = exp(lsc[g]);
    for (int j = 1; j < 3; ++j) {
      const double s = exp(lsc[(size_t)j * n + g]);
      if (s < sm) { sm = s; jm = j; }
    }
    acc += sm > floor_ ? sm : floor_;
    if (sm > floor_) glsc[(size_t)jm * n + g] += lam * sm / (double)n;
  }
  return lam * acc / (double)n;
}

/* Adam update of one parameter array (the optimiser the paper leaves open). */
OR_EXPORT void or_adam(int64_t n, double* p, const double* g, double* m,
                       double* v, double lr, double b1, double b2, double eps,
                       int step) {
  const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}

/* ---- Keyframe insertion (Eq. 6, with the accumulated-alpha mask). ---- */

/* Candidates are the 3x3 pixel patch around each centre (u, v) of pts_uvd
 * [K][3] = (u, v, inverse depth), visited patch by patch, pixels row-major
 * (dv = -1..1, then du = -1..1); centre_only visits just the centre.  A
 * candidate is kept when it lies inside the image and 1 - T_final <=
 * alpha_skip.  A kept candidate becomes a Gaussian at
 * X = R^T (((u - cx) / fx / d, (v - cy) / fy / d, 1 / d) - t), with the
 * keyframe colour at its pixel, opacity logit 0, identity rotation and
 * isotropic log-scale log(z / fx).  Outputs [3][cap] etc. in insertion
 * order; src [cap] is the candidate index (patch * 9 + pixel).  Returns the
 * number kept (which may exceed cap; only cap are written). */
/* Back-projection of a candidate pixel with inverse depth d (Eq. 6). */
static void back_project(const ocam* cam, int u, int v, double d, double* X) {
  const double z = 1.0 / d;
  const double xc[3] = {((double)u - cam->cx) / cam->fx * z,
                        ((double)v - cam->cy) / cam->fy * z, z};
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int j = 0; j < 3; ++j) s += cam->R[3 * j + i] * (xc[j] - cam->t[j]);
    X[i] = s;
  }
}

/* Distance test of Eq. 7: for every insertion candidate (index patch * per
 * + pixel, per = 9, or 1 with centre_only), the squared distance from its
 * back-projected point to the nearest of the n existing means [3][n]
 * (FP64, (x - m)^2 summed over the axes in order); -1 for candidates outside
 * the image or with d <= 0; +inf when n == 0. */
OR_EXPORT void or_nearest(const double* camd, const double* pts, int K,
                          int centre_only, const double* means, int n,
                          double* out_d2, int nthreads) {
  ocam cam;
  cam_load(camd, &cam);
  const int per = centre_only ? 1 : 9;
#ifdef _OPENMP
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
#endif
  for (int c = 0; c < K * per; ++c) {
    const int k = c / per, p = centre_only ? 4 : c % per;
    const double d = pts[3 * k + 2];
    const int u = (int)pts[3 * k] + (p % 3) - 1, v = (int)pts[3 * k + 1] + (p / 3) - 1;
    if (u < 0 || u >= cam.W || v < 0 || v >= cam.H || !(d > 0.0)) {
      out_d2[c] = -1.0;
      continue;
    }
    double X[3];
    back_project(&cam, u, v, d, X);
    double best = INFINITY;
    for (int g = 0; g < n; ++g) {
      const double a = X[0] - means[g], b = X[1] - means[(size_t)n + g],
                   e = X[2] - means[2 * (size_t)n + g];
      const double d2 = (a * a + b * b) + e * e;
      if (d2 < best) best = d2;
    }
    out_d2[c] = best;
  }
}

/* Insertion (Eq. 6).  The keep test is the accumulated-alpha mask
 * (1 - kf_T(u, v) <= alpha_skip) or, when cand_d2 is given, the distance
 * test of Eq. 7 (cand_d2[c] > tau2, cand_d2 from or_nearest). */
OR_EXPORT int or_insert(const double* camd, const double* kf_rgb,
                        const double* kf_T, const double* pts, int K,
                        double alpha_skip, int centre_only, int cap,
                        double* out_mean, double* out_lsc, double* out_quat,
                        double* out_opl, double* out_rgb, int32_t* src,
                        const double* cand_d2, double tau2) {
  ocam cam;
  cam_load(camd, &cam);
  int cnt = 0;
  const int per = centre_only ? 1 : 9;
  for (int k = 0; k < K; ++k) {
    const double uc = pts[3 * k], vc = pts[3 * k + 1], d = pts[3 * k + 2];
    for (int p = 0; p < 9; ++p) {
      if (centre_only && p != 4) continue;
      const int u = (int)uc + (p % 3) - 1, v = (int)vc + (p / 3) - 1;
      if (u < 0 || u >= cam.W || v < 0 || v >= cam.H) continue;
      if (!(d > 0.0)) continue;
      if (cand_d2) {
        if (!(cand_d2[k * per + (centre_only ? 0 : p)] > tau2)) continue;
      } else {
        const double acc = 1.0 - kf_T[(size_t)v * cam.W + u];
        if (acc > alpha_skip) continue;
      }
      if (cnt < cap) {
        const double z = 1.0 / d;
        double X[3];
        back_project(&cam, u, v, d, X);
        for (int i = 0; i < 3; ++i) {
          out_mean[(size_t)i * cap + cnt] = X[i];
          out_lsc[(size_t)i * cap + cnt] = log(z / cam.fx);
          out_rgb[(size_t)i * cap + cnt] =
              kf_rgb[((size_t)i * cam.H + v) * cam.W + u];
        }
        out_quat[cnt] = 1.0;
        out_quat[(size_t)cap + cnt] = 0.0;
        out_quat[2 * (size_t)cap + cnt] = 0.0;
        out_quat[3 * (size_t)cap + cnt] = 0.0;
        out_opl[cnt] = 0.0;
        src[cnt] = k * 9 + p;
      }
      ++cnt;
    }
  }
  return cnt;
}
