// Two small reductions of the mapping iteration as device functions, so
// that the window graph can run them as extra workgroups at the end of
// another launch (dispatched last, they fill that launch's tail) instead of
// as launches of their own:
//   planar_part     the planar regulariser of the map loss (Eq. 11) and its
//                   gradient, after the compositing backward's tiles;
//   l1_reduce_part  the per-tile fused L1 losses summed into the loss, after
//                   the projection backward's Gaussians.
// The stand-alone kernels (k_planar_reg, k_l1_reduce) call the same code.
#pragma once

#include "gs_internal.h"

namespace gs {

// lambda * mean_g max(floor, min_j exp(l_gj)) over the live Gaussians, its
// gradient added to the smallest log-scale's row.
struct PlanarJob {
  const float* lsc;      // [3][cap] log-scales
  const int32_t* n_dev;
  int cap;
  float lam;
  double floor_;
  float* dlsc;           // [3][cap] gradient rows, accumulated
  double* loss;          // accumulated
};

// Workgroup blk of nblk (any size, a multiple of 64 threads) takes the
// Gaussians blk * blockDim + tid, stepping nblk * blockDim, and adds its
// share of the loss with one FP64 atomic.  sh: blockDim / 64 doubles of LDS.
__device__ inline void planar_part(const PlanarJob& j, int blk, int nblk,
                                   double* sh) {
  const int nt = blockDim.x, tid = threadIdx.x;
  const int n = min(*j.n_dev, j.cap);
  double term = 0.0;
  for (int g = blk * nt + tid; g < n; g += nblk * nt) {
    const float l0 = j.lsc[g], l1 = j.lsc[j.cap + g], l2 = j.lsc[2 * j.cap + g];
    int jm = 0;
    float lm = l0;
    if (l1 < lm) { lm = l1; jm = 1; }
    if (l2 < lm) { lm = l2; jm = 2; }
    const double sm = exp((double)lm);
    term += sm > j.floor_ ? sm : j.floor_;
    if (sm > j.floor_)
      j.dlsc[jm * j.cap + g] += (float)((double)j.lam * sm / (double)n);
  }
  for (int off = 32; off > 0; off >>= 1) term += __shfl_down(term, off, 64);
  if ((tid & 63) == 0) sh[tid >> 6] = term;
  __syncthreads();
  if (tid == 0 && n > 0) {
    double t = 0.0;
    for (int w = 0; w < nt / 64; ++w) t += sh[w];
    atomicAdd(j.loss, (double)j.lam * t / (double)n);
  }
}

PlanarJob planar_job(const gs_params* p, float lambda, float floor_,
                     gs_params* grad, double* loss);
// The stand-alone regulariser kernel on a job.
hipError_t launch_planar_job(const PlanarJob& j, hipStream_t st);

// The fused L1 term's per-tile (loss, squared error) pairs of V views of tpv
// tiles.
struct L1ReduceJob {
  const double2* tile_loss;
  int V, tpv;
  double* loss;          // accumulated
  double* sqerr;         // [V], accumulated; may be null
};

L1ReduceJob l1_reduce_job(const gs_workspace* ws, double* loss, double* sqerr);

// One workgroup (a multiple of 64 threads): wave w sums the views w,
// w + waves, ..., each over its tiles in a fixed lane order and shuffle
// tree, and thread 0 adds the views' losses in view order, so the sums do
// not depend on the workgroup size or on scheduling.  One atomic add each
// (other calls may accumulate into the same buffers).  part: blockDim / 64
// doubles of LDS.
__device__ inline void l1_reduce_part(const L1ReduceJob& j, double* part) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nw = blockDim.x >> 6;
  double total = 0.0;
  for (int k0 = 0; k0 < j.V; k0 += nw) {
    const int k = k0 + w;
    if (k < j.V) {
      double la = 0.0, lq = 0.0;
      for (int i = lane; i < j.tpv; i += 64) {
        const double2 q = j.tile_loss[(size_t)k * j.tpv + i];
        la += q.x;
        lq += q.y;
      }
      for (int off = 32; off > 0; off >>= 1) {
        la += __shfl_down(la, off, 64);
        lq += __shfl_down(lq, off, 64);
      }
      if (lane == 0) {
        part[w] = la;
        if (j.sqerr) atomicAdd(&j.sqerr[k], lq);
      }
    }
    __syncthreads();
    if (tid == 0)
      for (int i = 0; i < nw && k0 + i < j.V; ++i) total += part[i];
    __syncthreads();
  }
  if (tid == 0) atomicAdd(j.loss, total);
}

}  // namespace gs
