// The two vector phases of a CG step (Algorithm 2 in z-space) as device
// functions that take their workgroup index and the workgroup count, so that
// they run either as launches of their own or as extra workgroups of another
// launch on the same stream (the joint CG + LOBPCG driver places the update in
// the LOBPCG Rayleigh-Ritz launch, whose one workgroup leaves the GPU almost
// idle, and the direction in the LOBPCG update launch).
//
// Every workgroup sums the previous phase's partials itself, in the same
// fixed order as a one-workgroup kernel, so all take bitwise the same
// scalars; workgroup 0 records them.  Scalars that other workgroups read in
// the same launch are never overwritten in it: r^T r is kept by step parity
// (step k's value in rhob[k & 1]) and the step index comes from the host.
#pragma once

#include "gsf_internal.h"
#include "solver_state.h"

namespace gsf {

// One phase of step k for `nblk` workgroups.  pbeta reads the r^T r partials
// of the last update (upd, 2 per workgroup of that update); aupdate reads the
// apply's p^T q partials (dots, ndots of them) and writes upd.
struct CgStepArgs {
  int prec;        // GSF_F32 / GSF_F64
  int nblk;        // workgroups of the phase
  int k;           // 1-based step
  int ndots;
  void* z;
  void* r;
  void* p;
  const void* q;
  int64_t n;
  const double* dots;
  double* upd;
  CgState* st;
};

// all threads get the fixed-order sum of NV partials per workgroup
template <int NV>
__device__ __forceinline__ void reduce_all(const double* partials, int nparts, double (&t)[NV], double* red,
                                           double* bc) {
  reduce_partials<NV>(partials, nparts, NV, t, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) bc[k] = t[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) t[k] = bc[k];
}

// step k >= 1: k = 1: p = r.  k > 1: rho_k and r_k^T r_{k-1} from the last
// update's partials, the tests before step k, beta = (rho_k - r_k^T r_{k-1}) /
// rho_{k-1}, p = r + beta p.
template <typename T>
__device__ __forceinline__ void cg_pbeta_body(const T* __restrict__ r, T* __restrict__ p, int64_t n,
                                              const double* __restrict__ partials, int nparts, CgState* st, int k,
                                              int bid, int nblk) {
  __shared__ double red[32];
  __shared__ double bc[2];
  if (!st->active) return;
  const int64_t stride = (int64_t)nblk * blockDim.x;
  if (k == 1) {
    for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = r[i];
    return;
  }
  double t[2];
  reduce_all<2>(partials, nparts, t, red, bc);
  const double rho = t[0];
  const bool stop_bd = !(__builtin_isfinite(rho) && rho > st->floor);
  const bool stop_tol = !stop_bd && st->tol2 > 0.0 && rho <= st->tol2;
  if (bid == 0 && threadIdx.x == 0) {
    st->rho = rho;
    st->rhob[k & 1] = rho;
    if (stop_bd) {
      st->status = GSF_EBREAKDOWN;
      st->active = 0;
    } else if (stop_tol) {
      st->active = 0;
    }
  }
  if (stop_bd || stop_tol) return;
  const double beta = (rho - t[1]) / st->rhob[(k - 1) & 1];
  if (bid == 0 && threadIdx.x == 0) st->beta = beta;
  const T b = (T)beta;
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = r[i] + b * p[i];
}

// step k: p^T q from the apply's partials, the breakdown test, alpha =
// rho_k / p^T q; z += alpha p, r -= alpha q; partials of r_new^T r_new and
// r_new^T r_old into upd (not the buffer the dot partials are read from).
template <typename T>
__device__ __forceinline__ void cg_aupdate_body(T* __restrict__ z, T* __restrict__ r, const T* __restrict__ p,
                                                const T* __restrict__ q, int64_t n, const double* __restrict__ dots,
                                                int ndots, double* __restrict__ upd, CgState* st, int k, int bid,
                                                int nblk) {
  __shared__ double red[32];
  __shared__ double bc[2];
  if (!st->active) return;
  double t[1];
  reduce_all<1>(dots, ndots, t, red, bc);
  const double pq = t[0];
  if (!(__builtin_isfinite(pq) && pq > 0.0)) {
    if (bid == 0 && threadIdx.x == 0) {
      st->pq = pq;
      st->status = GSF_EBREAKDOWN;
      st->active = 0;
    }
    return;
  }
  const double alpha_d = st->rhob[k & 1] / pq;
  if (bid == 0 && threadIdx.x == 0) {
    st->pq = pq;
    st->alpha = alpha_d;
    st->iters = k;
    st->k = k + 1;
  }
  const T alpha = (T)alpha_d;
  const int64_t stride = (int64_t)nblk * blockDim.x;
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n; i += stride) {
    z[i] += alpha * p[i];
    const T ro = r[i];
    const T rn = ro - alpha * q[i];
    r[i] = rn;
    v[0] += (double)rn * (double)rn;
    v[1] += (double)rn * (double)ro;
  }
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    upd[2 * bid] = v[0];
    upd[2 * bid + 1] = v[1];
  }
}

__device__ __forceinline__ void cg_aupdate_step(const CgStepArgs& a, int bid) {
  if (a.prec == GSF_F32)
    cg_aupdate_body<float>((float*)a.z, (float*)a.r, (const float*)a.p, (const float*)a.q, a.n, a.dots, a.ndots,
                           a.upd, a.st, a.k, bid, a.nblk);
  else
    cg_aupdate_body<double>((double*)a.z, (double*)a.r, (const double*)a.p, (const double*)a.q, a.n, a.dots,
                            a.ndots, a.upd, a.st, a.k, bid, a.nblk);
}

// workgroups of either phase (their count multiplies the redundant partial
// reads; 512 still stream the vectors at full bandwidth)
int cg_step_blocks(int64_t n);

}  // namespace gsf
