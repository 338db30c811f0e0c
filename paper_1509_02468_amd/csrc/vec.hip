// Vector kernels of the power iteration and of CG (Algorithm 2 in z-space, and
// in x-space for the re-guided filter, whose D changes every step), with
// deterministic FP64 reductions: each workgroup writes one partial per
// quantity, and a one-workgroup kernel that follows on the stream sums them in
// workgroup order and updates the solver state.  (Handing the partials over
// inside one launch would need an agent-scope release fence per workgroup,
// which writes back the whole L2 of its XCD.)
#include <cmath>

#include "cg_step.h"
#include "gsf_internal.h"
#include "solver_state.h"

namespace gsf {
namespace {

template <typename T>
__global__ void __launch_bounds__(kThreads) scale_kernel(const T* __restrict__ in, const T* __restrict__ s,
                                                         T* __restrict__ out, int64_t n, int divide) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = divide ? in[i] / s[i] : in[i] * s[i];
}

// r holds L_sym z on entry; r <- -L_sym z; state <- rho0, breakdown floor.
template <typename T>
__global__ void __launch_bounds__(kThreads) cg_init_kernel(const T* __restrict__ z, T* __restrict__ r, int64_t n,
                                                           double* __restrict__ partials, CgState*) {
  __shared__ double red[32];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T ri = -r[i];
    r[i] = ri;
    v[0] += (double)ri * (double)ri;
    v[1] += (double)z[i] * (double)z[i];
  }
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = v[0];
    partials[2 * blockIdx.x + 1] = v[1];
  }
}

// one workgroup: rho0, breakdown floor and the tests before the first step
__global__ void __launch_bounds__(kThreads) cg_init_final_kernel(const double* __restrict__ partials, int nparts,
                                                                 CgState* st) {
  __shared__ double red[32];
  double t[2];
  reduce_partials<2>(partials, nparts, 2, t, red);
  if (threadIdx.x == 0) {
    const double rho = t[0];
    st->rho = rho;
    st->rho0 = rho;
    st->rhob[1] = rho;
    st->res0 = sqrt(rho > 0.0 ? rho : 0.0);
    st->floor = st->tau * st->tau * t[1];
    st->tol2 = st->tol > 0.0 ? st->tol * st->tol * rho : -1.0;
    st->iters = 0;
    st->k = 1;
    st->beta = 0.0;
    st->status = GSF_OK;
    st->active = 1;
    if (!(__builtin_isfinite(rho) && rho > st->floor)) {
      st->status = GSF_EBREAKDOWN;
      st->active = 0;
    } else if (st->tol2 > 0.0 && rho <= st->tol2) {
      st->active = 0;
    }
  }
}

// p = r (k = 1) or p = r + beta p
template <typename T>
__global__ void __launch_bounds__(kThreads) cg_pupdate_kernel(const T* __restrict__ r, T* __restrict__ p, int64_t n,
                                                              const CgState* st) {
  if (!st->active) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (st->k == 1) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = r[i];
  } else {
    const T beta = (T)st->beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = r[i] + beta * p[i];
  }
}

// partials[b] = sum over workgroup b of a_i b_i
template <typename T>
__global__ void __launch_bounds__(kThreads) dot_kernel(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                                       double* __restrict__ partials, const CgState* st) {
  __shared__ double red[16];
  if (st != nullptr && !st->active) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    v[0] += (double)a[i] * (double)b[i];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// one workgroup: p^T q from the partials, alpha, breakdown test
__global__ void __launch_bounds__(kThreads) cg_alpha_kernel(const double* __restrict__ partials, int nparts,
                                                            CgState* st) {
  __shared__ double red[16];
  if (!st->active) return;
  double t[1];
  reduce_partials<1>(partials, nparts, 1, t, red);
  if (threadIdx.x == 0) {
    const double pq = t[0];
    st->pq = pq;
    if (!(__builtin_isfinite(pq) && pq > 0.0)) {
      st->status = GSF_EBREAKDOWN;
      st->active = 0;
    } else {
      st->alpha = st->rho / pq;
    }
  }
}

// z += alpha p; r -= alpha q; rho_new, beta = (rho_new - r_new.r_old) / rho_old;
// then the tests that precede the next step.
template <typename T>
__global__ void __launch_bounds__(kThreads) cg_update_kernel(T* __restrict__ z, T* __restrict__ r,
                                                             const T* __restrict__ p, const T* __restrict__ q,
                                                             int64_t n, double* __restrict__ partials, CgState* st) {
  __shared__ double red[32];
  if (!st->active) return;
  const T alpha = (T)st->alpha;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    z[i] += alpha * p[i];
    const T ro = r[i];
    const T rn = ro - alpha * q[i];
    r[i] = rn;
    v[0] += (double)rn * (double)rn;
    v[1] += (double)rn * (double)ro;
  }
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = v[0];
    partials[2 * blockIdx.x + 1] = v[1];
  }
}

// one workgroup: rho_new, beta = (rho_new - r_new.r_old) / rho_old, and the
// tests that precede the next step
__global__ void __launch_bounds__(kThreads) cg_beta_kernel(const double* __restrict__ partials, int nparts,
                                                           CgState* st) {
  __shared__ double red[32];
  if (!st->active) return;
  double t[2];
  reduce_partials<2>(partials, nparts, 2, t, red);
  if (threadIdx.x == 0) {
    const double rho_old = st->rho;
    const double rho = t[0];
    st->beta = (rho - t[1]) / rho_old;
    st->rho = rho;
    st->iters = st->k;
    st->k = st->k + 1;
    if (!(__builtin_isfinite(rho) && rho > st->floor)) {
      st->status = GSF_EBREAKDOWN;
      st->active = 0;
    } else if (st->tol2 > 0.0 && rho <= st->tol2) {
      st->active = 0;
    }
  }
}

// ---- fused CG step: three launches per step instead of five ----------------
// (the bodies are in cg_step.h, shared with the joint driver's launches)
template <typename T>
__global__ void __launch_bounds__(kThreads) cg_pbeta_kernel(const T* __restrict__ r, T* __restrict__ p, int64_t n,
                                                            const double* __restrict__ partials, int nparts,
                                                            CgState* st, int k) {
  cg_pbeta_body<T>(r, p, n, partials, nparts, st, k, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) cg_aupdate_kernel(T* __restrict__ z, T* __restrict__ r,
                                                              const T* __restrict__ p, const T* __restrict__ q,
                                                              int64_t n, const double* __restrict__ dots,
                                                              int ndots, double* __restrict__ upd, CgState* st,
                                                              int k) {
  cg_aupdate_body<T>(z, r, p, q, n, dots, ndots, upd, st, k, blockIdx.x, gridDim.x);
}

// one workgroup after the last step: the final residual and its tests
__global__ void __launch_bounds__(kThreads) cg_close_kernel(const double* __restrict__ partials, int nparts,
                                                            CgState* st) {
  __shared__ double red[32];
  if (!st->active) return;
  double t[2];
  reduce_partials<2>(partials, nparts, 2, t, red);
  if (threadIdx.x == 0) {
    const double rho = t[0];
    st->rho = rho;
    if (!(__builtin_isfinite(rho) && rho > st->floor)) {
      st->status = GSF_EBREAKDOWN;
      st->active = 0;
    } else if (st->tol2 > 0.0 && rho <= st->tol2) {
      st->active = 0;
    }
  }
}

// ---- re-guided CG: Algorithm 2 in x-space, the graph rebuilt every step ----
// r holds L x0 on entry: r <- -L x0 (r_0 of Algorithm 2 with b = 0); partial
// x0^T D x0 for the breakdown floor.
template <typename T>
__global__ void __launch_bounds__(kThreads) rg_init_kernel(const T* __restrict__ x, T* __restrict__ r,
                                                           const double* __restrict__ deg, int64_t n,
                                                           double* __restrict__ partials) {
  __shared__ double red[16];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    r[i] = -r[i];
    const double xi = (double)x[i];
    v[0] += xi * deg[i] * xi;
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// one workgroup: the breakdown floor (tau^2 x0^T D x0) and the state before step 1
__global__ void __launch_bounds__(kThreads) rg_init_final_kernel(const double* __restrict__ partials, int nparts,
                                                                 CgState* st) {
  __shared__ double red[16];
  double t[1];
  reduce_partials<1>(partials, nparts, 1, t, red);
  if (threadIdx.x == 0) {
    st->floor = st->tau * st->tau * t[0];
    st->rho = 0.0;
    st->rho0 = 0.0;
    st->res0 = 0.0;
    st->tol2 = -1.0;
    st->iters = 0;
    st->k = 1;
    st->beta = 0.0;
    st->status = GSF_OK;
    st->active = 1;
  }
}

// s = D_k^-1 r with the degrees of the graph built for this step; partials of
// s^T r and (from step 2 on) s^T r_old, both from the unrounded FP64 s
template <typename T>
__global__ void __launch_bounds__(kThreads) rg_s_kernel(const T* __restrict__ r, const T* __restrict__ r_old,
                                                        const double* __restrict__ deg, T* __restrict__ s,
                                                        int64_t n, double* __restrict__ partials,
                                                        const CgState* st) {
  __shared__ double red[32];
  if (!st->active) return;
  const bool later = st->k > 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double ri = (double)r[i];
    const double si = ri / deg[i];
    s[i] = (T)si;
    v[0] += si * ri;
    if (later) v[1] += si * (double)r_old[i];
  }
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = v[0];
    partials[2 * blockIdx.x + 1] = v[1];
  }
}

// one workgroup: rho = s^T r, the tests before step k, and the flexible
// beta = (s^T r - s^T r_old) / (s_old^T r_old)
__global__ void __launch_bounds__(kThreads) rg_beta_kernel(const double* __restrict__ partials, int nparts,
                                                           CgState* st) {
  __shared__ double red[32];
  if (!st->active) return;
  double t[2];
  reduce_partials<2>(partials, nparts, 2, t, red);
  if (threadIdx.x == 0) {
    const double rho = t[0];
    const int k = st->k;
    if (k == 1) {
      st->rho0 = rho;
      st->res0 = sqrt(rho > 0.0 ? rho : 0.0);
      st->tol2 = st->tol > 0.0 ? st->tol * st->tol * rho : -1.0;
    }
    if (!(__builtin_isfinite(rho) && rho > st->floor)) {
      st->status = GSF_EBREAKDOWN;
      st->active = 0;
    } else if (st->tol2 > 0.0 && rho <= st->tol2) {
      st->active = 0;
    } else {
      st->beta = k == 1 ? 0.0 : (rho - t[1]) / st->rho;
    }
    st->rho = rho;
  }
}

// one workgroup: p^T q, alpha = rho / p^T q, breakdown test; the step is then
// counted (the update that follows completes it)
__global__ void __launch_bounds__(kThreads) rg_alpha_kernel(const double* __restrict__ partials, int nparts,
                                                            CgState* st) {
  __shared__ double red[16];
  if (!st->active) return;
  double t[1];
  reduce_partials<1>(partials, nparts, 1, t, red);
  if (threadIdx.x == 0) {
    const double pq = t[0];
    st->pq = pq;
    if (!(__builtin_isfinite(pq) && pq > 0.0)) {
      st->status = GSF_EBREAKDOWN;
      st->active = 0;
    } else {
      st->alpha = st->rho / pq;
      st->iters = st->k;
      st->k = st->k + 1;
    }
  }
}

// x += alpha p; r_old = r; r -= alpha q
template <typename T>
__global__ void __launch_bounds__(kThreads) rg_update_kernel(T* __restrict__ x, T* __restrict__ r,
                                                             T* __restrict__ r_old, const T* __restrict__ p,
                                                             const T* __restrict__ q, int64_t n, const CgState* st) {
  if (!st->active) return;
  const T alpha = (T)st->alpha;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    x[i] += alpha * p[i];
    const T ri = r[i];
    r_old[i] = ri;
    r[i] = ri - alpha * q[i];
  }
}

}  // namespace

// Workgroups of the point-wise vector kernels: one point per thread up to
// 512 workgroups (grid-stride beyond).  Small problems get many short
// workgroups rather than a few long ones: at n = 4096 the LOBPCG update took
// 10.9 us on 4 workgroups of 4 points per thread.  The cap, compared in
// alternating runs on one GPU: 512 workgroups against 256 / 768 / 1024 / 2048
// took 9.49-9.51 against 9.62 / 9.51 / 9.54-9.58 / 9.73 ms per joint CG50 +
// LOBPCG50 call at 1024^2, and 2.83-2.84 against 2.84-2.85 / 2.87-2.89 /
// 2.87-2.88 ms per LOBPCG step at 4096^2, m = 8 (fewer, longer workgroups
// leave room for the CG phase that shares the update launch).
int vec_blocks(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 512) b = 512;
  return (int)b;
}

gsf_status launch_scale(const Operator& op, const void* in, void* out, int divide, hipStream_t s) {
  const int nb = vec_blocks(op.n);
  if (op.desc.prec == GSF_F32)
    scale_kernel<float><<<nb, kThreads, 0, s>>>((const float*)in, (const float*)op.sqd, (float*)out, op.n, divide);
  else
    scale_kernel<double><<<nb, kThreads, 0, s>>>((const double*)in, (const double*)op.sqd, (double*)out, op.n,
                                                 divide);
  return launch_status();
}

gsf_status launch_cg_init(const Operator& op, const void* z, void* r, double* partials, CgState* st,
                          hipStream_t s) {
  const int nb = vec_blocks(op.n);
  if (op.desc.prec == GSF_F32)
    cg_init_kernel<float><<<nb, kThreads, 0, s>>>((const float*)z, (float*)r, op.n, partials, st);
  else
    cg_init_kernel<double><<<nb, kThreads, 0, s>>>((const double*)z, (double*)r, op.n, partials, st);
  cg_init_final_kernel<<<1, kThreads, 0, s>>>(partials, nb, st);
  return launch_status();
}

gsf_status launch_cg_pupdate(const Operator& op, const void* r, void* p, const CgState* st, hipStream_t s) {
  const int nb = vec_blocks(op.n);
  if (op.desc.prec == GSF_F32)
    cg_pupdate_kernel<float><<<nb, kThreads, 0, s>>>((const float*)r, (float*)p, op.n, st);
  else
    cg_pupdate_kernel<double><<<nb, kThreads, 0, s>>>((const double*)r, (double*)p, op.n, st);
  return launch_status();
}

gsf_status launch_dot(const Operator& op, const void* a, const void* b, double* partials, int* nparts,
                      const CgState* st, hipStream_t s) {
  const int nb = vec_blocks(op.n);
  *nparts = nb;
  if (op.desc.prec == GSF_F32)
    dot_kernel<float><<<nb, kThreads, 0, s>>>((const float*)a, (const float*)b, op.n, partials, st);
  else
    dot_kernel<double><<<nb, kThreads, 0, s>>>((const double*)a, (const double*)b, op.n, partials, st);
  return launch_status();
}

gsf_status launch_cg_alpha(const double* partials, int nparts, CgState* st, hipStream_t s) {
  cg_alpha_kernel<<<1, kThreads, 0, s>>>(partials, nparts, st);
  return launch_status();
}

gsf_status launch_cg_update(const Operator& op, void* z, void* r, const void* p, const void* q, double* partials,
                            CgState* st, hipStream_t s) {
  const int nb = vec_blocks(op.n);
  if (op.desc.prec == GSF_F32)
    cg_update_kernel<float><<<nb, kThreads, 0, s>>>((float*)z, (float*)r, (const float*)p, (const float*)q, op.n,
                                                    partials, st);
  else
    cg_update_kernel<double><<<nb, kThreads, 0, s>>>((double*)z, (double*)r, (const double*)p, (const double*)q,
                                                     op.n, partials, st);
  cg_beta_kernel<<<1, kThreads, 0, s>>>(partials, nb, st);
  return launch_status();
}

// Workgroups of the fused CG step kernels: each of them first reduces all of
// the previous kernel's partials itself (the apply's, or the update's), so
// their count multiplies those redundant reads; 512 workgroups still stream
// the vectors at full bandwidth.
int cg_step_blocks(int64_t n) {
  const int nb = vec_blocks(n);
  return nb < 512 ? nb : 512;
}

gsf_status launch_cg_pbeta(const Operator& op, const void* r, void* p, const double* upd, CgState* st, int k,
                           hipStream_t s) {
  const int nb = cg_step_blocks(op.n);
  if (op.desc.prec == GSF_F32)
    cg_pbeta_kernel<float><<<nb, kThreads, 0, s>>>((const float*)r, (float*)p, op.n, upd, nb, st, k);
  else
    cg_pbeta_kernel<double><<<nb, kThreads, 0, s>>>((const double*)r, (double*)p, op.n, upd, nb, st, k);
  return launch_status();
}

gsf_status launch_cg_aupdate(const Operator& op, void* z, void* r, const void* p, const void* q, const double* dots,
                             int ndots, double* upd, CgState* st, int k, hipStream_t s) {
  const int nb = cg_step_blocks(op.n);
  if (op.desc.prec == GSF_F32)
    cg_aupdate_kernel<float><<<nb, kThreads, 0, s>>>((float*)z, (float*)r, (const float*)p, (const float*)q, op.n,
                                                     dots, ndots, upd, st, k);
  else
    cg_aupdate_kernel<double><<<nb, kThreads, 0, s>>>((double*)z, (double*)r, (const double*)p,
                                                      (const double*)q, op.n, dots, ndots, upd, st, k);
  return launch_status();
}

gsf_status launch_cg_close(const Operator& op, const double* upd, CgState* st, hipStream_t s) {
  cg_close_kernel<<<1, kThreads, 0, s>>>(upd, cg_step_blocks(op.n), st);
  return launch_status();
}

gsf_status launch_rg_init(const Operator& op, const void* x, void* r, double* partials, CgState* st, hipStream_t s) {
  const int nb = vec_blocks(op.n);
  if (op.desc.prec == GSF_F32)
    rg_init_kernel<float><<<nb, kThreads, 0, s>>>((const float*)x, (float*)r, op.deg, op.n, partials);
  else
    rg_init_kernel<double><<<nb, kThreads, 0, s>>>((const double*)x, (double*)r, op.deg, op.n, partials);
  rg_init_final_kernel<<<1, kThreads, 0, s>>>(partials, nb, st);
  return launch_status();
}

gsf_status launch_rg_s_beta(const Operator& op, const void* r, const void* r_old, void* sv, double* partials,
                            CgState* st, hipStream_t s) {
  const int nb = vec_blocks(op.n);
  if (op.desc.prec == GSF_F32)
    rg_s_kernel<float><<<nb, kThreads, 0, s>>>((const float*)r, (const float*)r_old, op.deg, (float*)sv, op.n,
                                               partials, st);
  else
    rg_s_kernel<double><<<nb, kThreads, 0, s>>>((const double*)r, (const double*)r_old, op.deg, (double*)sv,
                                                op.n, partials, st);
  rg_beta_kernel<<<1, kThreads, 0, s>>>(partials, nb, st);
  return launch_status();
}

gsf_status launch_rg_alpha(const double* partials, int nparts, CgState* st, hipStream_t s) {
  rg_alpha_kernel<<<1, kThreads, 0, s>>>(partials, nparts, st);
  return launch_status();
}

gsf_status launch_rg_update(const Operator& op, void* x, void* r, void* r_old, const void* p, const void* q,
                            const CgState* st, hipStream_t s) {
  const int nb = vec_blocks(op.n);
  if (op.desc.prec == GSF_F32)
    rg_update_kernel<float><<<nb, kThreads, 0, s>>>((float*)x, (float*)r, (float*)r_old, (const float*)p,
                                                    (const float*)q, op.n, st);
  else
    rg_update_kernel<double><<<nb, kThreads, 0, s>>>((double*)x, (double*)r, (double*)r_old, (const double*)p,
                                                     (const double*)q, op.n, st);
  return launch_status();
}

}  // namespace gsf
