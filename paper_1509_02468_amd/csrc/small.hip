// Small 1D signals in one workgroup: when a signal fits in LDS, the whole
// filter runs in one launch (the multi-kernel path pays a few launches and a
// grid-wide reduction per step, which dominate at a few thousand samples).
//
// Re-guided BF power filter (Sections 2-3, eq. (3) with the previous result
// as the guidance): each pass evaluates the weights of eq. (2) from the
// current iterate and takes x_i <- x_i - (1/d_i) sum_j w_ij (x_i - x_j), the
// random-walk form D^-1 W x of the chosen normalisation (d_i = 1 + sum_j w_ij
// with the self-loop, or diag L_i = sum_{j != i} w_ij, taken as 1 where it is
// 0).  Weights and sums are FP64; the iterate is stored in the data type after
// every pass (the guidance of the next pass is the stored iterate).
#include <cmath>

#include "gsf_internal.h"
#include "solver_state.h"

namespace gsf {
namespace {

constexpr int kSmallThreads = 1024;

template <typename T>
struct SmallMax {
  static constexpr int n = 65536 / (int)sizeof(T);  // two buffers in 128 KB of LDS
};

template <typename T>
__global__ void __launch_bounds__(kSmallThreads) rg_power1d_small_kernel(const T* __restrict__ x0,
                                                                         T* __restrict__ xout, int n, int kmax,
                                                                         int r, double cs, double cr, int diagl) {
  __shared__ T buf[2 * SmallMax<T>::n];
  T* a = buf;
  T* b = buf + SmallMax<T>::n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = x0[i];
  __syncthreads();
  for (int k = 0; k < kmax; ++k) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double gi = (double)a[i];
      double acc = 0.0, ws = 0.0;
      for (int o = 1; o <= r; ++o) {
        const double sp = (double)(o * o) * cs;
        if (i + o < n) {
          const double dg = gi - (double)a[i + o];
          const double w = exp(-(sp + dg * dg * cr));
          ws += w;
          acc = fma(w, dg, acc);
        }
        if (i - o >= 0) {
          const double dg = gi - (double)a[i - o];
          const double w = exp(-(sp + dg * dg * cr));
          ws += w;
          acc = fma(w, dg, acc);
        }
      }
      double d = diagl ? ws : 1.0 + ws;
      if (d == 0.0) d = 1.0;
      b[i] = (T)(gi - acc / d);
    }
    __syncthreads();
    T* t = a;
    a = b;
    b = t;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) xout[i] = a[i];
}

inline double inv_two_sigma2(double s) { return std::isinf(s) ? 0.0 : 1.0 / (2.0 * s * s); }

// CG filter (Algorithm 2 in z-space, as gsf_cg_filter) of a built 1D BF
// operator in one workgroup: every thread keeps its points' z, r, p, q in
// registers (point i = thread + 1024 j, j < kPts), u = D^-1/2 v is staged in
// LDS for the neighbour reads, the weights come from the operator's planes
// (own entry at i, mirrored at i - o; the pads are zeros), and the scalars are
// FP64 block sums broadcast through LDS.  The same recurrences, tests and
// state as the multi-kernel filter; the state is written once at the end.
constexpr int kPts = 8;

template <typename T>
__device__ __forceinline__ double block_all(double v, double* red, double* bc) {
  double t[1] = {v};
  block_sum<1>(t, red);
  if (threadIdx.x == 0) bc[0] = t[0];
  __syncthreads();
  return bc[0];
}

template <typename T>
__device__ __forceinline__ void block_all2(double& a, double& b, double* red, double* bc) {
  double t[2] = {a, b};
  block_sum<2>(t, red);
  if (threadIdx.x == 0) {
    bc[0] = t[0];
    bc[1] = t[1];
  }
  __syncthreads();
  a = bc[0];
  b = bc[1];
}

template <typename T>
__global__ void __launch_bounds__(kSmallThreads) cg1d_small_kernel(const T* __restrict__ planes, int64_t pstride,
                                                                   int64_t ppad, int r, const T* __restrict__ isqd,
                                                                   const T* __restrict__ sqd,
                                                                   const T* __restrict__ x0, T* __restrict__ xout,
                                                                   int n, int kmax, CgState* st) {
  __shared__ T u[kSmallThreads * kPts];
  __shared__ double red[32];
  __shared__ double bc[2];
  const int tid = threadIdx.x;
  T z[kPts], rv[kPts], p[kPts], q[kPts], is[kPts];
  // q = L_sym v: stage u = D^-1/2 v, then q_i = is_i sum_o w (u_i - u_j)
  auto apply = [&](const T (&v)[kPts]) {
#pragma unroll
    for (int j = 0; j < kPts; ++j) {
      const int i = tid + j * kSmallThreads;
      if (i < n) u[i] = v[j] * is[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPts; ++j) {
      const int i = tid + j * kSmallThreads;
      T acc = T(0);
      if (i < n) {
        const T ui = u[i];
        for (int o = 1; o <= r; ++o) {
          const T* pl = planes + ppad + (int64_t)(o - 1) * pstride;
          const T wo = pl[i], wm = pl[i - o];
          const T uo = i + o < n ? u[i + o] : T(0);
          const T um = i - o >= 0 ? u[i - o] : T(0);
          acc = fma(wo, ui - uo, acc);
          acc = fma(wm, ui - um, acc);
        }
      }
      q[j] = is[j] * acc;
    }
  };
  double zz = 0.0, rho = 0.0;
#pragma unroll
  for (int j = 0; j < kPts; ++j) {
    const int i = tid + j * kSmallThreads;
    is[j] = i < n ? isqd[i] : T(0);
    z[j] = i < n ? x0[i] * sqd[i] : T(0);
    zz += (double)z[j] * (double)z[j];
  }
  apply(z);
#pragma unroll
  for (int j = 0; j < kPts; ++j) {
    rv[j] = -q[j];
    rho += (double)rv[j] * (double)rv[j];
  }
  block_all2<T>(rho, zz, red, bc);
  const double tol = st->tol, tau = st->tau;
  const double floor = tau * tau * zz;
  const double tol2 = tol > 0.0 ? tol * tol * rho : -1.0;
  const double rho0 = rho;
  int status = GSF_OK, active = 1, iters = 0;
  if (!(__builtin_isfinite(rho) && rho > floor)) {
    status = GSF_EBREAKDOWN;
    active = 0;
  } else if (tol2 > 0.0 && rho <= tol2) {
    active = 0;
  }
  double beta = 0.0;
  for (int k = 1; k <= kmax && active; ++k) {
#pragma unroll
    for (int j = 0; j < kPts; ++j) p[j] = k == 1 ? rv[j] : rv[j] + (T)beta * p[j];
    __syncthreads();  // every read of u by the last apply is done
    apply(p);
    double pq = 0.0;
#pragma unroll
    for (int j = 0; j < kPts; ++j) pq += (double)p[j] * (double)q[j];
    pq = block_all<T>(pq, red, bc);
    if (!(__builtin_isfinite(pq) && pq > 0.0)) {
      status = GSF_EBREAKDOWN;
      active = 0;
      break;
    }
    const T alpha = (T)(rho / pq);
    double rn2 = 0.0, rno = 0.0;
#pragma unroll
    for (int j = 0; j < kPts; ++j) {
      z[j] += alpha * p[j];
      const T ro = rv[j];
      const T rn = ro - alpha * q[j];
      rv[j] = rn;
      rn2 += (double)rn * (double)rn;
      rno += (double)rn * (double)ro;
    }
    block_all2<T>(rn2, rno, red, bc);
    beta = (rn2 - rno) / rho;
    rho = rn2;
    iters = k;
    if (!(__builtin_isfinite(rho) && rho > floor)) {
      status = GSF_EBREAKDOWN;
      active = 0;
    } else if (tol2 > 0.0 && rho <= tol2) {
      active = 0;
    }
  }
#pragma unroll
  for (int j = 0; j < kPts; ++j) {
    const int i = tid + j * kSmallThreads;
    if (i < n) xout[i] = z[j] / sqd[i];
  }
  if (tid == 0) {
    st->rho = rho;
    st->rho0 = rho0;
    st->res0 = sqrt(rho0 > 0.0 ? rho0 : 0.0);
    st->floor = floor;
    st->tol2 = tol2;
    st->iters = iters;
    st->k = iters + 1;
    st->status = status;
    st->active = active;
  }
}

}  // namespace

// One-launch re-guided BF power filter for a 1D signal that fits in LDS;
// false (nothing launched) when the descriptor is not of that kind.
bool launch_rg_power_small(const gsf_operator_desc& d, const void* x0, void* x_out, int kmax, hipStream_t s) {
  const int64_t n = d.dims[0];
  if (d.kind != GSF_BF || d.ndim != 1 || desc_channels(d) != 1 || kmax < 1) return false;
  const double cs = inv_two_sigma2(d.sigma_d), cr = inv_two_sigma2(d.sigma_r);
  const int diagl = d.norm == GSF_NORM_DIAGL ? 1 : 0;
  if (d.prec == GSF_F32) {
    if (n > SmallMax<float>::n) return false;
    rg_power1d_small_kernel<float><<<1, kSmallThreads, 0, s>>>((const float*)x0, (float*)x_out, (int)n, kmax,
                                                               d.radius, cs, cr, diagl);
  } else {
    if (n > SmallMax<double>::n) return false;
    rg_power1d_small_kernel<double><<<1, kSmallThreads, 0, s>>>((const double*)x0, (double*)x_out, (int)n, kmax,
                                                                d.radius, cs, cr, diagl);
  }
  return true;
}

// One-launch CG filter of a built 1D BF operator whose signal fits in one
// workgroup (n <= 8192); false (nothing launched) otherwise.  The state must
// hold tol and tau (as after launch_cg_state_init).
bool launch_cg_small(const Operator& op, const void* x0, void* x_out, int kmax, CgState* st, hipStream_t s) {
  if (op.desc.kind != GSF_BF || op.desc.ndim != 1 || op.n > (int64_t)kSmallThreads * kPts) return false;
  if (op.desc.prec == GSF_F32)
    cg1d_small_kernel<float><<<1, kSmallThreads, 0, s>>>((const float*)op.planes, op.pstride, op.ppad,
                                                         op.desc.radius, (const float*)op.diag, (const float*)op.sqd,
                                                         (const float*)x0, (float*)x_out, (int)op.n, kmax, st);
  else
    cg1d_small_kernel<double><<<1, kSmallThreads, 0, s>>>((const double*)op.planes, op.pstride, op.ppad,
                                                          op.desc.radius, (const double*)op.diag,
                                                          (const double*)op.sqd, (const double*)x0,
                                                          (double*)x_out, (int)op.n, kmax, st);
  return true;
}

}  // namespace gsf
