// Multi-channel signals: the columns of a point-major n x m block share one
// graph (a colour image filtered under one guidance), so one m-column apply
// reads the weights once for all channels.  Block power iteration and block
// CG (Algorithm 2 per column, run in z-space as CG on L_sym like the
// single-vector filter; every column keeps its own scalars and stopping
// decisions), and the sRGB -> CIE-Lab conversion of a colour guidance
// (Section 2: the photometric distance of eq. (2) measured in CIE-Lab).
// Reductions are deterministic: per-workgroup FP64 partials summed in
// workgroup order by a one-workgroup kernel.
#include <cmath>

#include "gsf_internal.h"
#include "solver_state.h"

namespace gsf {

int vec_blocks(int64_t n);

namespace {

// out = in * sqrt(d) (or / sqrt(d)) for all m columns of every point
template <typename T, int M>
__global__ void __launch_bounds__(kThreads) bscale_kernel(const T* __restrict__ in, const T* __restrict__ s,
                                                          T* __restrict__ out, int64_t n, int divide) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T si = s[i];
#pragma unroll
    for (int c = 0; c < M; ++c) out[i * M + c] = divide ? in[i * M + c] / si : in[i * M + c] * si;
  }
}

// r holds L_sym z on entry: r <- -L_sym z; partials of r_c^T r_c and z_c^T z_c
template <typename T, int M>
__global__ void __launch_bounds__(kThreads) bcg_init_kernel(const T* __restrict__ z, T* __restrict__ r, int64_t n,
                                                            double* __restrict__ partials) {
  __shared__ double red[2 * M * 16];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[2 * M];
#pragma unroll
  for (int k = 0; k < 2 * M; ++k) v[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const T ri = -r[i * M + c];
      r[i * M + c] = ri;
      const double zi = (double)z[i * M + c];
      v[2 * c] += (double)ri * (double)ri;
      v[2 * c + 1] += zi * zi;
    }
  }
  block_sum<2 * M>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 2 * M; ++k) partials[(size_t)blockIdx.x * 2 * M + k] = v[k];
  }
}

__device__ void any_active(BlockCgState* st, int m) {
  int a = 0;
  for (int c = 0; c < m; ++c) a |= st->col[c].active;
  st->active = a;
}

// one workgroup: per column rho0, the breakdown floor and the tests before
// the first step (as for the single-vector filter)
template <int M>
__global__ void __launch_bounds__(kThreads) bcg_init_final_kernel(const double* __restrict__ partials, int nparts,
                                                                  BlockCgState* st) {
  __shared__ double red[2 * M * 16];
  double t[2 * M];
  reduce_partials<2 * M>(partials, nparts, 2 * M, t, red);
  if (threadIdx.x == 0) {
    for (int c = 0; c < M; ++c) {
      CgState& s = st->col[c];
      const double rho = t[2 * c];
      s.rho = rho;
      s.rho0 = rho;
      s.res0 = sqrt(rho > 0.0 ? rho : 0.0);
      s.floor = s.tau * s.tau * t[2 * c + 1];
      s.tol2 = s.tol > 0.0 ? s.tol * s.tol * rho : -1.0;
      s.iters = 0;
      s.k = 1;
      s.beta = 0.0;
      s.status = GSF_OK;
      s.active = 1;
      if (!(__builtin_isfinite(rho) && rho > s.floor)) {
        s.status = GSF_EBREAKDOWN;
        s.active = 0;
      } else if (s.tol2 > 0.0 && rho <= s.tol2) {
        s.active = 0;
      }
    }
    any_active(st, M);
  }
}

// p_c = r_c (first step of column c) or r_c + beta_c p_c; stopped columns keep p
template <typename T, int M>
__global__ void __launch_bounds__(kThreads) bcg_pupdate_kernel(const T* __restrict__ r, T* __restrict__ p, int64_t n,
                                                               const BlockCgState* st) {
  if (!st->active) return;
  T beta[M];
  bool on[M], first[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    on[c] = st->col[c].active != 0;
    first[c] = st->col[c].k == 1;
    beta[c] = (T)st->col[c].beta;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      if (!on[c]) continue;
      p[i * M + c] = first[c] ? r[i * M + c] : r[i * M + c] + beta[c] * p[i * M + c];
    }
  }
}

// partials of p_c^T q_c
template <typename T, int M>
__global__ void __launch_bounds__(kThreads) bdot_kernel(const T* __restrict__ p, const T* __restrict__ q, int64_t n,
                                                        double* __restrict__ partials, const BlockCgState* st) {
  __shared__ double red[M * 16];
  if (!st->active) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[M];
#pragma unroll
  for (int c = 0; c < M; ++c) v[c] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int c = 0; c < M; ++c) v[c] += (double)p[i * M + c] * (double)q[i * M + c];
  }
  block_sum<M>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < M; ++c) partials[(size_t)blockIdx.x * M + c] = v[c];
  }
}

// one workgroup: per active column p^T q, alpha = rho / p^T q, breakdown test
template <int M>
__global__ void __launch_bounds__(kThreads) bcg_alpha_kernel(const double* __restrict__ partials, int nparts,
                                                             BlockCgState* st) {
  __shared__ double red[M * 16];
  if (!st->active) return;
  double t[M];
  reduce_partials<M>(partials, nparts, M, t, red);
  if (threadIdx.x == 0) {
    for (int c = 0; c < M; ++c) {
      CgState& s = st->col[c];
      if (!s.active) continue;
      const double pq = t[c];
      s.pq = pq;
      if (!(__builtin_isfinite(pq) && pq > 0.0)) {
        s.status = GSF_EBREAKDOWN;
        s.active = 0;
      } else {
        s.alpha = s.rho / pq;
      }
    }
    any_active(st, M);
  }
}

// active columns: z += alpha p; r -= alpha q; partials of r_new^T r_new and
// r_new^T r_old
template <typename T, int M>
__global__ void __launch_bounds__(kThreads) bcg_update_kernel(T* __restrict__ z, T* __restrict__ r,
                                                              const T* __restrict__ p, const T* __restrict__ q,
                                                              int64_t n, double* __restrict__ partials,
                                                              const BlockCgState* st) {
  __shared__ double red[2 * M * 16];
  if (!st->active) return;
  T alpha[M];
  bool on[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    on[c] = st->col[c].active != 0;
    alpha[c] = (T)st->col[c].alpha;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[2 * M];
#pragma unroll
  for (int k = 0; k < 2 * M; ++k) v[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      if (!on[c]) continue;
      z[i * M + c] += alpha[c] * p[i * M + c];
      const T ro = r[i * M + c];
      const T rn = ro - alpha[c] * q[i * M + c];
      r[i * M + c] = rn;
      v[2 * c] += (double)rn * (double)rn;
      v[2 * c + 1] += (double)rn * (double)ro;
    }
  }
  block_sum<2 * M>(v, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 2 * M; ++k) partials[(size_t)blockIdx.x * 2 * M + k] = v[k];
  }
}

// one workgroup: per active column rho_new, beta = (rho_new - r_new.r_old) /
// rho_old, the step count and the tests that precede the next step
template <int M>
__global__ void __launch_bounds__(kThreads) bcg_beta_kernel(const double* __restrict__ partials, int nparts,
                                                            BlockCgState* st) {
  __shared__ double red[2 * M * 16];
  if (!st->active) return;
  double t[2 * M];
  reduce_partials<2 * M>(partials, nparts, 2 * M, t, red);
  if (threadIdx.x == 0) {
    for (int c = 0; c < M; ++c) {
      CgState& s = st->col[c];
      if (!s.active) continue;
      const double rho_old = s.rho;
      const double rho = t[2 * c];
      s.beta = (rho - t[2 * c + 1]) / rho_old;
      s.rho = rho;
      s.iters = s.k;
      s.k = s.k + 1;
      if (!(__builtin_isfinite(rho) && rho > s.floor)) {
        s.status = GSF_EBREAKDOWN;
        s.active = 0;
      } else if (s.tol2 > 0.0 && rho <= s.tol2) {
        s.active = 0;
      }
    }
    any_active(st, M);
  }
}

__global__ void bcg_state_init_kernel(BlockCgState* dst, BlockCgState v) { *dst = v; }

// sRGB (IEC 61966-2-1 transfer curve) -> XYZ (row-major matrix m) -> CIE 1976
// L*a*b* relative to the white (wx, wy, wz) of that matrix, FP64.
struct LabParams {
  double m[9];
  double wx, wy, wz;
};

__device__ __forceinline__ double srgb_lin(double c) {
  return c <= 0.04045 ? c / 12.92 : pow((c + 0.055) / 1.055, 2.4);
}

__device__ __forceinline__ double lab_f(double t) {
  constexpr double d = 6.0 / 29.0;
  return t > d * d * d ? cbrt(t) : t / (3.0 * d * d) + 4.0 / 29.0;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) srgb_to_lab_kernel(const T* __restrict__ rgb, T* __restrict__ lab,
                                                               int64_t n, LabParams p) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double r = srgb_lin((double)rgb[3 * i]);
    const double g = srgb_lin((double)rgb[3 * i + 1]);
    const double b = srgb_lin((double)rgb[3 * i + 2]);
    const double X = p.m[0] * r + p.m[1] * g + p.m[2] * b;
    const double Y = p.m[3] * r + p.m[4] * g + p.m[5] * b;
    const double Z = p.m[6] * r + p.m[7] * g + p.m[8] * b;
    const double fx = lab_f(X / p.wx), fy = lab_f(Y / p.wy), fz = lab_f(Z / p.wz);
    lab[3 * i] = (T)(116.0 * fy - 16.0);
    lab[3 * i + 1] = (T)(500.0 * (fx - fy));
    lab[3 * i + 2] = (T)(200.0 * (fy - fz));
  }
}

// Linear sRGB -> XYZ from the chromaticities of the primaries R (0.64, 0.33),
// G (0.30, 0.60), B (0.15, 0.06) and of the white D65 (0.3127, 0.3290):
// column k is the primary's XYZ at Y = 1 times the drive s_k that makes
// R = G = B = 1 the white with Y = 1 (Cramer's rule on the 3x3 system).
LabParams lab_params() {
  const double cx[3] = {0.64, 0.30, 0.15}, cy[3] = {0.33, 0.60, 0.06};
  double P[3][3];
  for (int k = 0; k < 3; ++k) {
    P[0][k] = cx[k] / cy[k];
    P[1][k] = 1.0;
    P[2][k] = (1.0 - cx[k] - cy[k]) / cy[k];
  }
  const double w[3] = {0.3127 / 0.3290, 1.0, (1.0 - 0.3127 - 0.3290) / 0.3290};
  auto det3 = [](double a[3][3]) {
    return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
           a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  };
  const double dp = det3(P);
  double s[3];
  for (int k = 0; k < 3; ++k) {
    double Q[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Q[i][j] = j == k ? w[i] : P[i][j];
    s[k] = det3(Q) / dp;
  }
  LabParams p{};
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) p.m[3 * i + k] = P[i][k] * s[k];
  // the white of the matrix: its row sums (R = G = B = 1)
  p.wx = p.m[0] + p.m[1] + p.m[2];
  p.wy = p.m[3] + p.m[4] + p.m[5];
  p.wz = p.m[6] + p.m[7] + p.m[8];
  return p;
}

template <typename T, int M>
void launch_bcg_m(int kind, const Operator& op, void* z, void* r, void* p, void* q, double* partials, int nparts,
                  BlockCgState* st, hipStream_t s) {
  const int nb = vec_blocks(op.n);
  switch (kind) {
    case 0:
      bcg_init_kernel<T, M><<<nb, kThreads, 0, s>>>((const T*)z, (T*)r, op.n, partials);
      bcg_init_final_kernel<M><<<1, kThreads, 0, s>>>(partials, nb, st);
      break;
    case 1:
      bcg_pupdate_kernel<T, M><<<nb, kThreads, 0, s>>>((const T*)r, (T*)p, op.n, st);
      break;
    case 2:
      bdot_kernel<T, M><<<nb, kThreads, 0, s>>>((const T*)p, (const T*)q, op.n, partials, st);
      bcg_alpha_kernel<M><<<1, kThreads, 0, s>>>(partials, nb, st);
      break;
    default:
      bcg_update_kernel<T, M><<<nb, kThreads, 0, s>>>((T*)z, (T*)r, (const T*)p, (const T*)q, op.n, partials, st);
      bcg_beta_kernel<M><<<1, kThreads, 0, s>>>(partials, nb, st);
      break;
  }
  (void)nparts;
}

template <typename T>
void launch_bcg_t(int kind, const Operator& op, int m, void* z, void* r, void* p, void* q, double* partials,
                  BlockCgState* st, hipStream_t s) {
  switch (m) {
    case 1: launch_bcg_m<T, 1>(kind, op, z, r, p, q, partials, 0, st, s); break;
    case 2: launch_bcg_m<T, 2>(kind, op, z, r, p, q, partials, 0, st, s); break;
    case 3: launch_bcg_m<T, 3>(kind, op, z, r, p, q, partials, 0, st, s); break;
    case 4: launch_bcg_m<T, 4>(kind, op, z, r, p, q, partials, 0, st, s); break;
    case 5: launch_bcg_m<T, 5>(kind, op, z, r, p, q, partials, 0, st, s); break;
    case 6: launch_bcg_m<T, 6>(kind, op, z, r, p, q, partials, 0, st, s); break;
    case 7: launch_bcg_m<T, 7>(kind, op, z, r, p, q, partials, 0, st, s); break;
    default: launch_bcg_m<T, 8>(kind, op, z, r, p, q, partials, 0, st, s); break;
  }
}

template <typename T>
void launch_bscale_t(const Operator& op, int m, const void* in, void* out, int divide, hipStream_t s) {
  const int nb = vec_blocks(op.n);
  const T* sq = (const T*)op.sqd;
  switch (m) {
    case 1: bscale_kernel<T, 1><<<nb, kThreads, 0, s>>>((const T*)in, sq, (T*)out, op.n, divide); break;
    case 2: bscale_kernel<T, 2><<<nb, kThreads, 0, s>>>((const T*)in, sq, (T*)out, op.n, divide); break;
    case 3: bscale_kernel<T, 3><<<nb, kThreads, 0, s>>>((const T*)in, sq, (T*)out, op.n, divide); break;
    case 4: bscale_kernel<T, 4><<<nb, kThreads, 0, s>>>((const T*)in, sq, (T*)out, op.n, divide); break;
    case 5: bscale_kernel<T, 5><<<nb, kThreads, 0, s>>>((const T*)in, sq, (T*)out, op.n, divide); break;
    case 6: bscale_kernel<T, 6><<<nb, kThreads, 0, s>>>((const T*)in, sq, (T*)out, op.n, divide); break;
    case 7: bscale_kernel<T, 7><<<nb, kThreads, 0, s>>>((const T*)in, sq, (T*)out, op.n, divide); break;
    default: bscale_kernel<T, 8><<<nb, kThreads, 0, s>>>((const T*)in, sq, (T*)out, op.n, divide); break;
  }
}

}  // namespace

gsf_status launch_bscale(const Operator& op, int m, const void* in, void* out, int divide, hipStream_t s) {
  if (op.desc.prec == GSF_F32)
    launch_bscale_t<float>(op, m, in, out, divide, s);
  else
    launch_bscale_t<double>(op, m, in, out, divide, s);
  return launch_status();
}

// kind: 0 init (r <- -r, per-column rho0 and floor), 1 p update, 2 p^T q and
// alpha, 3 z / r update and beta
gsf_status launch_bcg(int kind, const Operator& op, int m, void* z, void* r, void* p, void* q, double* partials,
                      BlockCgState* st, hipStream_t s) {
  if (op.desc.prec == GSF_F32)
    launch_bcg_t<float>(kind, op, m, z, r, p, q, partials, st, s);
  else
    launch_bcg_t<double>(kind, op, m, z, r, p, q, partials, st, s);
  return launch_status();
}

gsf_status launch_bcg_state_init(BlockCgState* st, const BlockCgState& v, hipStream_t s) {
  bcg_state_init_kernel<<<1, 1, 0, s>>>(st, v);
  return launch_status();
}

gsf_status launch_srgb_to_lab(int prec, int64_t n, const void* rgb, void* lab, hipStream_t s) {
  const LabParams p = lab_params();
  const int nb = vec_blocks(n);
  if (prec == GSF_F32)
    srgb_to_lab_kernel<float><<<nb, kThreads, 0, s>>>((const float*)rgb, (float*)lab, n, p);
  else
    srgb_to_lab_kernel<double><<<nb, kThreads, 0, s>>>((const double*)rgb, (double*)lab, n, p);
  return launch_status();
}

}  // namespace gsf
