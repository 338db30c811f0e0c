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

}  // namespace gsf
