// Operator construction: BF weights and normalisation (Section 2, eq. (2),
// eq. (4); Section 4 normalisation).  FP64 data and other channel counts:
// weights computed in FP64 and rounded once to the storage type, each
// undirected edge once (fold), then the degrees as FP64 row sums of the
// stored weights (so D 1 = W 1 holds for the operator that is applied).  FP32
// data with one or three guidance channels takes the one-pass build of the
// window kernels instead (FP32 exponentials, every weight of the window evaluated at
// its point, the forward half stored; the degrees are again FP64 sums of the
// stored values).  The
// (diag L) normalisation sums the off-diagonal weights only: the self-loop
// cancels in L = D - W, and leaving it out of the sum (rather than taking
// d_i - 1) keeps a small diag L_i exact to the sum's rounding.
#include <cmath>

#include "gsf_internal.h"

namespace gsf {
namespace {

struct BfParams {
  int64_t n, rows, cols;
  int radius, ndim;
  double cs;  // 1 / (2 sigma_d^2), 0 for sigma_d = inf
  double cr;  // 1 / (2 sigma_r^2), 0 for sigma_r = inf
  int cross;     // 2D cross stencil: offsets (0, 1..r) and (1..r, 0) only
  int diagl;     // normalise by diag L instead of D
  int channels;  // guidance values per point (point-major)
};

// 2D plane q -> half-window offset (dy, dx).  Square: q < r: (0, q + 1), else
// dy = 1 + (q - r) / (2r+1), dx = -r..r.  Cross: q < r: (0, q + 1), else
// (q - r + 1, 0).
__device__ __forceinline__ void plane_offset(int q, const BfParams& p, int& dy, int& dx) {
  const int r = p.radius;
  if (q < r) {
    dy = 0;
    dx = q + 1;
  } else if (p.cross) {
    dy = q - r + 1;
    dx = 0;
  } else {
    dy = 1 + (q - r) / (2 * r + 1);
    dx = (q - r) - (dy - 1) * (2 * r + 1) - r;
  }
}

// eq. (2) in one exponential: exp(-(|o|^2 cs + |g_i - g_j|^2 cr)), with
// |g_i - g_j|^2 summed over the guidance channels in channel order (the
// Euclidean distance of colour vectors, e.g. CIE-Lab).  The argument is
// bitwise the same for (i, j) and (j, i), so W is exactly symmetric wherever
// it is evaluated.
template <typename T>
__device__ __forceinline__ double bf_weight(const T* __restrict__ g, int64_t i, int64_t j, int o2,
                                            const BfParams& p) {
  double d2;
  if (p.channels == 1) {
    const double dg = (double)g[i] - (double)g[j];
    d2 = dg * dg;
  } else {
    d2 = 0.0;
    for (int c = 0; c < p.channels; ++c) {
      const double dg = (double)g[i * p.channels + c] - (double)g[j * p.channels + c];
      d2 += dg * dg;
    }
  }
  return exp(-((double)o2 * p.cs + d2 * p.cr));
}

// K1: half-window planes of the symmetric weights w_{i,i+o} (0 off the grid),
// each undirected edge evaluated once.  Plane order: 1D o = 1..r; 2D (0, 1..r)
// then dy = 1..r with dx = -r..r.  Plane q's data starts at
// planes + ppad + q * pstride; every element of the plane region that is not
// a weight (the ppad zeros before each plane and the tail up to the next one)
// is written as zero: thread i covers index i of every plane's stride window,
// threads i < ppad also the region's tail.
template <typename T>
__global__ void __launch_bounds__(kThreads) bf_fold_kernel(const T* __restrict__ g, T* __restrict__ planes,
                                                           BfParams p, int64_t pstride, int64_t ppad, int nplanes) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= pstride) return;
  if (t < ppad)
    planes[(int64_t)nplanes * pstride + t] = T(0);
  // region index t of every plane window: data point t - ppad, or a pad
  const int64_t i = t - ppad;
  if (i < 0 || i >= p.n) {
    for (int q = 0; q < nplanes; ++q) planes[(int64_t)q * pstride + t] = T(0);
    return;
  }
  planes += ppad;
  const int r = p.radius;
  int q = 0;
  if (p.ndim == 1) {
    for (int o = 1; o <= r; ++o, ++q) {
      const int64_t j = i + o;
      double v = 0.0;
      if (j < p.n) v = bf_weight(g, i, j, o * o, p);
      planes[(int64_t)q * pstride + i] = (T)v;
    }
  } else {
    const int64_t y = i / p.cols, x = i - y * p.cols;
    for (; q < nplanes; ++q) {
      int dy, dx;
      plane_offset(q, p, dy, dx);
      const int64_t yy = y + dy, xx = x + dx;
      double v = 0.0;
      if (yy < p.rows && xx >= 0 && xx < p.cols) {
        const int64_t j = yy * p.cols + xx;
        v = bf_weight(g, i, j, dy * dy + dx * dx, p);
      }
      planes[(int64_t)q * pstride + i] = (T)v;
    }
  }
}

// K2: d_i = 1 + sum_o w_{i,i+o} + sum_o w_{i-o,i} (the self-loop w_ii = 1 and
// both halves of the window), read from the stored planes, so that d is
// exactly the row sum of the stored weights; 1/sqrt(d_i) and sqrt(d_i).  The
// (diag L) normalisation leaves out the self-loop and takes 1 where the sum
// is 0 (a vertex with no edge of nonzero weight: its row and column of L are
// zero, so any positive scale leaves L_sym unchanged).  The mirrored reads
// use the zero pads and wrap-around zeros of the planes (as the apply does),
// so every load is unconditional.  FP64 sums.
template <typename T>
__global__ void __launch_bounds__(kThreads) bf_degree_kernel(const T* __restrict__ planes, double* __restrict__ deg,
                                                             T* __restrict__ diag, T* __restrict__ sqd, BfParams p,
                                                             int64_t pstride, int64_t ppad, int nplanes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const T* base = planes + ppad + i;
  const int r = p.radius;
  double d0 = p.diagl ? 0.0 : 1.0, d1 = 0.0;
  if (p.ndim == 1) {
    for (int o = 1; o <= r; ++o) {
      const T* pl = base + (int64_t)(o - 1) * pstride;
      d0 += (double)pl[0];
      d1 += (double)pl[-o];
    }
  } else {
    const int64_t W = p.cols;
#pragma unroll 4
    for (int q = 0; q < nplanes; ++q) {
      int dy, dx;
      plane_offset(q, p, dy, dx);
      const T* pl = base + (int64_t)q * pstride;
      d0 += (double)pl[0];
      d1 += (double)pl[-(dy * W + dx)];
    }
  }
  double d = d0 + d1;
  if (d == 0.0) d = 1.0;  // only reachable for diag L
  deg[i] = d;
  diag[i] = (T)(1.0 / sqrt(d));
  sqd[i] = (T)sqrt(d);
}

// 1 / (2 sigma^2), 0 for sigma = inf (the factor of eq. (2) is then 1)
inline double inv_two_sigma2(double s) { return std::isinf(s) ? 0.0 : 1.0 / (2.0 * s * s); }

}  // namespace

bool launch_bf_build_onepass(const Operator& op, const void* guidance, hipStream_t s);

gsf_status launch_bf_build(const Operator& op, const void* guidance, hipStream_t s) {
  // FP32 data with one or three guidance channels: one window pass (FP32 exponentials)
  if (launch_bf_build_onepass(op, guidance, s)) return launch_status();
  BfParams p{op.n,
             op.rows,
             op.cols,
             op.desc.radius,
             op.desc.ndim,
             inv_two_sigma2(op.desc.sigma_d),
             inv_two_sigma2(op.desc.sigma_r),
             bf_cross2d(op.desc) ? 1 : 0,
             op.desc.norm == GSF_NORM_DIAGL ? 1 : 0,
             desc_channels(op.desc)};
  const unsigned grid = (unsigned)((op.n + kThreads - 1) / kThreads);
  const unsigned fgrid = (unsigned)((op.pstride + kThreads - 1) / kThreads);
  if (op.desc.prec == GSF_F32) {
    bf_fold_kernel<float><<<fgrid, kThreads, 0, s>>>((const float*)guidance, (float*)op.planes, p, op.pstride,
                                                     op.ppad, op.nplanes);
    bf_degree_kernel<float><<<grid, kThreads, 0, s>>>((const float*)op.planes, op.deg, (float*)op.diag,
                                                      (float*)op.sqd, p, op.pstride, op.ppad, op.nplanes);
  } else {
    bf_fold_kernel<double><<<fgrid, kThreads, 0, s>>>((const double*)guidance, (double*)op.planes, p, op.pstride,
                                                      op.ppad, op.nplanes);
    bf_degree_kernel<double><<<grid, kThreads, 0, s>>>((const double*)op.planes, op.deg, (double*)op.diag,
                                                       (double*)op.sqd, p, op.pstride, op.ppad, op.nplanes);
  }
  return launch_status();
}

}  // namespace gsf
