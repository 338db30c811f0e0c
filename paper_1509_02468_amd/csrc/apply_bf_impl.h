// Normalized BF operator apply (kernel templates), Section 2 eqs. (1)-(4) and
// the normalisation of Section 4, evaluated in Laplacian form:
//   u = D^-1/2 z                      (z-space input; RW form: u = x)
//   (L u)_i = sum_j w_ij (u_i - u_j)  (eq. (4): L = D - W, self-loop cancels)
//   L_sym z = D^-1/2 L u,   N z = z - L_sym z,   D^-1 W x = x - D^-1 L x (eq. (3))
// Summing weighted neighbour differences keeps L_sym z accurate when z is
// smooth (forming z - N z would cancel all but a few digits of FP32).
//
// Each undirected edge is stored once, at its lower endpoint, in half-window
// planes w[o][i] = w_{i,i+o}; a point reads its own plane entry and, mirrored,
// the entry of the point i-o for the edge (i-o, i).  Every weight read is
// unconditional: a mirrored read above the first row (before the first
// sample) lands in the zeros that precede each plane, and one that wraps
// around a row end lands on an entry whose partner is off the grid, which is
// zero too.  Plane offsets are 32-bit per lane from a uniform plane base.
//
// Tiling: a workgroup of 256 threads owns a 64-wide tile of TY rows (2D) or
// 256*RPT consecutive samples (1D).  u for the tile plus an r-wide halo is
// staged once in LDS (zero outside the grid); the weight planes stream from
// HBM with coalesced row reads, and the mirrored reads hit rows that the L2 of
// the XCD owning the band of tiles already holds.
#pragma once
#include "gsf_internal.h"

namespace gsf {
namespace bfk {

struct ApplyArgs {
  const void* planes;  // padded start of plane 0
  int64_t pstride;     // elements between consecutive planes' padded starts
  int64_t ppad;        // zeros before each plane's data
  const void* isqd;  // 1/sqrt(d)
  const void* x;
  void* y;
  int64_t ldx, ldy;
  int64_t n, rows, cols;
  int form;
  int tiles_x, ntiles;
  double* dot;  // nullable, per-workgroup partial sum x.y (m = 1)
};

// Rows of points per thread (RPT) is a template choice in {1, 2, 4}: more rows
// amortise the LDS halo, fewer rows give more workgroups (and so more loads in
// flight per CU).  The default below keeps the LDS tile under ~64 KB; the
// apply tuner may pick another one per (type, m, r).
template <typename T, int M>
struct Rows {
  static constexpr int MB = M * (int)sizeof(T);
  static constexpr int RPT = MB <= 16 ? 4 : (MB <= 32 ? 2 : 1);
};

inline int default_rpt(int elem, int m) {
  const int mb = elem * m;
  return mb <= 16 ? 4 : (mb <= 32 ? 2 : 1);
}

// y from the Laplacian sum acc = sum_j w_ij (u_i - u_j) for one point.
template <typename T, int M>
__device__ __forceinline__ void finish_point(int form, T is, const T* __restrict__ xg, const T (&acc)[M],
                                             T (&out)[M]) {
  if (form == GSF_FORM_LSYM) {
#pragma unroll
    for (int c = 0; c < M; ++c) out[c] = is * acc[c];
  } else if (form == GSF_FORM_N) {
#pragma unroll
    for (int c = 0; c < M; ++c) out[c] = xg[c] - is * acc[c];
  } else {  // RW: x - D^-1 L x
    const T id = is * is;
#pragma unroll
    for (int c = 0; c < M; ++c) out[c] = xg[c] - id * acc[c];
  }
}

// How many offsets of one row of the window are scheduled together: all of
// them for narrow blocks; for wide blocks fewer, so that the loaded weights
// and neighbour values fit in registers at a useful occupancy.
template <typename T, int M>
struct DxUnroll {
  static constexpr int value = (M * (int)sizeof(T) >= 16) ? 4 : 17;
};

template <typename T, int M, int R, int RPT>
__global__ void __launch_bounds__(kThreads) bf_apply2d_kernel(ApplyArgs a) {
  constexpr int TX = 64;
  constexpr int TY = 4 * RPT;
  constexpr int LW = TX + 2 * R;
  constexpr int LH = TY + 2 * R;
  __shared__ T us[LH * LW * M];
  __shared__ double red[16];

  const T* __restrict__ planes = (const T*)a.planes;
  const T* __restrict__ isqd = (const T*)a.isqd;
  const T* __restrict__ x = (const T*)a.x;
  T* __restrict__ y = (T*)a.y;
  const int64_t W = a.cols, H = a.rows, n = a.n;

  const int tile = xcd_tile(blockIdx.x, a.ntiles);
  const int64_t ty0 = (int64_t)(tile / a.tiles_x) * TY;
  const int64_t tx0 = (int64_t)(tile % a.tiles_x) * TX;
  const bool zspace = (a.form != GSF_FORM_RW);

  // stage u = D^-1/2 z (or x) with halo
  for (int e = threadIdx.x; e < LH * LW; e += kThreads) {
    const int ly = e / LW, lx = e - (e / LW) * LW;
    const int64_t gy = ty0 - R + ly, gx = tx0 - R + lx;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const int64_t p = gy * W + gx;
    T s = T(1);
    if (zspace && in) s = isqd[p];
#pragma unroll
    for (int c = 0; c < M; ++c) us[e * M + c] = in ? x[p * a.ldx + c] * s : T(0);
  }
  __syncthreads();

  const int tx = threadIdx.x & 63, wy = threadIdx.x >> 6;
  const int64_t gx = tx0 + tx;
  double dotv = 0.0;
#pragma unroll 1
  for (int rr = 0; rr < RPT; ++rr) {
    const int ly = wy * RPT + rr;
    const int64_t gy = ty0 + ly;
    const bool valid = gy < H && gx < W;
    const int64_t p = valid ? gy * W + gx : 0;
    const T* uc = &us[((ly + R) * LW + tx + R) * M];
    T ui[M], acc[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      ui[c] = uc[c];
      acc[c] = T(0);
    }
    // byte offsets of this point in a padded plane (unsigned 32-bit, from a
    // uniform plane base)
    const uint32_t pv = ((uint32_t)p + (uint32_t)a.ppad) * (uint32_t)sizeof(T);
    const char* __restrict__ qb = (const char*)planes;  // padded start of the current plane
    const size_t qstep = (size_t)a.pstride * sizeof(T);
    // dy = 0: planes 0..R-1, offsets (0, dx)
#pragma unroll
    for (int dx = 1; dx <= R; ++dx) {
      const T wo = *(const T*)(qb + pv);
      const T wm = *(const T*)(qb + (pv - (uint32_t)(dx * (int)sizeof(T))));
      qb += qstep;
      const T* uo = uc + dx * M;
      const T* um = uc - dx * M;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        acc[c] = fma(wo, ui[c] - uo[c], acc[c]);
        acc[c] = fma(wm, ui[c] - um[c], acc[c]);
      }
    }
    // dy = 1..R, dx = -R..R: one row of 2R+1 planes per dy
#pragma unroll 1
    for (int dy = 1; dy <= R; ++dy) {
      const uint32_t mrow = pv - (uint32_t)(dy * (int)W) * (uint32_t)sizeof(T);
      const T* urow = uc + dy * LW * M;
      const T* umrow = uc - dy * LW * M;
#pragma unroll(DxUnroll<T, M>::value)
      for (int dx = -R; dx <= R; ++dx) {
        const T wo = *(const T*)(qb + pv);
        const T wm = *(const T*)(qb + (mrow - (uint32_t)(dx * (int)sizeof(T))));
        qb += qstep;
        const T* uo = urow + dx * M;
        const T* um = umrow - dx * M;
#pragma unroll
        for (int c = 0; c < M; ++c) {
          acc[c] = fma(wo, ui[c] - uo[c], acc[c]);
          acc[c] = fma(wm, ui[c] - um[c], acc[c]);
        }
      }
    }
    if (valid) {
      T xg[M], out[M];
#pragma unroll
      for (int c = 0; c < M; ++c) xg[c] = (a.form == GSF_FORM_LSYM) ? T(0) : x[p * a.ldx + c];
      finish_point<T, M>(a.form, isqd[p], xg, acc, out);
#pragma unroll
      for (int c = 0; c < M; ++c) y[p * a.ldy + c] = out[c];
      if (M == 1 && a.dot != nullptr) dotv += (double)x[p * a.ldx] * (double)out[0];
    }
  }
  if (a.dot != nullptr) {
    double v[1] = {dotv};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) a.dot[blockIdx.x] = v[0];
  }
}

template <typename T, int M, int R, int RPT>
__global__ void __launch_bounds__(kThreads) bf_apply1d_kernel(ApplyArgs a) {
  constexpr int TN = kThreads * RPT;
  constexpr int LN = TN + 2 * R;
  __shared__ T us[LN * M];
  __shared__ double red[16];

  const T* __restrict__ planes = (const T*)a.planes;
  const T* __restrict__ isqd = (const T*)a.isqd;
  const T* __restrict__ x = (const T*)a.x;
  T* __restrict__ y = (T*)a.y;
  const int64_t n = a.n;
  const int64_t base = (int64_t)blockIdx.x * TN;
  const bool zspace = (a.form != GSF_FORM_RW);

  for (int e = threadIdx.x; e < LN; e += kThreads) {
    const int64_t g = base - R + e;
    const bool in = g >= 0 && g < n;
    T s = T(1);
    if (zspace && in) s = isqd[g];
#pragma unroll
    for (int c = 0; c < M; ++c) us[e * M + c] = in ? x[g * a.ldx + c] * s : T(0);
  }
  __syncthreads();

  double dotv = 0.0;
#pragma unroll 1
  for (int rr = 0; rr < RPT; ++rr) {
    const int l = rr * kThreads + threadIdx.x;
    const int64_t p0 = base + l;
    const bool valid = p0 < n;
    const int64_t p = valid ? p0 : 0;
    const T* uc = &us[(l + R) * M];
    T ui[M], acc[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      ui[c] = uc[c];
      acc[c] = T(0);
    }
    const uint32_t pv = ((uint32_t)p + (uint32_t)a.ppad) * (uint32_t)sizeof(T);
    const char* __restrict__ qb = (const char*)planes;
    const size_t qstep = (size_t)a.pstride * sizeof(T);
#pragma unroll
    for (int o = 1; o <= R; ++o) {
      const T wo = *(const T*)(qb + pv);
      const T wm = *(const T*)(qb + (pv - (uint32_t)(o * (int)sizeof(T))));
      qb += qstep;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        acc[c] = fma(wo, ui[c] - uc[o * M + c], acc[c]);
        acc[c] = fma(wm, ui[c] - uc[-o * M + c], acc[c]);
      }
    }
    if (valid) {
      T xg[M], out[M];
#pragma unroll
      for (int c = 0; c < M; ++c) xg[c] = (a.form == GSF_FORM_LSYM) ? T(0) : x[p * a.ldx + c];
      finish_point<T, M>(a.form, isqd[p], xg, acc, out);
#pragma unroll
      for (int c = 0; c < M; ++c) y[p * a.ldy + c] = out[c];
      if (M == 1 && a.dot != nullptr) dotv += (double)x[p * a.ldx] * (double)out[0];
    }
  }
  if (a.dot != nullptr) {
    double v[1] = {dotv};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) a.dot[blockIdx.x] = v[0];
  }
}

template <typename T, int M, int R, int RPT>
void launch_bf_tile(const ApplyArgs& a, int ndim, hipStream_t s, int* nblocks) {
  if (ndim == 2) {
    constexpr int TY = 4 * RPT;
    ApplyArgs b = a;
    b.tiles_x = (int)((a.cols + 63) / 64);
    const int tiles_y = (int)((a.rows + TY - 1) / TY);
    b.ntiles = b.tiles_x * tiles_y;
    *nblocks = b.ntiles;
    bf_apply2d_kernel<T, M, R, RPT><<<b.ntiles, kThreads, 0, s>>>(b);
  } else {
    constexpr int TN = kThreads * RPT;
    const int nb = (int)((a.n + TN - 1) / TN);
    *nblocks = nb;
    bf_apply1d_kernel<T, M, R, RPT><<<nb, kThreads, 0, s>>>(a);
  }
}

template <typename T, int M, int R>
void launch_bf_rpt(const ApplyArgs& a, int ndim, int rpt, hipStream_t s, int* nb) {
  constexpr int MB = M * (int)sizeof(T);
  // taller tiles do not fit in LDS for wide FP64 blocks
  if constexpr (MB <= 32) {
    if (rpt >= 4) {
      launch_bf_tile<T, M, R, 4>(a, ndim, s, nb);
      return;
    }
    if (rpt >= 2) {
      launch_bf_tile<T, M, R, 2>(a, ndim, s, nb);
      return;
    }
  }
  launch_bf_tile<T, M, R, 1>(a, ndim, s, nb);
}

template <typename T, int M>
void launch_bf_r(const ApplyArgs& a, int ndim, int r, int rpt, hipStream_t s, int* nb) {
  switch (r) {
    case 1: launch_bf_rpt<T, M, 1>(a, ndim, rpt, s, nb); break;
    case 2: launch_bf_rpt<T, M, 2>(a, ndim, rpt, s, nb); break;
    case 3: launch_bf_rpt<T, M, 3>(a, ndim, rpt, s, nb); break;
    case 4: launch_bf_rpt<T, M, 4>(a, ndim, rpt, s, nb); break;
    case 5: launch_bf_rpt<T, M, 5>(a, ndim, rpt, s, nb); break;
    case 6: launch_bf_rpt<T, M, 6>(a, ndim, rpt, s, nb); break;
    case 7: launch_bf_rpt<T, M, 7>(a, ndim, rpt, s, nb); break;
    default: launch_bf_rpt<T, M, 8>(a, ndim, rpt, s, nb); break;
  }
}

}  // namespace bfk

// one translation unit per (T, M) instantiates this
template <typename T, int M>
void bf_apply_tm(const bfk::ApplyArgs& a, int ndim, int r, int rpt, hipStream_t s, int* nb);

}  // namespace gsf
