// Normalized BF operator apply (kernel templates), Section 2 eqs. (1)-(4) and
// the normalisation of Section 4, evaluated in Laplacian form:
//   u = D^-1/2 z                      (z-space input; RW and L forms: u = x)
//   (L u)_i = sum_j w_ij (u_i - u_j)  (eq. (4): L = D - W, self-loop cancels)
//   L_sym z = D^-1/2 L u,   N z = z - L_sym z,   D^-1 W x = x - D^-1 L x (eq. (3)),
//   L x = L u
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
#include <type_traits>
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
  int cross;  // 2D cross stencil (planes (0, 1..R) then (1..R, 0))
  // joint apply (kernels with M2 = 1): the last column comes from x2 / goes
  // to y2 (leading dimensions ldx2 / ldy2), the others from x / to y; the dot
  // partials are then those of that column
  const void* x2;
  void* y2;
  int64_t ldx2, ldy2;
  int tiles_x, ntiles;
  double* dot;  // nullable, per-workgroup partial sum x.y (m = 1)
};

// Rows of points per thread (RPT) is a template choice in {1, 2, 4}: more rows
// amortise the LDS halo, fewer rows give more workgroups (and so more loads in
// flight per CU).  In 2D, RPT = 2 is the paired kernel (two rows computed
// together, sharing each neighbour row); RPT = 1 and 4 take their rows one
// after the other.  The apply tuner may pick another one per (type, m, r).
// Defaults: for wide windows (r >= 3) one row for a single FP32 column and
// the paired kernel up to 32 bytes per point (measured at 1024^2, r = 5, FP32:
// m = 1: 46 / 52 / 67 us for 1 / 2 / 4 rows; m = 3: 61 / 59 / 93; m = 4:
// 73 / 66 / 77); for narrow windows four rows up to 16 bytes per point, where
// the halo is a larger share of the tile.
inline int default_rpt(int elem, int m, int radius) {
  const int mb = elem * m;
  if (radius >= 3) return mb <= 4 ? 1 : (mb <= 32 ? 2 : 1);
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
  } else if (form == GSF_FORM_L) {
#pragma unroll
    for (int c = 0; c < M; ++c) out[c] = acc[c];
  } else {  // RW: x - D^-1 L x
    const T id = is * is;
#pragma unroll
    for (int c = 0; c < M; ++c) out[c] = xg[c] - id * acc[c];
  }
}

// Column c (a compile-time index after unrolling) of point p of the input and
// output block: the first M - M2 columns in x / y, the last M2 in x2 / y2.
template <typename T, int M, int M2>
__device__ __forceinline__ T in_col(const ApplyArgs& a, int64_t p, int c) {
  if (M2 > 0 && c >= M - M2) return ((const T*)a.x2)[p * a.ldx2 + (c - (M - M2))];
  return ((const T*)a.x)[p * a.ldx + c];
}
template <typename T, int M, int M2>
__device__ __forceinline__ void out_col(const ApplyArgs& a, int64_t p, int c, T v) {
  if (M2 > 0 && c >= M - M2)
    ((T*)a.y2)[p * a.ldy2 + (c - (M - M2))] = v;
  else
    ((T*)a.y)[p * a.ldy + c] = v;
}
// the column whose x . y partial the kernel reports (m = 1, or the joint column)
// FP32 windows wider than 11 x 11 (R >= 6, up to 289 terms per point): each
// window row is summed in FP32 and the rows' sums in FP64, so that the sum's
// rounding does not grow with the window (one sequential FP32 sum of 2K
// sign-alternating terms reaches about 1e-5 of N x at R = 8); narrower windows
// and FP64 data sum in the data type.
template <typename T, int R>
struct RowSums {
  static constexpr bool on = R >= 6 && sizeof(T) == 4;
};

template <int M, int M2>
struct DotCol {
  static constexpr bool on = M == 1 || M2 > 0;
  static constexpr int c = M2 > 0 ? M - 1 : 0;
};

// How many offsets of one row of the window are scheduled together: all of
// them for narrow blocks; for wide blocks fewer, so that the loaded weights
// and neighbour values fit in registers at a useful occupancy.
template <typename T, int M>
struct DxUnroll {
  static constexpr int value = (M * (int)sizeof(T) >= 16) ? 4 : 17;
};

template <typename T, int M, int R, int RPT, int M2 = 0>
__global__ void __launch_bounds__(kThreads) bf_apply2d_kernel(ApplyArgs a) {
  constexpr int TX = 64;
  constexpr int TY = 4 * RPT;
  constexpr int LW = TX + 2 * R;
  constexpr int LH = TY + 2 * R;
  __shared__ T us[LH * LW * M];
  __shared__ double red[16];

  const T* __restrict__ planes = (const T*)a.planes;
  const T* __restrict__ isqd = (const T*)a.isqd;
  const int64_t W = a.cols, H = a.rows;

  const int tile = xcd_tile(blockIdx.x, a.ntiles);
  const int64_t ty0 = (int64_t)(tile / a.tiles_x) * TY;
  const int64_t tx0 = (int64_t)(tile % a.tiles_x) * TX;
  const bool zspace = (a.form == GSF_FORM_N || a.form == GSF_FORM_LSYM);

  // stage u = D^-1/2 z (or x) with halo
  for (int e = threadIdx.x; e < LH * LW; e += kThreads) {
    const int ly = e / LW, lx = e - (e / LW) * LW;
    const int64_t gy = ty0 - R + ly, gx = tx0 - R + lx;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const int64_t p = gy * W + gx;
    T s = T(1);
    if (zspace && in) s = isqd[p];
#pragma unroll
    for (int c = 0; c < M; ++c) us[e * M + c] = in ? in_col<T, M, M2>(a, p, c) * s : T(0);
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
    double dacc[M];  // RowSums<T, R>: the FP64 total of the window rows' sums
#pragma unroll
    for (int c = 0; c < M; ++c) {
      ui[c] = uc[c];
      acc[c] = T(0);
      dacc[c] = 0.0;
    }
    auto flush = [&]() {
      if constexpr (RowSums<T, R>::on) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          dacc[c] += (double)acc[c];
          acc[c] = T(0);
        }
      }
    };
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
    flush();
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
      flush();
    }
    if constexpr (RowSums<T, R>::on) {
#pragma unroll
      for (int c = 0; c < M; ++c) acc[c] = (T)dacc[c];
    }
    if (valid) {
      T xg[M], out[M];
#pragma unroll
      for (int c = 0; c < M; ++c) xg[c] = (a.form == GSF_FORM_LSYM || a.form == GSF_FORM_L) ? T(0) : in_col<T, M, M2>(a, p, c);
      finish_point<T, M>(a.form, isqd[p], xg, acc, out);
#pragma unroll
      for (int c = 0; c < M; ++c) out_col<T, M, M2>(a, p, c, out[c]);
      if (DotCol<M, M2>::on && a.dot != nullptr)
        dotv += (double)in_col<T, M, M2>(a, p, DotCol<M, M2>::c) * (double)out[DotCol<M, M2>::c];
    }
  }
  if (a.dot != nullptr) {
    double v[1] = {dotv};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) a.dot[blockIdx.x] = v[0];
  }
}

// Two vertically adjacent points per thread: rows 2w and 2w+1 (w = wave) of
// a 64 x TY tile (TY = 16 at launch: 512 threads; measured at 1024^2, 11x11,
// FP32, m = 4: 60 us against 65 us for 64 x 8 tiles and 62 us for 64 x 32,
// the taller tile re-reading fewer weight rows across tile borders).  Every staged neighbour row is read from LDS once and used
// by both points (2R+2 rows of 2R+1 neighbours per pair instead of two full
// windows).  The rows are taken in patterns in which every weight's plane and
// position are fixed at compile time up to the row: the rows of points 0 and
// 1, pairs of a mirrored row above and an own row below, and the two end
// rows, so no weight load sits behind a branch.  A point's own position
// (offset 0) gets a zero weight.  It pays where the one-row kernel is bound by
// its arithmetic and LDS reads (wide blocks).
template <typename T, int M, int R, int TY, int M2 = 0>
__global__ void __launch_bounds__(32 * TY) bf_apply2d_pair_kernel(ApplyArgs a) {
  constexpr int TX = 64;
  constexpr int NT = 32 * TY;  // threads: 64 columns x TY/2 row pairs
  constexpr int LW = TX + 2 * R;
  constexpr int LH = TY + 2 * R;
  constexpr int NQ = 2 * R + 1;  // planes per plane row dy >= 1
  __shared__ T us[LH * LW * M];
  __shared__ double red[16];

  const T* __restrict__ isqd = (const T*)a.isqd;
  const int64_t W = a.cols, H = a.rows;

  const int tile = xcd_tile(blockIdx.x, a.ntiles);
  const int64_t ty0 = (int64_t)(tile / a.tiles_x) * TY;
  const int64_t tx0 = (int64_t)(tile % a.tiles_x) * TX;
  const bool zspace = (a.form == GSF_FORM_N || a.form == GSF_FORM_LSYM);

  for (int e = threadIdx.x; e < LH * LW; e += NT) {
    const int ly = e / LW, lx = e - (e / LW) * LW;
    const int64_t gy = ty0 - R + ly, gx = tx0 - R + lx;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const int64_t p = gy * W + gx;
    T s = T(1);
    if (zspace && in) s = isqd[p];
#pragma unroll
    for (int c = 0; c < M; ++c) us[e * M + c] = in ? in_col<T, M, M2>(a, p, c) * s : T(0);
  }
  __syncthreads();

  const int tx = threadIdx.x & 63, ly0 = 2 * (threadIdx.x >> 6);
  const int64_t gx = tx0 + tx, gy0 = ty0 + ly0;
  const bool valid0 = gy0 < H && gx < W, valid1 = gy0 + 1 < H && gx < W;
  const int64_t p0 = valid0 ? gy0 * W + gx : 0;
  const int64_t p1 = valid1 ? p0 + W : 0;
  // byte offsets of the two points in a padded plane (32-bit, from uniform plane bases)
  const uint32_t pv0 = ((uint32_t)p0 + (uint32_t)a.ppad) * (uint32_t)sizeof(T);
  const uint32_t pv1 = ((uint32_t)p1 + (uint32_t)a.ppad) * (uint32_t)sizeof(T);
  const uint32_t wb = (uint32_t)W * (uint32_t)sizeof(T);
  const char* __restrict__ qb = (const char*)a.planes;
  const ptrdiff_t qs = (ptrdiff_t)a.pstride * (ptrdiff_t)sizeof(T);
  constexpr int TS = (int)sizeof(T);
  const T* c0 = &us[((ly0 + R) * LW + tx + R) * M];
  // Both points measure their neighbours against u0: acc0 = sum w0 (v - u0),
  // acc1 = sum w1 (v - u0) and sw1 = sum w1, so that the Laplacian sums are
  // -acc0 and (u1 - u0) sw1 - acc1.  One difference per neighbour and
  // channel serves both points, and every term stays a difference of nearby
  // values (no cancellation of whole values of u).  Skipped own positions
  // carry a zero weight.
  T u0[M], u1[M], acc0[M], acc1[M];
  T sw1 = T(0);
  double d0[M], d1[M], dsw1 = 0.0;  // RowSums<T, R>: FP64 totals of the rows' sums
#pragma unroll
  for (int c = 0; c < M; ++c) {
    u0[c] = c0[c];
    u1[c] = c0[LW * M + c];
    acc0[c] = T(0);
    acc1[c] = T(0);
    d0[c] = 0.0;
    d1[c] = 0.0;
  }
  auto flush = [&]() {
    if constexpr (RowSums<T, R>::on) {
#pragma unroll
      for (int c = 0; c < M; ++c) {
        d0[c] += (double)acc0[c];
        d1[c] += (double)acc1[c];
        acc0[c] = T(0);
        acc1[c] = T(0);
      }
      dsw1 += (double)sw1;
      sw1 = T(0);
    }
  };
  // A row of the window: the weights of both points are loaded first (one
  // uniform plane pointer per offset plus the lane's 32-bit byte offset),
  // then the LDS neighbour row is consumed.  The empty asm makes the byte
  // offsets opaque per row, so that the compiler keeps the plane pointers
  // uniform instead of hoisting 64-bit per-lane sums of them.  F0/F1: which
  // points take part; K0/K1: 0 own (plane q + dx, at o), 1 mirrored (q - dx,
  // at o + dx), 2 the split row of the point itself (dx < 0 mirrored from
  // plane -dx-1, dx > 0 own from plane dx-1, zero weight at dx = 0).
  auto row = [&](const T* ur, const char* q0, const char* q1, uint32_t o0, uint32_t o1, auto F0, auto F1, auto K0,
                 auto K1) {
    __asm__ volatile("" : "+v"(o0), "+v"(o1));
    T w0[NQ], w1[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int dx = i - R;
      if constexpr (decltype(F0)::value) {
        if constexpr (decltype(K0)::value == 0) w0[i] = *(const T*)(q0 + dx * qs + o0);
        if constexpr (decltype(K0)::value == 1) w0[i] = *(const T*)(q0 - dx * qs + (o0 + (uint32_t)(dx * TS)));
        if constexpr (decltype(K0)::value == 2) {
          if (dx < 0) w0[i] = *(const T*)(qb + (-dx - 1) * qs + (o0 + (uint32_t)(dx * TS)));
          if (dx > 0) w0[i] = *(const T*)(qb + (dx - 1) * qs + o0);
          if (dx == 0) w0[i] = T(0);
        }
      }
      if constexpr (decltype(F1)::value) {
        if constexpr (decltype(K1)::value == 0) w1[i] = *(const T*)(q1 + dx * qs + o1);
        if constexpr (decltype(K1)::value == 1) w1[i] = *(const T*)(q1 - dx * qs + (o1 + (uint32_t)(dx * TS)));
        if constexpr (decltype(K1)::value == 2) {
          if (dx < 0) w1[i] = *(const T*)(qb + (-dx - 1) * qs + (o1 + (uint32_t)(dx * TS)));
          if (dx > 0) w1[i] = *(const T*)(qb + (dx - 1) * qs + o1);
          if (dx == 0) w1[i] = T(0);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const int dx = i - R;
      if constexpr (decltype(F1)::value) sw1 += w1[i];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const T dv = ur[dx * M + c] - u0[c];
        if constexpr (decltype(F0)::value) acc0[c] = fma(w0[i], dv, acc0[c]);
        if constexpr (decltype(F1)::value) acc1[c] = fma(w1[i], dv, acc1[c]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  using Y = std::true_type;
  using N = std::false_type;
  using OWN = std::integral_constant<int, 0>;
  using MIR = std::integral_constant<int, 1>;
  using SPL = std::integral_constant<int, 2>;
  // plane q(0, dx) = dx - 1; q(dy, dx) = R + (dy - 1) (2R + 1) + dx + R for dy >= 1
  auto qrow = [&](int dy) -> const char* { return qb + (ptrdiff_t)(R + (dy - 1) * NQ + R) * qs; };

  // Row order -R, R+1, 0, 1, -1, 2, -2, 3, ..., -(R-1), R: plane rows k and
  // k+1 are read as own and as mirrored weights in neighbouring steps, so the
  // mirrored lines are still in L2 when they are needed again (measured: 1.2x
  // the algorithmic bytes, against 1.75x for the rows taken top to bottom).
  // The two end rows go first: that order leaves the fewest values live
  // (71 VGPRs for 4 FP32 columns, radius 5).
  // row -R: point 0 only, mirrored: plane q(R, -dx) at p0 - R W + dx
  row(c0 - R * LW * M, qrow(R), qb, pv0 - (uint32_t)R * wb, 0u, Y{}, N{}, MIR{}, MIR{});
  flush();
  // row R + 1: point 1 only, own q(R, dx) at p1
  row(c0 + (R + 1) * LW * M, qb, qrow(R), 0u, pv1, N{}, Y{}, OWN{}, OWN{});
  flush();

  // row 0 (point 0's): point 0 split at p0; point 1 mirrored, plane q(1, -dx) at p0 + dx
  row(c0, qb, qrow(1), pv0, pv0, Y{}, Y{}, SPL{}, MIR{});
  flush();
  // row 1 (point 1's): point 0 own q(1, dx) at p0; point 1 split at p1
  row(c0 + LW * M, qrow(1), qb, pv0, pv1, Y{}, Y{}, OWN{}, SPL{});
  flush();
  // (one row per step of the loop, which keeps one row's weights live)
#pragma unroll 1
  for (int j = 0; j < 2 * (R - 1); ++j) {
    const int k = 1 + (j >> 1);
    if ((j & 1) == 0) {
      // row -k: both mirrored at p0 - k W + dx, planes q(k, -dx) and q(k + 1, -dx)
      const uint32_t mrow = pv0 - (uint32_t)k * wb;
      row(c0 - k * LW * M, qrow(k), qrow(k + 1), mrow, mrow, Y{}, Y{}, MIR{}, MIR{});
    } else {
      // row k + 1: both own, planes q(k + 1, dx) at p0 and q(k, dx) at p1
      row(c0 + (k + 1) * LW * M, qrow(k + 1), qrow(k), pv0, pv1, Y{}, Y{}, OWN{}, OWN{});
    }
    flush();
  }
  if constexpr (RowSums<T, R>::on) {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      acc0[c] = (T)(-d0[c]);
      acc1[c] = (T)fma((double)(u1[c] - u0[c]), dsw1, -d1[c]);
    }
  } else {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      acc0[c] = -acc0[c];
      acc1[c] = fma(u1[c] - u0[c], sw1, -acc1[c]);
    }
  }
  double dotv = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const bool valid = h == 0 ? valid0 : valid1;
    const int64_t p = h == 0 ? p0 : p1;
    if (valid) {
      T xg[M], out[M];
#pragma unroll
      for (int c = 0; c < M; ++c) xg[c] = (a.form == GSF_FORM_LSYM || a.form == GSF_FORM_L) ? T(0) : in_col<T, M, M2>(a, p, c);
      finish_point<T, M>(a.form, isqd[p], xg, h == 0 ? acc0 : acc1, out);
#pragma unroll
      for (int c = 0; c < M; ++c) out_col<T, M, M2>(a, p, c, out[c]);
      if (DotCol<M, M2>::on && a.dot != nullptr)
        dotv += (double)in_col<T, M, M2>(a, p, DotCol<M, M2>::c) * (double)out[DotCol<M, M2>::c];
    }
  }
  if (a.dot != nullptr) {
    double v[1] = {dotv};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) a.dot[blockIdx.x] = v[0];
  }
}

// Cross stencil in 2D (the offsets along one axis, |o_k| <= R; R = 1 is the
// 5-point stencil): planes 0..R-1 hold the offsets (0, dx), planes R..2R-1
// the offsets (dy, 0).  Tiling and staging as in the square-window kernel;
// each point reads 2R own and 2R mirrored weights.
template <typename T, int M, int R, int RPT>
__global__ void __launch_bounds__(kThreads) bf_cross2d_kernel(ApplyArgs a) {
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
  const int64_t W = a.cols, H = a.rows;

  const int tile = xcd_tile(blockIdx.x, a.ntiles);
  const int64_t ty0 = (int64_t)(tile / a.tiles_x) * TY;
  const int64_t tx0 = (int64_t)(tile % a.tiles_x) * TX;
  const bool zspace = (a.form == GSF_FORM_N || a.form == GSF_FORM_LSYM);

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
  const size_t qstep = (size_t)a.pstride * sizeof(T);
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
    const uint32_t pv = ((uint32_t)p + (uint32_t)a.ppad) * (uint32_t)sizeof(T);
    const uint32_t wb = (uint32_t)W * (uint32_t)sizeof(T);
    const char* __restrict__ qh = (const char*)planes;                  // plane (0, 1)
    const char* __restrict__ qv = (const char*)planes + (size_t)R * qstep;  // plane (1, 0)
#pragma unroll
    for (int k = 1; k <= R; ++k) {
      const T wo = *(const T*)(qh + pv);
      const T wm = *(const T*)(qh + (pv - (uint32_t)(k * (int)sizeof(T))));
      const T vo = *(const T*)(qv + pv);
      const T vm = *(const T*)(qv + (pv - (uint32_t)k * wb));
      qh += qstep;
      qv += qstep;
      const T* ul = uc + k * M;
      const T* ur = uc - k * M;
      const T* ud = uc + k * LW * M;
      const T* uu = uc - k * LW * M;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        acc[c] = fma(wo, ui[c] - ul[c], acc[c]);
        acc[c] = fma(wm, ui[c] - ur[c], acc[c]);
        acc[c] = fma(vo, ui[c] - ud[c], acc[c]);
        acc[c] = fma(vm, ui[c] - uu[c], acc[c]);
      }
    }
    if (valid) {
      T xg[M], out[M];
#pragma unroll
      for (int c = 0; c < M; ++c) xg[c] = (a.form == GSF_FORM_LSYM || a.form == GSF_FORM_L) ? T(0) : x[p * a.ldx + c];
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

template <typename T, int M, int R, int RPT, int M2 = 0>
__global__ void __launch_bounds__(kThreads) bf_apply1d_kernel(ApplyArgs a) {
  constexpr int TN = kThreads * RPT;
  constexpr int LN = TN + 2 * R;
  __shared__ T us[LN * M];
  __shared__ double red[16];

  const T* __restrict__ planes = (const T*)a.planes;
  const T* __restrict__ isqd = (const T*)a.isqd;
  const int64_t n = a.n;
  const int64_t base = (int64_t)blockIdx.x * TN;
  const bool zspace = (a.form == GSF_FORM_N || a.form == GSF_FORM_LSYM);

  for (int e = threadIdx.x; e < LN; e += kThreads) {
    const int64_t g = base - R + e;
    const bool in = g >= 0 && g < n;
    T s = T(1);
    if (zspace && in) s = isqd[g];
#pragma unroll
    for (int c = 0; c < M; ++c) us[e * M + c] = in ? in_col<T, M, M2>(a, g, c) * s : T(0);
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
      for (int c = 0; c < M; ++c) xg[c] = (a.form == GSF_FORM_LSYM || a.form == GSF_FORM_L) ? T(0) : in_col<T, M, M2>(a, p, c);
      finish_point<T, M>(a.form, isqd[p], xg, acc, out);
#pragma unroll
      for (int c = 0; c < M; ++c) out_col<T, M, M2>(a, p, c, out[c]);
      if (DotCol<M, M2>::on && a.dot != nullptr)
        dotv += (double)in_col<T, M, M2>(a, p, DotCol<M, M2>::c) * (double)out[DotCol<M, M2>::c];
    }
  }
  if (a.dot != nullptr) {
    double v[1] = {dotv};
    block_sum<1>(v, red);
    if (threadIdx.x == 0) a.dot[blockIdx.x] = v[0];
  }
}

template <typename T, int M, int R, int RPT, int M2 = 0>
void launch_bf_tile(const ApplyArgs& a, int ndim, hipStream_t s, int* nblocks) {
  if constexpr (M2 == 0) {  // joint applies are not offered for the cross stencil
    if (ndim == 2 && a.cross) {
      constexpr int TY = 4 * RPT;
      ApplyArgs b = a;
      b.tiles_x = (int)((a.cols + 63) / 64);
      const int tiles_y = (int)((a.rows + TY - 1) / TY);
      b.ntiles = b.tiles_x * tiles_y;
      *nblocks = b.ntiles;
      bf_cross2d_kernel<T, M, R, RPT><<<b.ntiles, kThreads, 0, s>>>(b);
      return;
    }
  }
  if constexpr (RPT == 2) {
    if (ndim == 2) {  // two rows per thread computed together
      constexpr int PTY = 16;
      ApplyArgs b = a;
      b.tiles_x = (int)((a.cols + 63) / 64);
      const int tiles_y = (int)((a.rows + PTY - 1) / PTY);
      b.ntiles = b.tiles_x * tiles_y;
      *nblocks = b.ntiles;
      bf_apply2d_pair_kernel<T, M, R, PTY, M2><<<b.ntiles, 32 * PTY, 0, s>>>(b);
      return;
    }
  }
  if (ndim == 2) {
    constexpr int TY = 4 * RPT;
    ApplyArgs b = a;
    b.tiles_x = (int)((a.cols + 63) / 64);
    const int tiles_y = (int)((a.rows + TY - 1) / TY);
    b.ntiles = b.tiles_x * tiles_y;
    *nblocks = b.ntiles;
    bf_apply2d_kernel<T, M, R, RPT, M2><<<b.ntiles, kThreads, 0, s>>>(b);
  } else {
    constexpr int TN = kThreads * RPT;
    const int nb = (int)((a.n + TN - 1) / TN);
    *nblocks = nb;
    bf_apply1d_kernel<T, M, R, RPT, M2><<<nb, kThreads, 0, s>>>(a);
  }
}

template <typename T, int M, int R, int M2 = 0>
void launch_bf_rpt(const ApplyArgs& a, int ndim, int rpt, hipStream_t s, int* nb) {
  constexpr int MB = M * (int)sizeof(T);
  // taller tiles do not fit in LDS for wide FP64 blocks
  if constexpr (MB <= 32) {
    if (rpt >= 4) {
      launch_bf_tile<T, M, R, 4, M2>(a, ndim, s, nb);
      return;
    }
    if (rpt >= 2) {
      launch_bf_tile<T, M, R, 2, M2>(a, ndim, s, nb);
      return;
    }
  }
  launch_bf_tile<T, M, R, 1, M2>(a, ndim, s, nb);
}

template <typename T, int M, int M2 = 0>
void launch_bf_r(const ApplyArgs& a, int ndim, int r, int rpt, hipStream_t s, int* nb) {
  switch (r) {
    case 1: launch_bf_rpt<T, M, 1, M2>(a, ndim, rpt, s, nb); break;
    case 2: launch_bf_rpt<T, M, 2, M2>(a, ndim, rpt, s, nb); break;
    case 3: launch_bf_rpt<T, M, 3, M2>(a, ndim, rpt, s, nb); break;
    case 4: launch_bf_rpt<T, M, 4, M2>(a, ndim, rpt, s, nb); break;
    case 5: launch_bf_rpt<T, M, 5, M2>(a, ndim, rpt, s, nb); break;
    case 6: launch_bf_rpt<T, M, 6, M2>(a, ndim, rpt, s, nb); break;
    case 7: launch_bf_rpt<T, M, 7, M2>(a, ndim, rpt, s, nb); break;
    default: launch_bf_rpt<T, M, 8, M2>(a, ndim, rpt, s, nb); break;
  }
}

}  // namespace bfk

// one translation unit per (T, M) instantiates this
template <typename T, int M>
void bf_apply_tm(const bfk::ApplyArgs& a, int ndim, int r, int rpt, hipStream_t s, int* nb);
// joint applies: M - 1 columns from x plus one from x2 (one translation unit per (T, M))
template <typename T, int M>
void bf_apply_joint_tm(const bfk::ApplyArgs& a, int ndim, int r, int rpt, hipStream_t s, int* nb);

}  // namespace gsf
