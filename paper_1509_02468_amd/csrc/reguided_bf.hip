// Re-guided BF passes with the weights of eq. (2) evaluated where they are
// used.  The re-guided filters (Sections 2-3: the graph built from the
// current iterate at every step) use each graph for one or two passes, so
// storing it as half-window planes (a rebuild writes (K-1)/2 planes per point
// and the apply reads them back) costs more than evaluating eq. (2) again.
// One kernel stages a tile of the guidance g (and of the vector v) with its
// halo in LDS and evaluates every weight of its points' windows:
//   DEG  d_i = 1 + sum_{j != i} w_ij   (normalisation by D; by diag L: without
//        the 1, and 1 where the sum is 0), written as FP64
//   RW   y_i = v_i - (1/d_i) sum_{j != i} w_ij (v_i - v_j) = (D^-1 W v)_i, v = g
//   LAP  y_i = sum_{j != i} w_ij (v_i - v_j) = (L v)_i (the self-loop cancels
//        in L = D - W under both normalisations), and per workgroup the
//        partial sum of v_i y_i
//   BUILD the operator build of FP32 data in one pass: the weights of the
//        forward half-window written into the planes (w_{i,i+o}, 0 off the
//        grid), d_i as the FP64 sum of all the point's FP32 weights (the same
//        values the planes hold, since w_ij and w_ji are bitwise equal), and
//        1/sqrt(d_i), sqrt(d_i)
// FP32 data: w = 2^(-(|o|^2 cs + (g_i - g_j)^2 cr) log2 e) with the hardware
// base-2 exponential (the constants folded with log2 e; the relative error of
// a weight is a few units of 2^-24 times (1 + its exponent's magnitude)); the
// sums over one row of the window in FP32, the rows summed in FP64.  FP64
// data: exp in FP64 of the same argument as the operator build, all sums FP64.
// The argument is bitwise the same for (i, j) and (j, i): W stays exactly
// symmetric.
#include <cmath>

#include "gsf_internal.h"

namespace gsf {
namespace {

constexpr int kRgThreads = 256;
constexpr int kRgPts = 4;  // outputs per thread

enum { RG_DEG = 0, RG_RW = 1, RG_LAP = 2, RG_BUILD = 3 };

struct RgParams {
  int rows, cols;  // 1D: one row
  int ry, rx;      // window radii (1D: ry = 0)
  int cross;       // 2D cross stencil: offsets (dy, 0) and (0, dx) only
  int diagl;       // normalise by diag L
  double cs, cr;   // 1 / (2 sigma^2), 0 for sigma = inf
  float ncs2, ncr2;  // -cs log2 e, -cr log2 e
  int tiles_x, ntiles;
  // BUILD: the half-window planes (plane q's data at planes + ppad + q pstride)
  // and the 1/sqrt(d), sqrt(d) outputs
  void* planes;
  int64_t pstride, ppad;
  void* diag;
  void* sqd;
};

// Plane of the forward offset (dy, dx) (dy > 0, or dy = 0 and dx > 0), in the
// order of the operator build: (0, 1..r), then the rows dy = 1..r (all dx of
// the square window, dx = 0 only on the cross lattice).
__device__ __forceinline__ int rg_plane(int dy, int dx, int r, int cross) {
  if (dy == 0) return dx - 1;
  return cross ? r + dy - 1 : r + (dy - 1) * (2 * r + 1) + dx + r;
}

extern __shared__ double rg_smem[];

// Tile of TW x TH outputs (2D: 64 x 16; 1D: 1024 x 1); thread t computes the
// points t + 256 s (s < 4) of the tile in row-major order.  The LDS tile's
// pitch is fixed (TW plus the largest halo), so the four points of a thread
// are a compile-time distance apart and share one address per offset.
template <int TW>
struct RgPitch {
  static constexpr int v = TW + 2 * kMaxRadius;
};

// C > 1 (BUILD only): the guidance has C channels, staged as C LDS planes
// cplane values apart, and the photometric distance is the Euclidean one.
template <typename T, int MODE, int TW, int TH, bool BORDER, int C>
__device__ __forceinline__ void rg_tile(const T* __restrict__ gs, const T* __restrict__ vs, T* __restrict__ y,
                                        double* __restrict__ deg, double& dotv, const RgParams& p, int x0, int y0,
                                        int cplane) {
  constexpr int pitch = RgPitch<TW>::v;
  // LDS distance between a thread's consecutive points: 256 / TW rows, or 256
  // columns of one row
  constexpr int step = TW <= kRgThreads ? (kRgThreads / TW) * pitch : kRgThreads;
  const int tid = threadIdx.x;
  const int oy0 = tid / TW, ox0 = tid - (tid / TW) * TW;
  const int cc = (oy0 + p.ry) * pitch + ox0 + p.rx;  // centre of point 0
  int gyo[kRgPts], gxo[kRgPts];
  T gi[kRgPts], vi[kRgPts];
  T gic[C][kRgPts];  // C > 1: the point's channels
  double acc[kRgPts], ws[kRgPts];
#pragma unroll
  for (int t = 0; t < kRgPts; ++t) {
    const int l = tid + kRgThreads * t;
    gyo[t] = y0 + l / TW;
    gxo[t] = x0 + (l - (l / TW) * TW);
    gi[t] = gs[cc + t * step];
#pragma unroll
    for (int c = 0; c < C; ++c) gic[c][t] = gs[c * cplane + cc + t * step];
    vi[t] = MODE == RG_LAP ? vs[cc + t * step] : gi[t];
    acc[t] = 0.0;
    ws[t] = 0.0;
  }
  for (int dy = -p.ry; dy <= p.ry; ++dy) {
    const bool axis = p.cross && dy != 0;
    const int dxlo = axis ? 0 : -p.rx, dxhi = axis ? 0 : p.rx;
    T racc[kRgPts], rws[kRgPts];
#pragma unroll
    for (int t = 0; t < kRgPts; ++t) {
      racc[t] = T(0);
      rws[t] = T(0);
    }
    for (int dx = dxlo; dx <= dxhi; ++dx) {
      if (dy == 0 && dx == 0) continue;
      const int o2 = dy * dy + dx * dx;
      const T* gq = gs + cc + dy * pitch + dx;
      const T* vq = vs + cc + dy * pitch + dx;
      const float nsp = (float)o2 * p.ncs2;
#pragma unroll
      for (int t = 0; t < kRgPts; ++t) {
        const T gj = gq[t * step];
        const T d = gi[t] - gj;
        T w;
        if constexpr (C > 1) {
          // sum of the channels' squared differences, kept finite for cr = 0
          float d2 = 0.0f;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const float dc = gic[c][t] - gq[c * cplane + t * step];
            d2 = fmaf(dc, dc, d2);
          }
          w = __builtin_amdgcn_exp2f(fmaf(fminf(d2, 3.0e38f), p.ncr2, nsp));
        } else if constexpr (sizeof(T) == 4) {
          // d (d cr') rather than d^2 cr': with cr = 0 (sigma_r = inf) the
          // term is 0 for any finite d, and a huge d gives 2^-inf = 0
          w = __builtin_amdgcn_exp2f(fmaf(d, d * p.ncr2, nsp));
        } else {
          w = exp(-((double)o2 * p.cs + d * d * p.cr));
        }
        if (BORDER) {
          const bool ok = (unsigned)(gyo[t] + dy) < (unsigned)p.rows && (unsigned)(gxo[t] + dx) < (unsigned)p.cols;
          w = ok ? w : T(0);
        }
        if (MODE == RG_BUILD) {
          ws[t] += (double)w;
          const bool fwd = dy > 0 || (dy == 0 && dx > 0);
          if (fwd && (!BORDER || (gyo[t] < p.rows && gxo[t] < p.cols)))
            ((T*)p.planes)[p.ppad + (int64_t)rg_plane(dy, dx, p.rx, p.cross) * p.pstride + gyo[t] * p.cols +
                           gxo[t]] = w;
        } else {
          rws[t] += w;
        }
        if (MODE == RG_RW) racc[t] = fma(w, d, racc[t]);
        if (MODE == RG_LAP) racc[t] = fma(w, vi[t] - vq[t * step], racc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < kRgPts; ++t) {
      acc[t] += (double)racc[t];
      ws[t] += (double)rws[t];
    }
  }
#pragma unroll
  for (int t = 0; t < kRgPts; ++t) {
    if (BORDER && (gyo[t] >= p.rows || gxo[t] >= p.cols)) continue;
    const int i = gyo[t] * p.cols + gxo[t];
    double d = p.diagl ? ws[t] : 1.0 + ws[t];
    if (d == 0.0) d = 1.0;
    if (MODE == RG_DEG || MODE == RG_BUILD) deg[i] = d;
    if (MODE == RG_BUILD) {
      ((T*)p.diag)[i] = (T)(1.0 / sqrt(d));
      ((T*)p.sqd)[i] = (T)sqrt(d);
    }
    if (MODE == RG_RW) y[i] = (T)((double)vi[t] - acc[t] / d);
    if (MODE == RG_LAP) {
      const T yt = (T)acc[t];
      y[i] = yt;
      dotv += (double)vi[t] * (double)yt;
    }
  }
}

template <typename T, int MODE, int TW, int TH, int C = 1>
__global__ void __launch_bounds__(kRgThreads) rg_bf_kernel(const T* __restrict__ g, const T* __restrict__ v,
                                                           T* __restrict__ y, double* __restrict__ deg,
                                                           double* __restrict__ dot, RgParams p) {
  static_assert(TW * TH == kRgThreads * kRgPts, "one tile is 4 points per thread");
  __shared__ double red[16];
  const int b = xcd_tile((int)blockIdx.x, p.ntiles);
  const int ty = b / p.tiles_x, tx = b - ty * p.tiles_x;
  const int x0 = tx * TW, y0 = ty * TH;
  constexpr int pitch = RgPitch<TW>::v;
  const int width = TW + 2 * p.rx, hrows = TH + 2 * p.ry, cells = width * hrows;
  T* gs = (T*)rg_smem;
  T* vs = gs + pitch * hrows;
  for (int c = threadIdx.x; c < cells; c += kRgThreads) {
    const int ly = c / width, lx = c - ly * width;
    const int gy = y0 - p.ry + ly, gx = x0 - p.rx + lx;
    const bool in = (unsigned)gy < (unsigned)p.rows && (unsigned)gx < (unsigned)p.cols;
    const int i = in ? gy * p.cols + gx : 0;
    if constexpr (C == 1) {
      gs[ly * pitch + lx] = in ? g[i] : T(0);
    } else {
#pragma unroll
      for (int ch = 0; ch < C; ++ch) gs[ch * pitch * hrows + ly * pitch + lx] = in ? g[(int64_t)i * C + ch] : T(0);
    }
    if (MODE == RG_LAP) vs[ly * pitch + lx] = in ? v[i] : T(0);
  }
  __syncthreads();
  const bool interior = x0 - p.rx >= 0 && x0 + TW + p.rx <= p.cols && y0 - p.ry >= 0 && y0 + TH + p.ry <= p.rows;
  double dotv = 0.0;
  if (interior)
    rg_tile<T, MODE, TW, TH, false, C>(gs, vs, y, deg, dotv, p, x0, y0, pitch * hrows);
  else
    rg_tile<T, MODE, TW, TH, true, C>(gs, vs, y, deg, dotv, p, x0, y0, pitch * hrows);
  if (MODE == RG_LAP && dot != nullptr) {
    double t[1] = {dotv};
    block_sum<1>(t, red);
    if (threadIdx.x == 0) dot[blockIdx.x] = t[0];
  }
}

inline double inv_two_sigma2(double s) { return std::isinf(s) ? 0.0 : 1.0 / (2.0 * s * s); }

struct RgGeom {
  RgParams p;
  int tw, th;
  size_t lds;  // bytes of dynamic LDS
};

RgGeom rg_geom(const Operator& op, int mode) {
  RgGeom g{};
  const gsf_operator_desc& d = op.desc;
  const bool two = d.ndim == 2;
  g.tw = two ? 64 : 1024;
  g.th = two ? 16 : 1;
  g.p.rows = (int)op.rows;
  g.p.cols = (int)op.cols;
  g.p.ry = two ? d.radius : 0;
  g.p.rx = d.radius;
  g.p.cross = bf_cross2d(d) ? 1 : 0;
  g.p.diagl = d.norm == GSF_NORM_DIAGL ? 1 : 0;
  g.p.cs = inv_two_sigma2(d.sigma_d);
  g.p.cr = inv_two_sigma2(d.sigma_r);
  const double log2e = 1.4426950408889634;
  g.p.ncs2 = (float)(-g.p.cs * log2e);
  g.p.ncr2 = (float)(-g.p.cr * log2e);
  g.p.tiles_x = (int)((op.cols + g.tw - 1) / g.tw);
  const int tiles_y = (int)((op.rows + g.th - 1) / g.th);
  g.p.ntiles = g.p.tiles_x * tiles_y;
  const size_t cells = (size_t)(g.tw + 2 * kMaxRadius) * (g.th + 2 * g.p.ry);  // fixed pitch
  g.lds = cells * op.elem * (mode == RG_LAP ? 2 : 1);
  return g;
}

template <typename T, int MODE, int C = 1>
void rg_launch(const RgGeom& g, const void* gd, const void* v, void* y, double* deg, double* dot, hipStream_t s) {
  if (g.th == 16)
    rg_bf_kernel<T, MODE, 64, 16, C><<<g.p.ntiles, kRgThreads, g.lds * C, s>>>((const T*)gd, (const T*)v, (T*)y,
                                                                               deg, dot, g.p);
  else
    rg_bf_kernel<T, MODE, 1024, 1, C><<<g.p.ntiles, kRgThreads, g.lds * C, s>>>((const T*)gd, (const T*)v, (T*)y,
                                                                                deg, dot, g.p);
}

template <typename T>
void rg_dispatch(const RgGeom& g, int mode, const void* gd, const void* v, void* y, double* deg, double* dot,
                 hipStream_t s) {
  if (mode == RG_DEG)
    rg_launch<T, RG_DEG>(g, gd, v, y, deg, dot, s);
  else if (mode == RG_RW)
    rg_launch<T, RG_RW>(g, gd, v, y, deg, dot, s);
  else
    rg_launch<T, RG_LAP>(g, gd, v, y, deg, dot, s);
}

// Zeros of the plane region that are not weights: the ppad entries before
// each plane's data, the tail up to the next plane, and the ppad entries after
// the last plane (the apply's mirrored reads land there instead of branching).
template <typename T>
__global__ void __launch_bounds__(kRgThreads) rg_plane_pads_kernel(T* __restrict__ planes, int64_t n,
                                                                   int64_t pstride, int64_t ppad, int nplanes) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= pstride - n) return;
  const int64_t idx = t < ppad ? t : t + n;  // skips the data [ppad, ppad + n)
  for (int q = 0; q < nplanes; ++q) planes[(int64_t)q * pstride + idx] = T(0);
  if (t < ppad) planes[(int64_t)nplanes * pstride + t] = T(0);
}

}  // namespace

// Operator build of FP32 BF data with one or three guidance channels in one
// window pass (the weights of eq. (2) in FP32, the degrees as FP64 sums of
// exactly the stored values) plus the pad zeros; false (nothing launched) for
// other descriptors, which take the two-kernel build with FP64 exponentials.
bool launch_bf_build_onepass(const Operator& op, const void* guidance, hipStream_t s) {
  const int ch = desc_channels(op.desc);
  if (op.desc.kind != GSF_BF || op.desc.prec != GSF_F32 || (ch != 1 && ch != 3)) return false;
  RgGeom geo = rg_geom(op, RG_BUILD);
  geo.p.planes = op.planes;
  geo.p.pstride = op.pstride;
  geo.p.ppad = op.ppad;
  geo.p.diag = op.diag;
  geo.p.sqd = op.sqd;
  const int64_t npad = op.pstride - op.n;
  rg_plane_pads_kernel<float><<<(unsigned)((npad + kRgThreads - 1) / kRgThreads), kRgThreads, 0, s>>>(
      (float*)op.planes, op.n, op.pstride, op.ppad, op.nplanes);
  if (ch == 3)
    rg_launch<float, RG_BUILD, 3>(geo, guidance, nullptr, nullptr, op.deg, nullptr, s);  // e.g. CIE-Lab
  else
    rg_launch<float, RG_BUILD>(geo, guidance, nullptr, nullptr, op.deg, nullptr, s);
  return true;
}

// Workgroups (and so partials) of one fused pass.
int rg_bf_blocks(const Operator& op) { return rg_geom(op, RG_LAP).p.ntiles; }

// One fused pass on the BF graph of guidance g (mode 0: degrees into op.deg;
// 1: y = D^-1 W g; 2: y = L v with per-workgroup partials of v^T y in dot
// when it is not null).  Needs only op.desc, the grid and op.deg.
gsf_status launch_rg_bf(const Operator& op, int mode, const void* g, const void* v, void* y, double* dot,
                        int* nparts, hipStream_t s) {
  if (op.desc.kind != GSF_BF || mode < RG_DEG || mode > RG_LAP) return GSF_EINVAL;
  const RgGeom geo = rg_geom(op, mode);
  if (op.desc.prec == GSF_F32)
    rg_dispatch<float>(geo, mode, g, v, y, op.deg, dot, s);
  else
    rg_dispatch<double>(geo, mode, g, v, y, op.deg, dot, s);
  if (nparts != nullptr) *nparts = geo.p.ntiles;
  return launch_status();
}

}  // namespace gsf
