// Guided-filter operator apply in one pass (Section 3, Algorithm 1 with the
// fixed guidance g, eqs. (5)-(6)), one FP32 column: the two box-filter stages
// of Algorithm 1 chained through on-chip memory, so the window coefficients
// (a_k, b_k) never reach HBM.  (Blocks of columns and FP64 data take the
// two-pass kernels of apply_gf.hip: with the columns of a block interleaved
// per point, a pass over column pairs reads x at a stride and re-reads the
// guidance data per pair, 3.9 ms against 1.5 ms at m = 8, 4096^2, r = 8.)
//
// A workgroup of 256 threads owns a strip of 256 columns (thread t = strip
// column t, global column c0 - 2r + t) and a chunk of rows, and walks the
// window-centre rows k_y top to bottom.  Every step is done by the column's
// own thread; horizontal window sums are differences of a prefix sum along the
// strip row (a wave-wide scan by DPP lane shifts, plus the totals of the
// waves to the left), so no thread loops over a window.  Per centre row:
//   A  running FP64 vertical window sums of u = D^-1/2 x and g u over input
//      rows k_y - r .. k_y + r (add the entering row, subtract the leaving
//      one), scanned along the row;
//   C  the centre's horizontal sums from two prefix values and its
//      coefficients
//        a_k = (mean(g u)_k - mu_k mean(u)_k) / (sigma_k^2 + eps),
//        b_k = mean(u)_k - a_k mu_k
//      (mu_k and 1/(sigma_k^2 + eps) from the operator build), rounded to
//      FP32 as the two-pass path stores them, pushed into the column's
//      LDS ring of the last 2r + 1 centre rows and added to running FP64
//      vertical sums of (a, b), scanned along the row;
//   E  the output point of row k_y - r in this column: horizontal sums of
//      (a, b) from two prefix values and the output form
//        GF(u)_i = (g_i sum a + sum b) / N_i,  N x = D^1/2 GF(D^-1/2 x), ...;
//      then the oldest ring row leaves the (a, b) sums.
// Two barriers per row order the two prefix rows in LDS (LDS-only fences).  The strip's
// 256 - 4r output columns carry a 2r halo on each side (r for each box); a
// chunk of rb output rows walks rb + 2r centre rows.  Loads run D centre
// rows ahead in a register ring (entering and leaving input rows, the centre
// row's statistics, the output row's g and x).  HBM traffic per point is
// Algorithm 1's own: x, g, mu, 1/(var + eps) in and y out (the rows re-read
// for the leaving sums and the epilogue hit L2).  Counts and 1/sqrt(d) come
// from the border-truncated window sizes with the same expressions as the
// operator build (interior values computed once), so u equals the
// stored-diagonal product bit for bit.  A 1D signal is one row with no
// vertical window.
#include <cmath>

#include "gsf_internal.h"

namespace gsf {
namespace {

constexpr int kFT = 256;  // threads per workgroup = columns per strip

struct FusedArgs {
  const float* x;
  int ldx;
  const float* g;
  const float* mu;
  const float* inv;
  float* y;
  int ldy;
  int rows, cols;
  int rb;       // output rows per workgroup
  int form;
  double omega;  // |w| = (2r+1)^ndim
};

__device__ __forceinline__ int fcount(int v, int len, int r) {
  const int lo = v - r < 0 ? 0 : v - r;
  const int hi = v + r >= len ? len - 1 : v + r;
  return hi - lo + 1;
}

// DPP lane move of a double, 0 where the source lane is outside the row or
// the destination row is masked off
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp0(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4, 8
// within rows of 16 lanes, then the row totals broadcast to the rows above
__device__ __forceinline__ double wave_scan(double v) {
  v += dpp0<0x111, 0xf>(v);
  v += dpp0<0x112, 0xf>(v);
  v += dpp0<0x114, 0xf>(v);
  v += dpp0<0x118, 0xf>(v);
  v += dpp0<0x142, 0xa>(v);
  v += dpp0<0x143, 0xc>(v);
  return v;
}

// Workgroup barrier that orders LDS only: the fences name the local address
// space, so the loads of rows ahead stay in flight across it (a plain
// __syncthreads also waits for every outstanding global load).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// window sum over strip columns t - R .. t + R from the per-wave inclusive
// scans P and the wave totals T: the two ends are at most one wave apart
// (R < 64), so the sum is P[hi] - P[lo - 1] plus the total of lo - 1's wave
// when it is not hi's wave (lo - 1 = -1: the empty prefix)
template <int R>
__device__ __forceinline__ double box_sum(const double* P, const double* T, int t) {
  const int hi = t + R, lo = t - R - 1;
  double v = P[hi];
  if (lo >= 0) {
    v -= P[lo];
    if ((lo >> 6) != (hi >> 6)) v += T[lo >> 6];
  }
  return v;
}

// R: window radius; RV: vertical radius (R for images, 0 for a 1D signal);
// M: columns of the block (1 or 2); D: rows of loads in flight.
template <int R, int RV, int M, int D>
__global__ void __launch_bounds__(kFT) gf_fused_kernel(FusedArgs a) {
  constexpr int NC = 2 * M;            // channels per point: (u_j, g u_j), later (a_j, b_j)
  constexpr int NOUT = kFT - 4 * R;    // outputs per strip row (strip columns 2R .. 255 - 2R)
  constexpr int NR = 2 * RV + 1;       // rows of the (a, b) ring
  constexpr int NW = kFT / 64;
  __shared__ double P1[NC][kFT];
  __shared__ double P2[NC][kFT];
  __shared__ double T1[NC][NW];
  __shared__ double T2[NC][NW];
  __shared__ float ring[NR][NC][kFT];  // this column's (a, b) of the last NR centre rows

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int rows = a.rows, cols = a.cols;
  const int c0 = (int)blockIdx.x * NOUT;
  const int y0 = (int)blockIdx.y * a.rb;
  const int y1 = y0 + a.rb < rows ? y0 + a.rb : rows;
  const bool scale = a.form == GSF_FORM_N || a.form == GSF_FORM_LSYM;
  const int col = c0 - 2 * R + t;
  const bool cin = col >= 0 && col < cols;
  const int colc = cin ? col : 0;
  const bool centre_col = cin && t >= R && t < kFT - R;
  const bool out_col = cin && t >= 2 * R && t < kFT - 2 * R;
  const double rh = 1.0 / (double)fcount(colc, cols, R);
  const double srh = sqrt(rh);
  const double sro = 1.0 / sqrt(a.omega);
  // vertical window sizes: 2RV + 1 away from the top and bottom RV rows
  const double rv_in = 1.0 / (double)(2 * RV + 1 < rows ? 2 * RV + 1 : rows);
  const double srv_in = sqrt(rv_in);
  auto interior = [&](int v) { return v >= RV && v < rows - RV; };
  auto rv_of = [&](int v) { return interior(v) ? rv_in : 1.0 / (double)fcount(v, rows, RV); };
  // 1/sqrt(d) with d = N / |w|, as the operator build computes and stores it
  auto dinv_of_rv = [&](double rv) {
    const double d = 1.0 / ((rv * rh) * a.omega);
    return (double)(float)(1.0 / sqrt(d));
  };
  const double dinv_in = dinv_of_rv(rv_in);
  auto dinv_at = [&](int v) { return interior(v) ? dinv_in : dinv_of_rv(1.0 / (double)fcount(v, rows, RV)); };
  auto clamp_row = [&](int v) { return v < 0 ? 0 : (v >= rows ? rows - 1 : v); };

  struct Slot {
    float xin[M], gin, xl[M], gl, mu, inv, eg, ex[M];
  };
  auto fill = [&](Slot& s, int k) {
    const size_t pin = (size_t)clamp_row(k + RV) * cols + colc, pl = (size_t)clamp_row(k - RV - 1) * cols + colc;
    const size_t pk = (size_t)clamp_row(k) * cols + colc, po = (size_t)clamp_row(k - RV) * cols + colc;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      s.xin[j] = a.x[pin * a.ldx + j];
      s.xl[j] = a.x[pl * a.ldx + j];
      s.ex[j] = a.x[po * a.ldx + j];
    }
    s.gin = a.g[pin];
    s.gl = a.g[pl];
    s.mu = a.mu[pk];
    s.inv = a.inv[pk];
    s.eg = a.g[po];
  };

  // stage A warm-up: input rows y0 - 2RV .. y0 - 1 of the first centre row's window
  double sA[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) sA[c] = 0.0;
  const int wlo = y0 - 2 * RV < 0 ? 0 : y0 - 2 * RV;
  if (cin) {
    for (int yy = wlo; yy < y0 && yy < rows; ++yy) {
      const size_t p = (size_t)yy * cols + colc;
      const double di = scale ? dinv_at(yy) : 1.0;
      const double gv = (double)a.g[p];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const double u = (double)a.x[p * a.ldx + j] * di;
        sA[2 * j] += u;
        sA[2 * j + 1] += gv * u;
      }
    }
  }
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) ring[q][c][t] = 0.0f;
  double S[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) S[c] = 0.0;

  const int ks = y0 - RV, ke = y1 + RV;  // centre rows of this chunk
  Slot slot[D];
#pragma unroll
  for (int u = 0; u < D; ++u) fill(slot[u], ks + u);
  for (int kb = ks; kb < ke; kb += D) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int k = kb + u;
      const Slot cur = slot[u];
      fill(slot[u], k + D);
      if (k < ke) {  // uniform over the workgroup
        // A: the column's vertical sums for centre row k, scanned along the row
        const int yin = k + RV, yl = k - RV - 1;
        const bool ain = cin && yin >= 0 && yin < rows;
        const bool lin = cin && yl >= wlo && yl < rows;
        const double din = scale ? dinv_at(yin) : 1.0;
        const double dl = scale ? dinv_at(yl) : 1.0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const double ui = (double)cur.xin[j] * din, ul = (double)cur.xl[j] * dl;
          sA[2 * j] += (ain ? ui : 0.0) - (lin ? ul : 0.0);
          sA[2 * j + 1] += (ain ? (double)cur.gin * ui : 0.0) - (lin ? (double)cur.gl * ul : 0.0);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double p = wave_scan(cin ? sA[c] : 0.0);
          P1[c][t] = p;
          if (lane == 63) T1[c][wave] = p;
        }
        lds_barrier();
        // C: the centre's (a, b), into the ring and the vertical (a, b) sums
        float abn[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) abn[c] = 0.0f;
        if (centre_col && k >= 0 && k < rows) {
          const double rc = rv_of(k) * rh;
          const double mk = (double)cur.mu, ik = (double)cur.inv;
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const double su = box_sum<R>(P1[2 * j], T1[2 * j], t);
            const double sgu = box_sum<R>(P1[2 * j + 1], T1[2 * j + 1], t);
            const double mean_u = su * rc, mean_gu = sgu * rc;
            const double av = (mean_gu - mk * mean_u) * ik;
            abn[2 * j] = (float)av;
            abn[2 * j + 1] = (float)(mean_u - av * mk);
          }
        }
        // slot of centre row k: it held row k - NR, which already left the sums
        const int slot_k = ((k % NR) + NR) % NR;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          ring[slot_k][c][t] = abn[c];
          S[c] += (double)abn[c];
          const double p = wave_scan(S[c]);
          P2[c][t] = p;
          if (lane == 63) T2[c][wave] = p;
        }
        lds_barrier();
        // E: the output point of row k - RV in this column
        const int yo = k - RV;
        if (out_col && yo >= y0 && yo < y1) {
          const double rvo = rv_of(yo);
          const double rc = rvo * rh, src = (interior(yo) ? srv_in : sqrt(rvo)) * srh;
          const double gi = (double)cur.eg;
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const double sa = box_sum<R>(P2[2 * j], T2[2 * j], t);
            const double sb = box_sum<R>(P2[2 * j + 1], T2[2 * j + 1], t);
            const double gfu = gi * sa + sb;
            const double xi = (double)cur.ex[j];
            double out;
            if (a.form == GSF_FORM_RW) {
              out = gfu * rc;
            } else if (a.form == GSF_FORM_L) {
              out = (xi - gfu * rc) * (sro * sro / rc);
            } else {
              const double nx = gfu * (src * sro);
              out = a.form == GSF_FORM_LSYM ? xi - nx : nx;
            }
            a.y[((size_t)yo * cols + col) * a.ldy + j] = (float)out;
          }
        }
        // the oldest centre row, k - 2RV, leaves the (a, b) sums
        const int slot_o = (((k - 2 * RV) % NR) + NR) % NR;
#pragma unroll
        for (int c = 0; c < NC; ++c) S[c] -= (double)ring[slot_o][c][t];
      }
    }
  }
}

template <int R, int RV, int M>
void launch_fused_rm(const FusedArgs& a0, hipStream_t s) {
  constexpr int D = 2;
  constexpr int NOUT = kFT - 4 * R;
  FusedArgs a = a0;
  const int strips = (a.cols + NOUT - 1) / NOUT;
  // rows per workgroup: about 1024 workgroups (four per CU), at least 32 rows
  // so that the 2r extra centre rows of a chunk stay a modest share
  int rb = (int)(((int64_t)a.rows * strips + 1023) / 1024);
  rb = rb < 32 ? 32 : (rb > 256 ? 256 : rb);
  if (RV == 0) rb = 1;
  a.rb = rb;
  const dim3 grid((unsigned)strips, (unsigned)((a.rows + rb - 1) / rb));
  gf_fused_kernel<R, RV, M, D><<<grid, kFT, 0, s>>>(a);
}

template <int M>
void launch_fused_m(const FusedArgs& a, int r, bool two_d, hipStream_t s) {
#define GSF_FUSED_CASE(RR)                                        \
  case RR:                                                        \
    if (two_d) launch_fused_rm<RR, RR, M>(a, s);                   \
    else launch_fused_rm<RR, 0, M>(a, s);                          \
    break;
  switch (r) {
    GSF_FUSED_CASE(1)
    GSF_FUSED_CASE(2)
    GSF_FUSED_CASE(3)
    GSF_FUSED_CASE(4)
    GSF_FUSED_CASE(5)
    GSF_FUSED_CASE(6)
    GSF_FUSED_CASE(7)
    default: GSF_FUSED_CASE(8)
  }
#undef GSF_FUSED_CASE
}

}  // namespace

// One-pass GF apply of one FP32 column.
gsf_status launch_gf_apply_fused(const Operator& op, int form, const float* x, int64_t ldx, float* y, int64_t ldy,
                                 hipStream_t s) {
  FusedArgs a{};
  a.x = x;
  a.y = y;
  a.g = (const float*)op.g;
  a.mu = (const float*)op.mu;
  a.inv = (const float*)op.inv;
  a.ldx = (int)ldx;
  a.ldy = (int)ldy;
  a.rows = (int)op.rows;
  a.cols = (int)op.cols;
  a.form = form;
  const double w = 2.0 * op.desc.radius + 1.0;
  a.omega = op.desc.ndim == 1 ? w : w * w;
  launch_fused_m<1>(a, op.desc.radius, op.desc.ndim == 2, s);
  return launch_status();
}

}  // namespace gsf
