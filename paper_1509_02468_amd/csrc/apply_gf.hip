// Guided-filter operator (Section 3, Algorithm 1, eqs. (5)-(6)): the operator
// build (window statistics of the guidance) and the normalized apply
//   N x = D^1/2 GF(D^-1/2 x),  D = diag(N_i / |w|),
// where GF is Algorithm 1 with the fixed guidance g (a linear filter), mean
// filters over border-truncated windows (N_k points) and the window
// statistics mu_k, inv_k = 1/(sigma_k^2 + eps):
//   u      = D^-1/2 x            (RW form: u = x)
//   a_k    = (box(g u)_k / N_k - mu_k box(u)_k / N_k) inv_k
//   b_k    = box(u)_k / N_k - a_k mu_k
//   GF(u)_i = (g_i box(a)_i + box(b)_i) / N_i
//
// Every window sum runs in one streaming kernel of one wave per workgroup (see
// gf_box_kernel): running FP64 vertical sums in registers, sliding horizontal
// sums over the wave's own LDS row, no barriers.  Cost per point is O(1) in
// the radius.  The apply is two such kernels (u, g u) -> (a, b) and
// (a, b) -> output for up to 8 columns at once; the build is one kernel on
// (g, g^2).  A 1D signal is one row.
#include <cmath>

#include "gsf_internal.h"

namespace gsf {
namespace {

constexpr int kGfLanes = 64;   // one wave per workgroup; lane = halo column
// output rows per workgroup (fewer on small grids); 16 / 24 / 32 / 64 / 128
// compared in alternating runs on one GPU at 4096^2, r = 8, FP32: m = 8 apply
// 1485 / 1462 / 1438-1447 / 1474 / (step +1%) us, m = 4 820 / 798 / 787-791 /
// 807-810 us: more, shorter workgroups hide the row loads better than the
// fewer warm-up rows of long ones save
constexpr int kGfRowsMax = 32;

// 32-bit indices: the operator build rejects GF grids of 2^27 points or more,
// so point * 16 fits.
struct GfGeom {
  int rows, cols;
  int r;
  int rb;  // output rows per workgroup
};

__device__ __forceinline__ int win_count(int v, int len, int r) {
  const int lo = v - r < 0 ? 0 : v - r;
  const int hi = v + r >= len ? len - 1 : v + r;
  return hi - lo + 1;
}

// Keeps the compiler from moving LDS accesses across this point; a wave's
// own LDS operations complete in order, so no hardware barrier is needed.
__device__ __forceinline__ void wave_lds_fence() { __asm__ volatile("" ::: "memory"); }

// One wave owns a strip of 64 CPL - 2r output columns (64 CPL halo columns,
// CPL per lane: lane + 64 k) and g.rb rows (8..64).  Lane l keeps the FP64
// running vertical window sums of its columns c0 - r + l + 64 k for the 2M
// channels (P::M groups of two); per row it
// adds the entering row, writes its sums to the wave's LDS row, and then
// takes the horizontal window sums as lane (group, run of consecutive output
// columns) with a sliding sum over that LDS row, before subtracting the
// leaving row.  Loads are unconditional (clamped addresses, results selected)
// and issued D rows ahead (a register ring, the row loop unrolled by D), so
// a memory latency is spread over D rows.
//   P::Row       raw loads of one point (all groups)
//   P::fetch(i)  -> Row;    P::value(row, j) -> double2 (group j)
//   P::Epi / P::pre(k, j) / P::store(k, j, s0, s1, rc, src, e): epilogue at
//   point k with rc = 1 / (points in the window), src = sqrt(rc).
template <class P, int CPL>
__global__ void __launch_bounds__(kGfLanes) gf_box_kernel(P p, GfGeom g) {
  constexpr int M = P::M;
  constexpr int R = kGfLanes / M;  // runs per group
  constexpr int W = kGfLanes * CPL;  // halo columns of the strip
  constexpr int NO = M * CPL;        // most outputs of one lane's run
  typedef typename P::Row Row;
  typedef typename P::Epi Epi;
  __shared__ double vs[2 * M][W + 1];
  const int r = g.r, ow = W - 2 * r;
  const int lane = threadIdx.x;
  const int c0 = (int)blockIdx.x * ow;
  const int y0 = (int)blockIdx.y * g.rb;
  const int y1 = y0 + g.rb < g.rows ? y0 + g.rb : g.rows;
  // column role: halo columns lane + 64 k of the strip, k < CPL
  bool cok[CPL];
  int gcs[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    const int gc = c0 - r + lane + kGfLanes * k;
    cok[k] = gc >= 0 && gc < g.cols;
    gcs[k] = cok[k] ? gc : 0;
  }
  // run role: group j, output columns [run * L, run * L + L) of the strip
  const int L = (ow + R - 1) / R;
  const int j = lane / R, run = lane - (lane / R) * R;
  const int cb = run * L;
  int nout = ow - cb < L ? ow - cb : L;
  if (c0 + cb + nout > g.cols) nout = (int)(g.cols - c0 - cb);
  if (nout < 0) nout = 0;
  double rh[NO], srh[NO];  // L <= ceil((64 CPL - 2) M / 64) <= M CPL outputs per lane
#pragma unroll
  for (int t = 0; t < NO; ++t) {
    rh[t] = 1.0 / (double)win_count(c0 + cb + t, g.cols, r);
    srh[t] = sqrt(rh[t]);
  }

  double s[CPL][2 * M];
#pragma unroll
  for (int k = 0; k < CPL; ++k)
#pragma unroll
    for (int c = 0; c < 2 * M; ++c) s[k][c] = 0.0;
  auto clamp_row = [&](int y) { return y < 0 ? 0 : (y >= g.rows ? g.rows - 1 : y); };
  const int w0 = y0 - r < 0 ? 0 : y0 - r;
  const int w1 = y0 + r - 1 < g.rows - 1 ? y0 + r - 1 : g.rows - 1;
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    Row cur = p.fetch(clamp_row(w0) * g.cols + gcs[k]);
    for (int yy = w0; yy <= w1; ++yy) {
      const Row nxt = p.fetch(clamp_row(yy + 1) * g.cols + gcs[k]);
      if (cok[k]) {
#pragma unroll
        for (int q = 0; q < M; ++q) {
          const double2 v = p.value(cur, q);
          s[k][2 * q] += v.x;
          s[k][2 * q + 1] += v.y;
        }
      }
      cur = nxt;
    }
  }
  // ring of the entering / leaving points of the next D output rows
  constexpr int D = M <= 2 ? 4 : (M == 4 ? 2 : 1);
  // and of the epilogue's loads at the output points, the same D rows ahead
  Row fa[D][CPL], fd[D][CPL];
  Epi ep[D][NO];
  auto out_col = [&](int t) { return t < nout ? c0 + cb + t : c0; };
#pragma unroll
  for (int u = 0; u < D; ++u) {
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      fa[u][k] = p.fetch(clamp_row(y0 + u + r) * g.cols + gcs[k]);
      fd[u][k] = p.fetch(clamp_row(y0 + u - r) * g.cols + gcs[k]);
    }
#pragma unroll
    for (int t = 0; t < NO; ++t) ep[u][t] = p.pre(clamp_row(y0 + u) * g.cols + out_col(t), j);
  }
  // The body runs for every u, also past the workgroup's last row in the final
  // group (only the stores are skipped there): a ring slot refilled on some
  // paths only would need a register copy, and so a wait, every row.
  for (int yb = y0; yb < y1; yb += D) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int yo = yb + u;
      const bool live = yo < y1;
      const int ya = yo + r, yd = yo - r;
      Epi e[NO];
#pragma unroll
      for (int t = 0; t < NO; ++t) {
        e[t] = ep[u][t];
        ep[u][t] = p.pre(clamp_row(yo + D) * g.cols + out_col(t), j);
      }
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        const bool add = cok[k] && ya < g.rows;
#pragma unroll
        for (int q = 0; q < M; ++q) {
          const double2 v = p.value(fa[u][k], q);
          s[k][2 * q] += add ? v.x : 0.0;
          s[k][2 * q + 1] += add ? v.y : 0.0;
        }
      }
      wave_lds_fence();
#pragma unroll
      for (int k = 0; k < CPL; ++k)
#pragma unroll
        for (int c = 0; c < 2 * M; ++c) vs[c][lane + kGfLanes * k] = cok[k] ? s[k][c] : 0.0;
      wave_lds_fence();
      const int vc = (ya < g.rows ? ya : g.rows - 1) - (yd < 0 ? 0 : yd) + 1;
      const double rv = 1.0 / (double)vc, srv = sqrt(rv);
      if (nout > 0 && live) {
        const double* v0 = &vs[2 * j][cb];
        const double* v1 = &vs[2 * j + 1][cb];
        double a0 = 0.0, a1 = 0.0;
        for (int h = 0; h < 2 * r; ++h) {
          a0 += v0[h];
          a1 += v1[h];
        }
#pragma unroll
        for (int t = 0; t < NO; ++t) {
          if (t < nout) {
            a0 += v0[t + 2 * r];
            a1 += v1[t + 2 * r];
            p.store(yo * g.cols + c0 + cb + t, j, a0, a1, rv * rh[t], srv * srh[t], e[t]);
            a0 -= v0[t];
            a1 -= v1[t];
          }
        }
      }
      wave_lds_fence();
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        const bool sub = cok[k] && yd >= 0;
#pragma unroll
        for (int q = 0; q < M; ++q) {
          const double2 v = p.value(fd[u][k], q);
          s[k][2 * q] -= sub ? v.x : 0.0;
          s[k][2 * q + 1] -= sub ? v.y : 0.0;
        }
        fa[u][k] = p.fetch(clamp_row(ya + D) * g.cols + gcs[k]);
        fd[u][k] = p.fetch(clamp_row(yd + D) * g.cols + gcs[k]);
      }
    }
  }
}

// (u, g u) -> (a, b) at every window centre; AB point-major, pairs per group
template <typename T, int MM, bool SCALE>
struct GfStage1 {
  static constexpr int M = MM;
  const T* x;
  int ldx;
  const T* g;
  const T* dinv;  // 1/sqrt(d) (SCALE), else u = x (RW form)
  const T* mu;
  const T* inv;
  T* ab;
  struct Row {
    T x[M];
    T g, d;
  };
  __device__ __forceinline__ Row fetch(int i) const {
    Row w;
#pragma unroll
    for (int q = 0; q < M; ++q) w.x[q] = x[i * ldx + q];
    w.g = g[i];
    w.d = SCALE ? dinv[i] : T(1);
    return w;
  }
  __device__ __forceinline__ double2 value(const Row& w, int q) const {
    const double u = (double)w.x[q] * (double)w.d;
    return make_double2(u, (double)w.g * u);
  }
  struct Epi {
    T mu, inv;
  };
  __device__ __forceinline__ Epi pre(int k, int) const { return Epi{mu[k], inv[k]}; }
  __device__ __forceinline__ void store(int k, int j, double su, double sgu, double rc, double, const Epi& e) const {
    const double mk = (double)e.mu;
    const double mean_u = su * rc, mean_gu = sgu * rc;
    const double av = (mean_gu - mk * mean_u) * (double)e.inv;
    ab[(k * M + j) * 2] = (T)av;
    ab[(k * M + j) * 2 + 1] = (T)(mean_u - av * mk);
  }
};

// (a, b) -> y = D^1/2 GF(u) (N), x - D^1/2 GF(u) (L_sym), GF(x) (RW) or
// D (x - GF(x)) = L x (L, with d = N/|w|)
template <typename T, int MM>
struct GfStage2 {
  static constexpr int M = MM;
  const T* ab;
  const T* g;
  const T* x;
  int ldx;
  T* y;
  int ldy;
  int form;
  double sromega;  // 1 / sqrt(|w|)
  struct Row {
    T v[2 * M];
  };
  __device__ __forceinline__ Row fetch(int i) const {
    Row w;
#pragma unroll
    for (int q = 0; q < 2 * M; ++q) w.v[q] = ab[i * 2 * M + q];
    return w;
  }
  __device__ __forceinline__ double2 value(const Row& w, int q) const {
    return make_double2((double)w.v[2 * q], (double)w.v[2 * q + 1]);
  }
  struct Epi {
    T g, x;
  };
  __device__ __forceinline__ Epi pre(int i, int j) const {
    return Epi{g[i], (form == GSF_FORM_LSYM || form == GSF_FORM_L) ? x[i * ldx + j] : T(0)};
  }
  __device__ __forceinline__ void store(int i, int j, double sa, double sb, double rc, double src,
                                        const Epi& e) const {
    const double gfu = (double)e.g * sa + sb;
    double out;
    if (form == GSF_FORM_RW) {
      out = gfu * rc;
    } else if (form == GSF_FORM_L) {
      out = ((double)e.x - gfu * rc) * (sromega * sromega / rc);  // d (x - GF(x)), d = N/|w|
    } else {
      const double nx = gfu * (src * sromega);  // (g sum a + sum b) / sqrt(N_i |w|)
      out = form == GSF_FORM_LSYM ? (double)e.x - nx : nx;
    }
    y[i * ldy + j] = (T)out;
  }
};

// build: (g, g^2) -> mu, 1/(var + eps), d = N/|w|, sqrt(d), 1/sqrt(d), copy of g
template <typename T>
struct GfStats {
  static constexpr int M = 1;
  const T* gin;
  T* gcopy;
  T* mu;
  T* inv;
  T* sqd;
  T* dinv;
  double* deg;
  double eps, omega;
  struct Row {
    T v;
  };
  __device__ __forceinline__ Row fetch(int i) const { return Row{gin[i]}; }
  __device__ __forceinline__ double2 value(const Row& w, int) const {
    const double v = (double)w.v;
    return make_double2(v, v * v);
  }
  struct Epi {
    T gk;
  };
  __device__ __forceinline__ Epi pre(int k, int) const { return Epi{gin[k]}; }
  __device__ __forceinline__ void store(int k, int, double s1, double s2, double rc, double, const Epi& e) const {
    const double m = s1 * rc;
    const double var = s2 * rc - m * m;
    mu[k] = (T)m;
    inv[k] = (T)(1.0 / (var + eps));
    const double d = 1.0 / (rc * omega);
    deg[k] = d;
    sqd[k] = (T)sqrt(d);
    dinv[k] = (T)(1.0 / sqrt(d));
    gcopy[k] = e.gk;
  }
};

// Rows per workgroup: as many as possible up to kGfRowsMax (the 2r warm-up
// rows are amortised) while the grid still has about 2048 waves to hide
// memory latency.
template <int CPL>
GfGeom gf_geom(const Operator& op) {
  const int ow = kGfLanes * CPL - 2 * op.desc.radius;
  const int64_t strips = (op.cols + ow - 1) / ow;
  int64_t rb = (op.rows * strips + 2047) / 2048;
  rb = rb < 8 ? 8 : (rb > kGfRowsMax ? kGfRowsMax : rb);
  return GfGeom{(int)op.rows, (int)op.cols, op.desc.radius, (int)rb};
}

template <int CPL>
dim3 gf_grid(const Operator& op, const GfGeom& g) {
  const int ow = kGfLanes * CPL - 2 * op.desc.radius;
  return dim3((unsigned)((op.cols + ow - 1) / ow), (unsigned)((op.rows + g.rb - 1) / g.rb));
}

// Columns per lane: two for the one-column passes (half the LDS reads and
// horizontal adds per output, and a 1/(64 - r) instead of 2r/(64 - 2r) halo
// share), one for blocks, whose lanes already produce M outputs each.
template <int M>
struct GfCpl {
  static constexpr int v = M == 1 ? 2 : 1;
};

double gf_omega(const Operator& op) {
  const double w = 2.0 * op.desc.radius + 1.0;
  return op.desc.ndim == 1 ? w : w * w;
}

template <typename T, int M>
void gf_apply_group(const Operator& op, T* ab, int form, const T* x, int64_t ldx, T* y, int64_t ldy,
                    hipStream_t s) {
  constexpr int C = GfCpl<M>::v;
  const GfGeom geo = gf_geom<C>(op);
  const dim3 grid = gf_grid<C>(op, geo);
  if (form == GSF_FORM_RW || form == GSF_FORM_L) {
    GfStage1<T, M, false> p1{x, (int)ldx, (const T*)op.g, nullptr, (const T*)op.mu, (const T*)op.inv, ab};
    gf_box_kernel<GfStage1<T, M, false>, C><<<grid, kGfLanes, 0, s>>>(p1, geo);
  } else {
    GfStage1<T, M, true> p1{x, (int)ldx, (const T*)op.g, (const T*)op.diag, (const T*)op.mu, (const T*)op.inv, ab};
    gf_box_kernel<GfStage1<T, M, true>, C><<<grid, kGfLanes, 0, s>>>(p1, geo);
  }
  GfStage2<T, M> p2{ab, (const T*)op.g, x, (int)ldx, y, (int)ldy, form, 1.0 / sqrt(gf_omega(op))};
  gf_box_kernel<GfStage2<T, M>, C><<<grid, kGfLanes, 0, s>>>(p2, geo);
}

template <typename T>
void gf_apply_typed(const Operator& op, void* scratch, int form, int m, const T* x, int64_t ldx, T* y, int64_t ldy,
                    hipStream_t s) {
  T* ab = (T*)scratch;
  int c = 0;
  while (c < m) {
    const int left = m - c;
    if (left >= 8 && sizeof(T) == 4) {
      gf_apply_group<T, 8>(op, ab, form, x + c, ldx, y + c, ldy, s);
      c += 8;
    } else if (left >= 4) {
      gf_apply_group<T, 4>(op, ab, form, x + c, ldx, y + c, ldy, s);
      c += 4;
    } else if (left >= 2) {
      gf_apply_group<T, 2>(op, ab, form, x + c, ldx, y + c, ldy, s);
      c += 2;
    } else {
      gf_apply_group<T, 1>(op, ab, form, x + c, ldx, y + c, ldy, s);
      c += 1;
    }
  }
}

}  // namespace

gsf_status launch_gf_apply_fused(const Operator& op, int form, const float* x, int64_t ldx, float* y, int64_t ldy,
                                 hipStream_t s);

// One FP32 column: the one-pass kernel (apply_gf_fused.hip).  Blocks and FP64
// data: the two passes above; scratch: 2 * kMaxBlock planes of n elements
// (a, b of up to 8 columns).
gsf_status launch_gf_apply(const Operator& op, void* scratch, int form, int m, const void* x, int64_t ldx,
                           void* y, int64_t ldy, hipStream_t s) {
  if (op.desc.prec == GSF_F32 && m == 1)
    return launch_gf_apply_fused(op, form, (const float*)x, ldx, (float*)y, ldy, s);
  if (op.desc.prec == GSF_F32)
    gf_apply_typed<float>(op, scratch, form, m, (const float*)x, ldx, (float*)y, ldy, s);
  else
    gf_apply_typed<double>(op, scratch, form, m, (const double*)x, ldx, (double*)y, ldy, s);
  return launch_status();
}

gsf_status launch_gf_build(const Operator& op, const void* guidance, hipStream_t s) {
  const GfGeom geo = gf_geom<2>(op);
  const dim3 grid = gf_grid<2>(op, geo);
  if (op.desc.prec == GSF_F32) {
    GfStats<float> p{(const float*)guidance, (float*)op.g, (float*)op.mu, (float*)op.inv,
                     (float*)op.sqd, (float*)op.diag, op.deg, op.desc.gf_eps, gf_omega(op)};
    gf_box_kernel<GfStats<float>, 2><<<grid, kGfLanes, 0, s>>>(p, geo);
  } else {
    GfStats<double> p{(const double*)guidance, (double*)op.g, (double*)op.mu, (double*)op.inv,
                      (double*)op.sqd, (double*)op.diag, op.deg, op.desc.gf_eps, gf_omega(op)};
    gf_box_kernel<GfStats<double>, 2><<<grid, kGfLanes, 0, s>>>(p, geo);
  }
  return launch_status();
}

}  // namespace gsf
