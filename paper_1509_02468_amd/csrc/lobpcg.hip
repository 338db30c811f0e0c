// Block LOBPCG as a low-pass filter (Algorithm 3, Section 6, generalised to a
// block of m vectors), z-space operator A = L_sym, B = I, T = I.
//
// Kernels:
//   lob_ynorm      ||sqrt(d)|| for the constraint vector Y = sqrt(d)/||sqrt(d)||
//   lob_start      X0[:, j] = z0 * phi_j (Legendre modulations), Y^T X0
//   lob_project    B -= Y c (constraint projection of a block)
//   gram           partial Gram tiles S^T S, S^T (A S) of S = [X, W, P] with
//                  MFMA (FP32: v_mfma_f32_16x16x4f32 accumulated in FP32 over
//                  256 points then in FP64; FP64: v_mfma_f64_16x16x4f64)
//   gram_reduce /  fixed-order two-level reduction of the tiles, then the
//   gram_rr        Rayleigh-Ritz step on one workgroup in FP64: unit-diagonal scaling,
//                  column-dropping Cholesky, reduction to L^-1 A L^-T, cyclic
//                  parallel Jacobi eigensolver, m smallest Ritz pairs
//   lob_update     X = S C, AX = (AS) C, P = [W,P] C, AP likewise, the next
//                  residual W = AX - X Theta and its norms (and Y^T W)
//   lob_out_dots / lob_output: y = X X^T z0 (+ Y Y^T z0), x_out = y / sqrt(d)
#include <cmath>

#include "gsf_internal.h"
#include "solver_state.h"
#include "lobpcg_launch.h"

namespace gsf {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double legendre(int deg, double t) {
  double p0 = 1.0, p1 = t;
  if (deg == 0) return p0;
  for (int k = 1; k < deg; ++k) {
    const double p2 = ((2.0 * k + 1.0) * t * p1 - (double)k * p0) / (double)(k + 1);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// sum_i sqrt(d_i)^2 -> ynorm_inv
template <typename T>
__global__ void __launch_bounds__(kThreads) lob_ynorm_kernel(const T* __restrict__ sqd, int64_t n,
                                                             double* __restrict__ partials, LobpcgState* st) {
  __shared__ double red[16];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    v[0] += (double)sqd[i] * (double)sqd[i];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// one workgroup: sum the partials of a previous kernel in workgroup order;
// mode 0: ynorm_inv, 1: yx (M values), 2: update residuals (2M values),
// 3: output coefficients (M+1 values)
template <int NV>
__global__ void __launch_bounds__(kThreads) lob_final_kernel(const double* __restrict__ partials, int nparts,
                                                             LobpcgState* st, int mode, int m, int first,
                                                             int constraint) {
  __shared__ double red[16 * NV];
  if (mode == 2 && !st->active) return;
  double t[NV];
  reduce_partials<NV>(partials, nparts, NV, t, red);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    st->ynorm_inv = 1.0 / sqrt(t[0]);
  } else if (mode == 1 || mode == 3) {
    for (int j = 0; j < NV; ++j) st->yx[j] = t[j];
  } else {
    double mx = 0.0;
    for (int j = 0; j < m; ++j) {
      st->res[j] = sqrt(t[j]);
      st->yx[j] = constraint ? t[m + j] : 0.0;
      mx = st->res[j] > mx ? st->res[j] : mx;
    }
    if (!first) st->iters += 1;
    if (st->tol > 0.0 && mx <= st->tol) st->active = 0;
  }
}

// X0[i, j] = sqrt(d_i) x0_i phi_j(i); with the constraint also Y^T X0.
template <typename T, int M>
__global__ void __launch_bounds__(kThreads) lob_start_kernel(LobArgs a, StartDegrees deg) {
  __shared__ double red[16 * M];
  const T* __restrict__ x0 = (const T*)a.x0;
  const T* __restrict__ sqd = (const T*)a.sqd;
  T* __restrict__ X = (T*)a.X;
  const double yinv = a.st->ynorm_inv;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[M];
#pragma unroll
  for (int j = 0; j < M; ++j) v[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    const int64_t r = i / a.cols, c = i - r * a.cols;
    const double tr = 2.0 * ((double)r + 0.5) / (double)a.rows - 1.0;
    const double tc = 2.0 * ((double)c + 0.5) / (double)a.cols - 1.0;
    const double z = (double)sqd[i] * (double)x0[i];
    const double yi = (double)sqd[i] * yinv;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      double phi = legendre(deg.b[j], tc);
      if (a.ndim == 2) phi *= legendre(deg.a[j], tr);
      const T xv = (T)(z * phi);
      X[i * M + j] = xv;
      v[j] += yi * (double)xv;
    }
  }
  if (!a.constraint) return;
  block_sum<M>(v, red);
  if (threadIdx.x == 0)
    for (int j = 0; j < M; ++j) a.vpart[(size_t)blockIdx.x * M + j] = v[j];
}

// B[i, j] -= Y_i c_j with c = st->yx
template <typename T>
__global__ void __launch_bounds__(kThreads) lob_project_kernel(T* __restrict__ B, const T* __restrict__ sqd,
                                                               int64_t n, int m, const LobpcgState* st) {
  if (!st->active) return;
  const double yinv = st->ynorm_inv;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double yi = (double)sqd[i] * yinv;
    for (int j = 0; j < m; ++j) B[i * m + j] = (T)((double)B[i * m + j] - yi * st->yx[j]);
  }
}

// ---------------------------------------------------------------------------
// Gram tiles with MFMA
// ---------------------------------------------------------------------------
// Tiles of 16x16: nt = ceil(ns/16) tile rows.  S^T S: upper tiles (I <= J)
// in the order (0,0), (0,1), (1,1); S^T AS: all tiles (0,0), (0,1), (1,0), (1,1).
__device__ __forceinline__ int n_tiles_b(int nt) { return nt == 1 ? 1 : 3; }
__device__ __forceinline__ int n_tiles_a(int nt) { return nt == 1 ? 1 : 4; }

template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
  typedef floatx4 type;
  static __device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfmaAcc<double> {
  typedef doublex4 type;
  static __device__ __forceinline__ doublex4 mfma(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T, int NT>
__global__ void __launch_bounds__(kThreads) gram_kernel(GramArgs g) {
  typedef typename MfmaAcc<T>::type acc_t;
  typedef const __attribute__((address_space(1))) T* gptr;
  // groups of 4 points per stage (one MFMA k-step each); fewer for the wider
  // tiles and FP64, whose stages hold more registers
  constexpr int U = (NT == 1 && sizeof(T) == 4) ? 8 : 4;
  constexpr int G = 4 * U;      // points per stage
  constexpr int ntb = NT == 1 ? 1 : 3, nta = NT == 1 ? 1 : 4;
  constexpr int nt = NT;
  __shared__ double wsum[4][4][64];  // one tile at a time: wave, register, lane
  if (g.active != nullptr && *g.active == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ns = g.ns, m = g.m;
  const int col = lane & 15, krow = lane >> 4;

  // the S / AS column each lane feeds for tile row I; lanes past the last
  // column read column 0 and feed zeros
  gptr sp[2], ap[2];
  bool live[2];
#pragma unroll
  for (int I = 0; I < 2; ++I) {
    const int c = 16 * I + col;
    live[I] = I < nt && c < ns;
    const int cc = live[I] ? c : 0;
    const int b = cc / m, j = cc - (cc / m) * m;
    sp[I] = (gptr)g.S[b] + j;
    ap[I] = (gptr)g.AS[b] + j;
  }

  // FP32 partials move into FP64 every FL points (256); FP64 needs no flush
  constexpr int FL = sizeof(T) == 4 ? 256 : 2 * G;
  const int64_t nw = (int64_t)gridDim.x * 4;
  const int64_t wid = (int64_t)blockIdx.x * 4 + wave;
  int64_t chunk = (g.n + nw - 1) / nw;
  chunk = (chunk + FL - 1) / FL * FL;
  const int64_t p_begin = wid * chunk;
  const int64_t p_end = (p_begin + chunk < g.n) ? p_begin + chunk : g.n;

  double totb[ntb][4], tota[nta][4];
#pragma unroll
  for (int t = 0; t < ntb; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) totb[t][v] = 0.0;
#pragma unroll
  for (int t = 0; t < nta; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) tota[t][v] = 0.0;
  acc_t accb[ntb], acca[nta];
#pragma unroll
  for (int t = 0; t < ntb; ++t) accb[t] = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < nta; ++t) acca[t] = acc_t{0, 0, 0, 0};

  // one stage: the U point groups starting at p0.  Every load is issued
  // unconditionally (points past the end re-read p_begin); the 0/1 mask of a
  // point (and of a column past ns) multiplies only the A operand of its
  // MFMAs, when they run a stage later: A[i][k] = 0 removes point k from
  // every product, and the tile entries of the dead B columns are never read.
  // (Masking at load time lets the compiler sink the loads into branches or
  // wait for them at once.)  A non-finite value at p_begin already makes the
  // sums non-finite, so re-reading it changes nothing.
  auto load = [&](int64_t p0, T (&s)[2][U], T (&a)[2][U], T (&mk)[2][U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t p = p0 + 4 * u + krow;
      const bool ok = p < p_end;
      const int64_t off = (ok ? p : p_begin) * m;
#pragma unroll
      for (int I = 0; I < nt; ++I) {
        s[I][u] = sp[I][off];
        a[I][u] = ap[I][off];
        mk[I][u] = (ok && live[I]) ? T(1) : T(0);
      }
    }
  };
  auto mfmas = [&](const T (&s)[2][U], const T (&a)[2][U], const T (&mk)[2][U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T s0m = s[0][u] * mk[0][u];
      accb[0] = MfmaAcc<T>::mfma(s0m, s[0][u], accb[0]);
      acca[0] = MfmaAcc<T>::mfma(s0m, a[0][u], acca[0]);
      if constexpr (NT > 1) {
        const T s1m = s[1][u] * mk[1][u];
        accb[1] = MfmaAcc<T>::mfma(s0m, s[1][u], accb[1]);
        accb[2] = MfmaAcc<T>::mfma(s1m, s[1][u], accb[2]);
        acca[1] = MfmaAcc<T>::mfma(s0m, a[1][u], acca[1]);
        acca[2] = MfmaAcc<T>::mfma(s1m, a[0][u], acca[2]);
        acca[3] = MfmaAcc<T>::mfma(s1m, a[1][u], acca[3]);
      }
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int t = 0; t < ntb; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) totb[t][v] += (double)accb[t][v];
      accb[t] = acc_t{0, 0, 0, 0};
    }
#pragma unroll
    for (int t = 0; t < nta; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) tota[t][v] += (double)acca[t][v];
      acca[t] = acc_t{0, 0, 0, 0};
    }
  };

  // two register stages: the loads of the next stage are in flight while the
  // MFMAs of the current one run
  if (p_begin < p_end) {
    T s0[2][U], a0[2][U], k0[2][U], s1[2][U], a1[2][U], k1[2][U];
    load(p_begin, s0, a0, k0);
    for (int64_t pf = p_begin; pf < p_end; pf += FL) {
#pragma unroll
      for (int q = 0; q < FL / (2 * G); ++q) {
        const int64_t p0 = pf + (int64_t)q * 2 * G;
        // the scheduling barriers keep each stage's loads ahead of the other
        // stage's MFMAs (otherwise the mask products are hoisted next to the
        // loads and wait for them)
        load(p0 + G, s1, a1, k1);
        __builtin_amdgcn_sched_barrier(0);
        mfmas(s0, a0, k0);
        __builtin_amdgcn_sched_barrier(0);
        load(p0 + 2 * G, s0, a0, k0);
        __builtin_amdgcn_sched_barrier(0);
        mfmas(s1, a1, k1);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (sizeof(T) == 4) flush();
    }
  }
  flush();

  // fixed-order sum over the 4 waves, one tile at a time.  Output layouts of
  // the two MFMA variants (entry e = i*16 + j of a tile):
  //   16x16x4 f32: D[i][j] in lane j + 16*(i/4), register i%4
  //   16x16x4 f64: D[i][j] in lane j + 16*(i%4), register i/4
  const int ntot = ntb + nta;
  for (int t = 0; t < ntot; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double val = 0.0;
#pragma unroll
      for (int tt = 0; tt < ntb; ++tt)
        if (t == tt) val = totb[tt][v];
#pragma unroll
      for (int tt = 0; tt < nta; ++tt)
        if (t == ntb + tt) val = tota[tt][v];
      wsum[wave][v][lane] = val;
    }
    __syncthreads();
    {
      const int ij = threadIdx.x;  // 256 threads = 256 entries
      const int i = ij >> 4, j = ij & 15;
      const int ln = sizeof(T) == 4 ? j + 16 * (i >> 2) : j + 16 * (i & 3);
      const int v = sizeof(T) == 4 ? (i & 3) : (i >> 2);
      const double sm = wsum[0][v][ln] + wsum[1][v][ln] + wsum[2][v][ln] + wsum[3][v][ln];
      g.partials[((size_t)blockIdx.x * ntot + t) * 256 + ij] = sm;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz on one wave (FP64)
// ---------------------------------------------------------------------------
// The whole step runs on the first wave of the workgroup (the others only
// help to load the Gram pair).  Lanes of one wave issue their LDS accesses in
// program order and the LDS unit completes them in that order, so a store by
// one lane is seen by a later load of another lane of the same wave: the
// steps below need no workgroup barrier, only a compiler-level fence that
// keeps LDS accesses in program order.
__device__ __forceinline__ void wave_fence() { __asm__ volatile("" ::: "memory"); }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Reciprocal square root: the hardware approximation refined
// by one Newton step (a few ulp), short dependency chains for the Jacobi
// rotations.  The rotation stays orthogonal to rounding because c and s are
// both derived from the same t: c = (1 + t^2)^-1/2, s = t c.
__device__ __forceinline__ double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * r, r, 1.0);
  return fma(0.5 * r, e, r);
}
// Two Newton steps: full FP64 accuracy for the Cholesky pivots.
__device__ __forceinline__ double rsq_nr2(double x) {
  const double r = rsq_nr(x);
  const double e = fma(-x * r, r, 1.0);
  return fma(0.5 * r, e, r);
}
constexpr int KMAX = 24;
constexpr int LD = KMAX + 1;

struct RRShared {
  double A[KMAX * LD];   // Gram pair as loaded (A = S^T A S, B = S^T S)
  double B[KMAX * LD];
  double SA[KMAX * LD];  // symmetrised and scaled to unit diag(B)
  double SB[KMAX * LD];  // the same for B; work array of the Cholesky factorisation
  double L[KMAX * LD];   // Cholesky factor (dropped columns zero)
  double LK[KMAX * LD];  // compressed factor of the kept columns
  double M[KMAX * LD];   // Jacobi matrix, two buffers
  double M2[KMAX * LD];
  double V[KMAX * LD];   // accumulated rotations, two buffers
  double V2[KMAX * LD];
  double Cs[KMAX * 8];   // output coefficients, staged
  double delta[KMAX];
  double rinv[KMAX];
  double ev[KMAX];
  int good[KMAX];
  int kept[KMAX];
  int idx[KMAX];
  int order[KMAX];
};
// the Jacobi schedule table reuses A, B, SA and SB
static_assert((KMAX - 1) * 3 * 64 * sizeof(uint32_t) <= 4 * sizeof(double) * KMAX * LD, "schedule table");

// Players of pair `slot` in round `rnd` of the round-robin schedule over np
// players (np even): player 0 stays, the others rotate.  p < q.
__device__ __forceinline__ void rr_pair(int slot, int rnd, int np, int& p, int& q) {
  const int n1 = np - 1;
  int a = slot - 1 + rnd;
  a = a >= n1 ? a - n1 : a;
  int b = (np - 1 - slot) - 1 + rnd;
  b = b >= n1 ? b - n1 : b;
  const int pa = slot == 0 ? 0 : 1 + a, pb = 1 + b;
  p = pa < pb ? pa : pb;
  q = pa < pb ? pb : pa;
}

// The Jacobi rotation J = [[c, s], [-s, c]] (rows and columns p, q) that
// annihilates m_pq of the symmetric 2 x 2 block [[m_pp, m_pq], [m_pq, m_qq]]:
// with d = m_qq - m_pp, h = sqrt(d^2 + 4 m_pq^2) and u = d + sign(d) h (the
// root t = 2 m_pq / u of t^2 + 2 theta t - 1 = 0 of smaller magnitude,
// theta = d / (2 m_pq)), c = |u| / sqrt(2 h |u|) and s = sign(u) 2 m_pq /
// sqrt(2 h |u|), which is c = (1 + t^2)^-1/2, s = t c with one reciprocal
// square root for both (so c^2 + s^2 = 1 to rounding).  The rotated diagonal
// is m_pp - t m_pq, m_qq + t m_pq, with t m_pq = sign(u) 4 h m_pq^2 / (2 h |u|).
// The identity when `live` is false (m_pq = 0, or q is the dummy player);
// no branches, so every lane runs the same instruction stream.
struct JRot {
  double c, s, dp, dq;
};
__device__ __forceinline__ JRot jacobi_rot(double mpp, double mqq, double mpq, bool live) {
  live = live && mpq != 0.0;
  const double apq = live ? mpq : 1.0;  // keeps the dead lanes finite
  const double d = mqq - mpp;
  const double y = fma(d, d, 4.0 * apq * apq);
  const double h = y * rsq_nr(y);
  const double au = fabs(d) + h;
  const double r2 = rsq_nr(2.0 * h * au);
  const double sg = d >= 0.0 ? 1.0 : -1.0;
  const double s = sg * (2.0 * apq * r2);
  const double tm = sg * (4.0 * h * apq * apq * (r2 * r2));
  JRot r;
  r.c = live ? au * r2 : 1.0;
  r.s = live ? s : 0.0;
  r.dp = live ? mpp - tm : mpp;
  r.dq = live ? mqq + tm : mqq;
  return r;
}

// Solves the Rayleigh-Ritz problem for GA, GB (ns x ns, already loaded into
// sh.A and sh.B): C (ns x m, row-major with leading dimension m) and theta
// (ascending) of the m smallest Ritz pairs, the kept flags and their count.
// Called by the 64 lanes of one wave; KB >= ns is the padded size of the
// triangular solves (the kept block is extended by an identity factor and
// zero data there, which changes nothing and keeps the loops free of
// conditionals).  Steps: symmetrise; scale to unit diag(GB) (columns with a
// negligible diagonal are dropped); Cholesky GB = L L^T that drops columns
// with a pivot below drop_tol; M = L^-1 GA L^-T on the kept columns; cyclic
// Jacobi on M (parallel round-robin ordering, one 2 x 2 block of every
// rotated pair of rows and columns per lane); C = L^-T Z.  Loads are issued
// unconditionally (clamped indices) and only stores are masked, so a lane
// never waits on a load inside a branch.
template <int KB>
__device__ void rayleigh_ritz_kb(RRShared& sh, int ns, int m, double drop_tol, double zero_tol, double conv2,
                                 double* Cout, double* theta, int* kept_out, int* nkept_out) {
  const int lane = threadIdx.x & 63;
  // unit-diagonal scaling: delta_j = diag(GB)_j^-1/2, 0 for a negligible column
  const int lj = lane < ns ? lane : 0;
  const double dl = sh.B[lj * LD + lj];
  const double mx = wave_max(lane < ns && dl > 0.0 ? dl : 0.0);
  const int gd = lane < ns && dl > zero_tol * zero_tol * mx;
  if (lane < ns) {
    sh.good[lane] = gd;
    sh.delta[lane] = gd ? 1.0 / sqrt(dl) : 0.0;
  }
  wave_fence();
  for (int e = lane; e < ns * ns; e += 64) {
    const int i = e / ns, j = e - (e / ns) * ns;
    const double s = sh.delta[i] * sh.delta[j];
    const double aij = sh.A[i * LD + j], aji = sh.A[j * LD + i];
    const double bij = sh.B[i * LD + j], bji = sh.B[j * LD + i];
    const double a = i == j ? aij : 0.5 * (aij + aji);
    const double b = i == j ? bij : 0.5 * (bij + bji);
    sh.SA[i * LD + j] = a * s;
    sh.SB[i * LD + j] = b * s;
    sh.L[i * LD + j] = 0.0;
  }
  wave_fence();
  // right-looking Cholesky of SB with column dropping: every lane computes the
  // column entries it needs from SB itself (the same operations as the lane
  // that stores them into L)
  for (int j = 0; j < ns; ++j) {
    const double piv = sh.SB[j * LD + j];
    const int keep = sh.good[j] && piv > drop_tol;
    const double ip = rsq_nr2(keep ? piv : 1.0);  // 1 / L_jj
    if (lane == 0) {
      sh.kept[j] = keep;
      if (keep) sh.L[j * LD + j] = piv * ip;
    }
    const int rem = ns - j - 1;
    for (int e = lane; e < rem * rem; e += 64) {
      const int i = j + 1 + e / rem, l = j + 1 + (e - (e / rem) * rem);
      const double lij = sh.SB[i * LD + j] * ip;
      const double llj = sh.SB[l * LD + j] * ip;
      const double bil = sh.SB[i * LD + l];
      if (keep && l <= i) {
        sh.SB[i * LD + l] = bil - lij * llj;
        if (l == j + 1) sh.L[i * LD + j] = lij;
      }
    }
    wave_fence();
  }
  const int kp = lane < ns ? sh.kept[lane] : 0;
  const unsigned long long km = __ballot(kp);
  const int K = __popcll(km);
  if (kp) sh.idx[__popcll(km & ((1ull << lane) - 1ull))] = lane;
  if (lane < ns) kept_out[lane] = kp;
  if (lane == 0) *nkept_out = K;
  wave_fence();
  if (K < m) return;
  // compressed factor LK and reduced A (in M2), padded to KB x KB with the
  // identity and zeros; reciprocal pivots (1 on the padding)
  for (int e = lane; e < KB * KB; e += 64) {
    const int a = e / KB, b = e - (e / KB) * KB;
    const int ia = sh.idx[a < K ? a : 0], ib = sh.idx[b < K ? b : 0];
    const double lv = sh.L[ia * LD + ib], av = sh.SA[ia * LD + ib];
    const bool in = a < K && b < K;
    sh.LK[a * LD + b] = in ? (b <= a ? lv : 0.0) : (a == b ? 1.0 : 0.0);
    sh.M2[a * LD + b] = in ? av : 0.0;
  }
  if (lane < KB) {
    const int ia = sh.idx[lane < K ? lane : 0];
    const double lv = sh.L[ia * LD + ia];
    sh.rinv[lane] = lane < K ? 1.0 / lv : 1.0;
  }
  wave_fence();
  // T = LK^-1 A_K: lane c solves LK t = A_K[:, c] by forward substitution with
  // its column in registers (LK read as LDS broadcasts), then writes row c of
  // T^T.  A_K is symmetric, so M = T LK^-T = (LK^-1 T^T)^T.
  {
    const int c = lane < KB ? lane : 0;
    double col[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      double v = sh.M2[i * LD + c];
#pragma unroll
      for (int t = 0; t < i; ++t) v -= sh.LK[i * LD + t] * col[t];
      col[i] = v * sh.rinv[i];
    }
    if (lane < KB) {
#pragma unroll
      for (int i = 0; i < KB; ++i) sh.V[c * LD + i] = col[i];  // V = T^T
    }
  }
  wave_fence();
  {
    const int c = lane < KB ? lane : 0;
    double col[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      double v = sh.V[i * LD + c];
#pragma unroll
      for (int t = 0; t < i; ++t) v -= sh.LK[i * LD + t] * col[t];
      col[i] = v * sh.rinv[i];
    }
    if (lane < KB) {
#pragma unroll
      for (int i = 0; i < KB; ++i) sh.M2[c * LD + i] = col[i];  // M2 = (LK^-1 T^T)^T = M
    }
  }
  wave_fence();
  for (int e = lane; e < K * K; e += 64) {
    const int a = e / K, b = e - (e / K) * K;
    const double x = sh.M2[a * LD + b], y = sh.M2[b * LD + a];
    sh.M[a * LD + b] = 0.5 * (x + y);
    sh.V[a * LD + b] = (a == b) ? 1.0 : 0.0;
  }
  wave_fence();

  // cyclic Jacobi: in each round the np/2 disjoint pairs of the round-robin
  // schedule are rotated together, M <- J^T M J, V <- V J.  Lane b owns the
  // 2 x 2 block (pair P = b / nh rows, pair Q = b % nh columns) and computes
  // both rotations itself (bitwise the same on every lane that needs them).
  // The schedule is tabulated once per call (one word per round, block slot
  // and lane, in the Gram and scaled arrays, which are dead by now), and the
  // round loop alternates the two buffers explicitly so that every LDS
  // address is a table offset plus a constant.
  const int np = (K + 1) & ~1;  // players (a dummy when K is odd)
  const int nh = np >> 1, nblk = nh * nh, nr = np - 1;
  const int nslot = (nblk + 63) >> 6;
  uint32_t* tab = reinterpret_cast<uint32_t*>(sh.A);  // (KMAX-1) x 3 x 64 words fit in A, B, SA, SB
  for (int r = 0; r < nr; ++r) {
    for (int sl = 0; sl < nslot; ++sl) {
      const int bl = sl * 64 + lane;
      const int b = bl < nblk ? bl : 0;
      const int P = b / nh, Q = b - (b / nh) * nh;
      int i0, i1, j0, j1;
      rr_pair(P, r, np, i0, i1);
      rr_pair(Q, r, np, j0, j1);
      const uint32_t ri = i1 < K, rj = j1 < K;  // the second player is not the dummy
      const uint32_t i1c = ri ? i1 : i0, j1c = rj ? j1 : j0;
      tab[(r * nslot + sl) * 64 + lane] = (uint32_t)i0 | (i1c << 5) | ((uint32_t)j0 << 10) | (j1c << 15) |
                                          (ri << 20) | (rj << 21) | ((uint32_t)(bl < nblk) << 22) |
                                          ((uint32_t)(P == Q) << 23);
    }
  }
  wave_fence();
  auto jround = [&](int rnd, const double* __restrict__ Mc, double* __restrict__ Mn, const double* __restrict__ Vc,
                    double* __restrict__ Vn) {
    for (int sl = 0; sl < nslot; ++sl) {
      const uint32_t w = tab[(rnd * nslot + sl) * 64 + lane];
      const int i0 = w & 31, i1 = (w >> 5) & 31, j0 = (w >> 10) & 31, j1 = (w >> 15) & 31;
      const bool ri = (w >> 20) & 1, rj = (w >> 21) & 1, act = (w >> 22) & 1, dg = (w >> 23) & 1;
      const int a0 = i0 * LD, a1 = i1 * LD, b0 = j0 * LD, b1 = j1 * LD;
      const double m00 = Mc[a0 + j0], m01 = Mc[a0 + j1], m10 = Mc[a1 + j0], m11 = Mc[a1 + j1];
      const double pp = Mc[a0 + i0], qq = Mc[a1 + i1], pq = Mc[a0 + i1];
      const double rr = Mc[b0 + j0], ss = Mc[b1 + j1], rs = Mc[b0 + j1];
      const double v00 = Vc[a0 + j0], v01 = Vc[a0 + j1], v10 = Vc[a1 + j0], v11 = Vc[a1 + j1];
      const JRot jp = jacobi_rot(pp, qq, pq, ri);
      const JRot jq = jacobi_rot(rr, ss, rs, rj);
      // X = J_P^T B, B' = X J_Q
      const double x00 = jp.c * m00 - jp.s * m10, x01 = jp.c * m01 - jp.s * m11;
      const double x10 = jp.s * m00 + jp.c * m10, x11 = jp.s * m01 + jp.c * m11;
      double y00 = x00 * jq.c - x01 * jq.s, y01 = x00 * jq.s + x01 * jq.c;
      double y10 = x10 * jq.c - x11 * jq.s, y11 = x10 * jq.s + x11 * jq.c;
      if (dg) {  // the rotated pair itself: exact zero off the diagonal
        y00 = jp.dp;
        y11 = jp.dq;
        y01 = 0.0;
        y10 = 0.0;
      }
      if (act) {
        Mn[a0 + j0] = y00;
        Vn[a0 + j0] = v00 * jq.c - v01 * jq.s;
        if (rj) {
          Mn[a0 + j1] = y01;
          Vn[a0 + j1] = v00 * jq.s + v01 * jq.c;
        }
        if (ri) {
          Mn[a1 + j0] = y10;
          Vn[a1 + j0] = v10 * jq.c - v11 * jq.s;
        }
        if (ri && rj) {
          Mn[a1 + j1] = y11;
          Vn[a1 + j1] = v10 * jq.s + v11 * jq.c;
        }
      }
    }
  };
  // convergence: off-diagonal Frobenius mass below sqrt(conv2) of the whole
  // (relative: 1e-14 for FP64 data, 1e-10 for FP32 data, whose Gram entries
  // carry ~1e-7 relative errors anyway); the butterfly sum leaves the same
  // value on every lane
  const double c2 = conv2 > 0.0 ? conv2 : 1e-28;
  auto converged = [&](const double* Mc) {
    double off = 0.0, dia = 0.0;
    for (int e = lane; e < K * K; e += 64) {
      const int i = e / K, j = e - (e / K) * K;
      const double v = Mc[i * LD + j] * Mc[i * LD + j];
      off += i == j ? 0.0 : v;
      dia += i == j ? v : 0.0;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    return off <= c2 * (off + dia);
  };
  int rnd = 0, sweep = 0, cur = 0;  // cur = 1: the current matrix is in M2, V2
  while (true) {
    jround(rnd, sh.M, sh.M2, sh.V, sh.V2);
    wave_fence();
    cur = 1;
    if (++rnd == nr) {
      rnd = 0;
      if (converged(sh.M2) || ++sweep == 30) break;
    }
    jround(rnd, sh.M2, sh.M, sh.V2, sh.V);
    wave_fence();
    cur = 0;
    if (++rnd == nr) {
      rnd = 0;
      if (converged(sh.M) || ++sweep == 30) break;
    }
  }
  const double* Mc = cur ? sh.M2 : sh.M;
  const double* Vc = cur ? sh.V2 : sh.V;
  // order eigenvalues ascending (ties by index)
  {
    const int li = lane < K ? lane : 0;
    sh.ev[lane < KB ? lane : 0] = Mc[li * LD + li];  // lanes >= K store junk past K (never read)
  }
  for (int e = lane; e < ns * m; e += 64) sh.Cs[e] = 0.0;
  wave_fence();
  {
    const double e = sh.ev[lane < K ? lane : 0];
    int rank = 0;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const double ej = sh.ev[j];
      rank += (j < K && (ej < e || (ej == e && j < lane))) ? 1 : 0;
    }
    if (lane < K) sh.order[rank] = lane;
  }
  wave_fence();
  // C_K = LK^-T Z_m: lane t solves LK^T c = Z[:, order[t]] by back substitution
  {
    const int t = lane < m ? lane : 0;
    const int col = sh.order[t];
    if (lane < m) theta[lane] = sh.ev[col];
    double c[KB];
#pragma unroll
    for (int ii = KB - 1; ii >= 0; --ii) {
      const double z = Vc[(ii < K ? ii : 0) * LD + col];
      double v = ii < K ? z : 0.0;
      // oldest coefficients first: c[ii] then waits for c[ii + 1] through one FMA
#pragma unroll
      for (int b = KB - 1; b > ii; --b) v -= sh.LK[b * LD + ii] * c[b];
      c[ii] = v * sh.rinv[ii];
    }
    // sign: the largest-magnitude coefficient (first on ties) is positive, so
    // Ritz vectors (and residuals) have a fixed sign for a non-odd T
    double big = 0.0, sgn = 1.0;
#pragma unroll
    for (int a = 0; a < KB; ++a) {
      const double v = sh.delta[sh.idx[a < K ? a : 0]] * c[a];
      const bool more = a < K && fabs(v) > big;
      big = more ? fabs(v) : big;
      sgn = more ? (v < 0.0 ? -1.0 : 1.0) : sgn;
    }
    if (lane < m) {
#pragma unroll
      for (int a = 0; a < KB; ++a) {
        const int row = sh.idx[a < K ? a : 0];
        const double v = sgn * (sh.delta[row] * c[a]);
        if (a < K) sh.Cs[row * m + t] = v;
      }
    }
  }
  wave_fence();
  for (int e = lane; e < ns * m; e += 64) Cout[e] = sh.Cs[e];
}

__device__ void rayleigh_ritz(RRShared& sh, int ns, int m, double drop_tol, double zero_tol, double conv2,
                              double* Cout, double* theta, int* kept_out, int* nkept_out) {
  if (ns <= 4)
    rayleigh_ritz_kb<4>(sh, ns, m, drop_tol, zero_tol, conv2, Cout, theta, kept_out, nkept_out);
  else if (ns <= 8)
    rayleigh_ritz_kb<8>(sh, ns, m, drop_tol, zero_tol, conv2, Cout, theta, kept_out, nkept_out);
  else if (ns <= 12)
    rayleigh_ritz_kb<12>(sh, ns, m, drop_tol, zero_tol, conv2, Cout, theta, kept_out, nkept_out);
  else if (ns <= 16)
    rayleigh_ritz_kb<16>(sh, ns, m, drop_tol, zero_tol, conv2, Cout, theta, kept_out, nkept_out);
  else
    rayleigh_ritz_kb<KMAX>(sh, ns, m, drop_tol, zero_tol, conv2, Cout, theta, kept_out, nkept_out);
}

// First stage of the Gram reduction: workgroup (tile, chunk) sums the partials
// of its chunk of Gram workgroups for the 256 entries of one tile.
__global__ void __launch_bounds__(kThreads) gram_reduce_kernel(GramArgs g) {
  if (g.active != nullptr && *g.active == 0) return;
  const int nt = (g.ns + 15) >> 4;
  const int ntot = n_tiles_b(nt) + n_tiles_a(nt);
  const int tile = blockIdx.x, chunk = blockIdx.y, nchunks = gridDim.y;
  const int per = (g.nparts + nchunks - 1) / nchunks;
  const int b0 = chunk * per, b1 = (b0 + per < g.nparts) ? b0 + per : g.nparts;
  const int e = tile * 256 + threadIdx.x;
  const size_t st = (size_t)ntot * 256;
  // up to kGramPerChunk partials, loaded together, summed in order
  double v[kGramPerChunk];
#pragma unroll
  for (int k = 0; k < kGramPerChunk; ++k) v[k] = (b0 + k < b1) ? g.partials[(size_t)(b0 + k) * st + e] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kGramPerChunk; ++k) s += v[k];
  g.level2[(size_t)chunk * st + e] = s;
}

// One workgroup: sums the chunks and assembles GA and GB (ns x ns); its first
// wave then runs the Rayleigh-Ritz step.
__global__ void __launch_bounds__(kThreads) gram_rr_kernel(GramArgs g, RRArgs r) {
  __shared__ RRShared sh;
  __shared__ int nkept;
  __shared__ int keptf[KMAX];
  __shared__ double fred[8 * 16];
  __shared__ int live;
  if (r.st != nullptr && !r.st->active) return;
  if (r.fin_partials != nullptr) {
    // the previous update's residual norms, iteration count and convergence
    // test (what lob_final_kernel does after an update without the
    // constraint, in the same summation order)
    double t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = 0.0;
    for (int b = threadIdx.x; b < r.fin_nparts; b += blockDim.x) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < g.m) t[k] += r.fin_partials[(size_t)b * r.fin_stride + k];
    }
    block_sum<8>(t, fred);
    if (threadIdx.x == 0) {
      LobpcgState* st = r.st;
      double mx = 0.0;
      for (int j = 0; j < g.m; ++j) {
        st->res[j] = sqrt(t[j]);
        st->yx[j] = 0.0;
        mx = st->res[j] > mx ? st->res[j] : mx;
      }
      st->iters += 1;
      live = !(st->tol > 0.0 && mx <= st->tol);
      if (!live) st->active = 0;
    }
    __syncthreads();
    if (!live) return;
  }
  const int nt = (g.ns + 15) >> 4;
  const int ntb = n_tiles_b(nt), ntot = ntb + n_tiles_a(nt);
  for (int e = threadIdx.x; e < ntot * 256; e += blockDim.x) {
    double v[kGramChunks];
#pragma unroll
    for (int c = 0; c < kGramChunks; ++c) v[c] = g.level2[(size_t)c * (ntot * 256) + e];
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kGramChunks; ++c) s += v[c];
    const int t = e >> 8, i = (e & 255) >> 4, j = e & 15;
    int I, J;
    bool isb;
    if (t < ntb) {
      isb = true;
      I = (t == 2) ? 1 : 0;
      J = (t == 0) ? 0 : 1;
    } else {
      isb = false;
      const int ta = t - ntb;
      I = ta >> 1;
      J = ta & 1;
      if (nt == 1) I = J = 0;
    }
    const int row = 16 * I + i, colj = 16 * J + j;
    if (row < g.ns && colj < g.ns) {
      if (isb) {
        sh.B[row * LD + colj] = s;
        if (I != J) sh.B[colj * LD + row] = s;  // the lower off-diagonal tile is the mirror
      } else {
        sh.A[row * LD + colj] = s;
      }
    }
  }
  __syncthreads();
  if (r.gram_out != nullptr) {
    for (int e = threadIdx.x; e < g.ns * g.ns; e += blockDim.x) {
      const int i = e / g.ns, j = e - (e / g.ns) * g.ns;
      r.gram_out[e] = sh.A[i * LD + j];
      r.gram_out[g.ns * g.ns + e] = sh.B[i * LD + j];
    }
  }
  if (threadIdx.x >= 64) return;
  rayleigh_ritz(sh, g.ns, g.m, r.drop_tol, r.zero_tol, r.conv2, r.C, r.theta, keptf, &nkept);
  wave_fence();
  if (threadIdx.x == 0 && r.st != nullptr) {
    LobpcgState* st = r.st;
    st->nkept = nkept;
    for (int j = 0; j < g.ns; ++j) st->kept[j] = keptf[j];
    st->dropped += g.ns - nkept;
    if (nkept < g.m) {
      st->status = GSF_EBREAKDOWN;
      st->active = 0;
      if (r.init) st->start_failed = 1;
    } else {
      for (int j = 0; j < g.m; ++j) st->theta[j] = sh.ev[sh.order[j]];
    }
  }
  if (r.kept_out != nullptr && (int)threadIdx.x < g.ns) r.kept_out[threadIdx.x] = keptf[threadIdx.x];
  if (r.nkept_out != nullptr && threadIdx.x == 0) *r.nkept_out = nkept;
}

// ---------------------------------------------------------------------------
// update + next residual
// ---------------------------------------------------------------------------
// Row helpers: the M values of one point, as vector memory operations when
// the row is a whole number of 16-byte words.
template <typename T, int M>
__device__ __forceinline__ void load_row(const T* __restrict__ src, T (&v)[M]) {
  if constexpr (sizeof(T) * M % 16 == 0) {
    constexpr int W = (int)(sizeof(T) * M / 16);
    const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
    for (int w = 0; w < W; ++w) reinterpret_cast<float4*>(v)[w] = s4[w];
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = src[j];
  }
}

template <typename T, int M>
__device__ __forceinline__ void store_row(T* __restrict__ dst, const T (&v)[M]) {
  if constexpr (sizeof(T) * M % 16 == 0) {
    constexpr int W = (int)(sizeof(T) * M / 16);
    float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
    for (int w = 0; w < W; ++w) d4[w] = reinterpret_cast<const float4*>(v)[w];
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) dst[j] = v[j];
  }
}

// NB = number of blocks in the trial basis: 1 (start block), 2 ([X, W]),
// 3 ([X, W, P]).  Coefficients C (NB*M x M, FP64) are read from LDS; every
// output column is accumulated in FP64 and rounded once.
template <typename T, int M, int NB>
__global__ void __launch_bounds__(kThreads) lob_update_kernel(LobArgs a, int first) {
  __shared__ double Cs[3 * M * M];
  __shared__ double th[M];
  __shared__ double red[16 * 2 * M];
  LobpcgState* st = a.st;
  if (!st->active) return;
  for (int e = threadIdx.x; e < NB * M * M; e += blockDim.x) Cs[e] = a.C[e];
  if (threadIdx.x < M) th[threadIdx.x] = st->theta[threadIdx.x];
  __syncthreads();
  T* __restrict__ X = (T*)a.X;
  T* __restrict__ W = (T*)a.W;
  T* __restrict__ P = (T*)a.P;
  T* __restrict__ AX = (T*)a.AX;
  T* __restrict__ AW = (T*)a.AW;
  T* __restrict__ AP = (T*)a.AP;
  const T* __restrict__ sqd = (const T*)a.sqd;
  const double yinv = st->ynorm_inv;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[2 * M];
#pragma unroll
  for (int j = 0; j < 2 * M; ++j) v[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    // keep the coefficients in LDS: without this the loop-invariant reads are
    // hoisted into (NB*M*M doubles of) registers and occupancy collapses
    __asm__ volatile("" ::: "memory");
    T s[NB][M], as[NB][M];
    load_row<T, M>(X + i * M, s[0]);
    load_row<T, M>(AX + i * M, as[0]);
    if constexpr (NB > 1) {
      load_row<T, M>(W + i * M, s[1]);
      load_row<T, M>(AW + i * M, as[1]);
    }
    if constexpr (NB > 2) {
      load_row<T, M>(P + i * M, s[2]);
      load_row<T, M>(AP + i * M, as[2]);
    }
    const double yi = (double)sqd[i] * yinv;
    T xo[M], axo[M], po[M], apo[M], ro[M];
#pragma unroll
    for (int t = 0; t < M; ++t) {
      double px = 0.0, pax = 0.0, pp = 0.0, pap = 0.0;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const double c = Cs[j * M + t];
        px += (double)s[0][j] * c;
        pax += (double)as[0][j] * c;
      }
#pragma unroll
      for (int b = 1; b < NB; ++b) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const double c = Cs[(b * M + j) * M + t];
          pp += (double)s[b][j] * c;
          pap += (double)as[b][j] * c;
        }
      }
      const double xn = px + pp, axn = pax + pap;
      const double rt = axn - xn * th[t];
      xo[t] = (T)xn;
      axo[t] = (T)axn;
      po[t] = (T)pp;
      apo[t] = (T)pap;
      ro[t] = (T)rt;
      v[t] += rt * rt;
      v[M + t] += yi * rt;
    }
    store_row<T, M>(X + i * M, xo);
    store_row<T, M>(AX + i * M, axo);
    if (!first) {
      store_row<T, M>(P + i * M, po);
      store_row<T, M>(AP + i * M, apo);
    }
    store_row<T, M>(W + i * M, ro);
  }
  block_sum<2 * M>(v, red);
  if (threadIdx.x == 0)
    for (int j = 0; j < 2 * M; ++j) a.vpart[(size_t)blockIdx.x * (2 * M) + j] = v[j];
}

// ---------------------------------------------------------------------------
// output: y = X X^T z0 (+ Y Y^T z0), x_out = y / sqrt(d)
// ---------------------------------------------------------------------------
template <typename T, int M>
__global__ void __launch_bounds__(kThreads) lob_out_dots_kernel(LobArgs a) {
  __shared__ double red[16 * (M + 1)];
  LobpcgState* st = a.st;
  if (st->start_failed) return;
  const T* __restrict__ X = (const T*)a.X;
  const T* __restrict__ x0 = (const T*)a.x0;
  const T* __restrict__ sqd = (const T*)a.sqd;
  const double yinv = st->ynorm_inv;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[M + 1];
#pragma unroll
  for (int j = 0; j <= M; ++j) v[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    const double z = (double)sqd[i] * (double)x0[i];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] += (double)X[i * M + j] * z;
    v[M] += (double)sqd[i] * yinv * z;
  }
  block_sum<M + 1>(v, red);
  if (threadIdx.x == 0)
    for (int j = 0; j <= M; ++j) a.vpart[(size_t)blockIdx.x * (M + 1) + j] = v[j];
}

template <typename T, int M>
__global__ void __launch_bounds__(kThreads) lob_output_kernel(LobArgs a) {
  const LobpcgState* st = a.st;
  const bool broke = st->start_failed != 0;
  const T* __restrict__ X = (const T*)a.X;
  const T* __restrict__ x0 = (const T*)a.x0;
  const T* __restrict__ sqd = (const T*)a.sqd;
  T* __restrict__ out = (T*)a.xout;
  T* __restrict__ rv = (T*)a.ritz;
  double c[M], sg[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    c[j] = st->yx[j];
    sg[j] = c[j] >= 0.0 ? 1.0 : -1.0;
  }
  const double cy = a.constraint ? st->yx[M] : 0.0;
  const double yinv = st->ynorm_inv;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    if (broke) {
      out[i] = x0[i];
      continue;
    }
    const double sq = (double)sqd[i];
    double y = sq * yinv * cy;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const double xv = (double)X[i * M + j];
      y += xv * c[j];
      if (rv != nullptr) rv[i * M + j] = (T)(sg[j] * xv);
    }
    out[i] = (T)(y / sq);
  }
}

template <typename T, int M>
void launch_m_kernels(int which, const LobArgs& a, int nb, int ns, int first, StartDegrees deg, hipStream_t s) {
  switch (which) {
    case 0:
      lob_start_kernel<T, M><<<nb, kThreads, 0, s>>>(a, deg);
      if (a.constraint) lob_final_kernel<M><<<1, kThreads, 0, s>>>(a.vpart, nb, a.st, 1, M, 0, 1);
      break;
    case 1:
      if (ns == M)
        lob_update_kernel<T, M, 1><<<nb, kThreads, 0, s>>>(a, first);
      else if (ns == 2 * M)
        lob_update_kernel<T, M, 2><<<nb, kThreads, 0, s>>>(a, first);
      else
        lob_update_kernel<T, M, 3><<<nb, kThreads, 0, s>>>(a, first);
      lob_final_kernel<2 * M><<<1, kThreads, 0, s>>>(a.vpart, nb, a.st, 2, M, first, a.constraint);
      break;
    case 4:
      if (ns == M)
        lob_update_kernel<T, M, 1><<<nb, kThreads, 0, s>>>(a, first);
      else if (ns == 2 * M)
        lob_update_kernel<T, M, 2><<<nb, kThreads, 0, s>>>(a, first);
      else
        lob_update_kernel<T, M, 3><<<nb, kThreads, 0, s>>>(a, first);
      break;
    case 5:
      lob_final_kernel<2 * M><<<1, kThreads, 0, s>>>(a.vpart, nb, a.st, 2, M, first, a.constraint);
      break;
    case 2:
      lob_out_dots_kernel<T, M><<<nb, kThreads, 0, s>>>(a);
      lob_final_kernel<M + 1><<<1, kThreads, 0, s>>>(a.vpart, nb, a.st, 3, M, 0, a.constraint);
      break;
    default: lob_output_kernel<T, M><<<nb, kThreads, 0, s>>>(a); break;
  }
}

template <typename T>
void launch_m_dispatch(int which, const LobArgs& a, int nb, int ns, int first, StartDegrees deg, hipStream_t s) {
  switch (a.m) {
    case 1: launch_m_kernels<T, 1>(which, a, nb, ns, first, deg, s); break;
    case 2: launch_m_kernels<T, 2>(which, a, nb, ns, first, deg, s); break;
    case 3: launch_m_kernels<T, 3>(which, a, nb, ns, first, deg, s); break;
    case 4: launch_m_kernels<T, 4>(which, a, nb, ns, first, deg, s); break;
    case 5: launch_m_kernels<T, 5>(which, a, nb, ns, first, deg, s); break;
    case 6: launch_m_kernels<T, 6>(which, a, nb, ns, first, deg, s); break;
    case 7: launch_m_kernels<T, 7>(which, a, nb, ns, first, deg, s); break;
    default: launch_m_kernels<T, 8>(which, a, nb, ns, first, deg, s); break;
  }
}

}  // namespace

gsf_status lob_launch_ynorm(const LobArgs& a, int nb, hipStream_t s) {
  if (a.prec == GSF_F32)
    lob_ynorm_kernel<float><<<nb, kThreads, 0, s>>>((const float*)a.sqd, a.n, a.vpart, a.st);
  else
    lob_ynorm_kernel<double><<<nb, kThreads, 0, s>>>((const double*)a.sqd, a.n, a.vpart, a.st);
  lob_final_kernel<1><<<1, kThreads, 0, s>>>(a.vpart, nb, a.st, 0, a.m, 0, 0);
  return launch_status();
}

gsf_status lob_launch_mkernel(int which, const LobArgs& a, int nb, int ns, int first, StartDegrees deg,
                              hipStream_t s) {
  if (a.prec == GSF_F32)
    launch_m_dispatch<float>(which, a, nb, ns, first, deg, s);
  else
    launch_m_dispatch<double>(which, a, nb, ns, first, deg, s);
  return launch_status();
}

gsf_status lob_launch_project(const LobArgs& a, void* B, int nb, hipStream_t s) {
  if (a.prec == GSF_F32)
    lob_project_kernel<float><<<nb, kThreads, 0, s>>>((float*)B, (const float*)a.sqd, a.n, a.m, a.st);
  else
    lob_project_kernel<double><<<nb, kThreads, 0, s>>>((double*)B, (const double*)a.sqd, a.n, a.m, a.st);
  return launch_status();
}

// The Gram pair is loaded by one workgroup of four waves; the Rayleigh-Ritz
// step runs on its first wave.
int rr_threads(int ns) { return kThreads; }

int gram_tiles_total(int ns) {
  const int nt = (ns + 15) >> 4;
  return nt == 1 ? 2 : 7;
}

gsf_status lob_launch_gram(const GramArgs& g, const RRArgs& r, int prec, hipStream_t s) {
  const bool two = g.ns > 16;
  if (prec == GSF_F32) {
    if (two)
      gram_kernel<float, 2><<<g.nparts, kThreads, 0, s>>>(g);
    else
      gram_kernel<float, 1><<<g.nparts, kThreads, 0, s>>>(g);
  } else {
    if (two)
      gram_kernel<double, 2><<<g.nparts, kThreads, 0, s>>>(g);
    else
      gram_kernel<double, 1><<<g.nparts, kThreads, 0, s>>>(g);
  }
  dim3 grid(gram_tiles_total(g.ns), kGramChunks);
  gram_reduce_kernel<<<grid, kThreads, 0, s>>>(g);
  gram_rr_kernel<<<1, rr_threads(g.ns), 0, s>>>(g, r);
  return launch_status();
}

// Rayleigh-Ritz alone on a Gram pair already in device memory (GA then GB,
// ns x ns each, row-major) -- one workgroup, the step itself on its first wave.
__global__ void __launch_bounds__(kThreads) rr_only_kernel(const double* __restrict__ G, int ns, int m, RRArgs r) {
  __shared__ RRShared sh;
  __shared__ int nkept;
  __shared__ int keptf[KMAX];
  for (int e = threadIdx.x; e < ns * ns; e += blockDim.x) {
    const int i = e / ns, j = e - (e / ns) * ns;
    sh.A[i * LD + j] = G[e];
    sh.B[i * LD + j] = G[ns * ns + e];
  }
  __syncthreads();
  if (threadIdx.x >= 64) return;
  rayleigh_ritz(sh, ns, m, r.drop_tol, r.zero_tol, r.conv2, r.C, r.theta, keptf, &nkept);
  wave_fence();
  if ((int)threadIdx.x < ns) r.kept_out[threadIdx.x] = keptf[threadIdx.x];
  if (threadIdx.x == 0) *r.nkept_out = nkept;
}

gsf_status lob_launch_rr_only(const double* G, int ns, int m, const RRArgs& r, hipStream_t s) {
  rr_only_kernel<<<1, rr_threads(ns), 0, s>>>(G, ns, m, r);
  return launch_status();
}

}  // namespace gsf
