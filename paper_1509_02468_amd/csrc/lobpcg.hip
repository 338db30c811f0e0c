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

// Reciprocal and reciprocal square root: the hardware approximations refined
// by one Newton step (a few ulp), short dependency chains for the Jacobi
// rotations.  The rotation stays orthogonal to rounding because c and s are
// both derived from the same t: c = (1 + t^2)^-1/2, s = t c.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
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
  double M[KMAX * LD];   // reduced matrix L^-1 A L^-T, tridiagonalised in place
  double M2[KMAX * LD];  // work; then the Householder vectors (row k: v_k)
  double V[KMAX * LD];   // work; then the wanted eigenvectors (columns)
  double V2[KMAX * LD];  // Givens rotations of the tridiagonal QR, transposed (row j: column j)
  double Cs[KMAX * 8];   // output coefficients, staged
  double delta[KMAX];
  double rinv[KMAX];
  double ev[KMAX];
  int good[KMAX];
  int kept[KMAX];
  int idx[KMAX];
  int order[KMAX];
};
// Broadcast lane k's value of v to the whole wave (k uniform).
__device__ __forceinline__ double bcast(double v, int k) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, k);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Solves the Rayleigh-Ritz problem for GA, GB (ns x ns, already loaded into
// sh.A and sh.B): C (ns x m, row-major with leading dimension m) and theta
// (ascending) of the m smallest Ritz pairs, the kept flags and their count.
// Called by the 64 lanes of one wave; KB >= ns is the padded size of the
// triangular solves (the kept block is extended by an identity factor and
// zero data there, which changes nothing and keeps the loops free of
// conditionals).  Steps: symmetrise; scale to unit diag(GB) (columns with a
// negligible diagonal are dropped); Cholesky GB = L L^T that drops columns
// with a pivot below drop_tol; M = L^-1 GA L^-T on the kept columns; the
// eigenpairs of M by Householder tridiagonalisation and the implicit
// symmetric tridiagonal QR iteration with the Wilkinson shift (Golub and Van
// Loan, sections 8.3.1-8.3.3); C = L^-T Z for the m smallest.  Loads are
// issued unconditionally (clamped indices) and only stores are masked, so a
// lane never waits on a load inside a branch.
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

  // Householder tridiagonalisation of M (K x K) in place: step k maps the
  // column below the diagonal, x = M[k+1:, k], onto alpha e_1 with
  // H = I - beta v v^T, v = x - alpha e_1, alpha = -sign(x_0) ||x||,
  // beta = 1 / (||x||^2 - x_0 alpha), and updates the trailing block as
  // M <- M - v w^T - w v^T with p = beta M v, w = p - (beta/2)(v^T p) v.
  // Lane i holds entry i of x, v, p and w; row j of M is read at column i
  // (contiguous across lanes; M stays symmetric to rounding).  The tridiagonal
  // ends up distributed over the lanes: lane i holds d_i = T_ii and
  // e_i = T_{i,i+1}; v_k is kept in row k of M2 and beta_k in lane k of hb.
  double d = 0.0, e = 0.0, hb = 0.0;
  const bool lk = lane < K;
  for (int k = 0; k + 2 < K; ++k) {
    const bool in = lane > k && lk;
    const double xi = in ? sh.M[k * LD + (lane < K ? lane : 0)] : 0.0;
    const double s2 = wave_sum(xi * xi);
    const double x0 = bcast(xi, k + 1);
    const double dk = sh.M[k * LD + k];
    d = lane == k ? dk : d;
    double vi = 0.0, beta = 0.0, alpha = x0;
    if (s2 - x0 * x0 > 0.0) {  // uniform: something below the subdiagonal
      const double sig = sqrt(s2);
      alpha = x0 >= 0.0 ? -sig : sig;
      beta = 1.0 / (s2 - x0 * alpha);
      vi = lane == k + 1 ? x0 - alpha : xi;
      double pi = 0.0;
      for (int j = k + 1; j < K; ++j) pi = fma(sh.M[j * LD + (lane < K ? lane : 0)], bcast(vi, j), pi);
      pi = in ? beta * pi : 0.0;
      const double kc = 0.5 * beta * wave_sum(vi * pi);
      const double wi = pi - kc * vi;
      for (int j = k + 1; j < K; ++j) {
        const double vj = bcast(vi, j), wj = bcast(wi, j);
        const double mji = sh.M[j * LD + (lane < K ? lane : 0)];
        if (in) sh.M[j * LD + lane] = mji - (vj * wi + wj * vi);
      }
      wave_fence();
    }
    e = lane == k ? alpha : e;
    hb = lane == k ? beta : hb;
    if (lk) sh.M2[k * LD + lane] = vi;
  }
  // the trailing 1 x 1 or 2 x 2 block
  if (K >= 2) {
    const double a = sh.M[(K - 2) * LD + (K - 2)], b = sh.M[(K - 1) * LD + (K - 1)];
    const double f = sh.M[(K - 1) * LD + (K - 2)];
    d = lane == K - 2 ? a : (lane == K - 1 ? b : d);
    e = lane == K - 2 ? f : e;
  } else {
    d = lane == 0 ? sh.M[0] : d;
  }
  e = lane < K - 1 ? e : 0.0;
  // Z = I (stored transposed: row j of V2 is column j of Z)
  for (int q = lane; q < K * K; q += 64) {
    const int j = q / K, i = q - (q / K) * K;
    sh.V2[j * LD + i] = i == j ? 1.0 : 0.0;
  }
  wave_fence();
  // Implicit symmetric QR with the Wilkinson shift on the unreduced block
  // [l, h] at the bottom of the undeflated part; an off-diagonal entry is set
  // to zero once |e_i| <= tol (|d_i| + |d_{i+1}|).  Each step chases the
  // bulge down with Givens rotations G = [[c, -s], [s, c]] on (k, k+1),
  // T <- G^T T G, Z <- Z G.  All lanes compute the rotation chain (uniform
  // values); lane i updates row i of Z.
  const double tol = conv2 > 0.0 ? fmax(sqrt(conv2), 2.220446049250313e-16) : 2.220446049250313e-16;
  for (int it = 0; it < 30 * KB; ++it) {
    const double dn = __shfl_down(d, 1, 64);
    if (lane < K - 1 && fabs(e) <= tol * (fabs(d) + fabs(dn))) e = 0.0;
    const unsigned long long nz = __ballot(lane < K - 1 && e != 0.0);
    if (nz == 0ull) break;
    const int h = 64 - __clzll(nz);  // e_{h-1} != 0 and e_h, e_{h+1}, ... == 0
    const unsigned long long zero_below = ~nz & ((1ull << (h - 1)) - 1ull);
    const int l = zero_below ? 64 - __clzll(zero_below) : 0;
    const double dh1 = bcast(d, h - 1), dh = bcast(d, h), eh1 = bcast(e, h - 1);
    const double delta = 0.5 * (dh1 - dh);
    const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * sqrt(fma(delta, delta, eh1 * eh1));
    const double mu = dh - eh1 * (eh1 / den);
    double x = bcast(d, l) - mu, z = bcast(e, l);
    double a = bcast(d, l), f = bcast(e, l);
    for (int k = l; k < h; ++k) {
      const double q2 = fma(x, x, z * z);
      const double ir = q2 > 0.0 ? rsq_nr2(q2) : 0.0;
      const double c = q2 > 0.0 ? x * ir : 1.0, sn = q2 > 0.0 ? z * ir : 0.0;
      if (k > l) e = lane == k - 1 ? q2 * ir : e;  // r = hypot(x, z)
      const double b = bcast(d, k + 1);
      const double cc = c * c, ss = sn * sn, cs = c * sn;
      const double dk = fma(cc, a, fma(2.0 * cs, f, ss * b));
      const double dk1 = fma(ss, a, fma(-2.0 * cs, f, cc * b));
      const double ek = fma(cs, b - a, (cc - ss) * f);
      d = lane == k ? dk : (lane == k + 1 ? dk1 : d);
      e = lane == k ? ek : e;
      if (k + 1 < h) {
        const double en = bcast(e, k + 1);
        const double ecn = c * en;
        e = lane == k + 1 ? ecn : e;
        x = ek;
        z = sn * en;
        a = dk1;
        f = ecn;
      }
      const double z0 = sh.V2[k * LD + (lane < K ? lane : 0)], z1 = sh.V2[(k + 1) * LD + (lane < K ? lane : 0)];
      if (lk) {
        sh.V2[k * LD + lane] = fma(c, z0, sn * z1);
        sh.V2[(k + 1) * LD + lane] = fma(-sn, z0, c * z1);
      }
    }
    wave_fence();
  }
  // eigenvalues ascending (ties by index)
  if (lk) sh.ev[lane] = d;
  for (int q = lane; q < ns * m; q += 64) sh.Cs[q] = 0.0;
  wave_fence();
  {
    const double ei = sh.ev[lane < K ? lane : 0];
    int rank = 0;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const double ej = sh.ev[j < K ? j : 0];
      rank += (j < K && (ej < ei || (ej == ei && j < lane))) ? 1 : 0;
    }
    if (lk) sh.order[rank] = lane;
  }
  wave_fence();
  // eigenvectors of M for the m smallest: y = H_0 H_1 ... H_{K-3} z, lane i
  // holding entry i of every wanted vector; stored as columns order[t] of V
  {
    double y[kMaxBlock];
#pragma unroll
    for (int t = 0; t < kMaxBlock; ++t) {
      const int col = sh.order[t < m ? t : 0];
      y[t] = (t < m && lk) ? sh.V2[col * LD + lane] : 0.0;
    }
    for (int k = K - 3; k >= 0; --k) {
      const double vk = lk ? sh.M2[k * LD + lane] : 0.0;
      const double bk = bcast(hb, k);
      double dots[kMaxBlock];
#pragma unroll
      for (int t = 0; t < kMaxBlock; ++t) dots[t] = t < m ? vk * y[t] : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int t = 0; t < kMaxBlock; ++t) dots[t] += __shfl_xor(dots[t], off, 64);
      }
#pragma unroll
      for (int t = 0; t < kMaxBlock; ++t) y[t] = fma(-bk * dots[t], vk, y[t]);
    }
#pragma unroll
    for (int t = 0; t < kMaxBlock; ++t) {
      const int col = sh.order[t < m ? t : 0];
      if (t < m && lk) sh.V[lane * LD + col] = y[t];
    }
  }
  wave_fence();
  const double* Vc = sh.V;
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
  if (r.kept_out != nullptr && threadIdx.x < g.ns) r.kept_out[threadIdx.x] = keptf[threadIdx.x];
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
  return hipGetLastError() == hipSuccess ? GSF_OK : GSF_EDEVICE;
}

gsf_status lob_launch_mkernel(int which, const LobArgs& a, int nb, int ns, int first, StartDegrees deg,
                              hipStream_t s) {
  if (a.prec == GSF_F32)
    launch_m_dispatch<float>(which, a, nb, ns, first, deg, s);
  else
    launch_m_dispatch<double>(which, a, nb, ns, first, deg, s);
  return hipGetLastError() == hipSuccess ? GSF_OK : GSF_EDEVICE;
}

gsf_status lob_launch_project(const LobArgs& a, void* B, int nb, hipStream_t s) {
  if (a.prec == GSF_F32)
    lob_project_kernel<float><<<nb, kThreads, 0, s>>>((float*)B, (const float*)a.sqd, a.n, a.m, a.st);
  else
    lob_project_kernel<double><<<nb, kThreads, 0, s>>>((double*)B, (const double*)a.sqd, a.n, a.m, a.st);
  return hipGetLastError() == hipSuccess ? GSF_OK : GSF_EDEVICE;
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
  return hipGetLastError() == hipSuccess ? GSF_OK : GSF_EDEVICE;
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
  if (threadIdx.x < ns) r.kept_out[threadIdx.x] = keptf[threadIdx.x];
  if (threadIdx.x == 0) *r.nkept_out = nkept;
}

gsf_status lob_launch_rr_only(const double* G, int ns, int m, const RRArgs& r, hipStream_t s) {
  rr_only_kernel<<<1, rr_threads(ns), 0, s>>>(G, ns, m, r);
  return hipGetLastError() == hipSuccess ? GSF_OK : GSF_EDEVICE;
}

}  // namespace gsf
