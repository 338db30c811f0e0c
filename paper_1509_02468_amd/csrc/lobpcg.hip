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
  constexpr int U = 8;  // point groups of 4 loaded ahead of their MFMAs
  constexpr int ntb = NT == 1 ? 1 : 3, nta = NT == 1 ? 1 : 4;
  constexpr int nt = NT;
  __shared__ double wsum[4][4][64];  // one tile at a time: wave, register, lane
  if (g.active != nullptr && *g.active == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ns = g.ns, m = g.m;
  const int col = lane & 15, krow = lane >> 4;

  // the S / AS column each lane feeds for tile row I (0 past the last column)
  const T* sp[2] = {nullptr, nullptr};
  const T* ap[2] = {nullptr, nullptr};
  for (int I = 0; I < nt; ++I) {
    const int c = 16 * I + col;
    if (c < ns) {
      const int b = c / m, j = c - (c / m) * m;
      sp[I] = (const T*)g.S[b] + j;
      ap[I] = (const T*)g.AS[b] + j;
    }
  }

  const int64_t nw = (int64_t)gridDim.x * 4;
  const int64_t wid = (int64_t)blockIdx.x * 4 + wave;
  int64_t chunk = (g.n + nw - 1) / nw;
  chunk = (chunk + 4 * U - 1) / (4 * U) * (4 * U);
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

  int steps = 0;
  for (int64_t p0 = p_begin; p0 < p_end; p0 += 4 * U) {
    T s0[U], s1[U], a0[U], a1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t p = p0 + 4 * u + krow;
      const bool ok = p < p_end;
      s0[u] = (ok && sp[0]) ? sp[0][p * m] : T(0);
      a0[u] = (ok && sp[0]) ? ap[0][p * m] : T(0);
      s1[u] = (NT > 1 && ok && sp[1]) ? sp[1][p * m] : T(0);
      a1[u] = (NT > 1 && ok && sp[1]) ? ap[1][p * m] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      accb[0] = MfmaAcc<T>::mfma(s0[u], s0[u], accb[0]);
      acca[0] = MfmaAcc<T>::mfma(s0[u], a0[u], acca[0]);
      if constexpr (NT > 1) {
        accb[1] = MfmaAcc<T>::mfma(s0[u], s1[u], accb[1]);
        accb[2] = MfmaAcc<T>::mfma(s1[u], s1[u], accb[2]);
        acca[1] = MfmaAcc<T>::mfma(s0[u], a1[u], acca[1]);
        acca[2] = MfmaAcc<T>::mfma(s1[u], a0[u], acca[2]);
        acca[3] = MfmaAcc<T>::mfma(s1[u], a1[u], acca[3]);
      }
    }
    steps += U;
    if (sizeof(T) == 4 && steps >= 64) {  // FP32: move each 256-point partial into FP64
      steps = 0;
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
    }
  }
#pragma unroll
  for (int t = 0; t < ntb; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) totb[t][v] += (double)accb[t][v];
#pragma unroll
  for (int t = 0; t < nta; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) tota[t][v] += (double)acca[t][v];

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
// Rayleigh-Ritz on one workgroup (FP64)
// ---------------------------------------------------------------------------
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
constexpr int KMAX = 24;
constexpr int LD = KMAX + 1;

struct RRShared {
  double A[KMAX * LD];
  double B[KMAX * LD];
  double L[KMAX * LD];
  double LK[KMAX * LD];  // compressed Cholesky factor of the kept columns
  double M[KMAX * LD];
  double M2[KMAX * LD];
  double V[KMAX * LD];
  double V2[KMAX * LD];
  double delta[KMAX];
  double jself[KMAX + 1];
  double joff[KMAX + 1];
  double dnew[KMAX + 1];
  int partner[KMAX + 1];
  int good[KMAX];
  int kept[KMAX];
  int idx[KMAX];
  int order[KMAX];
  double ev[KMAX];
  double red[64];
  double piv;
  int keep;
  int nk;
  int stop;
};

// Solves the Rayleigh-Ritz problem for GA, GB (ns x ns, already loaded into
// sh.A and sh.B) and writes C (ns x m, row-major with leading dimension m),
// theta and the kept flags.  All threads of the workgroup take part.
__device__ __forceinline__ void rayleigh_ritz(RRShared& sh, int ns, int m, double drop_tol, double zero_tol, double* Cout,
                              double* theta, int* kept_out, int* nkept_out) {
  const int tid = threadIdx.x, nth = blockDim.x;
  // symmetrise
  for (int e = tid; e < ns * ns; e += nth) {
    const int i = e / ns, j = e - (e / ns) * ns;
    if (i < j) {
      const double a = 0.5 * (sh.A[i * LD + j] + sh.A[j * LD + i]);
      const double b = 0.5 * (sh.B[i * LD + j] + sh.B[j * LD + i]);
      sh.M[i * LD + j] = a;
      sh.M2[i * LD + j] = b;
    }
  }
  __syncthreads();
  for (int e = tid; e < ns * ns; e += nth) {
    const int i = e / ns, j = e - (e / ns) * ns;
    if (i < j) {
      sh.A[i * LD + j] = sh.A[j * LD + i] = sh.M[i * LD + j];
      sh.B[i * LD + j] = sh.B[j * LD + i] = sh.M2[i * LD + j];
    }
  }
  __syncthreads();
  // zero columns and unit-diagonal scaling
  if (tid == 0) {
    double mx = 0.0;
    for (int j = 0; j < ns; ++j) mx = sh.B[j * LD + j] > mx ? sh.B[j * LD + j] : mx;
    for (int j = 0; j < ns; ++j) {
      const double d = sh.B[j * LD + j];
      const int gd = d > zero_tol * zero_tol * mx;
      sh.good[j] = gd;
      sh.delta[j] = gd ? 1.0 / sqrt(d) : 0.0;
    }
  }
  __syncthreads();
  for (int e = tid; e < ns * ns; e += nth) {
    const int i = e / ns, j = e - (e / ns) * ns;
    const double s = sh.delta[i] * sh.delta[j];
    sh.A[i * LD + j] *= s;
    sh.B[i * LD + j] *= s;
    sh.L[i * LD + j] = 0.0;
  }
  __syncthreads();
  // right-looking Cholesky of B with column dropping (lower triangle of B is the work array)
  for (int j = 0; j < ns; ++j) {
    if (tid == 0) {
      const double piv = sh.B[j * LD + j];
      const int keep = sh.good[j] && (piv > drop_tol);
      sh.kept[j] = keep;
      sh.keep = keep;
      sh.piv = keep ? sqrt(piv) : 0.0;
      if (keep) sh.L[j * LD + j] = sh.piv;
    }
    __syncthreads();
    if (sh.keep) {
      for (int i = j + 1 + tid; i < ns; i += nth) sh.L[i * LD + j] = sh.B[i * LD + j] / sh.piv;
      __syncthreads();
      const int rem = ns - j - 1;
      for (int e = tid; e < rem * rem; e += nth) {
        const int i = j + 1 + e / rem, l = j + 1 + (e - (e / rem) * rem);
        if (l <= i) sh.B[i * LD + l] -= sh.L[i * LD + j] * sh.L[l * LD + j];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    int k = 0;
    for (int j = 0; j < ns; ++j)
      if (sh.kept[j]) sh.idx[k++] = j;
    sh.nk = k;
  }
  __syncthreads();
  const int K = sh.nk;
  if (tid < ns) kept_out[tid] = sh.kept[tid];
  if (tid == 0) *nkept_out = K;
  if (K < m) {
    __syncthreads();
    return;
  }
  // compressed factor LK (in L) and reduced A (in M2)
  for (int e = tid; e < K * K; e += nth) {
    const int a = e / K, b = e - (e / K) * K;
    sh.LK[a * LD + b] = (b <= a) ? sh.L[sh.idx[a] * LD + sh.idx[b]] : 0.0;
    sh.M2[a * LD + b] = sh.A[sh.idx[a] * LD + sh.idx[b]];
  }
  __syncthreads();
  // T = LK^-1 A_K: thread c solves LK t = A_K[:, c] by forward substitution
  // with its column in registers (LK read as LDS broadcasts), then writes row
  // c of T^T.  A_K is symmetric, so M = T LK^-T = (LK^-1 T^T)^T.
  if (tid < K) {
    const int c = tid;
    double col[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      if (i < K) {
        double v = sh.M2[i * LD + c];
#pragma unroll
        for (int t = 0; t < KMAX; ++t)
          if (t < i) v -= sh.LK[i * LD + t] * col[t];
        col[i] = v / sh.LK[i * LD + i];
      }
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
      if (i < K) sh.V[c * LD + i] = col[i];  // V = T^T
  }
  __syncthreads();
  if (tid < K) {
    const int c = tid;
    double col[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      if (i < K) {
        double v = sh.V[i * LD + c];
#pragma unroll
        for (int t = 0; t < KMAX; ++t)
          if (t < i) v -= sh.LK[i * LD + t] * col[t];
        col[i] = v / sh.LK[i * LD + i];
      }
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
      if (i < K) sh.M2[c * LD + i] = col[i];  // M2 = (LK^-1 T^T)^T = M
  }
  __syncthreads();
  for (int e = tid; e < K * K; e += nth) {
    const int a = e / K, b = e - (e / K) * K;
    sh.M[a * LD + b] = 0.5 * (sh.M2[a * LD + b] + sh.M2[b * LD + a]);
    sh.V[a * LD + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();

  // cyclic Jacobi with round-robin parallel ordering
  const int np = (K + 1) & ~1;  // players (a dummy when K is odd)
  // this thread's matrix elements, fixed for the whole eigensolve
  constexpr int EPT = (KMAX * KMAX + 63) / 64;  // enough for any launch of >= 64 threads
  int ei[EPT], ej[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = tid + k * nth;
    ei[k] = e < K * K ? e / K : -1;
    ej[k] = e < K * K ? e - (e / K) * K : 0;
  }
  double* Mc = sh.M;
  double* Mn = sh.M2;
  double* Vc = sh.V;
  double* Vn = sh.V2;
  for (int sweep = 0; sweep < 30; ++sweep) {
    for (int rnd = 0; rnd < np - 1; ++rnd) {
      if (tid < np / 2) {
        const int s0 = tid, s1 = np - 1 - tid;
        const int pa = (s0 == 0) ? 0 : 1 + ((s0 - 1 + rnd) % (np - 1));
        const int pb = 1 + ((s1 - 1 + rnd) % (np - 1));
        const int p = pa < pb ? pa : pb, q = pa < pb ? pb : pa;
        double c = 1.0, s = 0.0, t = 0.0, apq = 0.0;
        if (q < K) {
          apq = Mc[p * LD + q];
          if (apq != 0.0) {
            // t = tan of the rotation angle, the root of t^2 + 2 theta t - 1 = 0
            // of smaller magnitude, theta = (a_qq - a_pp) / (2 a_pq)
            const double d = Mc[q * LD + q] - Mc[p * LD + p];
            const double y = fma(d, d, 4.0 * apq * apq);
            const double h = y * rsq_nr(y);
            t = 2.0 * apq * rcp_nr(d >= 0.0 ? d + h : d - h);
            c = rsq_nr(fma(t, t, 1.0));
            s = t * c;
          }
        }
        sh.partner[p] = q;
        sh.partner[q] = p;
        sh.jself[p] = c;
        sh.jself[q] = c;
        sh.joff[p] = -s;  // J[q][p]
        sh.joff[q] = s;   // J[p][q]
        // the rotated pair: a_pq becomes exactly 0, the diagonal moves by t a_pq
        sh.dnew[p] = (q < K) ? Mc[p * LD + p] - t * apq : Mc[p * LD + p];
        if (q < K) sh.dnew[q] = Mc[q * LD + q] + t * apq;
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        if (ei[k] < 0) continue;
        const int i = ei[k], j = ej[k];
        const int pi = sh.partner[i], pj = sh.partner[j];
        const double ci = sh.jself[i], oi = sh.joff[i], cj = sh.jself[j], oj = sh.joff[j];
        double v;
        if (i == j) {
          v = sh.dnew[i];
        } else if (pi == j) {
          v = 0.0;
        } else {
          v = ci * cj * Mc[i * LD + j];
          if (pj < K) v += ci * oj * Mc[i * LD + pj];
          if (pi < K) {
            v += oi * cj * Mc[pi * LD + j];
            if (pj < K) v += oi * oj * Mc[pi * LD + pj];
          }
        }
        Mn[i * LD + j] = v;
        double w = Vc[i * LD + j] * cj;
        if (pj < K) w += Vc[i * LD + pj] * oj;
        Vn[i * LD + j] = w;
      }
      __syncthreads();
      double* t1 = Mc;
      Mc = Mn;
      Mn = t1;
      double* t2 = Vc;
      Vc = Vn;
      Vn = t2;
    }
    // convergence: off-diagonal mass relative to the whole
    double acc[2] = {0.0, 0.0};
    for (int e = tid; e < K * K; e += nth) {
      const int i = e / K, j = e - (e / K) * K;
      const double v = Mc[i * LD + j] * Mc[i * LD + j];
      if (i == j)
        acc[1] += v;
      else
        acc[0] += v;
    }
    block_sum<2>(acc, sh.red);
    // off-diagonal Frobenius mass below 1e-14 of the whole (relative)
    if (tid == 0) sh.stop = (acc[0] <= 1e-28 * (acc[0] + acc[1])) ? 1 : 0;
    __syncthreads();
    if (sh.stop) break;
  }
  // order eigenvalues ascending (ties by index)
  if (tid < K) sh.ev[tid] = Mc[tid * LD + tid];
  __syncthreads();
  if (tid < K) {
    int rank = 0;
    const double e = sh.ev[tid];
    for (int j = 0; j < K; ++j) rank += (sh.ev[j] < e || (sh.ev[j] == e && j < tid)) ? 1 : 0;
    sh.order[rank] = tid;
  }
  __syncthreads();
  if (tid < m) theta[tid] = sh.ev[sh.order[tid]];
  // C_K = LK^-T Z_m: thread t solves LK^T c = Z[:, order[t]] by back substitution
  for (int e = tid; e < ns * m; e += nth) Cout[e] = 0.0;
  __syncthreads();
  if (tid < m) {
    const int t = tid, col = sh.order[t];
    double c[KMAX];
#pragma unroll
    for (int ii = KMAX - 1; ii >= 0; --ii) {
      if (ii < K) {
        double v = Vc[ii * LD + col];
#pragma unroll
        for (int b = 0; b < KMAX; ++b)
          if (b > ii && b < K) v -= sh.LK[b * LD + ii] * c[b];
        c[ii] = v / sh.LK[ii * LD + ii];
      }
    }
    // sign: the largest-magnitude coefficient (first on ties) is positive, so
    // Ritz vectors (and residuals) have a fixed sign for a non-odd T
    double big = 0.0, sgn = 1.0;
#pragma unroll
    for (int a = 0; a < KMAX; ++a)
      if (a < K) {
        const double v = sh.delta[sh.idx[a]] * c[a];
        if (fabs(v) > big) {
          big = fabs(v);
          sgn = v < 0.0 ? -1.0 : 1.0;
        }
      }
#pragma unroll
    for (int a = 0; a < KMAX; ++a)
      if (a < K) {
        const int row = sh.idx[a];
        Cout[row * m + t] = sgn * (sh.delta[row] * c[a]);
      }
  }
  __syncthreads();
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

// One workgroup: sums the chunks, assembles GA and GB (ns x ns) and runs the
// Rayleigh-Ritz step.
__global__ void __launch_bounds__(kThreads) gram_rr_kernel(GramArgs g, RRArgs r) {
  __shared__ RRShared sh;
  if (r.st != nullptr && !r.st->active) return;
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
    __syncthreads();
  }
  __shared__ int nkept;
  __shared__ int keptf[KMAX];
  rayleigh_ritz(sh, g.ns, g.m, r.drop_tol, r.zero_tol, r.C, r.theta, keptf, &nkept);
  __syncthreads();
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
      for (int j = 0; j < g.m; ++j) st->theta[j] = r.theta[j];
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

// The Rayleigh-Ritz step runs on one workgroup of four waves.
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
// ns x ns each, row-major) -- one workgroup.
__global__ void __launch_bounds__(kThreads) rr_only_kernel(const double* __restrict__ G, int ns, int m, RRArgs r) {
  __shared__ RRShared sh;
  for (int e = threadIdx.x; e < ns * ns; e += blockDim.x) {
    const int i = e / ns, j = e - (e / ns) * ns;
    sh.A[i * LD + j] = G[e];
    sh.B[i * LD + j] = G[ns * ns + e];
  }
  __syncthreads();
  __shared__ int nkept;
  __shared__ int keptf[KMAX];
  rayleigh_ritz(sh, ns, m, r.drop_tol, r.zero_tol, r.C, r.theta, keptf, &nkept);
  if (threadIdx.x < ns) r.kept_out[threadIdx.x] = keptf[threadIdx.x];
  if (threadIdx.x == 0) *r.nkept_out = nkept;
}

gsf_status lob_launch_rr_only(const double* G, int ns, int m, const RRArgs& r, hipStream_t s) {
  rr_only_kernel<<<1, rr_threads(ns), 0, s>>>(G, ns, m, r);
  return hipGetLastError() == hipSuccess ? GSF_OK : GSF_EDEVICE;
}

}  // namespace gsf
