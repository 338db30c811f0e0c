// Block LOBPCG as a low-pass filter (Algorithm 3, Section 6, generalised to a
// block of m vectors), z-space operator A = L_sym, B = I, T = I.
//
// Kernels:
//   lob_ynorm      ||sqrt(d)|| for the constraint vector Y = sqrt(d)/||sqrt(d)||
//   lob_start      X0[:, j] = z0 * phi_j (Legendre modulations), Y^T X0
//   lob_project    B -= Y c (constraint projection of a block)
//   gram           partial Gram tiles S^T S, S^T (A S) of S = [X, W, P] with
//                  MFMA, 4x4 tiles of v_mfma_f64_4x4x4f64 for both data types
//                  (an FP32 value widened to FP64 loses nothing and the
//                  product of two is exact in FP64, so FP32 data get FP64 sums
//                  too)
//   gram_reduce /  fixed-order two-level reduction of the tiles (one level,
//   gram_rr        inside gram_rr, with at most 16 Gram workgroups), then the
//                  Rayleigh-Ritz step on one workgroup in FP64: unit-diagonal
//                  scaling, column-dropping Cholesky, reduction to
//                  L^-1 A L^-T, the m smallest eigenpairs (Householder
//                  tridiagonalisation, bisection, inverse iteration), m
//                  smallest Ritz pairs; extra workgroups of both launches run
//                  the joint driver's CG phases (cg_step.h)
//   lob_update     X = S C, AX = (AS) C, P = [W,P] C, AP likewise, the next
//                  residual W = AX - X Theta and its norms (and Y^T W)
//   lob_out_dots / lob_output: y = X X^T z0 (+ Y Y^T z0), x_out = y / sqrt(d)
#include <cmath>

#include "cg_step.h"
#include "gsf_internal.h"
#include "solver_state.h"
#include "lobpcg_launch.h"

namespace gsf {
namespace {


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
// Output format (read by the reductions and the Rayleigh-Ritz step): tiles of
// 16x16 entries, nt = ceil(ns/16) tile rows.  S^T S: upper tiles (I <= J) in
// the order (0,0), (0,1), (1,1); S^T AS: all tiles (0,0), (0,1), (1,0), (1,1).
__device__ __forceinline__ int n_tiles_b(int nt) { return nt == 1 ? 1 : 3; }
__device__ __forceinline__ int n_tiles_a(int nt) { return nt == 1 ? 1 : 4; }

// Gram matrix (GB = S^T S or GA = S^T AS), row and column of entry e of the
// tile sequence above (tile e >> 8, entry (e & 255) = 16 i + j)
__device__ __forceinline__ void tile_entry(int e, int nt, bool& isb, int& row, int& col) {
  const int t = e >> 8, i = (e & 255) >> 4, j = e & 15;
  const int ntb = n_tiles_b(nt);
  int I, J;
  if (t < ntb) {
    isb = true;
    I = (t == 2) ? 1 : 0;
    J = (t == 0) ? 0 : 1;
  } else {
    isb = false;
    I = (nt == 1) ? 0 : (t - ntb) >> 1;
    J = (nt == 1) ? 0 : (t - ntb) & 1;
  }
  row = 16 * I + i;
  col = 16 * J + j;
}

// v_mfma_f64_4x4x4f64 runs four independent 4x4x4 products (blocks q = 0..3).
// Lane l holds A[i = l%4][k = l/16] and B[k = l/16][j = l%4] of block
// q = (l/4)%4, and receives D[i = l/16][j = l%4] of that block (found with a
// probe of the instruction on the GPU).
__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// index of the S^T S tile (I, J), I <= J, of TG column groups (row-major upper)
template <int TG>
__device__ __forceinline__ constexpr int tile_b(int I, int J) {
  return I * TG - (I * (I - 1)) / 2 + (J - I);
}

// S^T S and S^T AS over the points of each workgroup, in FP64 for both data
// types: an FP32 value widened to FP64 loses nothing and the product of two is
// exact in FP64, so FP32 data get exact products and FP64 sums.  (The entries
// that steer a nearly converged column, X^T A W ~ ||r||, are far below the
// size of their terms; FP32 sums lose them.)
//
// The ns columns form TG groups of 4.  Every lane takes one point and one
// column of a group: lane l reads point p0 + l/4, column 4G + l%4, which
// makes each group's loads one contiguous run per instruction for m = 4 and
// 8.  With that mapping block q of the MFMA sums the points p0 + 4k + q, and
// one instruction adds 16 points to the 4x4 tile of groups (I, J):
// A = the S values of group I, B = the AS (or S) values of group J.  A stage
// of 16 points is TG loads of S and TG of AS per lane, TG^2 + TG(TG+1)/2
// MFMAs.  The four blocks are summed across lanes at the end, then the four
// waves, in fixed order.
template <typename T, int TG>
__global__ void __launch_bounds__(kThreads) gram_kernel(GramArgs g) {
  typedef const __attribute__((address_space(1))) T* gptr;
  constexpr int NA = TG * TG, NB = TG * (TG + 1) / 2;
  constexpr int NS = 3;        // register stages (loads of the next two in flight)
  constexpr int FL = NS * 16;  // points of one loop trip
  __shared__ double red[4][NA + NB][16];
  if (g.active != nullptr && *g.active == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ns = g.ns, m = g.m;
  const int pl = lane >> 2, cl = lane & 3;

  // the S / AS column this lane feeds for group G; lanes past the last
  // column read column 0 and feed zeros as A operands
  gptr sp[TG], ap[TG];
  float lv[TG];
#pragma unroll
  for (int G = 0; G < TG; ++G) {
    const int c = 4 * G + cl;
    const bool live = c < ns;
    const int cc = live ? c : 0;
    const int b = cc / m, j = cc - (cc / m) * m;
    sp[G] = (gptr)g.S[b] + j;
    ap[G] = (gptr)g.AS[b] + j;
    lv[G] = live ? 1.0f : 0.0f;
  }

  const int64_t nw = (int64_t)gridDim.x * 4;
  const int64_t wid = (int64_t)blockIdx.x * 4 + wave;
  int64_t chunk = (g.n + nw - 1) / nw;
  chunk = (chunk + FL - 1) / FL * FL;
  const int64_t p_begin = wid * chunk;
  const int64_t p_end = (p_begin + chunk < g.n) ? p_begin + chunk : g.n;

  double acca[NA], accb[NB];
#pragma unroll
  for (int t = 0; t < NA; ++t) acca[t] = 0.0;
#pragma unroll
  for (int t = 0; t < NB; ++t) accb[t] = 0.0;

  // loads are unconditional (a point past the end re-reads p_begin); its
  // 0/1 mask multiplies only the A operands, when the stage's MFMAs run
  auto load = [&](int64_t p0, T (&sv)[TG], T (&av)[TG], T& mk) {
    const int64_t p = p0 + pl;
    const bool ok = p < p_end;
    const int64_t off = (ok ? p : p_begin) * m;
#pragma unroll
    for (int G = 0; G < TG; ++G) {
      sv[G] = sp[G][off];
      av[G] = ap[G][off];
    }
    mk = ok ? T(1) : T(0);
  };
  auto mfmas = [&](const T (&sv)[TG], const T (&av)[TG], T mk) {
    double sa[TG], sb[TG], ab[TG];
#pragma unroll
    for (int G = 0; G < TG; ++G) {
      sa[G] = (double)(sv[G] * (mk * (T)lv[G]));
      sb[G] = (double)sv[G];
      ab[G] = (double)av[G];
    }
#pragma unroll
    for (int I = 0; I < TG; ++I)
#pragma unroll
      for (int J = 0; J < TG; ++J) acca[I * TG + J] = mfma4(sa[I], ab[J], acca[I * TG + J]);
#pragma unroll
    for (int I = 0; I < TG; ++I)
#pragma unroll
      for (int J = I; J < TG; ++J) accb[tile_b<TG>(I, J)] = mfma4(sa[I], sb[J], accb[tile_b<TG>(I, J)]);
  };

  if (p_begin < p_end) {
    T sv[NS][TG], av[NS][TG], mk[NS];
#pragma unroll
    for (int q = 0; q < NS - 1; ++q) load(p_begin + (int64_t)q * 16, sv[q], av[q], mk[q]);
    for (int64_t pf = p_begin; pf < p_end; pf += FL) {
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        // refill the slot the previous stage's MFMAs consumed; the scheduling
        // barriers keep each stage's loads ahead of the other stages' MFMAs
        const int lq = (q + NS - 1) % NS;
        load(pf + (int64_t)(q + NS - 1) * 16, sv[lq], av[lq], mk[lq]);
        __builtin_amdgcn_sched_barrier(0);
        mfmas(sv[q], av[q], mk[q]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  // blocks q = 0..3 (lanes 4q apart within each row of 16) summed as
  // (q0 + q1) + (q2 + q3); lane 16i + j then holds D[i][j]
#pragma unroll
  for (int t = 0; t < NA + NB; ++t) {
    double v = t < NA ? acca[t] : accb[t - NA];
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    if ((lane & 12) == 0) red[wave][t][4 * (lane >> 4) + cl] = v;
  }
  __syncthreads();

  // the 16x16 output tiles: entry (row, col) of GB or GA from its 4x4 tile,
  // the lower S^T S tiles as mirrors of the upper ones (the same products in
  // the same order); the four waves in order.  Entries past ns are neither
  // written nor read by the reductions.
  const int nt = (ns + 15) >> 4;
  const int ntot = n_tiles_b(nt) + n_tiles_a(nt);
  for (int e = threadIdx.x; e < ntot * 256; e += kThreads) {
    bool isb;
    int row, col;
    tile_entry(e, nt, isb, row, col);
    if (row >= ns || col >= ns) continue;
    const int GI = row >> 2, GJ = col >> 2;
    int t, sub;
    if (!isb) {
      t = GI * TG + GJ;
      sub = 4 * (row & 3) + (col & 3);
    } else if (GI <= GJ) {
      t = NA + tile_b<TG>(GI, GJ);
      sub = 4 * (row & 3) + (col & 3);
    } else {
      t = NA + tile_b<TG>(GJ, GI);
      sub = 4 * (col & 3) + (row & 3);
    }
    const double sm = red[0][t][sub] + red[1][t][sub] + red[2][t][sub] + red[3][t][sub];
    g.partials[(size_t)blockIdx.x * ntot * 256 + e] = sm;
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

// Reciprocal square root: the hardware approximation refined by one Newton
// step (a few ulp).
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
  double L[KMAX * LD];   // Cholesky factor (dropped columns zero)
  double LK[KMAX * LD];  // compressed factor of the kept columns
  double M[KMAX * LD];   // the reduced matrix L^-1 A L^-T, then the tridiagonal rows
  double M2[KMAX * LD];  // work array of the triangular solves
  double V[KMAX * LD];   // eigenvectors (columns 0..m-1)
  double Cs[KMAX * 8];   // output coefficients, staged
  double bc[2][KMAX];    // broadcast rows of the tridiagonalisation (v, w)
  double H[KMAX][KMAX];  // reflector vectors v_j (row j) of the tridiagonalisation
  double hb[KMAX];       // their factors beta_j
  double lu[8][5][KMAX]; // inverse iteration: per eigenvector LU of T - lambda I (u0, u1, u2, f, swap)
  double Y[8][KMAX];     // eigenvectors of T (rows of the lane-parallel phases)
  double delta[KMAX];
  double rinv[KMAX];
  double ev[KMAX];
  int idx[KMAX];
  int order[KMAX];
  int nk;                // kept columns (shared with the other waves)
};

// ---------------------------------------------------------------------------
// Small symmetric eigenproblem: the m smallest eigenpairs of the K x K matrix
// in sh.M (K <= KB <= 24), on the four waves of the workgroup:
//  1. Householder tridiagonalisation T = Q^T M Q on wave 0 (lane i owns row i
//     in registers; v and w of each reflector are read from their lanes;
//     column sums by DPP within rows of 16 lanes);
//  2. per eigenvalue, multisection bisection of the Sturm count: one wave per
//     eigenvalue (two for m > 4), its 64 (32) lanes evaluate the count at
//     evenly spaced shifts of the bracket, which shrinks by 65 (33) per round
//     down to about 2^-60 of the Gershgorin interval; rows past K are padded
//     with a diagonal far above the spectrum, so every loop has the fixed
//     length KB and no branch;
//  3. inverse iteration for its eigenvector in the first lane of the same
//     wave: Gaussian elimination with partial pivoting of T - lambda I in
//     registers, two solves from a fixed start vector;
//  4. classical Gram-Schmidt, twice, over the m vectors on wave 0, which keeps
//     the vectors of a cluster of eigenvalues orthonormal;
//  5. back-transform z = Q y by the reflectors, one wave per vector.
// Single-wave code is bound by the latency of its dependency chains; these
// chains are short, branch-free and spread over four SIMDs.  The cyclic Jacobi
// method this replaces ran 5-6 sweeps of K - 1 rounds, each an LDS round trip
// and two chained rotations (38-45 us per call at K = 12).
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
// Sum over the first KB lanes of the wave (lanes past the rows must hold 0),
// returned to every lane; every lane must be active.
template <int KB>
__device__ __forceinline__ double sum_rows(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);  // row_half_mirror: the other quad of the half row
  v += dpp_d<0x140>(v);  // row_mirror: the other half of the row
  if constexpr (KB <= 16) return readlane_d(v, 0);
  return readlane_d(v, 0) + readlane_d(v, 16);
}

constexpr double kPadDiag = 1e4;  // diagonal of the padding rows: far above any Ritz value of L_sym (<= 2)

// Number of eigenvalues of T below sigma: sign changes of the leading
// principal minors p_i of T - sigma I (Sturm), by the three-term recurrence
// p_i = (d_i - sigma) p_(i-1) - e_(i-1)^2 p_(i-2), no divisions; a zero minor
// takes the sign opposite to its predecessor.  With Ritz values in [0, 2] and
// at most 24 rows the minors stay within about 1e+-100 (the padding rows
// multiply by ~1e4 each), so no rescaling is needed.
template <int KB>
__device__ __forceinline__ int sturm_count(const double (&d)[KB], const double (&e2)[KB], double sigma) {
  double pm2 = 1.0, pm1 = d[0] - sigma;
  pm1 = pm1 == 0.0 ? -1e-300 : pm1;
  int c = pm1 < 0.0 ? 1 : 0;
#pragma unroll
  for (int i = 1; i < KB; ++i) {
    double p = fma(d[i] - sigma, pm1, -e2[i - 1] * pm2);
    p = p == 0.0 ? (pm1 < 0.0 ? 1e-300 : -1e-300) : p;
    c += ((p < 0.0) != (pm1 < 0.0)) ? 1 : 0;
    pm2 = pm1;
    pm1 = p;
  }
  return c;
}

// Step 1 (wave 0): T = Q^T M Q; the rows of T back into sh.M, the reflector
// vectors v_j into sh.H[j] and their factors into sh.hb.
template <int KB>
__device__ void tridiagonalize(RRShared& sh, int K) {
  const int lane = threadIdx.x & 63;
  const bool row = lane < KB;
  const int li = lane < K ? lane : 0;
  double a[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) a[k] = (lane < K && k < K) ? sh.M[li * LD + k] : 0.0;
#pragma unroll
  for (int j = 0; j + 2 < KB; ++j) {
    const double xj = (lane > j && row) ? a[j] : 0.0;
    const double s2 = sum_rows<KB>(xj * xj);
    const double x0 = readlane_d(a[j], j + 1);
    const double nrm = sqrt(s2);
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    const double v = lane == j + 1 ? x0 - alpha : xj;
    const double vtv = 2.0 * (s2 - alpha * x0);
    const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
    if (row) sh.H[j][lane] = v;
    if (lane == 0) sh.hb[j] = beta;
    // v_k and w_k come from lane k by lane reads (an LDS broadcast with its
    // waits cost about 1 us per call)
    double p0 = 0.0, p1 = 0.0;  // two chains: half the dependent FMAs
#pragma unroll
    for (int k = j + 1; k < KB; ++k) {
      if ((k & 1) == 0) p0 = fma(a[k], readlane_d(v, k), p0);
      else p1 = fma(a[k], readlane_d(v, k), p1);
    }
    const double p = (p0 + p1) * beta;
    const double kc = 0.5 * beta * sum_rows<KB>(row ? v * p : 0.0);
    const double w = p - kc * v;
    // A -= v w^T + w v^T: columns left of j are untouched (their rows are
    // already reduced, so w is zero there); column j takes w_j = p_j
#pragma unroll
    for (int k = j; k < KB; ++k) {
      const double vk = k > j ? readlane_d(v, k) : 0.0;
      a[k] -= v * readlane_d(w, k) + w * vk;
    }
  }
  wave_fence();
  if (row) {
#pragma unroll
    for (int k = 0; k < KB; ++k) sh.M[lane * LD + k] = a[k];
  }
}

// Steps 2-3 (every wave): eigenvalues t = wave (and wave + 4 for m > 4) into
// sh.ev[t], their eigenvectors of T into sh.Y[t].
template <int KB>
__device__ void eig_pairs(RRShared& sh, int K, int m) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // T with the padding rows: d = kPadDiag, e = 0 past row K - 1
  double d[KB], e2[KB], eo[KB];
  double glo = 0.0, ghi = 0.0, tnorm = 0.0;
#pragma unroll
  for (int i = 0; i < KB; ++i) {
    d[i] = i < K ? sh.M[i * LD + i] : kPadDiag;
    eo[i] = i + 1 < K ? sh.M[(i + 1) * LD + i] : 0.0;  // T[i+1][i] = T[i][i+1]
    e2[i] = eo[i] * eo[i];
    const double r = fabs(eo[i]) + (i > 0 ? fabs(eo[i - 1]) : 0.0);
    if (i < K) {
      glo = (i == 0 || d[i] - r < glo) ? d[i] - r : glo;
      ghi = (i == 0 || d[i] + r > ghi) ? d[i] + r : ghi;
      tnorm = fmax(tnorm, fabs(d[i]) + r);
    }
  }
  const int half = m > 4 ? 1 : 0;            // two eigenvalues per wave
  const int G = half ? 32 : 64;              // lanes per eigenvalue
  const int rounds = half ? 12 : 10;         // 33^12, 65^10 > 2^60
  const int sub = half ? (lane >> 5) : 0;
  const int t = wave + 4 * sub;              // this lane's eigenvalue (t >= m: idle copy)
  const int tc = t < m ? t : m - 1;
  const int s = lane & (G - 1);
  const double pad = 1e-14 * fmax(fabs(glo), fabs(ghi)) + 1e-300;
  double lo = glo - pad, hi = ghi + pad;
  for (int rnd = 0; rnd < rounds; ++rnd) {
    const double step = (hi - lo) * (1.0 / (double)(G + 1));
    const double sig = fma((double)(s + 1), step, lo);
    const int c = sturm_count<KB>(d, e2, sig);
    const unsigned long long bal = __ballot(c <= tc);
    const unsigned long long grp = half ? ((bal >> (32 * sub)) & 0xFFFFFFFFull) : bal;
    const int top = grp ? 63 - __clzll(grp) : -1;  // highest shift whose count is <= t
    const double nlo = top >= 0 ? fma((double)(top + 1), step, lo) : lo;
    const double nhi = top + 1 < G ? fma((double)(top + 2), step, lo) : hi;
    lo = nlo;
    hi = nhi;
  }
  const double lam = 0.5 * (lo + hi);
  // inverse iteration in the first lane of each group
  const double ptiny = 1e-16 * (tnorm > 0.0 ? tnorm : 1.0);
  double u0[KB], u1[KB], u2[KB], f[KB], y[KB];
  unsigned int sw = 0;
  {
    double c0 = d[0] - lam, c1 = eo[0], c2 = 0.0;
#pragma unroll
    for (int i = 0; i + 1 < KB; ++i) {
      const double sb = eo[i], dn = d[i + 1] - lam, sp = eo[i + 1 < KB ? i + 1 : 0] * (i + 1 < KB - 1 ? 1.0 : 0.0);
      const bool swp = fabs(sb) > fabs(c0);
      const double piv = fabs(c0) > ptiny ? c0 : (c0 < 0.0 ? -ptiny : ptiny);
      const double fi = swp ? c0 / sb : sb / piv;
      u0[i] = swp ? sb : piv;
      u1[i] = swp ? dn : c1;
      u2[i] = swp ? sp : c2;
      f[i] = fi;
      sw |= swp ? (1u << i) : 0u;
      const double n0 = swp ? c1 - fi * dn : dn - fi * c1;
      const double n1 = swp ? c2 - fi * sp : sp - fi * c2;
      c0 = n0;
      c1 = n1;
      c2 = 0.0;
    }
    u0[KB - 1] = fabs(c0) > ptiny ? c0 : (c0 < 0.0 ? -ptiny : ptiny);
    u1[KB - 1] = 0.0;
    u2[KB - 1] = 0.0;
    f[KB - 1] = 0.0;
#pragma unroll
    for (int i = 0; i < KB; ++i) u0[i] = 1.0 / u0[i];  // the back substitution multiplies
  }
#pragma unroll
  for (int i = 0; i < KB; ++i) y[i] = 1.0 + 0.05 * (double)(((i * 7 + tc * 13 + 3) % 11) - 5);
  for (int it = 0; it < 2; ++it) {
#pragma unroll
    for (int i = 0; i + 1 < KB; ++i) {
      const bool swp = (sw >> i) & 1u;
      const double ri = y[i], rn = y[i + 1];
      y[i] = swp ? rn : ri;
      y[i + 1] = swp ? ri - f[i] * rn : rn - f[i] * ri;
    }
#pragma unroll
    for (int i = KB - 1; i >= 0; --i) {
      double v = y[i];
      if (i + 1 < KB) v -= u1[i] * y[i + 1];
      if (i + 2 < KB) v -= u2[i] * y[i + 2];
      y[i] = v * u0[i];
    }
    double nn = 0.0;
#pragma unroll
    for (int i = 0; i < KB; ++i) nn = fma(y[i], y[i], nn);
    const double sc = 1.0 / sqrt(nn);
#pragma unroll
    for (int i = 0; i < KB; ++i) y[i] *= sc;
  }
  if (s == 0 && t < m) {
    sh.ev[t] = lam;
#pragma unroll
    for (int i = 0; i < KB; ++i) sh.Y[t][i] = i < K ? y[i] : 0.0;
  }
}

// Step 4 (wave 0): classical Gram-Schmidt twice over sh.Y[0..m), lane = row.
template <int KB>
__device__ void orthonormalize(RRShared& sh, int m) {
  const int lane = threadIdx.x & 63;
  const bool row = lane < KB;
  double z[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) z[q] = (q < m && row) ? sh.Y[q][row ? lane : 0] : 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (q < m) {
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        double dq[8];
#pragma unroll
        for (int s = 0; s < q; ++s) dq[s] = sum_rows<KB>(z[s] * z[q]);
#pragma unroll
        for (int s = 0; s < q; ++s) z[q] -= dq[s] * z[s];
      }
      const double nq = sum_rows<KB>(z[q] * z[q]);
      z[q] *= 1.0 / sqrt(nq);
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (q < m && row) sh.Y[q][lane] = z[q];
}

// Step 5 (every wave): z_t = Q y_t for t = wave (and wave + 4) into column t of sh.V.
template <int KB>
__device__ void back_transform(RRShared& sh, int K, int m) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool row = lane < KB;
  const int t0 = wave, t1 = wave + 4;
  double z0 = (t0 < m && row) ? sh.Y[t0][row ? lane : 0] : 0.0;
  double z1 = (t1 < m && row) ? sh.Y[t1 < 8 ? t1 : 0][row ? lane : 0] : 0.0;
#pragma unroll
  for (int j = KB - 3; j >= 0; --j) {
    const double vj = row ? sh.H[j][lane] : 0.0;
    const double bj = sh.hb[j];
    const double d0 = sum_rows<KB>(vj * z0);
    const double d1 = sum_rows<KB>(vj * z1);
    z0 -= (bj * d0) * vj;
    z1 -= (bj * d1) * vj;
  }
  if (lane < K) {
    if (t0 < m) sh.V[lane * LD + t0] = z0;
    if (t1 < m) sh.V[lane * LD + t1] = z1;
  }
}

// Solves the Rayleigh-Ritz problem for GA, GB (ns x ns, already loaded into
// sh.A and sh.B): C (ns x m, row-major with leading dimension m) and theta
// (ascending) of the m smallest Ritz pairs, the kept flags and their count.
// Called by all four waves of the workgroup (every thread must call it): the
// sequential steps run on wave 0, the eigenpairs on all four, with workgroup
// barriers between the phases.  KB >= ns is the padded size of the
// triangular solves (the kept block is extended by an identity factor and
// zero data there, which changes nothing and keeps the loops free of
// conditionals).  Steps: symmetrise; scale to unit diag(GB) (columns with a
// negligible diagonal are dropped); Cholesky GB = L L^T that drops columns
// with a pivot below drop_tol; M = L^-1 GA L^-T on the kept columns; the m
// smallest eigenpairs Z of M (tridiagonalisation, bisection, inverse
// iteration on all four waves); C = L^-T Z.  Loads are issued
// unconditionally (clamped indices) and only stores are masked, so a lane
// never waits on a load inside a branch.
template <int KB>
__device__ void rayleigh_ritz_kb(RRShared& sh, int ns, int m, double drop_tol, double zero_tol,
                                 double* Cout, double* theta, int* kept_out, int* nkept_out) {
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < 64) {
  // unit-diagonal scaling: delta_j = diag(GB)_j^-1/2, 0 for a negligible column
  const int lj = lane < ns ? lane : 0;
  const double dl = sh.B[lj * LD + lj];
  const double mx = wave_max(lane < ns && dl > 0.0 ? dl : 0.0);
  const int gd = lane < ns && dl > zero_tol * zero_tol * mx;
  const unsigned long long goodm = __ballot(gd);  // the flags as a wave-uniform mask
  if (lane < ns) sh.delta[lane] = gd ? 1.0 / sqrt(dl) : 0.0;
  wave_fence();
  // right-looking Cholesky of the symmetrised, scaled B with column dropping,
  // lane i owning row i (lower triangle) in registers: column j's pivot and
  // its entries come from their lanes by lane reads for the rank-1 update of
  // the rows below (an LDS broadcast instead cost 1 us per LOBPCG step at 9
  // columns); a dropped column leaves L and the trailing rows unchanged.  The
  // scaled entries (b_ij + b_ji) / 2 delta_i delta_j are formed as the rows
  // are loaded (and those of A where the compression reads them); only the
  // lower triangle of the kept columns of L is ever read.
  unsigned long long keptm = 0;  // kept columns, wave-uniform
  {
    double sb[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int kc = k < ns ? k : 0;
      const double bij = sh.B[lj * LD + kc], bji = sh.B[kc * LD + lj];
      const double b = lj == kc ? bij : 0.5 * (bij + bji);
      sb[k] = (lane < ns && k < ns) ? b * (sh.delta[lj] * sh.delta[kc]) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      if (j < ns) {
        const double piv = readlane_d(sb[j], j);
        const int keep = ((goodm >> j) & 1ull) && piv > drop_tol;
        const double ip = rsq_nr2(keep ? piv : 1.0);  // 1 / L_jj
        const double lij = sb[j] * ip;
        keptm |= (unsigned long long)keep << j;
        if (keep) {
          if (lane > j && lane < ns) sh.L[lane * LD + j] = lij;
          if (lane == j) sh.L[j * LD + j] = piv * ip;
#pragma unroll
          for (int l = j + 1; l < KB; ++l) {
            const double llj = readlane_d(lij, l);  // L[l][j], from lane l
            sb[l] = (lane > j && l <= lane) ? fma(-lij, llj, sb[l]) : sb[l];
          }
        }
      }
    }
  }
  wave_fence();
  const int kp = lane < ns ? (int)((keptm >> lane) & 1ull) : 0;
  const unsigned long long km = keptm;
  const int K = __popcll(km);
  if (kp) sh.idx[__popcll(km & ((1ull << lane) - 1ull))] = lane;
  if (lane < ns) kept_out[lane] = kp;
  if (lane == 0) {
    *nkept_out = K;
    sh.nk = K;
  }
  wave_fence();
  if (K >= m) {
  // compressed factor LK and reduced A (in M2), padded to KB x KB with the
  // identity and zeros; reciprocal pivots (1 on the padding)
  for (int e = lane; e < KB * KB; e += 64) {
    const int a = e / KB, b = e - (e / KB) * KB;
    const int ia = sh.idx[a < K ? a : 0], ib = sh.idx[b < K ? b : 0];
    const double aij = sh.A[ia * LD + ib], aji = sh.A[ib * LD + ia];
    const double lv = sh.L[ia * LD + ib];
    const double av = (ia == ib ? aij : 0.5 * (aij + aji)) * (sh.delta[ia] * sh.delta[ib]);
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
  }
  wave_fence();
  tridiagonalize<KB>(sh, K);
  }  // K >= m
  }  // wave 0
  __syncthreads();
  const int K = sh.nk;
  if (K < m) return;
  // the m smallest eigenpairs of M: eigenvalues ascending in ev[0..m),
  // eigenvectors in the columns 0..m-1 of V
  eig_pairs<KB>(sh, K, m);
  __syncthreads();
  if (threadIdx.x < 64) orthonormalize<KB>(sh, m);
  __syncthreads();
  back_transform<KB>(sh, K, m);
  __syncthreads();
  if (threadIdx.x >= 64) return;
  const double* Vc = sh.V;
  if (lane < m) sh.order[lane] = lane;
  for (int e = lane; e < ns * m; e += 64) sh.Cs[e] = 0.0;
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

__device__ void rayleigh_ritz(RRShared& sh, int ns, int m, double drop_tol, double zero_tol,
                              double* Cout, double* theta, int* kept_out, int* nkept_out) {
  if (ns <= 4)
    rayleigh_ritz_kb<4>(sh, ns, m, drop_tol, zero_tol, Cout, theta, kept_out, nkept_out);
  else if (ns <= 8)
    rayleigh_ritz_kb<8>(sh, ns, m, drop_tol, zero_tol, Cout, theta, kept_out, nkept_out);
  else if (ns <= 10)
    rayleigh_ritz_kb<10>(sh, ns, m, drop_tol, zero_tol, Cout, theta, kept_out, nkept_out);
  else if (ns <= 12)
    rayleigh_ritz_kb<12>(sh, ns, m, drop_tol, zero_tol, Cout, theta, kept_out, nkept_out);
  else if (ns <= 16)
    rayleigh_ritz_kb<16>(sh, ns, m, drop_tol, zero_tol, Cout, theta, kept_out, nkept_out);
  else
    rayleigh_ritz_kb<KMAX>(sh, ns, m, drop_tol, zero_tol, Cout, theta, kept_out, nkept_out);
}

// The previous update's residual sums (|R_j|^2 for j < m, summed over its
// workgroup partials in workgroup order) into fin[0..7], for the
// Rayleigh-Ritz step that finalizes them; one workgroup.
__device__ void fin_reduce(const RRArgs& r, int m, double* fin) {
  __shared__ double fred[8 * 16];
  double t[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) t[k] = 0.0;
  for (int b0 = 0; b0 < r.fin_nparts; b0 += 4 * (int)blockDim.x) {
    double fv[4][8];
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int b = b0 + it * (int)blockDim.x + (int)threadIdx.x;
      const int bb = b < r.fin_nparts ? b : 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) fv[it][k] = r.fin_partials[(size_t)bb * r.fin_stride + (k < m ? k : 0)];
    }
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const bool ok = b0 + it * (int)blockDim.x + (int)threadIdx.x < r.fin_nparts;
#pragma unroll
      for (int k = 0; k < 8; ++k) t[k] += (ok && k < m) ? fv[it][k] : 0.0;
    }
  }
  block_sum<8>(t, fred);
  if (threadIdx.x == 0)
    for (int k = 0; k < 8; ++k) fin[k] = t[k];
}

// First stage of the Gram reduction: workgroup (tile, chunk) sums the partials
// of its chunk of Gram workgroups for the 256 entries of one tile; the
// workgroup column after the tiles reduces the previous update's residual
// partials for the Rayleigh-Ritz step, off its critical path.
__global__ void __launch_bounds__(kThreads) gram_reduce_kernel(GramArgs g, RRArgs r) {
  const int ntiles = n_tiles_b((g.ns + 15) >> 4) + n_tiles_a((g.ns + 15) >> 4);
  if (g.active != nullptr && *g.active == 0) return;
  if ((int)blockIdx.x == ntiles) {
    if (blockIdx.y == 0 && r.fin_partials != nullptr) fin_reduce(r, g.m, g.level2 + kGramFinSlot);
    return;
  }
  const int nt = (g.ns + 15) >> 4;
  const int ntot = n_tiles_b(nt) + n_tiles_a(nt);
  const int tile = blockIdx.x, chunk = blockIdx.y, nchunks = gridDim.y;
  const int per = (g.nparts + nchunks - 1) / nchunks;
  const int b0 = chunk * per, b1 = (b0 + per < g.nparts) ? b0 + per : g.nparts;
  const int e = tile * 256 + threadIdx.x;
  const size_t st = (size_t)ntot * 256;
  {
    bool isb;
    int row, col;
    tile_entry(e, nt, isb, row, col);
    if (row >= g.ns || col >= g.ns) return;  // not written by the Gram kernel, not read
  }
  // up to kGramPerChunk partials, loaded together, summed in order
  double v[kGramPerChunk];
#pragma unroll
  for (int k = 0; k < kGramPerChunk; ++k) v[k] = (b0 + k < b1) ? g.partials[(size_t)(b0 + k) * st + e] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kGramPerChunk; ++k) s += v[k];
  g.level2[(size_t)chunk * st + e] = s;
}

// Workgroup 0: sums the chunks and assembles GA and GB (ns x ns); its first
// wave then runs the Rayleigh-Ritz step.  Workgroups 1.. (cg.nblk of them)
// run a CG update phase of the joint driver on the CUs the step leaves idle.
//
// direct != 0 (at most kGramDirect Gram workgroups): no
// reduction launch ran; the partials take the place of the chunk sums (the
// reduction would have copied them one to one, so the sums are bitwise the
// same) and this workgroup sums the previous update's residual partials.
__global__ void __launch_bounds__(kThreads) gram_rr_kernel(GramArgs g, RRArgs r, CgStepArgs cg, int direct) {
  if (blockIdx.x > 0) {
    cg_aupdate_step(cg, (int)blockIdx.x - 1);
    return;
  }
  __shared__ RRShared sh;
  __shared__ int nkept;
  __shared__ int keptf[KMAX];
  __shared__ int live;
  __shared__ int lockm;
  const int nt = (g.ns + 15) >> 4;
  const int ntot = n_tiles_b(nt) + n_tiles_a(nt);
  // Everything this kernel reads from global memory was written by earlier
  // kernels (other XCDs), so each load is a long trip: the chunk values of
  // every thread's first two entries (all entries for ns <= 16), the solver
  // state and the residual sums are all issued before any of them is used
  // (also before the state says whether the step runs at all).
  const double* chunks = direct ? g.partials : g.level2;
  const int nchunks = direct ? g.nparts : kGramChunks;
  const int e1 = (int)threadIdx.x + (int)blockDim.x;  // ntot >= 2: every thread has two entries
  double v0[kGramDirect], v1[kGramDirect];
#pragma unroll
  for (int c = 0; c < kGramDirect; ++c) {
    v0[c] = c < nchunks ? chunks[(size_t)c * (ntot * 256) + threadIdx.x] : 0.0;
    v1[c] = c < nchunks ? chunks[(size_t)c * (ntot * 256) + e1] : 0.0;
  }
  LobpcgState* st = r.st;
  const int active = st != nullptr ? st->active : 1;
  const double tol = st != nullptr ? st->tol : 0.0;
  const int iters0 = st != nullptr ? st->iters : 0;
  const int dropped0 = st != nullptr ? st->dropped : 0;
  if (!active) return;
  if (r.fin_partials != nullptr) {
    // the previous update's residual norms, iteration count and convergence
    // test (what lob_final_kernel does after an update without the
    // constraint, in the same summation order); the sums come reduced from
    // gram_reduce_kernel's extra workgroup, or from this workgroup (direct)
    __shared__ double fin_here[8];
    if (direct) fin_reduce(r, g.m, fin_here);
    const double* fin = direct ? fin_here : g.level2 + kGramFinSlot;
    double t[8];
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < 8; ++k) t[k] = fin[k];
    if (threadIdx.x == 0) {
      double mx = 0.0;
      for (int j = 0; j < g.m; ++j) {
        const double rj = sqrt(t[j]);
        st->res[j] = rj;
        st->yx[j] = 0.0;
        mx = rj > mx ? rj : mx;
      }
      st->iters = iters0 + 1;
      live = !(tol > 0.0 && mx <= tol);
      if (!live) st->active = 0;
    }
    __syncthreads();
    if (!live) return;
  }
  // entry e of the Gram tiles (chunk sums in v) into sh.A / sh.B
  auto place = [&](int e, const double (&v)[kGramDirect]) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kGramDirect; ++c) s += v[c];
    bool isb;
    int row, colj;
    tile_entry(e, nt, isb, row, colj);
    if (row < g.ns && colj < g.ns) {
      if (isb) {
        sh.B[row * LD + colj] = s;
        if ((row >> 4) != (colj >> 4)) sh.B[colj * LD + row] = s;  // the lower off-diagonal tile is the mirror
      } else {
        sh.A[row * LD + colj] = s;
      }
    }
  };
  place(threadIdx.x, v0);
  place(e1, v1);
  for (int e = e1 + blockDim.x; e < ntot * 256; e += blockDim.x) {
    double v[kGramDirect];
#pragma unroll
    for (int c = 0; c < kGramDirect; ++c) v[c] = c < nchunks ? chunks[(size_t)c * (ntot * 256) + e] : 0.0;
    place(e, v);
  }
  // soft locking (tol > 0): a column whose residual is already at the
  // tolerance adds no search direction, i.e. its W column counts as zero:
  // the W rows and columns of both Gram matrices are cleared, and the
  // Rayleigh-Ritz step drops the column
  // (tol, like the rest of the condition, is the same for every thread, so
  // a run without a tolerance skips the mask and its barrier)
  if (!r.init && st != nullptr && tol > 0.0 && g.ns > g.m) {
    if (threadIdx.x == 0) {
      int mask = 0;
      for (int j = 0; j < g.m; ++j)
        if (st->res[j] <= tol) mask |= 1 << j;
      lockm = mask;
    }
    __syncthreads();
    if (lockm != 0) {
      const int lk = lockm;
      for (int e = threadIdx.x; e < g.ns * g.ns; e += blockDim.x) {
        const int i = e / g.ns, j = e - (e / g.ns) * g.ns;
        const bool li = i >= g.m && i < 2 * g.m && ((lk >> (i - g.m)) & 1);
        const bool lj = j >= g.m && j < 2 * g.m && ((lk >> (j - g.m)) & 1);
        if (li || lj) {
          sh.A[i * LD + j] = 0.0;
          sh.B[i * LD + j] = 0.0;
        }
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
  rayleigh_ritz(sh, g.ns, g.m, r.drop_tol, r.zero_tol, r.C, r.theta, keptf, &nkept);
  if (threadIdx.x >= 64) return;
  wave_fence();
  if (threadIdx.x == 0 && st != nullptr) {
    st->nkept = nkept;
    for (int j = 0; j < g.ns; ++j) st->kept[j] = keptf[j];
    st->dropped = dropped0 + g.ns - nkept;
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

// store_row as streaming (non-temporal) stores: for the blocks that are read
// again only after the next stencil pass (X, AX, P, AP), so that they displace
// fewer of its weight planes from the caches (1024^2, 11x11, m = 4: the joint
// apply inside the steps 71.5 us against 72.3, the update 37.0 against 37.3;
// the joint CG50 + LOBPCG50 call 9.593-9.615 ms against 9.629-9.635 in
// alternating runs on one GPU; streaming loads of the update's inputs as well
// sped the apply up further but slowed the Gram and the update more).
template <typename T, int M>
__device__ __forceinline__ void store_row_nt(T* __restrict__ dst, const T (&v)[M]) {
  if constexpr (sizeof(T) * M % 16 == 0) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int W = (int)(sizeof(T) * M / 16);
    f4* d4 = reinterpret_cast<f4*>(dst);
#pragma unroll
    for (int w = 0; w < W; ++w) __builtin_nontemporal_store(reinterpret_cast<const f4*>(v)[w], d4 + w);
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) __builtin_nontemporal_store(v[j], dst + j);
  }
}

// NB = number of blocks in the trial basis: 1 (start block), 2 ([X, W]),
// 3 ([X, W, P]).  Coefficients C (NB*M x M, FP64) are read from LDS; every
// output column is accumulated in FP64 and rounded once.  The last cg.nblk
// workgroups run a CG direction phase of the joint driver (same element
// type): the update streams the LOBPCG block, and the direction's three
// vector passes share the launch instead of adding one to the step.
template <typename T, int M, int NB>
__global__ void __launch_bounds__(kThreads) lob_update_kernel(LobArgs a, int first, CgStepArgs cg) {
  __shared__ double Cs[3 * M * M];
  __shared__ double th[M];
  __shared__ double red[16 * 2 * M];
  const int nupd = (int)gridDim.x - cg.nblk;
  if ((int)blockIdx.x >= nupd) {
    cg_pbeta_body<T>((const T*)cg.r, (T*)cg.p, cg.n, cg.upd, cg.nblk, cg.st, cg.k, (int)blockIdx.x - nupd, cg.nblk);
    return;
  }
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
  const int64_t stride = (int64_t)nupd * blockDim.x;
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
    store_row_nt<T, M>(X + i * M, xo);
    store_row_nt<T, M>(AX + i * M, axo);
    if (!first) {
      store_row_nt<T, M>(P + i * M, po);
      store_row_nt<T, M>(AP + i * M, apo);
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
void launch_m_kernels(int which, const LobArgs& a, int nb, int ns, int first, StartDegrees deg,
                      const CgStepArgs& cg, hipStream_t s) {
  const CgStepArgs none{};
  const int nbc = nb + cg.nblk;  // the update launches, with the CG phase's workgroups
  switch (which) {
    case 0:
      lob_start_kernel<T, M><<<nb, kThreads, 0, s>>>(a, deg);
      if (a.constraint) lob_final_kernel<M><<<1, kThreads, 0, s>>>(a.vpart, nb, a.st, 1, M, 0, 1);
      break;
    case 1:
      if (ns == M)
        lob_update_kernel<T, M, 1><<<nbc, kThreads, 0, s>>>(a, first, cg);
      else if (ns == 2 * M)
        lob_update_kernel<T, M, 2><<<nbc, kThreads, 0, s>>>(a, first, cg);
      else
        lob_update_kernel<T, M, 3><<<nbc, kThreads, 0, s>>>(a, first, cg);
      lob_final_kernel<2 * M><<<1, kThreads, 0, s>>>(a.vpart, nb, a.st, 2, M, first, a.constraint);
      break;
    case 4:
      if (ns == M)
        lob_update_kernel<T, M, 1><<<nbc, kThreads, 0, s>>>(a, first, cg);
      else if (ns == 2 * M)
        lob_update_kernel<T, M, 2><<<nbc, kThreads, 0, s>>>(a, first, cg);
      else
        lob_update_kernel<T, M, 3><<<nbc, kThreads, 0, s>>>(a, first, cg);
      break;
    case 5:
      lob_final_kernel<2 * M><<<1, kThreads, 0, s>>>(a.vpart, nb, a.st, 2, M, first, a.constraint);
      break;
    case 6:  // W = AX - X Theta of a recomputed AX (a.C = I: X, AX copied, P, AP kept), finalized as an update
      lob_update_kernel<T, M, 1><<<nb, kThreads, 0, s>>>(a, 1, none);
      lob_final_kernel<2 * M><<<1, kThreads, 0, s>>>(a.vpart, nb, a.st, 2, M, 0, a.constraint);
      break;
    case 7:  // the same, its finalize folded into the next Rayleigh-Ritz step
      lob_update_kernel<T, M, 1><<<nb, kThreads, 0, s>>>(a, 1, none);
      break;
    case 2:
      lob_out_dots_kernel<T, M><<<nb, kThreads, 0, s>>>(a);
      lob_final_kernel<M + 1><<<1, kThreads, 0, s>>>(a.vpart, nb, a.st, 3, M, 0, a.constraint);
      break;
    default: lob_output_kernel<T, M><<<nb, kThreads, 0, s>>>(a); break;
  }
}

template <typename T>
void launch_m_dispatch(int which, const LobArgs& a, int nb, int ns, int first, StartDegrees deg, const CgStepArgs& cg,
                       hipStream_t s) {
  switch (a.m) {
    case 1: launch_m_kernels<T, 1>(which, a, nb, ns, first, deg, cg, s); break;
    case 2: launch_m_kernels<T, 2>(which, a, nb, ns, first, deg, cg, s); break;
    case 3: launch_m_kernels<T, 3>(which, a, nb, ns, first, deg, cg, s); break;
    case 4: launch_m_kernels<T, 4>(which, a, nb, ns, first, deg, cg, s); break;
    case 5: launch_m_kernels<T, 5>(which, a, nb, ns, first, deg, cg, s); break;
    case 6: launch_m_kernels<T, 6>(which, a, nb, ns, first, deg, cg, s); break;
    case 7: launch_m_kernels<T, 7>(which, a, nb, ns, first, deg, cg, s); break;
    default: launch_m_kernels<T, 8>(which, a, nb, ns, first, deg, cg, s); break;
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
                              hipStream_t s, const CgStepArgs* cg_direction) {
  const CgStepArgs none{};
  const CgStepArgs& cp = (cg_direction != nullptr && (which == 1 || which == 4)) ? *cg_direction : none;
  if (cp.nblk > 0 && cp.prec != a.prec) return GSF_EINVAL;
  if (a.prec == GSF_F32)
    launch_m_dispatch<float>(which, a, nb, ns, first, deg, cp, s);
  else
    launch_m_dispatch<double>(which, a, nb, ns, first, deg, cp, s);
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

template <typename T>
void launch_gram_kernel(const GramArgs& g, hipStream_t s) {
  switch ((g.ns + 3) >> 2) {
    case 1: gram_kernel<T, 1><<<g.nparts, kThreads, 0, s>>>(g); break;
    case 2: gram_kernel<T, 2><<<g.nparts, kThreads, 0, s>>>(g); break;
    case 3: gram_kernel<T, 3><<<g.nparts, kThreads, 0, s>>>(g); break;
    case 4: gram_kernel<T, 4><<<g.nparts, kThreads, 0, s>>>(g); break;
    case 5: gram_kernel<T, 5><<<g.nparts, kThreads, 0, s>>>(g); break;
    default: gram_kernel<T, 6><<<g.nparts, kThreads, 0, s>>>(g); break;
  }
}

gsf_status lob_launch_gram(const GramArgs& g, const RRArgs& r, int prec, hipStream_t s,
                           const CgStepArgs* cg_update) {
  if (g.ns < 1 || g.ns > KMAX) return GSF_EINVAL;
  if (prec == GSF_F32)
    launch_gram_kernel<float>(g, s);
  else
    launch_gram_kernel<double>(g, s);
  const CgStepArgs none{};
  const CgStepArgs& ca = cg_update != nullptr ? *cg_update : none;
  // with at most kGramDirect Gram workgroups the reduction launch would only
  // copy the partials: the Rayleigh-Ritz workgroup reads them itself
  const int direct = g.nparts <= kGramDirect ? 1 : 0;
  if (!direct) {
    dim3 grid(gram_tiles_total(g.ns) + 1, kGramChunks);
    gram_reduce_kernel<<<grid, kThreads, 0, s>>>(g, r);
  }
  // with a CG phase, unused LDS brings each workgroup above half of a CU's
  // 160 KB, which keeps a second workgroup off the Rayleigh-Ritz workgroup's
  // CU: 41.5 us per call at 1024^2, m = 4 against 42.3 us when a CG workgroup
  // shares it (the CG phase itself ends long before the step)
  constexpr size_t kHalfCu = 80 * 1024 + 1024;
  constexpr size_t kReserve = sizeof(RRShared) < kHalfCu ? kHalfCu - sizeof(RRShared) : 0;
  gram_rr_kernel<<<1 + ca.nblk, rr_threads(g.ns), ca.nblk > 0 ? kReserve : 0, s>>>(g, r, ca, direct);
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
  rayleigh_ritz(sh, ns, m, r.drop_tol, r.zero_tol, r.C, r.theta, keptf, &nkept);
  if (threadIdx.x >= 64) return;
  wave_fence();
  if ((int)threadIdx.x < ns) r.kept_out[threadIdx.x] = keptf[threadIdx.x];
  if (threadIdx.x == 0) *r.nkept_out = nkept;
}

gsf_status lob_launch_rr_only(const double* G, int ns, int m, const RRArgs& r, hipStream_t s) {
  rr_only_kernel<<<1, rr_threads(ns), 0, s>>>(G, ns, m, r);
  return launch_status();
}

}  // namespace gsf
