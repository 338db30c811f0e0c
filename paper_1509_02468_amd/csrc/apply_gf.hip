// Normalized guided-filter operator apply (Section 3, Algorithm 1, eqs. (5)-(6)):
//   N x = D^1/2 GF(D^-1/2 x),  D = diag(N_i / |w|),
// where GF is Algorithm 1 with the fixed guidance g (linear filter), mean
// filters over border-truncated windows (N_k points) and the precomputed window
// statistics mu_k, inv_k = 1/(sigma_k^2 + eps):
//   u      = D^-1/2 x            (RW form: u = x)
//   a_k    = (box(g u)_k / N_k - mu_k box(u)_k / N_k) inv_k
//   b_k    = box(u)_k / N_k - a_k mu_k
//   GF(u)_i = (g_i box(a)_i + box(b)_i) / N_i
// The separable window sums run as four passes (rows, columns, rows, columns)
// through two scratch planes of the operator; a 1D signal is a single row, so
// its column passes are the identity.
#include "gsf_internal.h"

namespace gsf {
namespace {

struct GfArgs {
  const void* g;
  const void* mu;
  const void* inv;
  const void* x;
  void* y;
  void* s0;
  void* s1;
  int64_t ldx, ldy;
  int64_t n, rows, cols;
  int r;
  int form;
  double omega;  // |w| = (2r+1)^ndim
};

__device__ __forceinline__ int64_t win_count(int64_t v, int64_t len, int r) {
  const int64_t lo = v - r < 0 ? 0 : v - r;
  const int64_t hi = v + r >= len ? len - 1 : v + r;
  return hi - lo + 1;
}

// pass 1: s0 = rowbox(u), s1 = rowbox(g u)
template <typename T>
__global__ void __launch_bounds__(kThreads) gf_pass1(GfArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const T* __restrict__ x = (const T*)a.x;
  const T* __restrict__ g = (const T*)a.g;
  const int64_t yy = i / a.cols, xx = i - yy * a.cols;
  const int64_t lo = xx - a.r < 0 ? 0 : xx - a.r;
  const int64_t hi = xx + a.r >= a.cols ? a.cols - 1 : xx + a.r;
  T su = T(0), sgu = T(0);
  for (int64_t c = lo; c <= hi; ++c) {
    const int64_t j = yy * a.cols + c;
    T u = x[j * a.ldx];
    if (a.form != GSF_FORM_RW) {
      const int64_t nj = win_count(yy, a.rows, a.r) * win_count(c, a.cols, a.r);
      u *= (T)sqrt(a.omega / (double)nj);
    }
    su += u;
    sgu += g[j] * u;
  }
  ((T*)a.s0)[i] = su;
  ((T*)a.s1)[i] = sgu;
}

// pass 2: column sums -> a_k, b_k (in place in s0, s1)
template <typename T>
__global__ void __launch_bounds__(kThreads) gf_pass2(GfArgs a, T* __restrict__ outa, T* __restrict__ outb) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n) return;
  const T* __restrict__ s0 = (const T*)a.s0;
  const T* __restrict__ s1 = (const T*)a.s1;
  const int64_t yy = k / a.cols, xx = k - yy * a.cols;
  const int64_t lo = yy - a.r < 0 ? 0 : yy - a.r;
  const int64_t hi = yy + a.r >= a.rows ? a.rows - 1 : yy + a.r;
  T su = T(0), sgu = T(0);
  for (int64_t rr = lo; rr <= hi; ++rr) {
    su += s0[rr * a.cols + xx];
    sgu += s1[rr * a.cols + xx];
  }
  const T nk = (T)((hi - lo + 1) * win_count(xx, a.cols, a.r));
  const T mean_u = su / nk, mean_gu = sgu / nk;
  const T m = ((const T*)a.mu)[k];
  const T av = (mean_gu - m * mean_u) * ((const T*)a.inv)[k];
  outa[k] = av;
  outb[k] = mean_u - av * m;
}

// pass 3: row sums of a and b
template <typename T>
__global__ void __launch_bounds__(kThreads) gf_pass3(GfArgs a, const T* __restrict__ ina, const T* __restrict__ inb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t yy = i / a.cols, xx = i - yy * a.cols;
  const int64_t lo = xx - a.r < 0 ? 0 : xx - a.r;
  const int64_t hi = xx + a.r >= a.cols ? a.cols - 1 : xx + a.r;
  T sa = T(0), sb = T(0);
  for (int64_t c = lo; c <= hi; ++c) {
    sa += ina[yy * a.cols + c];
    sb += inb[yy * a.cols + c];
  }
  ((T*)a.s0)[i] = sa;
  ((T*)a.s1)[i] = sb;
}

// pass 4: column sums -> output
template <typename T>
__global__ void __launch_bounds__(kThreads) gf_pass4(GfArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const T* __restrict__ s0 = (const T*)a.s0;
  const T* __restrict__ s1 = (const T*)a.s1;
  const int64_t yy = i / a.cols, xx = i - yy * a.cols;
  const int64_t lo = yy - a.r < 0 ? 0 : yy - a.r;
  const int64_t hi = yy + a.r >= a.rows ? a.rows - 1 : yy + a.r;
  T sa = T(0), sb = T(0);
  for (int64_t rr = lo; rr <= hi; ++rr) {
    sa += s0[rr * a.cols + xx];
    sb += s1[rr * a.cols + xx];
  }
  const double ni = (double)((hi - lo + 1) * win_count(xx, a.cols, a.r));
  const T gfu = (((const T*)a.g)[i] * sa + sb);
  T out;
  if (a.form == GSF_FORM_RW) {
    out = gfu / (T)ni;
  } else {
    const T nx = gfu / (T)sqrt(ni * a.omega);  // D^1/2 GF(u) = (g sum a + sum b) / sqrt(N_i |w|)
    out = (a.form == GSF_FORM_LSYM) ? ((const T*)a.x)[i * a.ldx] - nx : nx;
  }
  ((T*)a.y)[i * a.ldy] = out;
}

}  // namespace

// Scratch: 4 planes of n elements (two for the window sums, two for a and b).
gsf_status launch_gf_apply(const Operator& op, void* scratch, int form, int m, const void* x, int64_t ldx,
                           void* y, int64_t ldy, hipStream_t s) {
  GfArgs a{};
  a.g = op.g;
  a.mu = op.mu;
  a.inv = op.inv;
  a.ldx = ldx;
  a.ldy = ldy;
  a.n = op.n;
  a.rows = op.rows;
  a.cols = op.cols;
  a.r = op.desc.radius;
  a.form = form;
  a.omega = op.desc.ndim == 1 ? (double)(2 * a.r + 1) : (double)((2 * a.r + 1) * (2 * a.r + 1));
  const unsigned grid = (unsigned)((op.n + kThreads - 1) / kThreads);
  char* base = (char*)scratch;
  const size_t plane = align_up((size_t)op.n * op.elem, 256);
  a.s0 = base;
  a.s1 = base + plane;
  void* pa = base + 2 * plane;
  void* pb = base + 3 * plane;
  for (int c = 0; c < m; ++c) {
    a.x = (const char*)x + (size_t)c * op.elem;
    a.y = (char*)y + (size_t)c * op.elem;
    if (op.desc.prec == GSF_F32) {
      gf_pass1<float><<<grid, kThreads, 0, s>>>(a);
      gf_pass2<float><<<grid, kThreads, 0, s>>>(a, (float*)pa, (float*)pb);
      gf_pass3<float><<<grid, kThreads, 0, s>>>(a, (const float*)pa, (const float*)pb);
      gf_pass4<float><<<grid, kThreads, 0, s>>>(a);
    } else {
      gf_pass1<double><<<grid, kThreads, 0, s>>>(a);
      gf_pass2<double><<<grid, kThreads, 0, s>>>(a, (double*)pa, (double*)pb);
      gf_pass3<double><<<grid, kThreads, 0, s>>>(a, (const double*)pa, (const double*)pb);
      gf_pass4<double><<<grid, kThreads, 0, s>>>(a);
    }
  }
  return hipGetLastError() == hipSuccess ? GSF_OK : GSF_EDEVICE;
}

}  // namespace gsf
