// Learned preconditioner T for block LOBPCG (the preconditioner slot of
// Algorithm 3): a 3-layer 3x3 convolutional network
//   x = (bf16(r / s), bf16(g)),  a1 = bf16(relu(conv(x; W1))),  2 -> 16
//   a2 = bf16(relu(conv(a1; W2))),  16 -> 16,   y = conv(a2; W3),  16 -> 1
// with zero padding, no biases, s = RMS(r), T(r) = s * y.  BF16 weights and
// activations, FP32 accumulation.  Flat weight layout: W1[o][c][ky][kx]
// (offset 0), W2[o][c][ky][kx] (offset 288), W3[c][ky][kx] (offset 2592).
//
// Training (forward with stored activations, backward, weight gradients,
// Adam) runs on per-layer VALU kernels; inference inside LOBPCG runs on one
// fused kernel per 28x28 output tile that keeps the whole receptive field in
// LDS and does the three convolutions as implicit GEMMs on bf16 MFMA
// (v_mfma_f32_16x16x16bf16_1k: 16 output channels x 16 pixels per
// instruction; layer 3 as 9 per-tap 1x1 products summed over the taps).
#include <cmath>

#include "gsf_internal.h"
#include "solver_state.h"

namespace gsf {

int vec_blocks(int64_t n);

constexpr int kOffW1 = 0, kOffW2 = 288, kOffW3 = 2592, kNetWeights = 2736;

namespace {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest, ties to even (NaN stays NaN).
__device__ __forceinline__ uint32_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ float rbf(float f) { return bf2f(f2bf(f)); }

// FP64 -> BF16 with a single rounding: the FP32 conversion can create an
// exact BF16 tie that the FP64 value does not have; then the FP32 value is
// moved one unit towards the FP64 value, so the tie breaks the right way.
__device__ __forceinline__ uint32_t d2bf(double d) {
  const float f = (float)d;
  uint32_t u = __float_as_uint(f);
  if ((u & 0xffffu) == 0x8000u && (double)f != d && __builtin_isfinite(f))
    u = fabs(d) > fabs((double)f) ? u + 1u : u - 1u;
  return f2bf(__uint_as_float(u));
}

// ReLU that keeps NaN (so a NaN inside the network reaches the output and
// triggers the T = I fallback).
__device__ __forceinline__ float relu(float v) { return (v > 0.0f || v != v) ? v : 0.0f; }

__device__ __forceinline__ bool inside(int64_t y, int64_t x, int64_t rows, int64_t cols) {
  return y >= 0 && y < rows && x >= 0 && x < cols;
}

// ---------------------------------------------------------------------------
// training kernels (one thread per pixel of the batch)
// ---------------------------------------------------------------------------
struct NetTrainArgs {
  const float* wf;        // BF16-rounded weights as FP32
  const int32_t* idx;     // sample of each batch position
  int batch;
  int64_t rows, cols, hw;
  const float* inputs;    // [sample][hw][2]
  const float* targets;   // [sample][hw] (nullptr: forward only)
  uint16_t* a1;           // [b][hw][16]
  uint16_t* a2;           // [b][hw][16]
  float* y;               // [b][hw]
  float* dy;              // [b][hw]
  float* dz2;             // [b][hw][16]
  float* dz1;             // [b][hw][16]
  double* loss_part;      // one per workgroup
  float dscale;           // 2 / (batch * hw)
};

__global__ void __launch_bounds__(kThreads) net_round_weights_kernel(const uint16_t* __restrict__ w,
                                                                     float* __restrict__ wf) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kNetWeights; i += gridDim.x * blockDim.x)
    wf[i] = bf2f(w[i]);
}

__device__ __forceinline__ void load16_bf(const uint16_t* p, float (&v)[16]) {
  const uint4 a = *(const uint4*)p, b = *(const uint4*)(p + 8);
  const uint32_t u[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[2 * k] = bf2f(u[k] & 0xffffu);
    v[2 * k + 1] = bf2f(u[k] >> 16);
  }
}

__device__ __forceinline__ void store16_relu_bf(uint16_t* p, const float (&v)[16]) {
  uint32_t u[8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    u[k] = f2bf(relu(v[2 * k])) | (f2bf(relu(v[2 * k + 1])) << 16);
  *(uint4*)p = make_uint4(u[0], u[1], u[2], u[3]);
  *(uint4*)(p + 8) = make_uint4(u[4], u[5], u[6], u[7]);
}

__global__ void __launch_bounds__(kThreads) net_fwd1_kernel(NetTrainArgs a) {
  const int64_t total = (int64_t)a.batch * a.hw;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t b = t / a.hw, p = t - b * a.hw;
    const int64_t py = p / a.cols, px = p - py * a.cols;
    const float* in = a.inputs + (size_t)a.idx[b] * a.hw * 2;
    float acc[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) acc[o] = 0.0f;
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
      const int64_t gy = py + tap / 3 - 1, gx = px + tap % 3 - 1;
      float x0 = 0.0f, x1 = 0.0f;
      if (inside(gy, gx, a.rows, a.cols)) {
        const float2 v = *(const float2*)(in + (gy * a.cols + gx) * 2);
        x0 = rbf(v.x);
        x1 = rbf(v.y);
      }
#pragma unroll
      for (int o = 0; o < 16; ++o) {
        acc[o] = fmaf(a.wf[kOffW1 + o * 18 + tap], x0, acc[o]);
        acc[o] = fmaf(a.wf[kOffW1 + o * 18 + 9 + tap], x1, acc[o]);
      }
    }
    store16_relu_bf(a.a1 + t * 16, acc);
  }
}

__global__ void __launch_bounds__(kThreads) net_fwd2_kernel(NetTrainArgs a) {
  const int64_t total = (int64_t)a.batch * a.hw;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t b = t / a.hw, p = t - b * a.hw;
    const int64_t py = p / a.cols, px = p - py * a.cols;
    float acc[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) acc[o] = 0.0f;
    for (int tap = 0; tap < 9; ++tap) {
      const int64_t gy = py + tap / 3 - 1, gx = px + tap % 3 - 1;
      if (!inside(gy, gx, a.rows, a.cols)) continue;
      float v[16];
      load16_bf(a.a1 + (b * a.hw + gy * a.cols + gx) * 16, v);
#pragma unroll
      for (int c = 0; c < 16; ++c)
#pragma unroll
        for (int o = 0; o < 16; ++o) acc[o] = fmaf(a.wf[kOffW2 + o * 144 + c * 9 + tap], v[c], acc[o]);
    }
    store16_relu_bf(a.a2 + t * 16, acc);
  }
}

// y = conv(a2; W3); with targets also dy = dscale (y - t) and the loss partials.
__global__ void __launch_bounds__(kThreads) net_fwd3_kernel(NetTrainArgs a) {
  __shared__ double red[16];
  const int64_t total = (int64_t)a.batch * a.hw;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double v[1] = {0.0};
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t b = t / a.hw, p = t - b * a.hw;
    const int64_t py = p / a.cols, px = p - py * a.cols;
    float acc = 0.0f;
    for (int tap = 0; tap < 9; ++tap) {
      const int64_t gy = py + tap / 3 - 1, gx = px + tap % 3 - 1;
      if (!inside(gy, gx, a.rows, a.cols)) continue;
      float x[16];
      load16_bf(a.a2 + (b * a.hw + gy * a.cols + gx) * 16, x);
#pragma unroll
      for (int c = 0; c < 16; ++c) acc = fmaf(a.wf[kOffW3 + c * 9 + tap], x[c], acc);
    }
    a.y[t] = acc;
    if (a.targets != nullptr) {
      const float e = acc - a.targets[(size_t)a.idx[b] * a.hw + p];
      a.dy[t] = a.dscale * e;
      v[0] += (double)e * (double)e;
    }
  }
  if (a.targets == nullptr) return;
  block_sum<1>(v, red);
  if (threadIdx.x == 0) a.loss_part[blockIdx.x] = v[0];
}

// dz2[q][c] = [a2[q][c] > 0] sum_tap W3[c][tap] dy[q - off(tap)]
__global__ void __launch_bounds__(kThreads) net_bwd3_kernel(NetTrainArgs a) {
  const int64_t total = (int64_t)a.batch * a.hw;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t b = t / a.hw, p = t - b * a.hw;
    const int64_t py = p / a.cols, px = p - py * a.cols;
    float acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0f;
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
      const int64_t gy = py - (tap / 3 - 1), gx = px - (tap % 3 - 1);
      if (!inside(gy, gx, a.rows, a.cols)) continue;
      const float d = a.dy[b * a.hw + gy * a.cols + gx];
#pragma unroll
      for (int c = 0; c < 16; ++c) acc[c] = fmaf(a.wf[kOffW3 + c * 9 + tap], d, acc[c]);
    }
    float act[16];
    load16_bf(a.a2 + t * 16, act);
    float4* out = (float4*)(a.dz2 + t * 16);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      out[k] = make_float4(act[4 * k] > 0.0f ? acc[4 * k] : 0.0f, act[4 * k + 1] > 0.0f ? acc[4 * k + 1] : 0.0f,
                           act[4 * k + 2] > 0.0f ? acc[4 * k + 2] : 0.0f,
                           act[4 * k + 3] > 0.0f ? acc[4 * k + 3] : 0.0f);
  }
}

// dz1[q][c] = [a1[q][c] > 0] sum_tap sum_o W2[o][c][tap] dz2[q - off(tap)][o]
__global__ void __launch_bounds__(kThreads) net_bwd2_kernel(NetTrainArgs a) {
  const int64_t total = (int64_t)a.batch * a.hw;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    const int64_t b = t / a.hw, p = t - b * a.hw;
    const int64_t py = p / a.cols, px = p - py * a.cols;
    float acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0f;
    for (int tap = 0; tap < 9; ++tap) {
      const int64_t gy = py - (tap / 3 - 1), gx = px - (tap % 3 - 1);
      if (!inside(gy, gx, a.rows, a.cols)) continue;
      const float4* d4 = (const float4*)(a.dz2 + (b * a.hw + gy * a.cols + gx) * 16);
      float d[16];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 q = d4[k];
        d[4 * k] = q.x;
        d[4 * k + 1] = q.y;
        d[4 * k + 2] = q.z;
        d[4 * k + 3] = q.w;
      }
#pragma unroll
      for (int o = 0; o < 16; ++o)
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = fmaf(a.wf[kOffW2 + o * 144 + c * 9 + tap], d[o], acc[c]);
    }
    float act[16];
    load16_bf(a.a1 + t * 16, act);
    float4* out = (float4*)(a.dz1 + t * 16);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      out[k] = make_float4(act[4 * k] > 0.0f ? acc[4 * k] : 0.0f, act[4 * k + 1] > 0.0f ? acc[4 * k + 1] : 0.0f,
                           act[4 * k + 2] > 0.0f ? acc[4 * k + 2] : 0.0f,
                           act[4 * k + 3] > 0.0f ? acc[4 * k + 3] : 0.0f);
  }
}

// Weight gradient of one layer, dW[o][c][tap] = sum_p dz[p][o] act[p + off(tap)][c],
// over 16x16 pixel tiles (grid-stride over batch x tiles).  Each thread owns
// one (o, c) pair and a fixed subset of the tile's pixels; per tile the sums
// are FP32, across tiles FP64; the per-workgroup partials are reduced later
// in workgroup order.
template <int LAYER>
__global__ void __launch_bounds__(kThreads) net_wgrad_kernel(NetTrainArgs a, int tiles_x, int tiles_per_sample,
                                                             double* __restrict__ partials) {
  constexpr int CIN = LAYER == 1 ? 2 : 16, COUT = LAYER == 3 ? 1 : 16;
  constexpr int P = CIN * COUT, S = kThreads / P;
  __shared__ float acts[18 * 18 * CIN];
  __shared__ float dzs[256 * COUT];
  __shared__ double red[kThreads * 9];
  const int tid = threadIdx.x, pair = tid % P, sub = tid / P;
  const int o = pair / CIN, c = pair - (pair / CIN) * CIN;
  double accd[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) accd[k] = 0.0;
  const int64_t ntiles = (int64_t)a.batch * tiles_per_sample;
  for (int64_t tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
    const int64_t b = tt / tiles_per_sample;
    const int tl = (int)(tt - b * tiles_per_sample);
    const int64_t ty = (tl / tiles_x) * 16, tx = (tl % tiles_x) * 16;
    __syncthreads();
    for (int e = tid; e < 18 * 18; e += kThreads) {
      const int64_t gy = ty - 1 + e / 18, gx = tx - 1 + e % 18;
      const bool in = inside(gy, gx, a.rows, a.cols);
      const int64_t q = gy * a.cols + gx;
      if constexpr (LAYER == 1) {
        float2 v = make_float2(0.0f, 0.0f);
        if (in) v = *(const float2*)(a.inputs + ((size_t)a.idx[b] * a.hw + q) * 2);
        acts[e * 2] = rbf(v.x);
        acts[e * 2 + 1] = rbf(v.y);
      } else {
        float v[16];
        if (in) {
          load16_bf((LAYER == 2 ? a.a1 : a.a2) + (b * a.hw + q) * 16, v);
        } else {
#pragma unroll
          for (int k = 0; k < 16; ++k) v[k] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) acts[e * 16 + k] = v[k];
      }
    }
    for (int e = tid; e < 256 * COUT; e += kThreads) {
      const int px = e / COUT, oo = e - (e / COUT) * COUT;
      const int64_t gy = ty + px / 16, gx = tx + px % 16;
      float v = 0.0f;
      if (inside(gy, gx, a.rows, a.cols)) {
        const int64_t q = b * a.hw + gy * a.cols + gx;
        v = LAYER == 3 ? a.dy[q] : (LAYER == 2 ? a.dz2[q * 16 + oo] : a.dz1[q * 16 + oo]);
      }
      dzs[e] = v;
    }
    __syncthreads();
    float acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.0f;
    for (int px = sub; px < 256; px += S) {
      const float d = dzs[px * COUT + o];
      const int ly = px >> 4, lx = px & 15;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap)
        acc[tap] = fmaf(d, acts[((ly + tap / 3) * 18 + lx + tap % 3) * CIN + c], acc[tap]);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) accd[k] += (double)acc[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 9; ++k) red[tid * 9 + k] = accd[k];
  __syncthreads();
  if (tid < P) {
    for (int k = 0; k < 9; ++k) {
      double s = 0.0;
      for (int q = 0; q < S; ++q) s += red[(q * P + tid) * 9 + k];
      partials[((size_t)blockIdx.x * P + tid) * 9 + k] = s;
    }
  }
}

__global__ void __launch_bounds__(kThreads) net_wgrad_reduce_kernel(const double* __restrict__ partials, int nparts,
                                                                    int nw, float* __restrict__ grad) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  double s = 0.0;
  for (int g = 0; g < nparts; ++g) s += partials[(size_t)g * nw + w];
  grad[w] = (float)s;
}

__global__ void __launch_bounds__(kThreads) net_loss_final_kernel(const double* __restrict__ partials, int nparts,
                                                                  double inv_count, double* __restrict__ loss) {
  __shared__ double red[16];
  double t[1];
  reduce_partials<1>(partials, nparts, 1, t, red);
  if (threadIdx.x == 0) *loss = t[0] * inv_count;
}

__global__ void __launch_bounds__(kThreads) net_adam_kernel(int64_t count, float b1, float b2, float eps,
                                                            float step, float bc1, float bc2, float* __restrict__ w,
                                                            float* __restrict__ mom, float* __restrict__ vel,
                                                            const float* __restrict__ grad,
                                                            uint16_t* __restrict__ wb) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const float g = grad[i];
    const float m = b1 * mom[i] + (1.0f - b1) * g;
    const float v = b2 * vel[i] + (1.0f - b2) * g * g;
    mom[i] = m;
    vel[i] = v;
    const float wn = w[i] - step * (m / bc1) / (sqrtf(v / bc2) + eps);
    w[i] = wn;
    wb[i] = (uint16_t)f2bf(wn);
  }
}

__global__ void __launch_bounds__(kThreads) net_to_bf16_kernel(int64_t count, const float* __restrict__ w,
                                                               uint16_t* __restrict__ wb) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    wb[i] = (uint16_t)f2bf(w[i]);
}

// ---------------------------------------------------------------------------
// fused inference
// ---------------------------------------------------------------------------
constexpr int kOT = 28;             // output tile side
constexpr int kA2 = kOT + 2;        // layer-2 output region side (30)
constexpr int kA1 = kOT + 4;        // layer-1 output region side (32)
constexpr int kXS = kOT + 6;        // input region side (34)
constexpr int kA2N = kA2 * kA2;     // 900
constexpr int kA1N = kA1 * kA1;     // 1024
constexpr int kXN = kXS * kXS;      // 1156
constexpr int kA2Chunks = (kA2N + 15) / 16;  // 57
static_assert(kA1N / 16 % 16 == 0, "layer-1 chunks must split into pairs over 8 waves");

struct NetInferArgs {
  const uint16_t* w;       // BF16 weights (flat layout)
  const void* R;           // n x m, point-major
  void* Z;                 // n x m output T(R)
  const void* g;           // guidance, n values
  const void* sqd;         // sqrt(d) (constraint dots), or nullptr
  const double* colnorm;   // ||R_j||
  const LobpcgState* st;   // LOBPCG state (skip when inactive; Y norm), or nullptr
  int64_t rows, cols, n;
  int m;
  int tiles_x, ntiles;
  double* partials;        // [tile][3m]: r_j.w_j, y.w_j, non-finite count
};

__device__ __forceinline__ floatx4 mfma_bf16(short4_t a, short4_t b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ short4_t as_short4(uint32_t lo, uint32_t hi) {
  short4_t r;
  r[0] = (short)(lo & 0xffffu);
  r[1] = (short)(lo >> 16);
  r[2] = (short)(hi & 0xffffu);
  r[3] = (short)(hi >> 16);
  return r;
}

constexpr int kNetThreads = 512;    // 8 waves per tile
constexpr int kNetWaves = kNetThreads / 64;
constexpr int kA2PerWave = (kA2Chunks + kNetWaves - 1) / kNetWaves;  // 8

// Two independent 16-pixel chunks per step keep two MFMA chains in flight.
// Layer 1 writes a1 to LDS; layer 2 feeds its BF16 output (already in the
// layer-3 operand layout) straight into the layer-3 per-tap products.
template <typename T>
__global__ void __launch_bounds__(kNetThreads) net_infer_kernel(NetInferArgs a) {
  __shared__ uint32_t xs[kXN];                         // (r/s, g) as a BF16 pair per pixel
  __shared__ __align__(16) uint16_t a1s[kA1N * 16];    // layer-1 output
  __shared__ float c3[9 * kA2N];                       // layer-3 per-tap products
  __shared__ double red[16 * 3];
  if (a.st != nullptr && !a.st->active) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, l16 = lane & 15;
  const int tile = xcd_tile(blockIdx.x, a.ntiles);
  const int ty = tile / a.tiles_x, tx = tile - (tile / a.tiles_x) * a.tiles_x;
  const int64_t y0 = (int64_t)ty * kOT, x0 = (int64_t)tx * kOT;

  // MFMA A operands (weights): lane holds A[row = l16][k = 4q + i]
  short4_t w1a[2], w2a[9], w3a;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 16 * h + 4 * q + i, tap = k >> 1, c = k & 1;
      w1a[h][i] = tap < 9 ? (short)a.w[kOffW1 + l16 * 18 + c * 9 + tap] : (short)0;
    }
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int i = 0; i < 4; ++i) w2a[tap][i] = (short)a.w[kOffW2 + l16 * 144 + (4 * q + i) * 9 + tap];
#pragma unroll
  for (int i = 0; i < 4; ++i) w3a[i] = l16 < 9 ? (short)a.w[kOffW3 + (4 * q + i) * 9 + l16] : (short)0;

  // layer-1 B operand taps of this lane: k = 16h + 4q + i -> taps 8h + 2q, 8h + 2q + 1
  const int t0 = 2 * q, t1 = 2 * q + 1;
  const int xo0 = (t0 / 3) * kXS + t0 % 3, xo1 = (t1 / 3) * kXS + t1 % 3, xo8 = 2 * kXS + 2;

  const T* R = (const T*)a.R;
  T* Z = (T*)a.Z;
  const T* G = (const T*)a.g;
  const T* sqd = (const T*)a.sqd;
  const double yinv = (a.st != nullptr && sqd != nullptr) ? a.st->ynorm_inv : 0.0;
  const double rn = sqrt((double)a.n);

  for (int j = 0; j < a.m; ++j) {
    const double s = a.colnorm[j] / rn;
    // stage the input region
    for (int e = threadIdx.x; e < kXN; e += kNetThreads) {
      const int64_t gy = y0 - 3 + e / kXS, gx = x0 - 3 + e % kXS;
      uint32_t v = 0;
      if (inside(gy, gx, a.rows, a.cols)) {
        const int64_t i = gy * a.cols + gx;
        const double r = (double)R[i * a.m + j];
        v = (s > 0.0 ? d2bf(r / s) : 0u) | (d2bf((double)G[i]) << 16);
      }
      xs[e] = v;
    }
    __syncthreads();
    // layer 1: 2 -> 16 channels on the 32 x 32 region, K = 9 taps x 2 (padded to 32)
#pragma unroll
    for (int k = 0; k < kA1N / 16 / kNetWaves; k += 2) {
      floatx4 acc[2];
      int pp[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int p = (wave + kNetWaves * (k + u)) * 16 + l16, py = p >> 5, px = p & 31;
        const int base = py * kXS + px;
        const short4_t b0 = as_short4(xs[base + xo0], xs[base + xo1]);
        const short4_t b1 = as_short4(q == 0 ? xs[base + xo8] : 0u, 0u);
        floatx4 c = {0.0f, 0.0f, 0.0f, 0.0f};
        c = mfma_bf16(w1a[0], b0, c);
        acc[u] = mfma_bf16(w1a[1], b1, c);
        pp[u] = p;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int p = pp[u], py = p >> 5, px = p & 31;
        uint32_t u0 = 0, u1 = 0;
        if (inside(y0 - 2 + py, x0 - 2 + px, a.rows, a.cols)) {
          u0 = f2bf(relu(acc[u][0])) | (f2bf(relu(acc[u][1])) << 16);
          u1 = f2bf(relu(acc[u][2])) | (f2bf(relu(acc[u][3])) << 16);
        }
        *(uint2*)&a1s[p * 16 + 4 * q] = make_uint2(u0, u1);
      }
    }
    __syncthreads();
    // layer 2 (16 -> 16 channels on the 30 x 30 region, K = 9 taps x 16) and
    // layer 3 as 9 per-tap 1x1 products c3[tap][p] = sum_c W3[c][tap] a2[p][c]
#pragma unroll
    for (int k = 0; k < kA2PerWave; k += 2) {
      int base[2];
      bool in[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        int ch = wave + kNetWaves * (k + u);
        ch = ch < kA2Chunks ? ch : kA2Chunks - 1;
        const int pv = ch * 16 + l16;
        const int p = pv < kA2N ? pv : kA2N - 1;
        const int py = p / kA2, px = p - (p / kA2) * kA2;
        base[u] = (py * kA1 + px) * 16 + 4 * q;
        in[u] = inside(y0 - 1 + py, x0 - 1 + px, a.rows, a.cols);
      }
      floatx4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int off = ((tap / 3) * kA1 + tap % 3) * 16;
        const uint2 bv0 = *(const uint2*)&a1s[base[0] + off];
        const uint2 bv1 = *(const uint2*)&a1s[base[1] + off];
        acc0 = mfma_bf16(w2a[tap], as_short4(bv0.x, bv0.y), acc0);
        acc1 = mfma_bf16(w2a[tap], as_short4(bv1.x, bv1.y), acc1);
      }
      const floatx4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const floatx4 acc = u == 0 ? acc0 : acc1;
        uint32_t u0 = 0, u1 = 0;
        if (in[u]) {
          u0 = f2bf(relu(acc[0])) | (f2bf(relu(acc[1])) << 16);
          u1 = f2bf(relu(acc[2])) | (f2bf(relu(acc[3])) << 16);
        }
        const floatx4 t = mfma_bf16(w3a, as_short4(u0, u1), zero);
        const int ch = wave + kNetWaves * (k + u);
        const int pv = ch * 16 + l16;
        if (ch < kA2Chunks && pv < kA2N) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (4 * q + i < 9) c3[(4 * q + i) * kA2N + pv] = t[i];
        }
      }
    }
    __syncthreads();
    // output: y[o] = sum_tap c3[tap][o + off(tap)], w = s y
    double v[3] = {0.0, 0.0, 0.0};
    for (int e = threadIdx.x; e < kOT * kOT; e += kNetThreads) {
      const int oy = e / kOT, ox = e - (e / kOT) * kOT;
      const int64_t gy = y0 + oy, gx = x0 + ox;
      if (gy >= a.rows || gx >= a.cols) continue;
      float yv = 0.0f;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) yv += c3[tap * kA2N + (oy + tap / 3) * kA2 + ox + tap % 3];
      const int64_t i = gy * a.cols + gx;
      const T wt = (T)(s * (double)yv);
      Z[i * a.m + j] = wt;
      const double wd = (double)wt;
      v[0] += (double)R[i * a.m + j] * wd;
      if (sqd != nullptr) v[1] += (double)sqd[i] * yinv * wd;
      if (!__builtin_isfinite(wd)) v[2] += 1.0;
    }
    block_sum<3>(v, red);
    if (threadIdx.x == 0) {
      double* pp = a.partials + ((size_t)blockIdx.x * a.m + j) * 3;
      pp[0] = v[0];
      pp[1] = v[1];
      pp[2] = v[2];
    }
  }
}

// LOBPCG: per column, use T(r) unless it has a non-finite entry or
// r^T T(r) <= 0 (then T = I); Y^T T(r) for the constraint projection.
__global__ void __launch_bounds__(kThreads) net_final_kernel(const double* __restrict__ partials, int nparts, int m,
                                                             LobpcgState* st) {
  __shared__ double red[16 * 3];
  if (!st->active) return;
  for (int j = 0; j < m; ++j) {
    double t[3];
    reduce_partials<3>(partials + 3 * j, nparts, 3 * m, t, red);
    if (threadIdx.x == 0) {
      const bool use = t[2] == 0.0 && __builtin_isfinite(t[0]) && t[0] > 0.0 && st->res[j] > 0.0;
      st->tuse[j] = use ? 1 : 0;
      st->yz[j] = t[1];
      if (!use) st->fallbacks += 1;
    }
  }
}

// W <- T(R) or R per column (W holds R on entry), minus its Y component
template <typename T>
__global__ void __launch_bounds__(kThreads) net_select_kernel(T* __restrict__ W, const T* __restrict__ Z,
                                                              const T* __restrict__ sqd, int64_t n, int m,
                                                              int constraint, const LobpcgState* st) {
  if (!st->active) return;
  const double yinv = st->ynorm_inv;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double yi = constraint ? (double)sqd[i] * yinv : 0.0;
    for (int j = 0; j < m; ++j) {
      const bool use = st->tuse[j] != 0;
      double v = use ? (double)Z[i * m + j] : (double)W[i * m + j];
      if (constraint) v -= yi * (use ? st->yz[j] : st->yx[j]);
      W[i * m + j] = (T)v;
    }
  }
}

// Partials of the fallback test for a preconditioner output Z computed
// outside the network kernel: per column r^T z, (Y^T z with Y = sqrt(d) /
// ||sqrt(d)||, when sqd != nullptr) and the count of non-finite entries, in
// the layout net_final_kernel reads (3 values per column, 3m per workgroup).
template <typename T>
__global__ void __launch_bounds__(kThreads) tz_partials_kernel(const T* __restrict__ R, const T* __restrict__ Z,
                                                               const T* __restrict__ sqd, int64_t n, int m,
                                                               const LobpcgState* st, double* __restrict__ partials) {
  __shared__ double red[16 * 3 * kMaxBlock];
  double v[3 * kMaxBlock];
#pragma unroll
  for (int k = 0; k < 3 * kMaxBlock; ++k) v[k] = 0.0;
  const double yinv = sqd != nullptr ? st->ynorm_inv : 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double yi = sqd != nullptr ? (double)sqd[i] * yinv : 0.0;
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j)
      if (j < m) {
        const double z = (double)Z[i * m + j];
        v[3 * j] += (double)R[i * m + j] * z;
        v[3 * j + 1] += yi * z;
        if (!__builtin_isfinite(z)) v[3 * j + 2] += 1.0;
      }
  }
  block_sum<3 * kMaxBlock>(v, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3 * m; ++k) partials[(size_t)blockIdx.x * 3 * m + k] = v[k];
}

// dst[i * ldd] = src[i * lds]
template <typename T>
__global__ void __launch_bounds__(kThreads) col_copy_kernel(const T* __restrict__ src, int64_t lds, T* __restrict__ dst,
                                                            int64_t ldd, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i * ldd] = src[i * lds];
}

// ||R_j||^2 partials of an n x m block
template <typename T>
__global__ void __launch_bounds__(kThreads) colnorm_kernel(const T* __restrict__ R, int64_t n, int m,
                                                           int64_t ld, double* __restrict__ partials) {
  __shared__ double red[16 * kMaxBlock];
  double v[kMaxBlock];
#pragma unroll
  for (int j = 0; j < kMaxBlock; ++j) v[j] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j)
      if (j < m) {
        const double r = (double)R[i * ld + j];
        v[j] += r * r;
      }
  }
  block_sum<kMaxBlock>(v, red);
  if (threadIdx.x == 0)
    for (int j = 0; j < kMaxBlock; ++j) partials[(size_t)blockIdx.x * kMaxBlock + j] = v[j];
}

__global__ void __launch_bounds__(kThreads) colnorm_final_kernel(const double* __restrict__ partials, int nparts,
                                                                 double* __restrict__ out) {
  __shared__ double red[16 * kMaxBlock];
  double t[kMaxBlock];
  reduce_partials<kMaxBlock>(partials, nparts, kMaxBlock, t, red);
  if (threadIdx.x == 0)
    for (int j = 0; j < kMaxBlock; ++j) out[j] = sqrt(t[j]);
}

// training pair: inputs = (r/s, g), targets = y/s with s = ||r|| / sqrt(n)
template <typename T>
__global__ void __launch_bounds__(kThreads) net_pair_kernel(const T* __restrict__ r, int64_t ldr,
                                                            const T* __restrict__ y, int64_t ldy,
                                                            const T* __restrict__ g, int64_t n,
                                                            const double* __restrict__ norm, float* __restrict__ in,
                                                            float* __restrict__ tg) {
  const double s = norm[0] / sqrt((double)n);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double rs = s > 0.0 ? (double)r[i * ldr] / s : 0.0;
    const double ys = s > 0.0 ? (double)y[i * ldy] / s : 0.0;
    in[2 * i] = (float)rs;
    in[2 * i + 1] = (float)g[i];
    tg[i] = (float)ys;
  }
}

struct Theta8 {
  double v[kMaxBlock];
};

template <typename T>
__global__ void __launch_bounds__(kThreads) residual_kernel(const T* __restrict__ X, T* __restrict__ R, int64_t n,
                                                            int m, Theta8 th) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    for (int j = 0; j < m; ++j) R[i * m + j] = (T)((double)R[i * m + j] - th.v[j] * (double)X[i * m + j]);
}

// ---- shifted CG: (L_sym + alpha I) y = b ---------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads) scg_init_kernel(const T* __restrict__ b, int64_t ldb,
                                                            T* __restrict__ y, T* __restrict__ r, int64_t n,
                                                            double* __restrict__ partials) {
  __shared__ double red[16];
  double v[1] = {0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T bi = b[i * ldb];
    y[i] = (T)0;
    r[i] = bi;
    v[0] += (double)bi * (double)bi;
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(kThreads) scg_init_final_kernel(const double* __restrict__ partials, int nparts,
                                                                  CgState* st) {
  __shared__ double red[16];
  double t[1];
  reduce_partials<1>(partials, nparts, 1, t, red);
  if (threadIdx.x == 0) {
    const double rho = t[0];
    st->rho = rho;
    st->rho0 = rho;
    st->res0 = sqrt(rho);
    st->floor = -1.0;  // no breakdown floor: the right-hand side is given
    st->tol2 = st->tol * st->tol * rho;
    st->iters = 0;
    st->k = 1;
    st->beta = 0.0;
    st->status = GSF_OK;
    st->active = (__builtin_isfinite(rho) && rho > st->tol2) ? 1 : 0;
    if (!__builtin_isfinite(rho)) st->status = GSF_EBREAKDOWN;
  }
}

// q += alpha_shift p; partials of p^T q
template <typename T>
__global__ void __launch_bounds__(kThreads) scg_shift_kernel(const T* __restrict__ p, T* __restrict__ q, int64_t n,
                                                             double shift, double* __restrict__ partials,
                                                             const CgState* st) {
  __shared__ double red[16];
  if (!st->active) return;
  double v[1] = {0.0};
  const T sh = (T)shift;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T pi = p[i];
    const T qi = q[i] + sh * pi;
    q[i] = qi;
    v[0] += (double)pi * (double)qi;
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t net_train_bytes(int batch, int64_t hw) {
  const size_t px = (size_t)batch * (size_t)hw;
  const size_t wg = (size_t)1024 * kNetWeights;  // wgrad partials (at most 1024 workgroups per layer)
  return align_up(kNetWeights * 4, 256) + 2 * align_up(px * 32, 256) + 2 * align_up(px * 4, 256) +
         2 * align_up(px * 64, 256) + align_up(1024 * 8, 256) + align_up(wg * 8, 256);
}

struct NetTrainWs {
  float* wf;
  uint16_t *a1, *a2;
  float *y, *dy, *dz2, *dz1;
  double *loss_part, *wpart;
};

static NetTrainWs carve_train(void* ws, int batch, int64_t hw) {
  const size_t px = (size_t)batch * (size_t)hw;
  char* p = (char*)ws;
  NetTrainWs w;
  w.wf = (float*)p;
  p += align_up(kNetWeights * 4, 256);
  w.a1 = (uint16_t*)p;
  p += align_up(px * 32, 256);
  w.a2 = (uint16_t*)p;
  p += align_up(px * 32, 256);
  w.y = (float*)p;
  p += align_up(px * 4, 256);
  w.dy = (float*)p;
  p += align_up(px * 4, 256);
  w.dz2 = (float*)p;
  p += align_up(px * 64, 256);
  w.dz1 = (float*)p;
  p += align_up(px * 64, 256);
  w.loss_part = (double*)p;
  p += align_up(1024 * 8, 256);
  w.wpart = (double*)p;
  return w;
}

static int px_blocks(int64_t total) {
  int64_t b = (total + kThreads - 1) / kThreads;
  if (b > 4096) b = 4096;
  return (int)(b < 1 ? 1 : b);
}

gsf_status net_forward_train(const uint16_t* w, int batch, const int32_t* idx, int64_t rows, int64_t cols,
                             const float* inputs, const float* targets, float* y_out, float* grad, double* loss,
                             void* ws, hipStream_t s) {
  const int64_t hw = rows * cols;
  NetTrainWs t = carve_train(ws, batch, hw);
  NetTrainArgs a{};
  a.wf = t.wf;
  a.idx = idx;
  a.batch = batch;
  a.rows = rows;
  a.cols = cols;
  a.hw = hw;
  a.inputs = inputs;
  a.targets = targets;
  a.a1 = t.a1;
  a.a2 = t.a2;
  a.y = y_out != nullptr ? y_out : t.y;
  a.dy = t.dy;
  a.dz2 = t.dz2;
  a.dz1 = t.dz1;
  a.loss_part = t.loss_part;
  a.dscale = (float)(2.0 / ((double)batch * (double)hw));
  const int nb = px_blocks((int64_t)batch * hw);
  const int nbl = nb < 1024 ? nb : 1024;
  net_round_weights_kernel<<<(kNetWeights + kThreads - 1) / kThreads, kThreads, 0, s>>>(w, t.wf);
  net_fwd1_kernel<<<nb, kThreads, 0, s>>>(a);
  net_fwd2_kernel<<<nb, kThreads, 0, s>>>(a);
  net_fwd3_kernel<<<targets != nullptr ? nbl : nb, kThreads, 0, s>>>(a);
  if (targets == nullptr) return launch_status();
  net_loss_final_kernel<<<1, kThreads, 0, s>>>(t.loss_part, nbl, 1.0 / ((double)batch * (double)hw), loss);
  net_bwd3_kernel<<<nb, kThreads, 0, s>>>(a);
  net_bwd2_kernel<<<nb, kThreads, 0, s>>>(a);
  const int tiles_x = (int)((cols + 15) / 16), tiles_y = (int)((rows + 15) / 16);
  const int tps = tiles_x * tiles_y;
  const int64_t ntiles = (int64_t)batch * tps;
  const int gw = (int)(ntiles < 1024 ? ntiles : 1024);
  double* p1 = t.wpart;
  double* p2 = p1 + (size_t)gw * kOffW2;
  double* p3 = p2 + (size_t)gw * (kOffW3 - kOffW2);
  net_wgrad_kernel<1><<<gw, kThreads, 0, s>>>(a, tiles_x, tps, p1);
  net_wgrad_kernel<2><<<gw, kThreads, 0, s>>>(a, tiles_x, tps, p2);
  net_wgrad_kernel<3><<<gw, kThreads, 0, s>>>(a, tiles_x, tps, p3);
  net_wgrad_reduce_kernel<<<(kOffW2 + kThreads - 1) / kThreads, kThreads, 0, s>>>(p1, gw, kOffW2, grad + kOffW1);
  net_wgrad_reduce_kernel<<<(kOffW3 - kOffW2 + kThreads - 1) / kThreads, kThreads, 0, s>>>(p2, gw, kOffW3 - kOffW2,
                                                                                        grad + kOffW2);
  net_wgrad_reduce_kernel<<<1, kThreads, 0, s>>>(p3, gw, kNetWeights - kOffW3, grad + kOffW3);
  return launch_status();
}

gsf_status net_adam(int64_t count, int t, double lr, double b1, double b2, double eps, float* w, float* mom,
                    float* vel, const float* grad, uint16_t* wb, hipStream_t s) {
  const float bc1 = (float)(1.0 - std::pow(b1, t)), bc2 = (float)(1.0 - std::pow(b2, t));
  net_adam_kernel<<<px_blocks(count), kThreads, 0, s>>>(count, (float)b1, (float)b2, (float)eps, (float)lr, bc1, bc2,
                                                        w, mom, vel, grad, wb);
  return launch_status();
}

gsf_status net_to_bf16(int64_t count, const float* w, uint16_t* wb, hipStream_t s) {
  net_to_bf16_kernel<<<px_blocks(count), kThreads, 0, s>>>(count, w, wb);
  return launch_status();
}

int net_tiles(int64_t rows, int64_t cols) {
  return (int)(((rows + kOT - 1) / kOT) * ((cols + kOT - 1) / kOT));
}

gsf_status net_infer(int prec, const uint16_t* w, int64_t rows, int64_t cols, int m, const void* R, void* Z,
                     const void* g, const void* sqd, const double* colnorm, const LobpcgState* st, double* partials,
                     hipStream_t s) {
  NetInferArgs a{};
  a.w = w;
  a.R = R;
  a.Z = Z;
  a.g = g;
  a.sqd = sqd;
  a.colnorm = colnorm;
  a.st = st;
  a.rows = rows;
  a.cols = cols;
  a.n = rows * cols;
  a.m = m;
  a.tiles_x = (int)((cols + kOT - 1) / kOT);
  a.ntiles = net_tiles(rows, cols);
  a.partials = partials;
  if (prec == GSF_F32)
    net_infer_kernel<float><<<a.ntiles, kNetThreads, 0, s>>>(a);
  else
    net_infer_kernel<double><<<a.ntiles, kNetThreads, 0, s>>>(a);
  return launch_status();
}

gsf_status net_lob_select(int prec, int64_t rows, int64_t cols, int m, int constraint, void* W, const void* Z,
                          const void* sqd, const double* partials, int nparts, LobpcgState* st, hipStream_t s) {
  const int64_t n = rows * cols;
  net_final_kernel<<<1, kThreads, 0, s>>>(partials, nparts, m, st);
  const int nb = vec_blocks(n);
  if (prec == GSF_F32)
    net_select_kernel<float><<<nb, kThreads, 0, s>>>((float*)W, (const float*)Z, (const float*)sqd, n, m, constraint,
                                                     st);
  else
    net_select_kernel<double><<<nb, kThreads, 0, s>>>((double*)W, (const double*)Z, (const double*)sqd, n, m,
                                                      constraint, st);
  return launch_status();
}

int tz_blocks(int64_t rows, int64_t cols) {
  const int a = vec_blocks(rows * cols), b = net_tiles(rows, cols);
  return a < b ? a : b;
}

gsf_status launch_tz_partials(int prec, const void* R, const void* Z, const void* sqd, int64_t rows, int64_t cols,
                              int m, const LobpcgState* st, double* partials, hipStream_t s) {
  const int nb = tz_blocks(rows, cols);
  const int64_t n = rows * cols;
  if (prec == GSF_F32)
    tz_partials_kernel<float><<<nb, kThreads, 0, s>>>((const float*)R, (const float*)Z, (const float*)sqd, n, m, st,
                                                      partials);
  else
    tz_partials_kernel<double><<<nb, kThreads, 0, s>>>((const double*)R, (const double*)Z, (const double*)sqd, n, m,
                                                       st, partials);
  return launch_status();
}

gsf_status launch_col_copy(int prec, const void* src, int64_t lds, void* dst, int64_t ldd, int64_t n, hipStream_t s) {
  const int nb = vec_blocks(n);
  if (prec == GSF_F32)
    col_copy_kernel<float><<<nb, kThreads, 0, s>>>((const float*)src, lds, (float*)dst, ldd, n);
  else
    col_copy_kernel<double><<<nb, kThreads, 0, s>>>((const double*)src, lds, (double*)dst, ldd, n);
  return launch_status();
}

gsf_status launch_colnorm(int prec, const void* R, int64_t n, int m, int64_t ld, double* partials, double* out,
                          hipStream_t s) {
  const int nb = vec_blocks(n);
  if (prec == GSF_F32)
    colnorm_kernel<float><<<nb, kThreads, 0, s>>>((const float*)R, n, m, ld, partials);
  else
    colnorm_kernel<double><<<nb, kThreads, 0, s>>>((const double*)R, n, m, ld, partials);
  colnorm_final_kernel<<<1, kThreads, 0, s>>>(partials, nb, out);
  return launch_status();
}

gsf_status launch_net_pair(int prec, const void* r, int64_t ldr, const void* y, int64_t ldy, const void* g,
                           int64_t n, const double* norm, float* in, float* tg, hipStream_t s) {
  const int nb = vec_blocks(n);
  if (prec == GSF_F32)
    net_pair_kernel<float><<<nb, kThreads, 0, s>>>((const float*)r, ldr, (const float*)y, ldy, (const float*)g, n,
                                                   norm, in, tg);
  else
    net_pair_kernel<double><<<nb, kThreads, 0, s>>>((const double*)r, ldr, (const double*)y, ldy, (const double*)g,
                                                    n, norm, in, tg);
  return launch_status();
}

gsf_status launch_residual(int prec, const void* X, void* R, int64_t n, int m, const double* theta, hipStream_t s) {
  Theta8 th{};
  for (int j = 0; j < m; ++j) th.v[j] = theta[j];
  const int nb = vec_blocks(n);
  if (prec == GSF_F32)
    residual_kernel<float><<<nb, kThreads, 0, s>>>((const float*)X, (float*)R, n, m, th);
  else
    residual_kernel<double><<<nb, kThreads, 0, s>>>((const double*)X, (double*)R, n, m, th);
  return launch_status();
}

gsf_status launch_scg_init(int prec, const void* b, int64_t ldb, void* y, void* r, int64_t n, double* partials,
                           CgState* st, hipStream_t s) {
  const int nb = vec_blocks(n);
  if (prec == GSF_F32)
    scg_init_kernel<float><<<nb, kThreads, 0, s>>>((const float*)b, ldb, (float*)y, (float*)r, n, partials);
  else
    scg_init_kernel<double><<<nb, kThreads, 0, s>>>((const double*)b, ldb, (double*)y, (double*)r, n, partials);
  scg_init_final_kernel<<<1, kThreads, 0, s>>>(partials, nb, st);
  return launch_status();
}

gsf_status launch_scg_shift(int prec, const void* p, void* q, int64_t n, double shift, double* partials, int* nparts,
                            const CgState* st, hipStream_t s) {
  const int nb = vec_blocks(n);
  *nparts = nb;
  if (prec == GSF_F32)
    scg_shift_kernel<float><<<nb, kThreads, 0, s>>>((const float*)p, (float*)q, n, shift, partials, st);
  else
    scg_shift_kernel<double><<<nb, kThreads, 0, s>>>((const double*)p, (double*)q, n, shift, partials, st);
  return launch_status();
}

}  // namespace gsf
