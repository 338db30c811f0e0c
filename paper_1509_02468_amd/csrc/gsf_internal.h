// Internal declarations of libgsf (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "gsf.h"

namespace gsf {

constexpr int kMaxRadius = 8;
constexpr int kMaxBlock = 8;   // largest LOBPCG block size m
constexpr int kThreads = 256;  // threads per workgroup of the streaming kernels

// Host-side description of a built operator.  All device pointers point into
// the caller's operator workspace.
struct Operator {
  gsf_operator_desc desc;
  int64_t n;        // grid points
  int64_t rows;     // 2D: H, 1D: 1
  int64_t cols;     // 2D: W, 1D: n
  int nplanes;      // BF half-window planes
  size_t elem;      // sizeof element type
  void* planes;     // BF: padded start of plane 0 (see pstride, ppad); GF: apply scratch
  int64_t pstride;  // BF: elements from one plane's padded start to the next
  int64_t ppad;     // BF: zeros before each plane's data (r W + r in 2D, r in 1D)
  void* diag;       // BF: 1/sqrt(d)
  void* sqd;        // sqrt(d)
  double* deg;      // d (FP64)
  void* g;          // GF: guidance copy
  void* mu;         // GF: window means
  void* inv;        // GF: 1/(var + eps)
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// BF: the 2D cross stencil (1D cross is the square window's interval).
inline bool bf_cross2d(const gsf_operator_desc& d) { return d.ndim == 2 && d.stencil == GSF_STENCIL_CROSS; }

// Guidance channels (0 in a descriptor means 1).
inline int desc_channels(const gsf_operator_desc& d) { return d.channels > 1 ? d.channels : 1; }

// BF half-window planes: one per undirected offset pair {o, -o}, o != 0.
inline int bf_num_planes(const gsf_operator_desc& d) {
  if (d.ndim == 1) return d.radius;
  if (d.stencil == GSF_STENCIL_CROSS) return 2 * d.radius;
  return ((2 * d.radius + 1) * (2 * d.radius + 1) - 1) / 2;
}

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum NV values over the whole workgroup (blockDim.x a multiple of 64,
// at most 1024 threads) in a fixed order; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* NV * 16 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) lds[k * 16 + wave] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nwaves; ++w) s += lds[k * 16 + w];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Sum partials[b * stride + k] over b = 0..nparts-1 for k < NV in a fixed
// order (the partials were written by an earlier kernel on the stream).
// Result valid in thread 0.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double* partials, int nparts, int stride,
                                                double (&out)[NV], double* lds) {
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] += partials[(size_t)b * stride + k];
  }
  block_sum<NV>(out, lds);
}

// Map a workgroup index to a tile so that each of the 8 XCDs (workgroups are
// dispatched round-robin over them) walks a contiguous band of tiles: tiles
// sharing halos then share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  const int q = ntiles >> 3, rem = ntiles & 7;
  const int k = b & 7, l = b >> 3;
  return k * q + (k < rem ? k : rem) + l;
}

// Status of a HIP call (GSF_EDEVICE on failure, the code kept for
// gsf_last_device_error) and of the launches so far in this thread.
gsf_status device_status(hipError_t e);
inline gsf_status launch_status() { return device_status(hipGetLastError()); }
// Drops a HIP error that other code left in this thread (the runtime keeps
// the last failed call's error until hipGetLastError reads it), so that the
// launch checks of a call report only that call's own launches.
inline void clear_stale_errors() { (void)hipGetLastError(); }

// ---------------------------------------------------------------------------
// launchers (implemented in the .hip files)
// ---------------------------------------------------------------------------
gsf_status launch_bf_build(const Operator& op, const void* guidance, hipStream_t s);
gsf_status launch_gf_build(const Operator& op, const void* guidance, hipStream_t s);

// y = F x (F: form) for an m-column block; x and y have leading dimensions
// ldx / ldy (elements between consecutive grid points) and start at column
// offsets already applied by the caller.  If dot_partials != nullptr (m = 1
// only) every workgroup b writes sum_i x_i y_i of its points to
// dot_partials[b]; *nparts receives the number of workgroups.
gsf_status launch_apply(const Operator& op, int form, int m, const void* x, int64_t ldx, void* y,
                        int64_t ldy, double* dot_partials, int* nparts, hipStream_t s);
int apply_num_blocks(const Operator& op, int m);

}  // namespace gsf

struct gsf_operator {
  gsf::Operator op;
};

// Preconditioner handle: the learned network (grid, precision and borrowed
// device pointers) or the shifted solve T(r) = `inner` CG steps on
// (L_sym + alpha I) y = r from y = 0 (the operator borrowed, the CG scratch
// owned by the handle).
constexpr int kPrecondNet = 0, kPrecondShifted = 1;
struct gsf_precond {
  int64_t n, rows, cols;
  int prec;
  int kind = kPrecondNet;
  const void* g = nullptr;       // guidance, n elements of the operator's type
  const uint16_t* w = nullptr;   // BF16 weights
  const gsf_operator* op = nullptr;
  double alpha = 0.0;
  int inner = 0;
  void* mem = nullptr;           // device scratch of the shifted solve
};
