// C ABI of libgsf: validation, workspace layout and the solver drivers.
#include <cmath>
#include <cstddef>
#include <mutex>
#include <cstring>
#include <new>
#include <string>
#include <cstdio>

#include "cg_step.h"
#include "gsf_internal.h"
#include "lobpcg_launch.h"
#include "solver_state.h"

namespace gsf {

thread_local int g_last_device_error = 0;

gsf_status device_status(hipError_t e) {
  if (e == hipSuccess) return GSF_OK;
  g_last_device_error = (int)e;
  return GSF_EDEVICE;
}

gsf_status launch_bf_apply(const Operator& op, int form, int m, const void* x, int64_t ldx, void* y,
                           int64_t ldy, double* dot, int* nparts, hipStream_t s);
int bf_apply_blocks(const Operator& op, int m);
int bf_rpt(const Operator& op, int w);
void bf_set_rpt(const Operator& op, int w, int rpt);
gsf_status launch_bf_apply_rpt(const Operator& op, int form, int m, const void* x, int64_t ldx, void* y,
                               int64_t ldy, double* dot, int* nparts, int rpt_override, hipStream_t s);
gsf_status launch_gf_apply(const Operator& op, void* scratch, int form, int m, const void* x, int64_t ldx,
                           void* y, int64_t ldy, hipStream_t s);
int vec_blocks(int64_t n);
int rg_bf_blocks(const Operator& op);
gsf_status launch_rg_bf(const Operator& op, int mode, const void* g, const void* v, void* y, double* dot,
                        int* nparts, hipStream_t s);
gsf_status launch_bscale(const Operator& op, int m, const void* in, void* out, int divide, hipStream_t s);
gsf_status launch_bcg(int kind, const Operator& op, int m, void* z, void* r, void* p, void* q, double* partials,
                      BlockCgState* st, hipStream_t s);
gsf_status launch_bcg_state_init(BlockCgState* st, const BlockCgState& v, hipStream_t s);
gsf_status launch_srgb_to_lab(int prec, int64_t n, const void* rgb, void* lab, hipStream_t s);
bool launch_bf_apply_joint(const Operator& op, int form, int m, const void* x, int64_t ldx, void* y, int64_t ldy,
                           const void* x2, int64_t ldx2, void* y2, int64_t ldy2, double* dot, int* nparts,
                           hipStream_t s);
bool launch_rg_power_small(const gsf_operator_desc& d, const void* x0, void* x_out, int kmax, hipStream_t s);
bool launch_cg_small(const Operator& op, const void* x0, void* x_out, int kmax, CgState* st, hipStream_t s);
gsf_status launch_scale(const Operator& op, const void* in, void* out, int divide, hipStream_t s);
gsf_status launch_cg_init(const Operator& op, const void* z, void* r, double* partials, CgState* st,
                          hipStream_t s);
gsf_status launch_cg_pupdate(const Operator& op, const void* r, void* p, const CgState* st, hipStream_t s);
gsf_status launch_dot(const Operator& op, const void* a, const void* b, double* partials, int* nparts,
                      const CgState* st, hipStream_t s);
gsf_status launch_cg_alpha(const double* partials, int nparts, CgState* st, hipStream_t s);
gsf_status launch_cg_pbeta(const Operator& op, const void* r, void* p, const double* upd, CgState* st, int k,
                           hipStream_t s);
gsf_status launch_cg_aupdate(const Operator& op, void* z, void* r, const void* p, const void* q, const double* dots,
                             int ndots, double* upd, CgState* st, int k, hipStream_t s);
gsf_status launch_cg_close(const Operator& op, const double* upd, CgState* st, hipStream_t s);
gsf_status launch_rg_init(const Operator& op, const void* x, void* r, double* partials, CgState* st, hipStream_t s);
gsf_status launch_rg_s_beta(const Operator& op, const void* r, const void* r_old, void* sv, double* partials,
                            CgState* st, hipStream_t s);
gsf_status launch_rg_alpha(const double* partials, int nparts, CgState* st, hipStream_t s);
gsf_status launch_rg_update(const Operator& op, void* x, void* r, void* r_old, const void* p, const void* q,
                            const CgState* st, hipStream_t s);
gsf_status launch_cg_update(const Operator& op, void* z, void* r, const void* p, const void* q, double* partials,
                            CgState* st, hipStream_t s);

// learned preconditioner (net.hip)
size_t net_train_bytes(int batch, int64_t hw);
gsf_status net_forward_train(const uint16_t* w, int batch, const int32_t* idx, int64_t rows, int64_t cols,
                             const float* inputs, const float* targets, float* y_out, float* grad, double* loss,
                             void* ws, hipStream_t s);
gsf_status net_adam(int64_t count, int t, double lr, double b1, double b2, double eps, float* w, float* mom,
                    float* vel, const float* grad, uint16_t* wb, hipStream_t s);
gsf_status net_to_bf16(int64_t count, const float* w, uint16_t* wb, hipStream_t s);
int net_tiles(int64_t rows, int64_t cols);
gsf_status net_infer(int prec, const uint16_t* w, int64_t rows, int64_t cols, int m, const void* R, void* Z,
                     const void* g, const void* sqd, const double* colnorm, const LobpcgState* st, double* partials,
                     hipStream_t s);
gsf_status net_lob_select(int prec, int64_t rows, int64_t cols, int m, int constraint, void* W, const void* Z,
                          const void* sqd, const double* partials, int nparts, LobpcgState* st, hipStream_t s);
int tz_blocks(int64_t rows, int64_t cols);
int tune_table_write(FILE* f);
int tune_table_read(const std::string& text);
void tune_table_clear();
gsf_status shifted_precond_apply(const gsf_precond* T, int m, const void* R, void* Z, hipStream_t s);
gsf_status launch_tz_partials(int prec, const void* R, const void* Z, const void* sqd, int64_t rows, int64_t cols,
                              int m, const LobpcgState* st, double* partials, hipStream_t s);
gsf_status launch_col_copy(int prec, const void* src, int64_t lds, void* dst, int64_t ldd, int64_t n, hipStream_t s);
gsf_status launch_colnorm(int prec, const void* R, int64_t n, int m, int64_t ld, double* partials, double* out,
                          hipStream_t s);
gsf_status launch_net_pair(int prec, const void* r, int64_t ldr, const void* y, int64_t ldy, const void* g,
                           int64_t n, const double* norm, float* in, float* tg, hipStream_t s);
gsf_status launch_residual(int prec, const void* X, void* R, int64_t n, int m, const double* theta, hipStream_t s);
gsf_status launch_scg_init(int prec, const void* b, int64_t ldb, void* y, void* r, int64_t n, double* partials,
                           CgState* st, hipStream_t s);
gsf_status launch_scg_shift(int prec, const void* p, void* q, int64_t n, double shift, double* partials, int* nparts,
                            const CgState* st, hipStream_t s);

namespace {

constexpr size_t kAlign = 256;

__global__ void lob_state_init_kernel(LobpcgState* dst, LobpcgState v) { *dst = v; }
__global__ void cg_state_init_kernel(CgState* dst, CgState v) { *dst = v; }

gsf_status validate_desc(const gsf_operator_desc* d) {
  if (d == nullptr) return GSF_EINVAL;
  if (d->kind != GSF_BF && d->kind != GSF_GF) return GSF_EINVAL;
  if (d->ndim != 1 && d->ndim != 2) return GSF_EINVAL;
  if (d->prec != GSF_F32 && d->prec != GSF_F64) return GSF_EINVAL;
  if (d->radius < 1 || d->radius > kMaxRadius) return GSF_EINVAL;
  if (d->stencil != GSF_STENCIL_SQUARE && d->stencil != GSF_STENCIL_CROSS) return GSF_EINVAL;
  if (d->norm != GSF_NORM_D && d->norm != GSF_NORM_DIAGL) return GSF_EINVAL;
  if (d->channels < 0 || d->channels > kMaxBlock || d->reserved != 0) return GSF_EINVAL;
  if (d->kind == GSF_GF && (d->stencil != GSF_STENCIL_SQUARE || d->norm != GSF_NORM_D || desc_channels(*d) != 1))
    return GSF_EINVAL;
  if (d->dims[0] < 1) return GSF_EINVAL;
  if (d->ndim == 2 && d->dims[1] < 1) return GSF_EINVAL;
  const int64_t n = d->ndim == 1 ? d->dims[0] : d->dims[0] * d->dims[1];
  if (d->ndim == 2 && (d->dims[0] > (int64_t)1 << 30 || d->dims[1] > (int64_t)1 << 30)) return GSF_EINVAL;
  if (n > ((int64_t)1 << 34)) return GSF_EINVAL;
  if (d->kind == GSF_BF) {
    // the BF apply addresses a padded plane with 32-bit byte offsets: the
    // padded plane (ppad zeros, then n weights) must fit in 4 GiB
    const int64_t ppad = d->ndim == 1 ? d->radius : (int64_t)d->radius * d->dims[1] + d->radius;
    const int64_t elem = d->prec == GSF_F32 ? 4 : 8;
    if (n >= ((int64_t)1 << 30) || (n + ppad) * elem > ((int64_t)1 << 32)) return GSF_EINVAL;
    if (!(d->sigma_d > 0.0) || std::isnan(d->sigma_d)) return GSF_EINVAL;
    if (!(d->sigma_r > 0.0) || std::isnan(d->sigma_r)) return GSF_EINVAL;
  } else {
    if (!(d->gf_eps >= 0.0) || !std::isfinite(d->gf_eps)) return GSF_EINVAL;
    if (n >= ((int64_t)1 << 27)) return GSF_EINVAL;  // the GF kernels index with 32 bits
  }
  return GSF_OK;
}

// Operator workspace layout, in order, each region 256-byte aligned:
//   BF: planes (nplanes padded planes, see layout_operator), diag (n), sqd (n),
//       deg (n doubles)
//   GF: g (n), mu (n), inv (n), sqd (n), diag (n), deg (n doubles), 16 scratch
//       planes (n): (a, b) of up to 8 columns for the apply
size_t layout_operator(const gsf_operator_desc* d, Operator* op, char* base) {
  const int64_t n = d->ndim == 1 ? d->dims[0] : d->dims[0] * d->dims[1];
  const size_t elem = d->prec == GSF_F32 ? 4 : 8;
  const size_t plane = align_up((size_t)n * elem, kAlign);
  const size_t dplane = align_up((size_t)n * 8, kAlign);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  if (op) {
    std::memset(op, 0, sizeof(*op));
    op->desc = *d;
    op->n = n;
    op->rows = d->ndim == 1 ? 1 : d->dims[0];
    op->cols = d->ndim == 1 ? d->dims[0] : d->dims[1];
    op->elem = elem;
  }
  if (d->kind == GSF_BF) {
    const int np = bf_num_planes(*d);
    // every plane is preceded by ppad zeros, so that the apply's mirrored
    // reads w_{i-o,i} above the first row (or before the first sample) read
    // zeros instead of branching
    const int64_t cols = d->ndim == 1 ? d->dims[0] : d->dims[1];
    const int64_t ppad = d->ndim == 1 ? d->radius : (int64_t)d->radius * cols + d->radius;
    const int64_t pstride = (int64_t)align_up((size_t)(n + ppad), 64);
    void* planes = take(align_up((size_t)(np * pstride + ppad) * elem, kAlign));
    void* diag = take(plane);
    void* sqd = take(plane);
    void* deg = take(dplane);
    if (op) {
      op->nplanes = np;
      op->planes = planes;
      op->pstride = pstride;
      op->ppad = ppad;
      op->diag = diag;
      op->sqd = sqd;
      op->deg = (double*)deg;
    }
  } else {
    void* g = take(plane);
    void* mu = take(plane);
    void* inv = take(plane);
    void* sqd = take(plane);
    void* diag = take(plane);
    void* deg = take(dplane);
    void* scratch = take(align_up((size_t)2 * kMaxBlock * n * elem, kAlign));  // apply: (a, b) of 8 columns
    if (op) {
      op->g = g;
      op->mu = mu;
      op->inv = inv;
      op->sqd = sqd;
      op->diag = diag;
      op->deg = (double*)deg;
      op->planes = scratch;
    }
  }
  return off;
}

void* gf_scratch(const Operator& op) { return op.planes; }

gsf_status apply_any(const Operator& op, int form, int m, const void* x, int64_t ldx, void* y, int64_t ldy,
                     double* dot, int* nparts, hipStream_t s) {
  if (op.desc.kind == GSF_BF) return launch_bf_apply(op, form, m, x, ldx, y, ldy, dot, nparts, s);
  return launch_gf_apply(op, gf_scratch(op), form, m, x, ldx, y, ldy, s);
}

// Bump allocator over a caller workspace (nullptr base: size query).
struct Carve {
  char* base;
  size_t off = 0;
  void* take(size_t bytes) {
    void* p = base ? base + off : nullptr;
    off += align_up(bytes, kAlign);
    return p;
  }
};

double breakdown_tau(int prec) { return prec == GSF_F32 ? 1e-6 : 1e-13; }
// LOBPCG recomputes AX = A X after every kAxRefresh-th step
constexpr int kAxRefresh = 20;
double drop_tol_of(int prec) { return prec == GSF_F32 ? 1e-6 : 1e-10; }

struct CgWs {
  void *z, *r, *p, *q;
  double* partials;   // per-workgroup partials (the apply's p^T q, and the step kernels')
  double* partials2;  // the fused update's r^T r partials
  CgState* st;
};

size_t carve_cg(const Operator& op, char* base, CgWs* w) {
  Carve c{base};
  const size_t v = (size_t)op.n * op.elem;
  w->z = c.take(v);
  w->r = c.take(v);
  w->p = c.take(v);
  w->q = c.take(v);
  int nb = vec_blocks(op.n);
  if (op.desc.kind == GSF_BF) {
    const int ab = bf_apply_blocks(op, 1);
    nb = ab > nb ? ab : nb;
  }
  w->partials = (double*)c.take((size_t)nb * 2 * sizeof(double));
  w->partials2 = (double*)c.take((size_t)vec_blocks(op.n) * 2 * sizeof(double));
  w->st = (CgState*)c.take(sizeof(CgState));
  return c.off;
}

// Block CG over m columns: z, r, p, q (n x m each), partials (2m per
// workgroup) and the per-column state.
struct BcgWs {
  void *z, *r, *p, *q;
  double* partials;
  BlockCgState* st;
};

size_t carve_bcg(const Operator& op, int m, char* base, BcgWs* w) {
  Carve c{base};
  const size_t v = (size_t)op.n * m * op.elem;
  w->z = c.take(v);
  w->r = c.take(v);
  w->p = c.take(v);
  w->q = c.take(v);
  w->partials = (double*)c.take((size_t)vec_blocks(op.n) * 2 * m * sizeof(double));
  w->st = (BlockCgState*)c.take(sizeof(BlockCgState));
  return c.off;
}

// Re-guided filters: the operator (rebuilt in place every step), then for CG
// x-space r, r_old, s, p, q, partials and state; for the power filter one
// spare iterate.
struct RgWs {
  Operator op;
  void *r, *r_old, *s, *p, *q, *tmp;
  double* partials;
  CgState* st;
};

size_t carve_rg(const gsf_operator_desc* d, int method, char* base, RgWs* w) {
  Carve c{base};
  if (d->kind == GSF_BF) {
    // the fused passes evaluate the weights of eq. (2) where they are used:
    // of the operator only the grid, the descriptor and the degrees
    layout_operator(d, &w->op, nullptr);
    w->op.deg = (double*)c.take((size_t)w->op.n * sizeof(double));
  } else {
    char* ob = (char*)c.take(align_up(layout_operator(d, nullptr, nullptr), kAlign));
    layout_operator(d, &w->op, ob);
  }
  const size_t v = (size_t)w->op.n * w->op.elem;
  if (method == GSF_METHOD_POWER) {
    w->tmp = c.take(v);
    return c.off;
  }
  w->r = c.take(v);
  w->r_old = c.take(v);
  w->s = c.take(v);
  w->p = c.take(v);
  w->q = c.take(v);
  int nb = vec_blocks(w->op.n);
  if (d->kind == GSF_BF) {
    const int ab = rg_bf_blocks(w->op);
    nb = ab > nb ? ab : nb;
  }
  w->partials = (double*)c.take((size_t)nb * 2 * sizeof(double));
  w->st = (CgState*)c.take(sizeof(CgState));
  return c.off;
}

gsf_status build_any(const Operator& op, const void* guidance, hipStream_t s) {
  return op.desc.kind == GSF_BF ? launch_bf_build(op, guidance, s) : launch_gf_build(op, guidance, s);
}

struct LobWs {
  void *X, *W, *P, *AX, *AW, *AP;
  void* Z;               // learned preconditioner output T(R)
  double* net_partials;  // per-tile partials of the preconditioner
  double* gram_partials;
  double* gram_level2;
  double* C;
  double* theta;
  double* vpart;
  LobpcgState* st;
};

// Workgroups of the Gram kernel: 256 points each (64 per wave) up to
// kGramBlocks (512); at n = 4096 the Gram took 9.5 us on 4 workgroups of 1024.
int gram_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > kGramBlocks) b = kGramBlocks;
  return (int)b;
}

size_t carve_lob(const Operator& op, int m, char* base, LobWs* w) {
  Carve c{base};
  const size_t blk = (size_t)op.n * m * op.elem;
  w->X = c.take(blk);
  w->W = c.take(blk);
  w->P = c.take(blk);
  w->AX = c.take(blk);
  w->AW = c.take(blk);
  w->AP = c.take(blk);
  w->gram_partials = (double*)c.take((size_t)gram_blocks(op.n) * 7 * 256 * sizeof(double));
  w->gram_level2 = (double*)c.take((size_t)kGramLevel2Doubles * sizeof(double));
  w->C = (double*)c.take(24 * 8 * sizeof(double));
  w->theta = (double*)c.take(8 * sizeof(double));
  w->vpart = (double*)c.take((size_t)vec_blocks(op.n) * 17 * sizeof(double));
  w->st = (LobpcgState*)c.take(sizeof(LobpcgState));
  w->Z = c.take(blk);
  w->net_partials = (double*)c.take((size_t)net_tiles(op.rows, op.cols) * 3 * m * sizeof(double));
  return c.off;
}

StartDegrees start_degrees(int ndim, int m) {
  StartDegrees d{};
  if (ndim == 1) {
    for (int j = 0; j < m; ++j) {
      d.a[j] = 0;
      d.b[j] = j;
    }
    return d;
  }
  int j = 0;
  for (int s = 0; j < m; ++s)
    for (int a = 0; a <= s && j < m; ++a, ++j) {
      d.a[j] = a;
      d.b[j] = s - a;
    }
  return d;
}

gsf_status hip_ok(hipError_t e) { return device_status(e); }

#define GSF_TRY(expr)                 \
  do {                                \
    gsf_status _st = (expr);          \
    if (_st != GSF_OK) return _st;    \
  } while (0)

// Stops a solver's host loop once its device state reports convergence or
// breakdown: every kPoll steps the state's `active` flag is copied to pinned
// host memory behind the queued work, and the copy from the previous poll is
// read (so kPoll steps stay queued on the GPU while the host waits).  Off
// under stream capture and when the caller asked for no info (no host sync).
class Poller {
 public:
  static constexpr int kPoll = 16;
  Poller(hipStream_t s, const int32_t* flag, bool enabled) : s_(s), flag_(flag) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!enabled || hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    static thread_local int32_t* pinned = nullptr;
    if (pinned == nullptr && hipHostMalloc((void**)&pinned, 64, hipHostMallocDefault) != hipSuccess) {
      pinned = nullptr;
      return;
    }
    host_ = pinned;
    for (int i = 0; i < 2; ++i)
      if (hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming) != hipSuccess) return;
    on_ = true;
  }
  ~Poller() {
    if (pending_ >= 0) (void)hipEventSynchronize(ev_[pending_]);
    for (int i = 0; i < 2; ++i)
      if (ev_[i]) (void)hipEventDestroy(ev_[i]);
  }
  // false once the solver is known to have stopped (call before step k)
  bool keep_going(int k) {
    if (!on_ || k == 0 || k % kPoll != 0) return true;
    if (pending_ >= 0) {
      if (hipEventSynchronize(ev_[pending_]) != hipSuccess) return true;
      if (host_[pending_] == 0) return false;
    }
    const int slot = (k / kPoll) & 1;
    if (hipMemcpyAsync(&host_[slot], flag_, sizeof(int32_t), hipMemcpyDeviceToHost, s_) != hipSuccess ||
        hipEventRecord(ev_[slot], s_) != hipSuccess) {
      on_ = false;
      return true;
    }
    pending_ = slot;
    return true;
  }

 private:
  hipStream_t s_;
  const int32_t* flag_;
  int32_t* host_ = nullptr;
  hipEvent_t ev_[2] = {nullptr, nullptr};
  int pending_ = -1;
  bool on_ = false;
};

}  // namespace

// Host description of an operator without device memory (pointers null):
// used to size workspaces before anything is built.
gsf_status describe_operator(const gsf_operator_desc* d, Operator* out) {
  GSF_TRY(validate_desc(d));
  layout_operator(d, out, nullptr);
  return GSF_OK;
}

size_t solver_bytes(const Operator& op, int method, int m) {
  if (method == GSF_METHOD_POWER) return 2 * align_up((size_t)op.n * op.elem, 256);
  if (method == GSF_METHOD_CG) {
    CgWs w;
    return carve_cg(op, nullptr, &w);
  }
  LobWs w;
  return carve_lob(op, m, nullptr, &w);
}

CgState* cg_state_ptr(const Operator& op, void* ws) {
  CgWs w;
  carve_cg(op, (char*)ws, &w);
  return w.st;
}

LobpcgState* lob_state_ptr(const Operator& op, int m, void* ws) {
  LobWs w;
  carve_lob(op, m, (char*)ws, &w);
  return w.st;
}

gsf_status launch_lob_state_init(LobpcgState* dst, const LobpcgState& v, hipStream_t s) {
  lob_state_init_kernel<<<1, 1, 0, s>>>(dst, v);
  return hip_ok(hipGetLastError());
}
gsf_status launch_cg_state_init(CgState* dst, const CgState& v, hipStream_t s) {
  cg_state_init_kernel<<<1, 1, 0, s>>>(dst, v);
  return hip_ok(hipGetLastError());
}

}  // namespace gsf

using namespace gsf;

extern "C" {

gsf_status gsf_block_gram_workspace_bytes(int64_t n, size_t* bytes);

int gsf_version(void) { return 1; }

int gsf_last_device_error(void) {
  const int e = g_last_device_error;
  g_last_device_error = 0;
  return e;
}

const char* gsf_device_error_string(int code) { return hipGetErrorString((hipError_t)code); }

const char* gsf_status_string(int status) {
  switch (status) {
    case GSF_OK: return "ok";
    case GSF_EINVAL: return "invalid argument";
    case GSF_ENOMEM: return "workspace too small";
    case GSF_EDEVICE: return "HIP runtime error";
    case GSF_ENOTCONV: return "tolerance not reached";
    case GSF_EBREAKDOWN: return "iteration broke down";
    case GSF_ESCRATCH: return "problem larger than the static scratch";
    default: return "unknown status";
  }
}

gsf_status gsf_operator_workspace_bytes(const gsf_operator_desc* desc, size_t* bytes) {
  if (bytes == nullptr) return GSF_EINVAL;
  GSF_TRY(validate_desc(desc));
  *bytes = layout_operator(desc, nullptr, nullptr);
  return GSF_OK;
}

gsf_status gsf_build_operator(const gsf_operator_desc* desc, const void* guidance, void* ws, size_t ws_bytes,
                              void* stream, gsf_operator** out) {
  clear_stale_errors();
  if (out == nullptr || guidance == nullptr || ws == nullptr) return GSF_EINVAL;
  GSF_TRY(validate_desc(desc));
  if (ws_bytes < layout_operator(desc, nullptr, nullptr)) return GSF_ENOMEM;
  gsf_operator* h = new (std::nothrow) gsf_operator;
  if (h == nullptr) return GSF_EDEVICE;
  layout_operator(desc, &h->op, (char*)ws);
  hipStream_t s = (hipStream_t)stream;
  gsf_status st = desc->kind == GSF_BF ? launch_bf_build(h->op, guidance, s) : launch_gf_build(h->op, guidance, s);
  if (st != GSF_OK) {
    delete h;
    return st;
  }
  *out = h;
  return GSF_OK;
}

gsf_status gsf_operator_get_layout(const gsf_operator* h, gsf_operator_layout* out) {
  if (h == nullptr || out == nullptr) return GSF_EINVAL;
  const Operator& op = h->op;
  std::memset(out, 0, sizeof(*out));
  out->kind = op.desc.kind;
  out->ndim = op.desc.ndim;
  out->prec = op.desc.prec;
  out->radius = op.desc.radius;
  out->n = op.n;
  out->nplanes = op.nplanes;
  out->planes = op.desc.kind == GSF_BF ? (const char*)op.planes + op.ppad * op.elem : nullptr;
  out->plane_stride = op.desc.kind == GSF_BF ? op.pstride : 0;
  out->inv_sqrt_d = op.diag;
  out->sqrt_d = op.sqd;
  out->degree = op.deg;
  out->guidance = op.g;
  out->mu = op.mu;
  out->inv = op.inv;
  return GSF_OK;
}

void gsf_destroy_operator(gsf_operator* h) { delete h; }

gsf_status gsf_apply(const gsf_operator* h, int form, int m, const void* x, int64_t ldx, void* y, int64_t ldy,
                     void* stream) {
  clear_stale_errors();
  if (h == nullptr || x == nullptr || y == nullptr) return GSF_EINVAL;
  if (form != GSF_FORM_N && form != GSF_FORM_LSYM && form != GSF_FORM_RW && form != GSF_FORM_L) return GSF_EINVAL;
  if (m < 1 || m > kMaxBlock) return GSF_EINVAL;
  if (ldx == 0) ldx = m;
  if (ldy == 0) ldy = m;
  if (ldx < m || ldy < m) return GSF_EINVAL;
  const Operator& op = h->op;
  // extents: (n - 1) ld + m elements
  const size_t xb = ((size_t)(op.n - 1) * (size_t)ldx + (size_t)m) * op.elem;
  const size_t yb = ((size_t)(op.n - 1) * (size_t)ldy + (size_t)m) * op.elem;
  const char *xa = (const char*)x, *ya = (const char*)y;
  if (xa < ya + yb && ya < xa + xb) return GSF_EINVAL;  // overlap
  return apply_any(op, form, m, x, ldx, y, ldy, nullptr, nullptr, (hipStream_t)stream);
}

gsf_status gsf_apply_joint(const gsf_operator* h, int form, int m, const void* x, void* y, const void* x2, void* y2,
                           void* stream) {
  clear_stale_errors();
  if (h == nullptr || x == nullptr || y == nullptr || x2 == nullptr || y2 == nullptr) return GSF_EINVAL;
  if (form != GSF_FORM_N && form != GSF_FORM_LSYM && form != GSF_FORM_RW && form != GSF_FORM_L) return GSF_EINVAL;
  if (m < 1 || m > kMaxBlock) return GSF_EINVAL;
  const Operator& op = h->op;
  const size_t bytes = (size_t)op.n * m * op.elem, b1 = (size_t)op.n * op.elem;
  auto overlap = [](const void* a, size_t na, const void* b, size_t nb) {
    const char *pa = (const char*)a, *pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
  };
  if (overlap(x, bytes, y, bytes) || overlap(x, bytes, y2, b1) || overlap(x2, b1, y, bytes) ||
      overlap(x2, b1, y2, b1) || overlap(y, bytes, y2, b1))
    return GSF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (launch_bf_apply_joint(op, form, m, x, m, y, m, x2, 1, y2, 1, nullptr, nullptr, s))
    return hip_ok(hipGetLastError());
  GSF_TRY(apply_any(op, form, m, x, m, y, m, nullptr, nullptr, s));
  return apply_any(op, form, 1, x2, 1, y2, 1, nullptr, nullptr, s);
}

gsf_status gsf_solver_workspace_bytes(const gsf_operator* h, int method, int m, size_t* bytes) {
  if (h == nullptr || bytes == nullptr) return GSF_EINVAL;
  const Operator& op = h->op;
  if (method == GSF_METHOD_POWER) {
    if (m < 1 || m > kMaxBlock) return GSF_EINVAL;
    *bytes = 2 * align_up((size_t)op.n * m * op.elem, 256);
  } else if (method == GSF_METHOD_CG) {
    if (m < 1 || m > kMaxBlock) return GSF_EINVAL;
    CgWs w;
    BcgWs bw;
    const size_t a = carve_cg(op, nullptr, &w), b = carve_bcg(op, m, nullptr, &bw);
    *bytes = a > b ? a : b;
  } else if (method == GSF_METHOD_LOBPCG) {
    if (m < 1 || m > kMaxBlock) return GSF_EINVAL;
    LobWs w;
    *bytes = carve_lob(op, m, nullptr, &w);
  } else {
    return GSF_EINVAL;
  }
  return GSF_OK;
}

gsf_status gsf_power_filter(const gsf_operator* h, const void* x0, void* x_out, int kmax, void* ws,
                            size_t ws_bytes, void* stream) {
  clear_stale_errors();
  if (h == nullptr || x0 == nullptr || x_out == nullptr || kmax < 0) return GSF_EINVAL;
  const Operator& op = h->op;
  const size_t v = align_up((size_t)op.n * op.elem, 256);
  if (kmax > 0 && (ws == nullptr || ws_bytes < 2 * v)) return GSF_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  if (kmax == 0) return hip_ok(hipMemcpyAsync(x_out, x0, (size_t)op.n * op.elem, hipMemcpyDeviceToDevice, s));
  char* a = (char*)ws;
  char* b = a + v;
  GSF_TRY(launch_scale(op, x0, a, 0, s));  // z = D^1/2 x
  for (int k = 0; k < kmax; ++k) {
    GSF_TRY(apply_any(op, GSF_FORM_N, 1, a, 1, b, 1, nullptr, nullptr, s));
    char* t = a;
    a = b;
    b = t;
  }
  return launch_scale(op, a, x_out, 1, s);  // x = D^-1/2 z
}

gsf_status gsf_power_filter_block(const gsf_operator* h, int m, const void* x0, void* x_out, int kmax, void* ws,
                                  size_t ws_bytes, void* stream) {
  clear_stale_errors();
  if (h == nullptr || x0 == nullptr || x_out == nullptr || kmax < 0 || m < 1 || m > kMaxBlock) return GSF_EINVAL;
  const Operator& op = h->op;
  const size_t v = align_up((size_t)op.n * m * op.elem, 256);
  if (kmax > 0 && (ws == nullptr || ws_bytes < 2 * v)) return GSF_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  if (kmax == 0)
    return hip_ok(hipMemcpyAsync(x_out, x0, (size_t)op.n * m * op.elem, hipMemcpyDeviceToDevice, s));
  char* a = (char*)ws;
  char* b = a + v;
  GSF_TRY(launch_bscale(op, m, x0, a, 0, s));  // z = D^1/2 x, column by column
  for (int k = 0; k < kmax; ++k) {
    GSF_TRY(apply_any(op, GSF_FORM_N, m, a, m, b, m, nullptr, nullptr, s));
    char* t = a;
    a = b;
    b = t;
  }
  return launch_bscale(op, m, a, x_out, 1, s);
}

gsf_status gsf_cg_filter_block(const gsf_operator* h, int m, const void* x0, void* x_out, int kmax, double tol,
                               void* ws, size_t ws_bytes, gsf_cg_info* info, void* stream) {
  clear_stale_errors();
  if (h == nullptr || x0 == nullptr || x_out == nullptr || kmax < 0 || !(tol >= 0.0) || !std::isfinite(tol))
    return GSF_EINVAL;
  if (m < 1 || m > kMaxBlock) return GSF_EINVAL;
  const Operator& op = h->op;
  BcgWs w;
  if (ws == nullptr || ws_bytes < carve_bcg(op, m, nullptr, &w)) return GSF_ENOMEM;
  carve_bcg(op, m, (char*)ws, &w);
  hipStream_t s = (hipStream_t)stream;
  BlockCgState init{};
  init.m = m;
  init.active = 1;
  for (int c = 0; c < m; ++c) {
    init.col[c].tol = tol;
    init.col[c].tau = breakdown_tau(op.desc.prec);
  }
  GSF_TRY(launch_bcg_state_init(w.st, init, s));
  GSF_TRY(launch_bscale(op, m, x0, w.z, 0, s));
  GSF_TRY(apply_any(op, GSF_FORM_LSYM, m, w.z, m, w.r, m, nullptr, nullptr, s));
  GSF_TRY(launch_bcg(0, op, m, w.z, w.r, w.p, w.q, w.partials, w.st, s));
  Poller poll(s, &w.st->active, info != nullptr && tol > 0.0);
  for (int k = 1; k <= kmax; ++k) {
    if (!poll.keep_going(k - 1)) break;
    GSF_TRY(launch_bcg(1, op, m, w.z, w.r, w.p, w.q, w.partials, w.st, s));
    GSF_TRY(apply_any(op, GSF_FORM_LSYM, m, w.p, m, w.q, m, nullptr, nullptr, s));
    GSF_TRY(launch_bcg(2, op, m, w.z, w.r, w.p, w.q, w.partials, w.st, s));
    GSF_TRY(launch_bcg(3, op, m, w.z, w.r, w.p, w.q, w.partials, w.st, s));
  }
  GSF_TRY(launch_bscale(op, m, w.z, x_out, 1, s));
  if (info == nullptr) return GSF_OK;
  BlockCgState host{};
  GSF_TRY(hip_ok(hipMemcpyAsync(&host, w.st, sizeof(host), hipMemcpyDeviceToHost, s)));
  GSF_TRY(hip_ok(hipStreamSynchronize(s)));
  gsf_status first = GSF_OK;
  for (int c = 0; c < m; ++c) {
    const CgState& cs = host.col[c];
    gsf_status status = (gsf_status)cs.status;
    if (status == GSF_OK && tol > 0.0 && cs.active && !(cs.rho <= cs.tol2)) status = GSF_ENOTCONV;
    info[c].iters = cs.iters;
    info[c].status = status;
    info[c].res0 = cs.res0;
    info[c].res = std::sqrt(cs.rho > 0.0 ? cs.rho : 0.0);
    if (first == GSF_OK) first = status;
  }
  return first;
}

gsf_status gsf_srgb_to_lab(int prec, int64_t n, const void* rgb, void* lab, void* stream) {
  clear_stale_errors();
  if (n < 0 || (prec != GSF_F32 && prec != GSF_F64)) return GSF_EINVAL;
  if (n == 0) return GSF_OK;
  if (rgb == nullptr || lab == nullptr) return GSF_EINVAL;
  return launch_srgb_to_lab(prec, n, rgb, lab, (hipStream_t)stream);
}

namespace {

// The CG filter (Algorithm 2 in z-space) as a sequence of enqueued phases, so
// that the single filter and the joint CG + LOBPCG driver share them.
struct CgRun {
  const Operator& op;
  CgWs w;
  hipStream_t s;
  int nparts = 0;
  int steps = 0;  // steps issued
  CgRun(const Operator& o, char* ws, hipStream_t st) : op(o), s(st) { carve_cg(op, ws, &w); }
  // the start: z0, r0 = -L_sym z0 and the initial scalars (begin_pre, the
  // apply z -> r, begin_post; the joint driver applies z with the LOBPCG block)
  gsf_status begin(const void* x0, double tol) {
    GSF_TRY(begin_pre(x0, tol));
    GSF_TRY(apply_any(op, GSF_FORM_LSYM, 1, w.z, 1, w.r, 1, nullptr, nullptr, s));
    return begin_post();
  }
  gsf_status begin_pre(const void* x0, double tol) {
    CgState init{};
    init.tol = tol;
    init.tau = breakdown_tau(op.desc.prec);
    GSF_TRY(launch_cg_state_init(w.st, init, s));
    return launch_scale(op, x0, w.z, 0, s);
  }
  gsf_status begin_post() { return launch_cg_init(op, w.z, w.r, w.partials, w.st, s); }
  // step k (1-based): p from r (with beta from the last update's partials)
  gsf_status pre(int k) { return launch_cg_pbeta(op, w.r, w.p, w.partials2, w.st, k, s); }
  gsf_status apply() {  // q = L_sym p and the p^T q partials
    if (op.desc.kind == GSF_BF) return apply_any(op, GSF_FORM_LSYM, 1, w.p, 1, w.q, 1, w.partials, &nparts, s);
    GSF_TRY(apply_any(op, GSF_FORM_LSYM, 1, w.p, 1, w.q, 1, nullptr, nullptr, s));
    return launch_dot(op, w.p, w.q, w.partials, &nparts, w.st, s);
  }
  gsf_status post(int k) {  // alpha and the update of step k
    steps = k;
    return launch_cg_aupdate(op, w.z, w.r, w.p, w.q, w.partials, nparts, w.partials2, w.st, k, s);
  }
  // step k's update (or direction) phase, to run as extra workgroups of
  // another launch on s (the update reads the p^T q partials of the last apply)
  CgStepArgs phase(int k) const {
    CgStepArgs a{};
    a.prec = op.desc.prec;
    a.nblk = cg_step_blocks(op.n);
    a.k = k;
    a.ndots = nparts;
    a.z = w.z;
    a.r = w.r;
    a.p = w.p;
    a.q = w.q;
    a.n = op.n;
    a.dots = w.partials;
    a.upd = w.partials2;
    a.st = w.st;
    return a;
  }
  gsf_status finish(void* x_out, double tol, gsf_cg_info* info) {
    if (steps > 0) GSF_TRY(launch_cg_close(op, w.partials2, w.st, s));
    GSF_TRY(launch_scale(op, w.z, x_out, 1, s));
    return report(tol, info);
  }
  gsf_status report(double tol, gsf_cg_info* info) {  // info from the device state
    if (info == nullptr) return GSF_OK;
    CgState host{};
    GSF_TRY(hip_ok(hipMemcpyAsync(&host, w.st, sizeof(host), hipMemcpyDeviceToHost, s)));
    GSF_TRY(hip_ok(hipStreamSynchronize(s)));
    gsf_status status = (gsf_status)host.status;
    if (status == GSF_OK && tol > 0.0 && host.active && !(host.rho <= host.tol2)) status = GSF_ENOTCONV;
    info->iters = host.iters;
    info->status = status;
    info->res0 = host.res0;
    info->res = std::sqrt(host.rho > 0.0 ? host.rho : 0.0);
    return status;
  }
};

// Shifted-solve preconditioner: for every column j of the n x m block R,
// Z[:, j] = y after T->inner CG steps on (L_sym + alpha I) y = R[:, j] from
// y = 0 (the recurrences of gsf_shifted_cg with tol 0: every step runs unless
// the column is zero or p^T q <= 0 stops it early).
}  // namespace
}  // extern "C"

namespace gsf {
gsf_status shifted_precond_apply(const gsf_precond* T, int m, const void* R, void* Z, hipStream_t s) {
  const Operator& op = T->op->op;
  CgWs cw;
  carve_cg(op, (char*)T->mem, &cw);
  void* y = cw.z;
  for (int j = 0; j < m; ++j) {
    CgState init{};
    init.tol = 0.0;
    GSF_TRY(launch_cg_state_init(cw.st, init, s));
    GSF_TRY(launch_scg_init(op.desc.prec, (const char*)R + (size_t)j * op.elem, m, y, cw.r, op.n, cw.partials,
                            cw.st, s));
    for (int k = 1; k <= T->inner; ++k) {
      GSF_TRY(launch_cg_pupdate(op, cw.r, cw.p, cw.st, s));
      GSF_TRY(apply_any(op, GSF_FORM_LSYM, 1, cw.p, 1, cw.q, 1, nullptr, nullptr, s));
      int nparts = 0;
      GSF_TRY(launch_scg_shift(op.desc.prec, cw.p, cw.q, op.n, T->alpha, cw.partials, &nparts, cw.st, s));
      GSF_TRY(launch_cg_alpha(cw.partials, nparts, cw.st, s));
      GSF_TRY(launch_cg_update(op, y, cw.r, cw.p, cw.q, cw.partials, cw.st, s));
    }
    GSF_TRY(launch_col_copy(op.desc.prec, y, 1, (char*)Z + (size_t)j * op.elem, m, op.n, s));
  }
  return GSF_OK;
}
}  // namespace gsf

extern "C" {
namespace {

// The LOBPCG filter (Algorithm 3, block form) as enqueued phases.
struct LobRun {
  const Operator& op;
  LobWs w;
  hipStream_t s;
  int m;
  bool constraint;
  const gsf_precond* T;
  LobArgs a{};
  GramArgs g{};
  RRArgs rr{};
  int nb = 0;
  StartDegrees deg{};
  bool fold = false, pending = false;
  // the joint driver's CG phases carried by the next post() (nullable)
  const CgStepArgs* cg_update = nullptr;
  const CgStepArgs* cg_direction = nullptr;
  LobRun(const Operator& o, int m_, bool con, const gsf_precond* T_, char* ws, hipStream_t st)
      : op(o), s(st), m(m_), constraint(con), T(T_) {
    carve_lob(op, m, ws, &w);
  }
  // the start (begin_pre: state, X0; the apply X0 -> AX; begin_post: the
  // start-block Rayleigh-Ritz step and update; the joint driver applies X0
  // together with the CG start vector)
  gsf_status begin(const void* x0, void* x_out, void* ritz_vecs, double tol) {
    GSF_TRY(begin_pre(x0, x_out, ritz_vecs, tol));
    GSF_TRY(apply_any(op, GSF_FORM_LSYM, m, w.X, m, w.AX, m, nullptr, nullptr, s));
    return begin_post();
  }
  gsf_status begin_pre(const void* x0, void* x_out, void* ritz_vecs, double tol) {
    LobpcgState init{};
    init.tol = tol;
    init.drop_tol = drop_tol_of(op.desc.prec);
    init.zero_tol = breakdown_tau(op.desc.prec);
    init.m = m;
    init.active = 1;
    init.status = GSF_OK;
    for (int j = 0; j < m; ++j) init.cid[j * m + j] = 1.0;
    GSF_TRY(launch_lob_state_init(w.st, init, s));
    a.prec = op.desc.prec;
    a.n = op.n;
    a.rows = op.rows;
    a.cols = op.cols;
    a.ndim = op.desc.ndim;
    a.m = m;
    a.constraint = constraint ? 1 : 0;
    a.x0 = x0;
    a.sqd = op.sqd;
    a.X = w.X;
    a.W = w.W;
    a.P = w.P;
    a.AX = w.AX;
    a.AW = w.AW;
    a.AP = w.AP;
    a.C = w.C;
    a.vpart = w.vpart;
    a.st = w.st;
    a.xout = x_out;
    a.ritz = ritz_vecs;
    nb = vec_blocks(op.n);
    deg = start_degrees(op.desc.ndim, m);
    g.m = m;
    g.n = op.n;
    g.nparts = gram_blocks(op.n);
    g.partials = w.gram_partials;
    g.level2 = w.gram_level2;
    g.active = &w.st->active;
    rr.C = w.C;
    rr.theta = w.theta;
    rr.st = w.st;
    rr.drop_tol = init.drop_tol;
    rr.zero_tol = init.zero_tol;
    if (constraint) GSF_TRY(lob_launch_ynorm(a, nb, s));
    GSF_TRY(lob_launch_mkernel(0, a, nb, m, 1, deg, s));  // X0
    if (constraint) GSF_TRY(lob_launch_project(a, w.X, nb, s));
    return GSF_OK;
  }
  gsf_status begin_post() {
    // start-block Rayleigh-Ritz
    g.ns = m;
    g.S[0] = w.X;
    g.AS[0] = w.AX;
    rr.init = 1;
    GSF_TRY(lob_launch_gram(g, rr, op.desc.prec, s));
    rr.init = 0;
    GSF_TRY(lob_launch_mkernel(1, a, nb, m, 1, deg, s));  // X = X0 C, AX, W = R
    // Without a preconditioner network or the constraint nothing between an
    // update and the next Rayleigh-Ritz step reads the residual norms, so that
    // step finalizes them (one launch less per iteration); the last update is
    // finalized at the end.
    fold = T == nullptr && !constraint;
    return GSF_OK;
  }
  gsf_status pre() {  // W = T(R), or the projected R
    if (T != nullptr && T->kind == kPrecondShifted) {
      GSF_TRY(shifted_precond_apply(T, m, w.W, w.Z, s));
      GSF_TRY(launch_tz_partials(op.desc.prec, w.W, w.Z, constraint ? op.sqd : nullptr, op.rows, op.cols, m, w.st,
                                 w.net_partials, s));
      return net_lob_select(op.desc.prec, op.rows, op.cols, m, constraint ? 1 : 0, w.W, w.Z, op.sqd,
                            w.net_partials, tz_blocks(op.rows, op.cols), w.st, s);
    }
    if (T != nullptr) {
      GSF_TRY(net_infer(op.desc.prec, T->w, op.rows, op.cols, m, w.W, w.Z, T->g, constraint ? op.sqd : nullptr,
                        w.st->res, w.st, w.net_partials, s));
      return net_lob_select(op.desc.prec, op.rows, op.cols, m, constraint ? 1 : 0, w.W, w.Z, op.sqd,
                            w.net_partials, net_tiles(op.rows, op.cols), w.st, s);
    }
    if (constraint) return lob_launch_project(a, w.W, nb, s);
    return GSF_OK;
  }
  gsf_status apply() { return apply_any(op, GSF_FORM_LSYM, m, w.W, m, w.AW, m, nullptr, nullptr, s); }
  gsf_status post(int k) {  // Rayleigh-Ritz on [X, W, P] and the update
    const int ns = (k == 0) ? 2 * m : 3 * m;
    g.ns = ns;
    g.S[0] = w.X;
    g.S[1] = w.W;
    g.S[2] = w.P;
    g.AS[0] = w.AX;
    g.AS[1] = w.AW;
    g.AS[2] = w.AP;
    rr.fin_partials = pending ? w.vpart : nullptr;
    rr.fin_nparts = nb;
    rr.fin_stride = 2 * m;
    GSF_TRY(lob_launch_gram(g, rr, op.desc.prec, s, cg_update));
    if ((k + 1) % kAxRefresh != 0) {
      GSF_TRY(lob_launch_mkernel(fold ? 4 : 1, a, nb, ns, 0, deg, s, cg_direction));
    } else {
      // every kAxRefresh steps AX = A X explicitly (the update's linear
      // combinations accumulate rounding that would floor the residual), then
      // the residual of that AX: it, not the carried one, makes this step's
      // convergence decision
      GSF_TRY(lob_launch_mkernel(4, a, nb, ns, 0, deg, s, cg_direction));
      GSF_TRY(apply_any(op, GSF_FORM_LSYM, m, w.X, m, w.AX, m, nullptr, nullptr, s));
      LobArgs ai = a;
      ai.C = reinterpret_cast<const double*>(reinterpret_cast<const char*>(w.st) + offsetof(LobpcgState, cid));
      GSF_TRY(lob_launch_mkernel(fold ? 7 : 6, ai, nb, m, 1, deg, s));
    }
    pending = fold;
    return GSF_OK;
  }
  gsf_status finish(double tol, gsf_lobpcg_info* info) {
    if (pending) GSF_TRY(lob_launch_mkernel(5, a, nb, m, 0, deg, s));
    pending = false;
    GSF_TRY(lob_launch_mkernel(2, a, nb, m, 0, deg, s));  // X^T z0, Y^T z0
    GSF_TRY(lob_launch_mkernel(3, a, nb, m, 0, deg, s));  // x_out
    if (info == nullptr) return GSF_OK;
    LobpcgState host{};
    GSF_TRY(hip_ok(hipMemcpyAsync(&host, w.st, sizeof(host), hipMemcpyDeviceToHost, s)));
    GSF_TRY(hip_ok(hipStreamSynchronize(s)));
    gsf_status status = (gsf_status)host.status;
    double mx = 0.0;
    for (int j = 0; j < m; ++j) mx = host.res[j] > mx ? host.res[j] : mx;
    if (status == GSF_OK && tol > 0.0 && mx > tol) status = GSF_ENOTCONV;
    info->iters = host.iters;
    info->status = status;
    info->dropped = host.dropped;
    info->m = m;
    info->fallbacks = host.fallbacks;
    info->pad = 0;
    for (int j = 0; j < 8; ++j) {
      info->res[j] = j < m ? host.res[j] : 0.0;
      info->theta[j] = j < m ? host.theta[j] : 0.0;
    }
    return status;
  }
};

}  // namespace

namespace {

// The CG filter on a carved workspace `ws` (arguments already validated).
// poll: the host may stop issuing steps once the device state reports the
// stop (pinned host memory, allocated once per thread); without it every
// step is issued and the steps after a stop are no-ops on the device.
gsf_status cg_filter_run(const Operator& op, const void* x0, void* x_out, int kmax, double tol, char* ws,
                         gsf_cg_info* info, hipStream_t stream, bool poll_host) {
  CgRun cg(op, ws, stream);
  {
    // a 1D BF signal that fits in one workgroup: the whole filter in one launch
    CgState init{};
    init.tol = tol;
    init.tau = breakdown_tau(op.desc.prec);
    if (op.desc.kind == GSF_BF && op.desc.ndim == 1 && op.n <= 8192) {
      GSF_TRY(launch_cg_state_init(cg.w.st, init, cg.s));
      if (launch_cg_small(op, x0, x_out, kmax, cg.w.st, cg.s)) {
        GSF_TRY(hip_ok(hipGetLastError()));
        return cg.report(tol, info);
      }
    }
  }
  GSF_TRY(cg.begin(x0, tol));
  Poller poll(cg.s, &cg.w.st->active, poll_host && info != nullptr && tol > 0.0);
  for (int k = 1; k <= kmax; ++k) {
    if (!poll.keep_going(k - 1)) break;
    GSF_TRY(cg.pre(k));
    GSF_TRY(cg.apply());
    GSF_TRY(cg.post(k));
  }
  return cg.finish(x_out, tol, info);
}

// Workspace of gsf_cg_filter_noalloc: one array per device, in the code
// object's device memory, kept until the process ends.  Host code must not
// pass `scratch` itself to a kernel (on the host the name is a stand-in, not
// a device address): the address comes from hipGetSymbolAddress, taken once
// per device with that device current.
constexpr size_t kNoAllocScratchBytes = (size_t)GSF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_address[kMaxDevices] = {};

gsf_status scratch_address(void** out) {
  int dev = -1;
  GSF_TRY(hip_ok(hipGetDevice(&dev)));
  if (dev < 0 || dev >= kMaxDevices) return GSF_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_address[dev] == nullptr) {
    void* p = nullptr;
    GSF_TRY(hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))));
    if (p == nullptr) return GSF_EDEVICE;
    g_scratch_address[dev] = p;
  }
  *out = g_scratch_address[dev];
  return GSF_OK;
}

}  // namespace

gsf_status gsf_cg_filter(const gsf_operator* h, const void* x0, void* x_out, int kmax, double tol, void* ws,
                         size_t ws_bytes, gsf_cg_info* info, void* stream) {
  clear_stale_errors();
  if (h == nullptr || x0 == nullptr || x_out == nullptr || kmax < 0 || !(tol >= 0.0) || !std::isfinite(tol))
    return GSF_EINVAL;
  const Operator& op = h->op;
  CgWs w0;
  if (ws == nullptr || ws_bytes < carve_cg(op, nullptr, &w0)) return GSF_ENOMEM;
  return cg_filter_run(op, x0, x_out, kmax, tol, (char*)ws, info, (hipStream_t)stream, true);
}

gsf_status gsf_cg_filter_noalloc(const gsf_operator* h, const void* x0, void* x_out, int kmax, double tol,
                                 gsf_cg_info* info, void* stream) {
  clear_stale_errors();
  if (h == nullptr || x0 == nullptr || x_out == nullptr || kmax < 0 || !(tol >= 0.0) || !std::isfinite(tol))
    return GSF_EINVAL;
  const Operator& op = h->op;
  CgWs w0;
  if (carve_cg(op, nullptr, &w0) > kNoAllocScratchBytes) return GSF_ESCRATCH;
  void* ws = nullptr;
  GSF_TRY(scratch_address(&ws));
  return cg_filter_run(op, x0, x_out, kmax, tol, (char*)ws, info, (hipStream_t)stream, false);
}

gsf_status gsf_lobpcg_filter(const gsf_operator* h, const void* x0, void* x_out, int m, int kmax, double tol,
                             int constraint, const gsf_precond* T, void* ritz_vecs, double* ritz_vals_host, void* ws,
                             size_t ws_bytes, gsf_lobpcg_info* info, void* stream) {
  clear_stale_errors();
  if (h == nullptr || x0 == nullptr || x_out == nullptr || kmax < 0 || !(tol >= 0.0) || !std::isfinite(tol))
    return GSF_EINVAL;
  if (m < 1 || m > kMaxBlock) return GSF_EINVAL;
  const Operator& op = h->op;
  if (T != nullptr && (T->n != op.n || T->rows != op.rows || T->cols != op.cols || T->prec != op.desc.prec))
    return GSF_EINVAL;
  LobWs w0;
  if (ws == nullptr || ws_bytes < carve_lob(op, m, nullptr, &w0)) return GSF_ENOMEM;
  LobRun lob(op, m, constraint != 0, T, (char*)ws, (hipStream_t)stream);
  GSF_TRY(lob.begin(x0, x_out, ritz_vecs, tol));
  Poller poll(lob.s, &lob.w.st->active, info != nullptr && tol > 0.0);
  for (int k = 0; k < kmax; ++k) {
    if (!poll.keep_going(k)) break;
    GSF_TRY(lob.pre());
    GSF_TRY(lob.apply());
    GSF_TRY(lob.post(k));
  }
  if (ritz_vals_host == nullptr) return lob.finish(tol, info);
  gsf_lobpcg_info local{};
  gsf_lobpcg_info* out = info != nullptr ? info : &local;
  const gsf_status st = lob.finish(tol, out);
  for (int j = 0; j < m; ++j) ritz_vals_host[j] = out->theta[j];
  return st;
}

// Joint CG + LOBPCG filters of one operator: step k of both runs shares one
// stencil pass, [A W | A p] from [W | p] (the CG vector as one more column of
// the LOBPCG block), where the operator offers a joint apply; so do the
// starts, [A X0 | L_sym z0].  Everything runs
// on the caller's stream: the CG update of step k runs as extra workgroups of
// the LOBPCG Rayleigh-Ritz launch (one workgroup of its own), and the
// direction of step k + 1 as extra workgroups of the LOBPCG update launch.
// (A second stream for the CG phases cost two event waits per step, each
// delaying the next launch by about 6 us.)
gsf_status gsf_joint_workspace_bytes(const gsf_operator* h, int m, size_t* bytes) {
  if (h == nullptr || bytes == nullptr || m < 1 || m > kMaxBlock) return GSF_EINVAL;
  CgWs cw;
  LobWs lw;
  *bytes = align_up(carve_cg(h->op, nullptr, &cw), kAlign) + carve_lob(h->op, m, nullptr, &lw);
  return GSF_OK;
}

gsf_status gsf_joint_filter(gsf_operator* h, const void* x0_cg, void* x_cg, int kmax_cg, const void* x0_lob,
                            void* x_lob, int m, int kmax_lob, int constraint, void* ws, size_t ws_bytes,
                            gsf_cg_info* cg_info, gsf_lobpcg_info* lob_info, void* stream) {
  clear_stale_errors();
  if (h == nullptr || x0_cg == nullptr || x_cg == nullptr || x0_lob == nullptr || x_lob == nullptr)
    return GSF_EINVAL;
  if (kmax_cg < 0 || kmax_lob < 0 || m < 1 || m > kMaxBlock) return GSF_EINVAL;
  size_t need = 0;
  GSF_TRY(gsf_joint_workspace_bytes(h, m, &need));
  if (ws == nullptr || ws_bytes < need) return GSF_ENOMEM;
  const Operator& op = h->op;
  hipStream_t s = (hipStream_t)stream;
  CgWs cw;
  char* base = (char*)ws;
  CgRun cg(op, base, s);
  LobRun lob(op, m, constraint != 0, nullptr, base + align_up(carve_cg(op, nullptr, &cw), kAlign), s);
  // the two starts share one stencil pass too: [X0 | z0] -> [A X0 | L_sym z0]
  GSF_TRY(cg.begin_pre(x0_cg, 0.0));
  GSF_TRY(lob.begin_pre(x0_lob, x_lob, nullptr, 0.0));
  const bool joint0 = launch_bf_apply_joint(op, GSF_FORM_LSYM, m, lob.w.X, m, lob.w.AX, m, cg.w.z, 1, cg.w.r, 1,
                                            cg.w.partials, &cg.nparts, s);
  if (joint0) {
    GSF_TRY(hip_ok(hipGetLastError()));
  } else {
    GSF_TRY(apply_any(op, GSF_FORM_LSYM, 1, cg.w.z, 1, cg.w.r, 1, nullptr, nullptr, s));
    GSF_TRY(apply_any(op, GSF_FORM_LSYM, m, lob.w.X, m, lob.w.AX, m, nullptr, nullptr, s));
  }
  GSF_TRY(cg.begin_post());
  GSF_TRY(lob.begin_post());
  const int kj = kmax_cg < kmax_lob ? kmax_cg : kmax_lob;
  bool p_ready = false;  // the next CG direction was formed in the last Rayleigh-Ritz launch
  for (int k = 0; k < kmax_cg || k < kmax_lob; ++k) {
    const bool both = k < kj;
    if (k < kmax_cg && !p_ready) GSF_TRY(cg.pre(k + 1));
    p_ready = false;
    if (k < kmax_lob) GSF_TRY(lob.pre());
    bool joint = false;
    if (both) {
      joint = launch_bf_apply_joint(op, GSF_FORM_LSYM, m, lob.w.W, m, lob.w.AW, m, cg.w.p, 1, cg.w.q, 1,
                                    cg.w.partials, &cg.nparts, s);
      if (joint) GSF_TRY(hip_ok(hipGetLastError()));
    }
    if (!joint) {
      if (k < kmax_cg) GSF_TRY(cg.apply());
      if (k < kmax_lob) GSF_TRY(lob.apply());
    }
    if (both) {
      // CG's update of step k + 1 in the Rayleigh-Ritz launch, the direction
      // of step k + 2 (when there is one) in the LOBPCG update launch
      const CgStepArgs upd = cg.phase(k + 1), dir = cg.phase(k + 2);
      cg.steps = k + 1;
      lob.cg_update = &upd;
      lob.cg_direction = k + 1 < kmax_cg ? &dir : nullptr;
      const gsf_status st = lob.post(k);
      lob.cg_update = lob.cg_direction = nullptr;
      GSF_TRY(st);
      p_ready = k + 1 < kmax_cg;
    } else {
      if (k < kmax_cg) GSF_TRY(cg.post(k + 1));
      if (k < kmax_lob) GSF_TRY(lob.post(k));
    }
  }
  gsf_status st_cg = cg.finish(x_cg, 0.0, cg_info);
  gsf_status st_lob = lob.finish(0.0, lob_info);
  if (st_cg != GSF_OK && st_cg != GSF_EBREAKDOWN) return st_cg;
  if (st_lob != GSF_OK) return st_lob;
  return st_cg;
}

// ---- re-guided (non-linear) filters -----------------------------------------
gsf_status gsf_reguided_workspace_bytes(const gsf_operator_desc* desc, int method, size_t* bytes) {
  if (bytes == nullptr || (method != GSF_METHOD_POWER && method != GSF_METHOD_CG)) return GSF_EINVAL;
  GSF_TRY(validate_desc(desc));
  if (desc_channels(*desc) != 1) return GSF_EINVAL;
  RgWs w;
  *bytes = carve_rg(desc, method, nullptr, &w);
  return GSF_OK;
}

gsf_status gsf_reguided_filter(const gsf_operator_desc* desc, int method, const void* x0, void* x_out, int kmax,
                               double tol, void* ws, size_t ws_bytes, gsf_cg_info* info, void* stream) {
  clear_stale_errors();
  if (x0 == nullptr || x_out == nullptr || kmax < 0 || !(tol >= 0.0) || !std::isfinite(tol)) return GSF_EINVAL;
  if (method != GSF_METHOD_POWER && method != GSF_METHOD_CG) return GSF_EINVAL;
  GSF_TRY(validate_desc(desc));
  if (desc_channels(*desc) != 1) return GSF_EINVAL;
  RgWs w;
  if (ws == nullptr || ws_bytes < carve_rg(desc, method, nullptr, &w)) return GSF_ENOMEM;
  carve_rg(desc, method, (char*)ws, &w);
  const Operator& op = w.op;
  hipStream_t s = (hipStream_t)stream;
  const size_t v = (size_t)op.n * op.elem;
  if (method == GSF_METHOD_POWER && launch_rg_power_small(*desc, x0, x_out, kmax, s)) {
    // a 1D BF signal that fits in one workgroup's LDS: all passes in one launch
    GSF_TRY(hip_ok(hipGetLastError()));
    if (info != nullptr) {
      info->iters = kmax;
      info->status = GSF_OK;
      info->res0 = 0.0;
      info->res = 0.0;
    }
    return GSF_OK;
  }
  if (x_out != x0) GSF_TRY(hip_ok(hipMemcpyAsync(x_out, x0, v, hipMemcpyDeviceToDevice, s)));
  // BF: fused passes (mode 0 degrees, 1 D^-1 W g, 2 L v) that evaluate the
  // weights of the current iterate's graph where they are used; GF: the
  // operator build (window statistics) and its apply
  const bool bf = op.desc.kind == GSF_BF;
  auto rebuild = [&]() -> gsf_status {
    return bf ? launch_rg_bf(op, 0, x_out, nullptr, nullptr, nullptr, nullptr, s) : build_any(op, x_out, s);
  };
  auto lap = [&](const void* v, void* y, double* dot, int* nparts) -> gsf_status {
    if (bf) return launch_rg_bf(op, 2, x_out, v, y, dot, nparts, s);
    return apply_any(op, GSF_FORM_L, 1, v, 1, y, 1, dot, nparts, s);
  };
  if (method == GSF_METHOD_POWER) {
    // x <- D(x)^-1 W(x) x, the graph built from the current iterate each pass
    char* a = (char*)x_out;
    char* b = (char*)w.tmp;
    for (int k = 0; k < kmax; ++k) {
      if (bf) {
        GSF_TRY(launch_rg_bf(op, 1, a, a, b, nullptr, nullptr, s));
      } else {
        GSF_TRY(build_any(op, a, s));
        GSF_TRY(apply_any(op, GSF_FORM_RW, 1, a, 1, b, 1, nullptr, nullptr, s));
      }
      char* t = a;
      a = b;
      b = t;
    }
    if (a != (char*)x_out) GSF_TRY(hip_ok(hipMemcpyAsync(x_out, a, v, hipMemcpyDeviceToDevice, s)));
    if (info != nullptr) {
      info->iters = kmax;
      info->status = GSF_OK;
      info->res0 = 0.0;
      info->res = 0.0;
    }
    return GSF_OK;
  }
  // Algorithm 2 in x-space with L_k, D_k from the current iterate x (x_out)
  CgState init{};
  init.tol = tol;
  init.tau = breakdown_tau(op.desc.prec);
  GSF_TRY(launch_cg_state_init(w.st, init, s));
  GSF_TRY(rebuild());
  GSF_TRY(lap(x_out, w.r, nullptr, nullptr));
  GSF_TRY(launch_rg_init(op, x_out, w.r, w.partials, w.st, s));
  Poller poll(s, &w.st->active, info != nullptr && tol > 0.0);
  for (int k = 1; k <= kmax; ++k) {
    if (!poll.keep_going(k - 1)) break;
    if (k > 1) GSF_TRY(rebuild());
    GSF_TRY(launch_rg_s_beta(op, w.r, w.r_old, w.s, w.partials, w.st, s));
    GSF_TRY(launch_cg_pupdate(op, w.s, w.p, w.st, s));
    int nparts = 0;
    if (bf) {
      GSF_TRY(lap(w.p, w.q, w.partials, &nparts));
    } else {
      GSF_TRY(lap(w.p, w.q, nullptr, nullptr));
      GSF_TRY(launch_dot(op, w.p, w.q, w.partials, &nparts, w.st, s));
    }
    GSF_TRY(launch_rg_alpha(w.partials, nparts, w.st, s));
    GSF_TRY(launch_rg_update(op, x_out, w.r, w.r_old, w.p, w.q, w.st, s));
  }
  if (info == nullptr) return GSF_OK;
  CgState host{};
  GSF_TRY(hip_ok(hipMemcpyAsync(&host, w.st, sizeof(host), hipMemcpyDeviceToHost, s)));
  GSF_TRY(hip_ok(hipStreamSynchronize(s)));
  gsf_status status = (gsf_status)host.status;
  if (status == GSF_OK && tol > 0.0 && host.active && !(host.rho <= host.tol2)) status = GSF_ENOTCONV;
  info->iters = host.iters;
  info->status = status;
  info->res0 = host.res0;
  info->res = std::sqrt(host.rho > 0.0 ? host.rho : 0.0);
  return status;
}

// ---- diagnostics: the Gram and Rayleigh-Ritz kernels on caller data ----------
// Gram pair (S^T A S, S^T S) of S = [S0, S1, S2] (nb blocks of m columns,
// point-major, element type prec) with AS = [A0, A1, A2]; results copied to
// host arrays GA, GB (ns x ns, ns = nb*m).  Synchronizes the stream.
gsf_status gsf_block_gram(int prec, int64_t n, int m, int nb, const void* const* S, const void* const* AS,
                          double* GA, double* GB, void* ws, size_t ws_bytes, void* stream) {
  clear_stale_errors();
  if (n < 1 || m < 1 || m > 8 || nb < 1 || nb > 3 || S == nullptr || AS == nullptr || GA == nullptr ||
      GB == nullptr)
    return GSF_EINVAL;
  if (prec != GSF_F32 && prec != GSF_F64) return GSF_EINVAL;
  size_t need = 0;
  gsf_block_gram_workspace_bytes(n, &need);
  if (ws == nullptr || ws_bytes < need) return GSF_ENOMEM;
  const int gb = gram_blocks(n);
  Carve w{(char*)ws};
  GramArgs g{};
  g.ns = nb * m;
  g.m = m;
  g.n = n;
  g.nparts = gb;
  g.partials = (double*)w.take((size_t)gb * 7 * 256 * 8);
  g.level2 = (double*)w.take((size_t)kGramLevel2Doubles * 8);
  double* gout = (double*)w.take(2 * 24 * 24 * 8);
  double* C = (double*)w.take(24 * 8 * 8);
  double* th = (double*)w.take(64);
  int* kept = (int*)w.take(256);
  for (int b = 0; b < nb; ++b) {
    g.S[b] = S[b];
    g.AS[b] = AS[b];
  }
  RRArgs r{};
  r.C = C;
  r.theta = th;
  r.drop_tol = 1e-10;
  r.zero_tol = 0.0;
  r.gram_out = gout;
  r.kept_out = kept;
  r.nkept_out = kept + 32;
  hipStream_t s = (hipStream_t)stream;
  GSF_TRY(lob_launch_gram(g, r, prec, s));
  const int ns = nb * m;
  GSF_TRY(hip_ok(hipMemcpyAsync(GA, gout, (size_t)ns * ns * 8, hipMemcpyDeviceToHost, s)));
  GSF_TRY(hip_ok(hipMemcpyAsync(GB, gout + ns * ns, (size_t)ns * ns * 8, hipMemcpyDeviceToHost, s)));
  return hip_ok(hipStreamSynchronize(s));
}

gsf_status gsf_block_gram_workspace_bytes(int64_t n, size_t* bytes) {
  if (n < 1 || bytes == nullptr) return GSF_EINVAL;
  Carve c{nullptr};
  const int gb = gram_blocks(n);
  c.take((size_t)gb * 7 * 256 * 8);
  c.take((size_t)kGramLevel2Doubles * 8);
  c.take(2 * 24 * 24 * 8);
  c.take(24 * 8 * 8);
  c.take(64);
  c.take(256);
  *bytes = c.off;
  return GSF_OK;
}

// Rayleigh-Ritz step alone: GA, GB (ns x ns, host, row-major) -> theta (m),
// C (ns x m, row-major), kept (ns), *nkept.  Uses a device workspace of
// gsf_rr_workspace_bytes() bytes; synchronizes the stream.
gsf_status gsf_rayleigh_ritz(int ns, int m, const double* GA, const double* GB, double drop_tol, double zero_tol,
                             double* theta, double* C, int* kept, int* nkept, void* ws, size_t ws_bytes,
                             void* stream) {
  clear_stale_errors();
  if (ns < 1 || ns > 24 || m < 1 || m > 8 || m > ns || !GA || !GB || !theta || !C || !kept || !nkept)
    return GSF_EINVAL;
  if (ws == nullptr || ws_bytes < 8192 + 4096) return GSF_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  double* G = (double*)ws;
  double* Cd = G + 2 * 24 * 24;
  double* thd = Cd + 24 * 8;
  int* kd = (int*)(thd + 8);
  GSF_TRY(hip_ok(hipMemcpyAsync(G, GA, (size_t)ns * ns * 8, hipMemcpyHostToDevice, s)));
  GSF_TRY(hip_ok(hipMemcpyAsync(G + ns * ns, GB, (size_t)ns * ns * 8, hipMemcpyHostToDevice, s)));
  RRArgs r{};
  r.C = Cd;
  r.theta = thd;
  r.drop_tol = drop_tol;
  r.zero_tol = zero_tol;
  r.kept_out = kd;
  r.nkept_out = kd + 32;
  GSF_TRY(lob_launch_rr_only(G, ns, m, r, s));
  GSF_TRY(hip_ok(hipMemcpyAsync(theta, thd, (size_t)m * 8, hipMemcpyDeviceToHost, s)));
  GSF_TRY(hip_ok(hipMemcpyAsync(C, Cd, (size_t)ns * m * 8, hipMemcpyDeviceToHost, s)));
  GSF_TRY(hip_ok(hipMemcpyAsync(kept, kd, (size_t)ns * 4, hipMemcpyDeviceToHost, s)));
  GSF_TRY(hip_ok(hipMemcpyAsync(nkept, kd + 32, 4, hipMemcpyDeviceToHost, s)));
  return hip_ok(hipStreamSynchronize(s));
}

size_t gsf_rr_workspace_bytes(void) { return 8192 + 4096; }

gsf_status gsf_tune_apply(const gsf_operator* h, int m, const void* x, void* y, int reps, int* best_rpt,
                          float* times_us, void* stream) {
  clear_stale_errors();
  if (h == nullptr || x == nullptr || y == nullptr || m < 1 || m > kMaxBlock || reps < 1) return GSF_EINVAL;
  const Operator& op = h->op;
  const int w = m >= 8 ? 8 : (m >= 4 ? 4 : m);
  if (w != m) return GSF_EINVAL;  // tune the supported widths 1, 2, 3, 4, 8
  if (op.desc.kind != GSF_BF) {
    if (best_rpt) *best_rpt = 0;
    return GSF_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return GSF_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return GSF_EDEVICE;
  }
  // Candidates timed in interleaved rounds, each keeping its best round, so
  // that a clock or cache drift during tuning (a cold GPU) moves all of them
  // alike; the current choice stays unless another is faster by over 3%.
  const int cand[3] = {1, 2, 4};
  constexpr int kRounds = 3;
  float tbest[3] = {1e30f, 1e30f, 1e30f};
  gsf_status st = GSF_OK;
  for (int c = 0; c < 3 && st == GSF_OK; ++c)  // warm-up
    st = launch_bf_apply_rpt(op, GSF_FORM_LSYM, m, x, m, y, m, nullptr, nullptr, cand[c], s);
  for (int round = 0; round < kRounds && st == GSF_OK; ++round) {
    for (int c = 0; c < 3 && st == GSF_OK; ++c) {
      if (hipEventRecord(e0, s) != hipSuccess) { st = GSF_EDEVICE; break; }
      for (int k = 0; k < reps && st == GSF_OK; ++k)
        st = launch_bf_apply_rpt(op, GSF_FORM_LSYM, m, x, m, y, m, nullptr, nullptr, cand[c], s);
      if (st != GSF_OK) break;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { st = GSF_EDEVICE; break; }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = GSF_EDEVICE; break; }
      const float us = ms * 1000.f / (float)reps;
      if (us < tbest[c]) tbest[c] = us;
    }
  }
  int best = bf_rpt(op, w);
  float best_t = 1e30f;
  for (int c = 0; c < 3; ++c)
    if (cand[c] == best) best_t = tbest[c];
  for (int c = 0; c < 3; ++c) {
    if (times_us) times_us[c] = tbest[c];
    if (tbest[c] < 0.97f * best_t) {
      best_t = tbest[c];
      best = cand[c];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != GSF_OK) return st;
  bf_set_rpt(op, w, best);
  if (best_rpt) *best_rpt = best;
  return GSF_OK;
}

gsf_status gsf_shifted_cg(const gsf_operator* h, double alpha, const void* b, int64_t ldb, void* y, int kmax,
                          double tol, void* ws, size_t ws_bytes, gsf_cg_info* info, void* stream) {
  clear_stale_errors();
  if (h == nullptr || b == nullptr || y == nullptr || ldb < 1 || kmax < 0 || !(alpha >= 0.0) ||
      !std::isfinite(alpha) || !(tol >= 0.0) || !std::isfinite(tol))
    return GSF_EINVAL;
  const Operator& op = h->op;
  CgWs w;
  if (ws == nullptr || ws_bytes < carve_cg(op, nullptr, &w)) return GSF_ENOMEM;
  carve_cg(op, (char*)ws, &w);
  hipStream_t s = (hipStream_t)stream;
  CgState init{};
  init.tol = tol;
  GSF_TRY(launch_cg_state_init(w.st, init, s));
  GSF_TRY(launch_scg_init(op.desc.prec, b, ldb, y, w.r, op.n, w.partials, w.st, s));
  Poller poll(s, &w.st->active, info != nullptr && tol > 0.0);
  for (int k = 1; k <= kmax; ++k) {
    if (!poll.keep_going(k - 1)) break;
    GSF_TRY(launch_cg_pupdate(op, w.r, w.p, w.st, s));
    GSF_TRY(apply_any(op, GSF_FORM_LSYM, 1, w.p, 1, w.q, 1, nullptr, nullptr, s));
    int nparts = 0;
    GSF_TRY(launch_scg_shift(op.desc.prec, w.p, w.q, op.n, alpha, w.partials, &nparts, w.st, s));
    GSF_TRY(launch_cg_alpha(w.partials, nparts, w.st, s));
    GSF_TRY(launch_cg_update(op, y, w.r, w.p, w.q, w.partials, w.st, s));
  }
  if (info == nullptr) return GSF_OK;
  CgState host{};
  GSF_TRY(hip_ok(hipMemcpyAsync(&host, w.st, sizeof(host), hipMemcpyDeviceToHost, s)));
  GSF_TRY(hip_ok(hipStreamSynchronize(s)));
  gsf_status status = (gsf_status)host.status;
  if (status == GSF_OK && tol > 0.0 && !(host.rho <= host.tol2)) status = GSF_ENOTCONV;
  info->iters = host.iters;
  info->status = status;
  info->res0 = host.res0;
  info->res = std::sqrt(host.rho > 0.0 ? host.rho : 0.0);
  return status;
}

gsf_status gsf_precond_create_shifted(const gsf_operator* h, double alpha, int inner_steps, gsf_precond** out) {
  clear_stale_errors();
  if (h == nullptr || out == nullptr || !(alpha > 0.0) || !std::isfinite(alpha) || inner_steps < 1) return GSF_EINVAL;
  CgWs cw;
  const size_t bytes = carve_cg(h->op, nullptr, &cw);
  gsf_precond* T = new (std::nothrow) gsf_precond;
  if (T == nullptr) return GSF_EDEVICE;
  if (hipMalloc(&T->mem, bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete T;
    return GSF_ENOMEM;
  }
  T->n = h->op.n;
  T->rows = h->op.rows;
  T->cols = h->op.cols;
  T->prec = h->op.desc.prec;
  T->kind = kPrecondShifted;
  T->op = h;
  T->alpha = alpha;
  T->inner = inner_steps;
  *out = T;
  return GSF_OK;
}

gsf_status gsf_lobpcg_residual(const gsf_operator* h, int m, const void* X, const double* theta, void* R,
                               void* stream) {
  clear_stale_errors();
  if (h == nullptr || X == nullptr || theta == nullptr || R == nullptr || m < 1 || m > kMaxBlock) return GSF_EINVAL;
  const Operator& op = h->op;
  hipStream_t s = (hipStream_t)stream;
  GSF_TRY(apply_any(op, GSF_FORM_LSYM, m, X, m, R, m, nullptr, nullptr, s));
  return launch_residual(op.desc.prec, X, R, op.n, m, theta, s);
}

gsf_status gsf_get_apply_rows(const gsf_operator* h, int m, int* rows_per_thread) {
  if (h == nullptr || rows_per_thread == nullptr || m < 1 || m > kMaxBlock) return GSF_EINVAL;
  if (h->op.desc.kind != GSF_BF) {
    *rows_per_thread = 0;
    return GSF_OK;
  }
  const int w = m >= 8 ? 8 : (m >= 4 ? 4 : m);
  *rows_per_thread = bf_rpt(h->op, w);
  return GSF_OK;
}

gsf_status gsf_tune_table_save(const char* path, int* entries) {
  if (path == nullptr) return GSF_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (f == nullptr) return GSF_EINVAL;
  const int count = tune_table_write(f);
  const bool bad = std::ferror(f) != 0;
  if (std::fclose(f) != 0 || bad) return GSF_EINVAL;
  if (entries) *entries = count;
  return GSF_OK;
}

gsf_status gsf_tune_table_load(const char* path, int* entries) {
  if (path == nullptr) return GSF_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return GSF_EINVAL;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  const int count = tune_table_read(text);
  if (count < 0) return GSF_EINVAL;
  if (entries) *entries = count;
  return GSF_OK;
}

void gsf_tune_table_clear(void) { tune_table_clear(); }

gsf_status gsf_set_apply_rows(const gsf_operator* h, int m, int rows_per_thread) {
  if (h == nullptr || m < 1 || m > kMaxBlock || h->op.desc.kind != GSF_BF) return GSF_EINVAL;
  if (rows_per_thread != 1 && rows_per_thread != 2 && rows_per_thread != 4) return GSF_EINVAL;
  const int w = m >= 8 ? 8 : (m >= 4 ? 4 : m);
  bf_set_rpt(h->op, w, rows_per_thread);
  return GSF_OK;
}

}  // extern "C"
