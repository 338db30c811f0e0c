// C ABI of the learned preconditioner: training entry points, training
// pairs and the preconditioner handle used by gsf_lobpcg_filter.
#include <cmath>
#include <new>

#include "gsf_internal.h"
#include "solver_state.h"

namespace gsf {
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
gsf_status launch_colnorm(int prec, const void* R, int64_t n, int m, int64_t ld, double* partials, double* out,
                          hipStream_t s);
gsf_status launch_net_pair(int prec, const void* r, int64_t ldr, const void* y, int64_t ldy, const void* g,
                           int64_t n, const double* norm, float* in, float* tg, hipStream_t s);
int vec_blocks(int64_t n);
gsf_status shifted_precond_apply(const gsf_precond* T, int m, const void* R, void* Z, hipStream_t s);
}  // namespace gsf

using namespace gsf;

namespace {
size_t a256(size_t v) { return (v + 255) / 256 * 256; }
}  // namespace

#define GSF_TRY(expr)              \
  do {                             \
    gsf_status _st = (expr);       \
    if (_st != GSF_OK) return _st; \
  } while (0)

extern "C" {

gsf_status gsf_net_workspace_bytes(int batch, int64_t rows, int64_t cols, size_t* bytes) {
  if (bytes == nullptr || batch < 1 || rows < 1 || cols < 1) return GSF_EINVAL;
  *bytes = net_train_bytes(batch, rows * cols);
  return GSF_OK;
}

gsf_status gsf_net_forward(const uint16_t* w, int batch, const int32_t* idx, int64_t rows, int64_t cols,
                           const float* inputs, float* y, void* ws, size_t ws_bytes, void* stream) {
  clear_stale_errors();
  if (w == nullptr || idx == nullptr || inputs == nullptr || y == nullptr || batch < 1 || rows < 1 || cols < 1)
    return GSF_EINVAL;
  if (ws == nullptr || ws_bytes < net_train_bytes(batch, rows * cols)) return GSF_ENOMEM;
  return net_forward_train(w, batch, idx, rows, cols, inputs, nullptr, y, nullptr, nullptr, ws,
                           (hipStream_t)stream);
}

gsf_status gsf_net_loss_grad(const uint16_t* w, int batch, const int32_t* idx, int64_t rows, int64_t cols,
                             const float* inputs, const float* targets, float* grad, double* loss, void* ws,
                             size_t ws_bytes, void* stream) {
  clear_stale_errors();
  if (w == nullptr || idx == nullptr || inputs == nullptr || targets == nullptr || grad == nullptr ||
      loss == nullptr || batch < 1 || rows < 1 || cols < 1)
    return GSF_EINVAL;
  if (ws == nullptr || ws_bytes < net_train_bytes(batch, rows * cols)) return GSF_ENOMEM;
  return net_forward_train(w, batch, idx, rows, cols, inputs, targets, nullptr, grad, loss, ws,
                           (hipStream_t)stream);
}

gsf_status gsf_net_adam(int64_t count, int t, double lr, double beta1, double beta2, double eps, float* w, float* mom,
                        float* vel, const float* grad, uint16_t* w_bf16, void* stream) {
  clear_stale_errors();
  if (count < 1 || t < 1 || w == nullptr || mom == nullptr || vel == nullptr || grad == nullptr ||
      w_bf16 == nullptr || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0))
    return GSF_EINVAL;
  return net_adam(count, t, lr, beta1, beta2, eps, w, mom, vel, grad, w_bf16, (hipStream_t)stream);
}

gsf_status gsf_net_to_bf16(int64_t count, const float* w, uint16_t* w_bf16, void* stream) {
  clear_stale_errors();
  if (count < 1 || w == nullptr || w_bf16 == nullptr) return GSF_EINVAL;
  return net_to_bf16(count, w, w_bf16, (hipStream_t)stream);
}

gsf_status gsf_net_pair_workspace_bytes(const gsf_operator* op, size_t* bytes) {
  if (op == nullptr || bytes == nullptr) return GSF_EINVAL;
  *bytes = a256((size_t)vec_blocks(op->op.n) * kMaxBlock * 8) + 256;
  return GSF_OK;
}

gsf_status gsf_net_make_pair(const gsf_operator* h, const void* r, int64_t ldr, const void* y, int64_t ldy,
                             const void* g, float* inputs, float* targets, void* ws, size_t ws_bytes, void* stream) {
  clear_stale_errors();
  if (h == nullptr || r == nullptr || y == nullptr || g == nullptr || inputs == nullptr || targets == nullptr ||
      ldr < 1 || ldy < 1)
    return GSF_EINVAL;
  size_t need = 0;
  gsf_net_pair_workspace_bytes(h, &need);
  if (ws == nullptr || ws_bytes < need) return GSF_ENOMEM;
  const Operator& op = h->op;
  double* partials = (double*)ws;
  double* norm = (double*)((char*)ws + a256((size_t)vec_blocks(op.n) * kMaxBlock * 8));
  hipStream_t s = (hipStream_t)stream;
  GSF_TRY(launch_colnorm(op.desc.prec, r, op.n, 1, ldr, partials, norm, s));
  return launch_net_pair(op.desc.prec, r, ldr, y, ldy, g, op.n, norm, inputs, targets, s);
}

gsf_status gsf_precond_create(const gsf_operator* h, const void* g, const uint16_t* w, gsf_precond** out) {
  if (h == nullptr || g == nullptr || w == nullptr || out == nullptr) return GSF_EINVAL;
  gsf_precond* T = new (std::nothrow) gsf_precond;
  if (T == nullptr) return GSF_EDEVICE;
  T->n = h->op.n;
  T->rows = h->op.rows;
  T->cols = h->op.cols;
  T->prec = h->op.desc.prec;
  T->g = g;
  T->w = w;
  *out = T;
  return GSF_OK;
}

void gsf_precond_destroy(gsf_precond* T) {
  if (T == nullptr) return;
  if (T->mem != nullptr) (void)hipFree(T->mem);
  delete T;
}

gsf_status gsf_precond_workspace_bytes(const gsf_precond* T, int m, size_t* bytes) {
  if (T == nullptr || bytes == nullptr || m < 1 || m > kMaxBlock) return GSF_EINVAL;
  *bytes = a256((size_t)vec_blocks(T->n) * kMaxBlock * 8) + 256 +
           a256((size_t)net_tiles(T->rows, T->cols) * 3 * m * 8);
  return GSF_OK;
}

gsf_status gsf_precond_apply(const gsf_precond* T, int m, const void* R, void* W, void* ws, size_t ws_bytes,
                             void* stream) {
  clear_stale_errors();
  if (T == nullptr || R == nullptr || W == nullptr || m < 1 || m > kMaxBlock) return GSF_EINVAL;
  size_t need = 0;
  gsf_precond_workspace_bytes(T, m, &need);
  if (ws == nullptr || ws_bytes < need) return GSF_ENOMEM;
  const size_t pb = a256((size_t)vec_blocks(T->n) * kMaxBlock * 8);
  double* cpart = (double*)ws;
  double* norms = (double*)((char*)ws + pb);
  double* npart = (double*)((char*)ws + pb + 256);
  hipStream_t s = (hipStream_t)stream;
  if (T->kind == kPrecondShifted) return shifted_precond_apply(T, m, R, W, s);
  GSF_TRY(launch_colnorm(T->prec, R, T->n, m, m, cpart, norms, s));
  return net_infer(T->prec, T->w, T->rows, T->cols, m, R, W, T->g, nullptr, norms, nullptr, npart, s);
}

}  // extern "C"
