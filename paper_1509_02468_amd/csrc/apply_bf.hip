// BF apply: host dispatch over element type and block width.
#include "apply_bf_impl.h"

namespace gsf {
namespace {
template <typename T>
void launch_bf_m(const bfk::ApplyArgs& a, int ndim, int r, int m, hipStream_t s, int* nb) {
  switch (m) {
    case 1: bf_apply_tm<T, 1>(a, ndim, r, s, nb); break;
    case 2: bf_apply_tm<T, 2>(a, ndim, r, s, nb); break;
    case 3: bf_apply_tm<T, 3>(a, ndim, r, s, nb); break;
    case 4: bf_apply_tm<T, 4>(a, ndim, r, s, nb); break;
    default: bf_apply_tm<T, 8>(a, ndim, r, s, nb); break;
  }
}
}  // namespace

gsf_status launch_bf_apply(const Operator& op, int form, int m, const void* x, int64_t ldx, void* y,
                           int64_t ldy, double* dot, int* nparts, hipStream_t s) {
  bfk::ApplyArgs a{};
  a.planes = op.planes;
  a.isqd = op.diag;
  a.ldx = ldx;
  a.ldy = ldy;
  a.n = op.n;
  a.rows = op.rows;
  a.cols = op.cols;
  a.form = form;
  a.dot = dot;
  // split m into supported block widths (8, 4, 3, 2, 1)
  int c0 = 0;
  int nb = 0;
  while (c0 < m) {
    const int left = m - c0;
    const int w = left >= 8 ? 8 : (left >= 4 ? 4 : left);
    a.x = (const char*)x + (size_t)c0 * op.elem;
    a.y = (char*)y + (size_t)c0 * op.elem;
    if (op.desc.prec == GSF_F32)
      launch_bf_m<float>(a, op.desc.ndim, op.desc.radius, w, s, &nb);
    else
      launch_bf_m<double>(a, op.desc.ndim, op.desc.radius, w, s, &nb);
    c0 += w;
  }
  if (nparts) *nparts = nb;
  return hipGetLastError() == hipSuccess ? GSF_OK : GSF_EDEVICE;
}

int bf_apply_blocks(const Operator& op, int m) {
  const int w = m >= 8 ? 8 : (m >= 4 ? 4 : m);
  const int mb = w * (int)op.elem;
  const int rpt = mb <= 16 ? 4 : (mb <= 32 ? 2 : 1);
  if (op.desc.ndim == 2) {
    const int64_t tiles_x = (op.cols + 63) / 64, tiles_y = (op.rows + 4 * rpt - 1) / (4 * rpt);
    return (int)(tiles_x * tiles_y);
  }
  const int64_t tn = (int64_t)kThreads * rpt;
  return (int)((op.n + tn - 1) / tn);
}

}  // namespace gsf
