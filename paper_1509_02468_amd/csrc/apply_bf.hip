// BF apply: host dispatch over element type and block width, and the table
// of tuned tile heights (with its JSON file form).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "apply_bf_impl.h"

namespace gsf {
namespace {
template <typename T>
void launch_bf_m(const bfk::ApplyArgs& a, int ndim, int r, int m, int rpt, hipStream_t s, int* nb) {
  switch (m) {
    case 1: bf_apply_tm<T, 1>(a, ndim, r, rpt, s, nb); break;
    case 2: bf_apply_tm<T, 2>(a, ndim, r, rpt, s, nb); break;
    case 3: bf_apply_tm<T, 3>(a, ndim, r, rpt, s, nb); break;
    case 4: bf_apply_tm<T, 4>(a, ndim, r, rpt, s, nb); break;
    default: bf_apply_tm<T, 8>(a, ndim, r, rpt, s, nb); break;
  }
}

// Tuned rows-per-thread choices, per (precision, geometry, radius, block
// width, size class); geometry 0 = 1D, 1 = 2D square window, 2 = 2D cross;
// 0 = not tuned (use the default).  Written by the apply tuner.
int g_rpt[2][3][kMaxRadius + 1][kMaxBlock + 1][4];

int geometry(const Operator& op) { return op.desc.ndim == 1 ? 0 : (bf_cross2d(op.desc) ? 2 : 1); }

int size_class(int64_t n) { return n < (1 << 16) ? 0 : (n < (1 << 20) ? 1 : (n < (1 << 23) ? 2 : 3)); }

int width_of(int left) { return left >= 8 ? 8 : (left >= 4 ? 4 : left); }

}  // namespace

int bf_rpt(const Operator& op, int w) {
  const int t = g_rpt[op.desc.prec][geometry(op)][op.desc.radius][w][size_class(op.n)];
  if (t > 0) return t;
  // cross stencil (measured at 1024^2, r = 1, FP32, us for 1 / 2 / 4 rows:
  // m = 1 7.6 / 8.2 / 8.3, m = 4 10.0 / 8.7 / 10.0)
  if (bf_cross2d(op.desc)) return (int)op.elem * w <= 4 ? 1 : 2;
  return bfk::default_rpt((int)op.elem, w, op.desc.radius);
}

void bf_set_rpt(const Operator& op, int w, int rpt) {
  g_rpt[op.desc.prec][geometry(op)][op.desc.radius][w][size_class(op.n)] = rpt;
}

// Tuned-tile table as JSON: {"gsf_apply_tiles": [{"prec": p, "geometry": g,
// "radius": r, "width": w, "size_class": c, "rows_per_thread": t}, ...]}
// (only the tuned entries; geometry 0 = 1D, 1 = 2D square window, 2 = 2D
// cross; size class 0..3 = n below 2^16, 2^20, 2^23, above).
static const char* kTileKeys[6] = {"prec", "geometry", "radius", "width", "size_class", "rows_per_thread"};

int tune_table_write(FILE* f) {
  int count = 0;
  std::fputs("{\"gsf_apply_tiles\": [", f);
  for (int p = 0; p < 2; ++p)
    for (int g = 0; g < 3; ++g)
      for (int r = 0; r <= kMaxRadius; ++r)
        for (int w = 0; w <= kMaxBlock; ++w)
          for (int c = 0; c < 4; ++c) {
            const int t = g_rpt[p][g][r][w][c];
            if (t <= 0) continue;
            std::fprintf(f, "%s\n  {\"prec\": %d, \"geometry\": %d, \"radius\": %d, \"width\": %d, "
                            "\"size_class\": %d, \"rows_per_thread\": %d}",
                         count ? "," : "", p, g, r, w, c, t);
            ++count;
          }
  std::fputs("\n]}\n", f);
  return count;
}

// Parses the table; entries replace the current values of their keys only if
// the whole text is valid.  Returns the entry count, or -1 if malformed.
int tune_table_read(const std::string& text) {
  struct E { int v[6]; };
  std::vector<E> es;
  const size_t lst = text.find("\"gsf_apply_tiles\"");
  if (lst == std::string::npos) return -1;
  size_t pos = text.find('[', lst);
  if (pos == std::string::npos) return -1;
  const size_t end = text.find(']', pos);
  if (end == std::string::npos) return -1;
  while (true) {
    const size_t o = text.find('{', pos);
    if (o == std::string::npos || o > end) break;
    const size_t cl = text.find('}', o);
    if (cl == std::string::npos || cl > end) return -1;
    const std::string obj = text.substr(o, cl - o + 1);
    E e;
    for (int k = 0; k < 6; ++k) {
      const std::string key = std::string("\"") + kTileKeys[k] + "\"";
      const size_t kp = obj.find(key);
      if (kp == std::string::npos) return -1;
      const size_t colon = obj.find(':', kp + key.size());
      if (colon == std::string::npos) return -1;
      char* stop = nullptr;
      const long v = std::strtol(obj.c_str() + colon + 1, &stop, 10);
      if (stop == obj.c_str() + colon + 1) return -1;
      e.v[k] = (int)v;
    }
    const bool ok = e.v[0] >= 0 && e.v[0] < 2 && e.v[1] >= 0 && e.v[1] < 3 && e.v[2] >= 1 && e.v[2] <= kMaxRadius &&
                    (e.v[3] == 1 || e.v[3] == 2 || e.v[3] == 3 || e.v[3] == 4 || e.v[3] == 8) && e.v[4] >= 0 &&
                    e.v[4] < 4 && (e.v[5] == 1 || e.v[5] == 2 || e.v[5] == 4);
    if (!ok) return -1;
    es.push_back(e);
    pos = cl + 1;
  }
  for (const E& e : es) g_rpt[e.v[0]][e.v[1]][e.v[2]][e.v[3]][e.v[4]] = e.v[5];
  return (int)es.size();
}

void tune_table_clear() { std::memset(g_rpt, 0, sizeof(g_rpt)); }

gsf_status launch_bf_apply_rpt(const Operator& op, int form, int m, const void* x, int64_t ldx, void* y,
                               int64_t ldy, double* dot, int* nparts, int rpt_override, hipStream_t s);

gsf_status launch_bf_apply_rpt(const Operator& op, int form, int m, const void* x, int64_t ldx, void* y,
                               int64_t ldy, double* dot, int* nparts, int rpt_override, hipStream_t s) {
  bfk::ApplyArgs a{};
  a.planes = op.planes;
  a.pstride = op.pstride;
  a.ppad = op.ppad;
  a.isqd = op.diag;
  a.ldx = ldx;
  a.ldy = ldy;
  a.n = op.n;
  a.rows = op.rows;
  a.cols = op.cols;
  a.form = form;
  a.cross = bf_cross2d(op.desc) ? 1 : 0;
  a.dot = dot;
  // split m into supported block widths (8, 4, 3, 2, 1)
  int c0 = 0;
  int nb = 0;
  while (c0 < m) {
    const int w = width_of(m - c0);
    const int rpt = rpt_override > 0 ? rpt_override : bf_rpt(op, w);
    a.x = (const char*)x + (size_t)c0 * op.elem;
    a.y = (char*)y + (size_t)c0 * op.elem;
    if (op.desc.prec == GSF_F32)
      launch_bf_m<float>(a, op.desc.ndim, op.desc.radius, w, rpt, s, &nb);
    else
      launch_bf_m<double>(a, op.desc.ndim, op.desc.radius, w, rpt, s, &nb);
    c0 += w;
  }
  if (nparts) *nparts = nb;
  return launch_status();
}

gsf_status launch_bf_apply(const Operator& op, int form, int m, const void* x, int64_t ldx, void* y,
                           int64_t ldy, double* dot, int* nparts, hipStream_t s) {
  return launch_bf_apply_rpt(op, form, m, x, ldx, y, ldy, dot, nparts, 0, s);
}

// Joint apply: y = F x for m columns (x, y with leading dimensions ldx, ldy)
// and y2 = F x2 for one more column (ldx2, ldy2) in one launch that reads the
// operator once; the dot partials are those of x2 . y2.  Offered for BF
// operators on the square window (or 1D) with m = 1 or 4; returns false
// (nothing launched) otherwise.
bool launch_bf_apply_joint(const Operator& op, int form, int m, const void* x, int64_t ldx, void* y, int64_t ldy,
                           const void* x2, int64_t ldx2, void* y2, int64_t ldy2, double* dot, int* nparts,
                           hipStream_t s) {
  if (op.desc.kind != GSF_BF || bf_cross2d(op.desc) || (m != 1 && m != 4)) return false;
  bfk::ApplyArgs a{};
  a.planes = op.planes;
  a.pstride = op.pstride;
  a.ppad = op.ppad;
  a.isqd = op.diag;
  a.x = x;
  a.y = y;
  a.ldx = ldx;
  a.ldy = ldy;
  a.x2 = x2;
  a.y2 = y2;
  a.ldx2 = ldx2;
  a.ldy2 = ldy2;
  a.n = op.n;
  a.rows = op.rows;
  a.cols = op.cols;
  a.form = form;
  a.dot = dot;
  const int rpt = bf_rpt(op, m);  // the tile tuned for the m-column block
  int nb = 0;
  if (op.desc.prec == GSF_F32) {
    if (m == 1) bf_apply_joint_tm<float, 2>(a, op.desc.ndim, op.desc.radius, rpt, s, &nb);
    else bf_apply_joint_tm<float, 5>(a, op.desc.ndim, op.desc.radius, rpt, s, &nb);
  } else {
    if (m == 1) bf_apply_joint_tm<double, 2>(a, op.desc.ndim, op.desc.radius, rpt, s, &nb);
    else bf_apply_joint_tm<double, 5>(a, op.desc.ndim, op.desc.radius, rpt, s, &nb);
  }
  if (nparts) *nparts = nb;
  return true;
}

// Upper bound of the workgroups (and so of the dot partials) of an apply.
int bf_apply_blocks(const Operator& op, int m) {
  const int rpt = 1;  // fewest rows per thread = most workgroups
  (void)m;
  if (op.desc.ndim == 2) {
    const int64_t tiles_x = (op.cols + 63) / 64, tiles_y = (op.rows + 4 * rpt - 1) / (4 * rpt);
    return (int)(tiles_x * tiles_y);
  }
  const int64_t tn = (int64_t)kThreads * rpt;
  return (int)((op.n + tn - 1) / tn);
}

}  // namespace gsf
