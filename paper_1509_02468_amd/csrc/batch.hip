// Batching: many independent items filtered side by side.
//
// Items are spread over kBranches branches (longest-processing-time first),
// each with a stream of the plan's own, forked from and joined back to the
// caller's stream, so small items that cannot fill the chip run concurrently.
// A run issues, per item, the operator build and the solver call of the
// single-item entry points onto its branch stream; optionally each branch is
// recorded once as a HIP graph and replayed (a single graph with parallel
// branches is executed one node after the other by the runtime, so graphs are
// per branch).  Every item runs exactly the kernels of its single-item call,
// so its result is bitwise the same; an item whose solver has converged
// (tol > 0) or broken down turns its remaining kernels into early returns
// through its own device-side state.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "gsf_internal.h"
#include "solver_state.h"

namespace gsf {
gsf_status describe_operator(const gsf_operator_desc* d, Operator* out);
size_t solver_bytes(const Operator& op, int method, int m);
CgState* cg_state_ptr(const Operator& op, void* ws);
LobpcgState* lob_state_ptr(const Operator& op, int m, void* ws);
}  // namespace gsf

constexpr int kBranches = 8;

struct gsf_batch {
  std::vector<gsf_batch_item> items;
  std::vector<gsf_operator*> ops;
  std::vector<void*> solver_ws;
  std::vector<size_t> solver_ws_bytes;
  hipGraph_t graph[kBranches] = {};
  hipGraphExec_t exec[kBranches] = {};
  hipStream_t stream[kBranches] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kBranches] = {};
  std::vector<int> order;      // items, longest first
  std::vector<int> branch_of;  // branch of each item
  std::vector<char*> op_ws;
  std::vector<size_t> op_bytes;
  std::vector<gsf::Operator> desc;  // sizes of each item's operator
  bool graphs = false;
};

namespace {

using namespace gsf;

constexpr size_t kAlignB = 256;

size_t ceil_align(size_t v) { return (v + kAlignB - 1) / kAlignB * kAlignB; }

gsf_status check_item(const gsf_batch_item& it, int prec0, Operator* op) {
  if (it.guidance == nullptr || it.x0 == nullptr || it.x_out == nullptr) return GSF_EINVAL;
  if (it.method != GSF_METHOD_POWER && it.method != GSF_METHOD_CG && it.method != GSF_METHOD_LOBPCG)
    return GSF_EINVAL;
  if (it.kmax < 0 || !(it.tol >= 0.0) || !std::isfinite(it.tol)) return GSF_EINVAL;
  if (it.method == GSF_METHOD_LOBPCG && (it.m < 1 || it.m > kMaxBlock)) return GSF_EINVAL;
  if (it.op.prec != prec0) return GSF_EINVAL;
  return describe_operator(&it.op, op);
}

int item_m(const gsf_batch_item& it) { return it.method == GSF_METHOD_LOBPCG ? it.m : 1; }

// Rough work estimate (point-vector applies) used to balance the branches.
double item_work(const gsf_batch_item& it, const Operator& op) {
  const double n = (double)op.n, k = (double)it.kmax + 1.0;
  return it.method == GSF_METHOD_LOBPCG ? n * k * (2.0 * it.m + 8.0) : n * k * 2.0;
}

gsf_status hip_ok(hipError_t e) { return device_status(e); }

__global__ void batch_touch_kernel() {}

// Streams per device that have run work before any branch stream of a plan
// does (created with the first plan on the device, kept until the process
// ends; default priority); the first also carries the tile tuning.  Measured
// on the 320-item batch (graph replay, four hardware queues): 455-474 ms when
// fewer than three other streams of the process had run work before the
// branch streams, 352-356 ms with three, whatever the order of the branch
// streams' own first launches (an empty kernel on each at creation changed
// nothing).
constexpr int kHelpers = 3;
gsf_status helper_streams(hipStream_t* first) {
  static std::mutex mu;
  static hipStream_t helpers[64][kHelpers] = {};
  int dev = 0;
  gsf_status st = hip_ok(hipGetDevice(&dev));
  if (st != GSF_OK) return st;
  if (dev < 0 || dev >= 64) return GSF_EDEVICE;
  std::lock_guard<std::mutex> lock(mu);
  for (int k = 0; k < kHelpers; ++k) {
    if (helpers[dev][k] != nullptr) continue;
    hipStream_t h = nullptr;
    st = hip_ok(hipStreamCreateWithFlags(&h, hipStreamNonBlocking));
    if (st != GSF_OK) return st;
    batch_touch_kernel<<<1, 64, 0, h>>>();
    st = launch_status();
    if (st == GSF_OK) st = hip_ok(hipStreamSynchronize(h));
    if (st != GSF_OK) {
      (void)hipStreamDestroy(h);
      return st;
    }
    helpers[dev][k] = h;
  }
  *first = helpers[dev][0];
  return GSF_OK;
}

void free_batch(gsf_batch* b) {
  if (b == nullptr) return;
  for (gsf_operator* op : b->ops) gsf_destroy_operator(op);
  for (int k = 0; k < kBranches; ++k) {
    if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
    if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
    if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    if (b->stream[k]) (void)hipStreamDestroy(b->stream[k]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
}

// Operator build and solve of item i on stream s (the single-item calls).
gsf_status issue_item(gsf_batch* b, int i, hipStream_t s) {
  const gsf_batch_item& it = b->items[i];
  if (b->ops[i] != nullptr) {
    gsf_destroy_operator(b->ops[i]);
    b->ops[i] = nullptr;
  }
  gsf_status st = gsf_build_operator(&it.op, it.guidance, b->op_ws[i], b->op_bytes[i], s, &b->ops[i]);
  if (st != GSF_OK) return st;
  void* sw = b->solver_ws[i];
  const size_t sb = b->solver_ws_bytes[i];
  if (it.method == GSF_METHOD_POWER) return gsf_power_filter(b->ops[i], it.x0, it.x_out, it.kmax, sw, sb, s);
  if (it.method == GSF_METHOD_CG)
    return gsf_cg_filter(b->ops[i], it.x0, it.x_out, it.kmax, it.tol, sw, sb, nullptr, s);
  return gsf_lobpcg_filter(b->ops[i], it.x0, it.x_out, it.m, it.kmax, it.tol, it.constraint, nullptr, nullptr, nullptr,
                           sw, sb,
                           nullptr, s);
}

}  // namespace

extern "C" {

gsf_status gsf_batch_workspace_bytes(const gsf_batch_item* items, int count, size_t* bytes) {
  if (items == nullptr || count < 1 || bytes == nullptr) return GSF_EINVAL;
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    Operator op;
    gsf_status st = check_item(items[i], items[0].op.prec, &op);
    if (st != GSF_OK) return st;
    size_t ob = 0;
    gsf_operator_workspace_bytes(&items[i].op, &ob);
    total += ceil_align(ob) + ceil_align(solver_bytes(op, items[i].method, item_m(items[i])));
  }
  *bytes = total;
  return GSF_OK;
}

gsf_status gsf_batch_create(const gsf_batch_item* items, int count, void* ws, size_t ws_bytes, int flags,
                            gsf_batch** out) {
  const int autotune = flags & GSF_BATCH_AUTOTUNE;
  if (out == nullptr || ws == nullptr) return GSF_EINVAL;
  size_t need = 0;
  gsf_status st = gsf_batch_workspace_bytes(items, count, &need);
  if (st != GSF_OK) return st;
  if (ws_bytes < need) return GSF_ENOMEM;

  gsf_batch* b = new (std::nothrow) gsf_batch;
  if (b == nullptr) return GSF_EDEVICE;
  b->items.assign(items, items + count);
  std::vector<Operator> desc(count);
  std::vector<char*> op_ws(count);
  std::vector<size_t> op_bytes(count);
  char* p = (char*)ws;
  for (int i = 0; i < count; ++i) {
    describe_operator(&items[i].op, &desc[i]);
    gsf_operator_workspace_bytes(&items[i].op, &op_bytes[i]);
    op_ws[i] = p;
    p += ceil_align(op_bytes[i]);
    const size_t sb = solver_bytes(desc[i], items[i].method, item_m(items[i]));
    b->solver_ws.push_back(p);
    b->solver_ws_bytes.push_back(sb);
    p += ceil_align(sb);
  }

  hipStream_t s0 = nullptr;
  st = helper_streams(&s0);
  for (int k = 0; k < kBranches && st == GSF_OK; ++k) {
    st = hip_ok(hipStreamCreateWithFlags(&b->stream[k], hipStreamNonBlocking));
    if (st == GSF_OK) st = hip_ok(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming));
  }
  if (st == GSF_OK) st = hip_ok(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));

  // BF apply tile per class (precision, geometry, radius, width, size): built
  // operator of the first item of each class, its solver workspace as scratch.
  if (st == GSF_OK && autotune) {
    std::map<std::tuple<int, int, int, int, int, int>, bool> done;
    for (int i = 0; i < count && st == GSF_OK; ++i) {
      const gsf_batch_item& it = items[i];
      if (it.op.kind != GSF_BF || it.method == GSF_METHOD_POWER) continue;
      const int w = item_m(it) >= 8 ? 8 : (item_m(it) >= 4 ? 4 : item_m(it));
      const int64_t n = desc[i].n;
      const int sc = n < (1 << 16) ? 0 : (n < (1 << 20) ? 1 : (n < (1 << 23) ? 2 : 3));
      const int cross = bf_cross2d(it.op) ? 1 : 0;
      auto key = std::make_tuple(it.op.prec, it.op.ndim, cross, it.op.radius, w, sc);
      if (done.count(key)) continue;
      done[key] = true;
      gsf_operator* tmp = nullptr;
      st = gsf_build_operator(&it.op, it.guidance, op_ws[i], op_bytes[i], s0, &tmp);
      if (st != GSF_OK) break;
      char* x = (char*)b->solver_ws[i];
      char* y = x + ceil_align((size_t)n * w * desc[i].elem);
      st = gsf_tune_apply(tmp, w, x, y, 5, nullptr, nullptr, s0);
      gsf_destroy_operator(tmp);
    }
  }
  if (st == GSF_OK && s0 != nullptr) st = hip_ok(hipStreamSynchronize(s0));

  // items over the branches, longest first onto the least loaded branch
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return item_work(items[a], desc[a]) > item_work(items[c], desc[c]);
  });
  std::vector<int> branch_of(count, 0);
  double load[kBranches] = {};
  for (int idx = 0; idx < count; ++idx) {
    const int i = order[idx];
    int k = 0;
    for (int t = 1; t < kBranches; ++t)
      if (load[t] < load[k]) k = t;
    load[k] += item_work(items[i], desc[i]);
    branch_of[i] = k;
  }
  b->order = order;
  b->branch_of = branch_of;
  b->op_ws = op_ws;
  b->op_bytes = op_bytes;
  b->desc = desc;
  b->graphs = (flags & GSF_BATCH_GRAPHS) != 0;
  b->ops.assign(count, nullptr);
  // one graph per branch: operator builds and solves of its items, in order
  for (int k = 0; k < kBranches && st == GSF_OK && b->graphs; ++k) {
    hipStream_t sk = b->stream[k];
    st = hip_ok(hipStreamBeginCapture(sk, hipStreamCaptureModeThreadLocal));
    if (st != GSF_OK) break;
    for (int idx = 0; idx < count && st == GSF_OK; ++idx) {
      const int i = order[idx];
      if (branch_of[i] == k) st = issue_item(b, i, sk);
    }
    hipGraph_t g = nullptr;
    const gsf_status se = hip_ok(hipStreamEndCapture(sk, &g));
    if (st == GSF_OK) st = se;
    b->graph[k] = g;
    if (st == GSF_OK) st = hip_ok(hipGraphInstantiate(&b->exec[k], g, nullptr, nullptr, 0));
  }
  if (st != GSF_OK) {
    free_batch(b);
    return st;
  }
  *out = b;
  return GSF_OK;
}

gsf_status gsf_batch_run(gsf_batch* b, void* stream) {
  clear_stale_errors();
  if (b == nullptr) return GSF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipEventRecord(b->fork, s) != hipSuccess) return GSF_EDEVICE;
  for (int k = 0; k < kBranches; ++k)
    if (hipStreamWaitEvent(b->stream[k], b->fork, 0) != hipSuccess) return GSF_EDEVICE;
  if (b->graphs) {
    for (int k = 0; k < kBranches; ++k)
      if (b->exec[k] != nullptr && hipGraphLaunch(b->exec[k], b->stream[k]) != hipSuccess) return GSF_EDEVICE;
  } else {
    for (int i : b->order) {
      const gsf_status st = issue_item(b, i, b->stream[b->branch_of[i]]);
      if (st != GSF_OK) return st;
    }
  }
  for (int k = 0; k < kBranches; ++k) {
    if (hipEventRecord(b->join[k], b->stream[k]) != hipSuccess) return GSF_EDEVICE;
    if (hipStreamWaitEvent(s, b->join[k], 0) != hipSuccess) return GSF_EDEVICE;
  }
  return GSF_OK;
}

gsf_status gsf_batch_get_info(const gsf_batch* b, gsf_batch_info* info, void* stream) {
  clear_stale_errors();
  if (b == nullptr || info == nullptr) return GSF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int count = (int)b->items.size();
  std::vector<CgState> cg(count);
  std::vector<LobpcgState> lob(count);
  for (int i = 0; i < count; ++i) {
    const gsf_batch_item& it = b->items[i];
    const Operator& op = b->desc[i];
    if (it.method == GSF_METHOD_CG) {
      if (hipMemcpyAsync(&cg[i], cg_state_ptr(op, b->solver_ws[i]), sizeof(CgState), hipMemcpyDeviceToHost, s) !=
          hipSuccess)
        return GSF_EDEVICE;
    } else if (it.method == GSF_METHOD_LOBPCG) {
      if (hipMemcpyAsync(&lob[i], lob_state_ptr(op, it.m, b->solver_ws[i]), sizeof(LobpcgState),
                         hipMemcpyDeviceToHost, s) != hipSuccess)
        return GSF_EDEVICE;
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess) return GSF_EDEVICE;
  for (int i = 0; i < count; ++i) {
    const gsf_batch_item& it = b->items[i];
    gsf_batch_info& o = info[i];
    if (it.method == GSF_METHOD_POWER) {
      o.iters = it.kmax;
      o.status = GSF_OK;
      o.res0 = o.res = 0.0;
    } else if (it.method == GSF_METHOD_CG) {
      const CgState& h = cg[i];
      gsf_status status = (gsf_status)h.status;
      if (status == GSF_OK && it.tol > 0.0 && h.active && !(h.rho <= h.tol2)) status = GSF_ENOTCONV;
      o.iters = h.iters;
      o.status = status;
      o.res0 = h.res0;
      o.res = std::sqrt(h.rho > 0.0 ? h.rho : 0.0);
    } else {
      const LobpcgState& h = lob[i];
      gsf_status status = (gsf_status)h.status;
      double mx = 0.0;
      for (int j = 0; j < it.m; ++j) mx = h.res[j] > mx ? h.res[j] : mx;
      if (status == GSF_OK && it.tol > 0.0 && mx > it.tol) status = GSF_ENOTCONV;
      o.iters = h.iters;
      o.status = status;
      o.res0 = 0.0;
      o.res = mx;
    }
  }
  return GSF_OK;
}

void gsf_batch_destroy(gsf_batch* b) { free_batch(b); }

gsf_status gsf_batch_filter(const gsf_batch_item* items, int count, void* ws, size_t ws_bytes, gsf_batch_info* info,
                            void* stream) {
  gsf_batch* b = nullptr;
  gsf_status st = gsf_batch_create(items, count, ws, ws_bytes, 0, &b);
  if (st != GSF_OK) return st;
  st = gsf_batch_run(b, stream);
  if (st == GSF_OK) {
    std::vector<gsf_batch_info> local;
    if (info == nullptr) local.resize(count);
    gsf_batch_info* out = info != nullptr ? info : local.data();
    st = gsf_batch_get_info(b, out, stream);  // synchronizes the stream
    for (int i = 0; st == GSF_OK && i < count; ++i)
      if (out[i].status != GSF_OK && out[i].status != GSF_ENOTCONV && out[i].status != GSF_EBREAKDOWN)
        st = (gsf_status)out[i].status;
  } else {
    (void)hipStreamSynchronize((hipStream_t)stream);
  }
  gsf_batch_destroy(b);
  return st;
}

}  // extern "C"
