// Batches of patches: many independent single-patch problems (plans) formed
// together.  Rows of different patches, like rows of one patch, are
// independent (Section 1: each row of the matrices is formed on its own), so
// a batch only reorganises the launches: per class of patches (degree p,
// dimension d, precision) one first-contraction launch over all their blocks
// and one persistent pencil-kernel launch over a device work queue of
// (patch, work item) pairs.  A project autotuner picks, per class, the
// runs of rows per pencil (the row-to-workgroup schedule) and the persistent
// grid; the launch sequence can be captured once into a HIP graph and
// replayed.  See include/wq.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "wq_internal.h"

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Candidates of the autotuner: total work items per class (0: one run of
// rows per pencil) and persistent workgroups per compute unit.
constexpr int kSegTargets[] = {0, 2048, 8192};
constexpr int kWgsPerCu[] = {1, 2, 4};

}  // namespace

constexpr size_t kSideStreams = 4;   // streams the classes of a batch run on

struct wq_batch {
  struct Class {
    int p = 0, d = 3, prec = 0;
    std::vector<int> members;   // plan indices
    int seg_target = 2048, wgs_per_cu = 2;
    size_t views = 0, outm = 0, outs = 0, itm = 0, its = 0, nsm = 0, nss = 0, blk = 0;
    int first_blocks = 0;
    int total[2] = {0, 0};      // work items (mass, stiffness)
  };
  std::vector<wq_plan*> plans;
  std::vector<Class> classes;
  size_t counters = 0, total_bytes = 0;
  char* ws = nullptr;
  bool bound = false;
  int n_cu = 256;
  std::vector<void*> mass, stiff;
  std::vector<char> img;        // host image of the descriptors
  hipGraphExec_t graph = nullptr;
  int graph_which = 0;
  hipStream_t graph_stream = nullptr;
  // classes run concurrently on side streams forked from the caller's
  // stream (a class's tail, when its queue drains, overlaps the next one)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev_done;
  hipEvent_t ev_fork = nullptr;
  std::string err;
  ~wq_batch() {
    if (graph) (void)hipGraphExecDestroy(graph);
    for (hipStream_t s : side) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : ev_done) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
  }
  hipError_t make_side() {
    const size_t ns = std::min<size_t>(kSideStreams, 2 * classes.size());
    hipError_t e = hipSuccess;
    while (e == hipSuccess && side.size() < ns) {
      hipStream_t s = nullptr;
      e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
      if (e == hipSuccess) side.push_back(s);
    }
    while (e == hipSuccess && ev_done.size() < 2 * classes.size()) {
      hipEvent_t ev = nullptr;
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) ev_done.push_back(ev);
    }
    if (e == hipSuccess && !ev_fork) e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming);
    return e;
  }
  void drop_graph() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
  }
  wq::BatchClassView view(const Class& c) const {
    wq::BatchClassView v{};
    v.views = reinterpret_cast<const wq::PlanView*>(ws + c.views);
    v.out_mass = reinterpret_cast<void* const*>(ws + c.outm);
    v.out_stiff = reinterpret_cast<void* const*>(ws + c.outs);
    v.items_mass = reinterpret_cast<const int*>(ws + c.itm);
    v.items_stiff = reinterpret_cast<const int*>(ws + c.its);
    v.nsegs_mass = reinterpret_cast<const int*>(ws + c.nsm);
    v.nsegs_stiff = reinterpret_cast<const int*>(ws + c.nss);
    v.blocks = reinterpret_cast<const int*>(ws + c.blk);
    v.counter = reinterpret_cast<int*>(ws + counters) + 2 * (&c - classes.data());
    v.np = int(c.members.size());
    return v;
  }
};

namespace {

wq_status bfail(wq_batch* b, wq_status st, const std::string& msg) {
  if (b) b->err = msg;
  return st;
}

wq_status bhip(wq_batch* b, hipError_t e, const char* where) {
  return bfail(b, WQ_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Work items and runs of rows of every member of class c (both matrices),
// written into the host image; the first-contraction block prefix too.
void fill_schedule(wq_batch* b, wq_batch::Class& c) {
  const int np = int(c.members.size());
  for (int stiff = 0; stiff < 2; ++stiff) {
    int* items = reinterpret_cast<int*>(b->img.data() + (stiff ? c.its : c.itm));
    int* nsegs = reinterpret_cast<int*>(b->img.data() + (stiff ? c.nss : c.nsm));
    int acc = 0;
    for (int k = 0; k < np; ++k) {
      const wq_plan* pl = b->plans[c.members[k]];
      const int64_t wgs = wq::push_units(c.p, c.d, c.prec, stiff != 0, int(pl->n[1]), int(pl->n[2]));
      const int max_seg = std::max<int>(1, int(pl->n[0] / (2 * c.p)));
      const int64_t want = c.seg_target > 0 ? (int64_t(c.seg_target) + np * wgs - 1) / (np * wgs) : 1;
      const int nseg = int(std::min<int64_t>(max_seg, std::max<int64_t>(1, want)));
      items[k] = acc;
      nsegs[k] = nseg;
      acc += int(wgs * nseg);
    }
    items[np] = acc;
    c.total[stiff] = acc;
  }
  // first-contraction blocks (a plane class has no first contraction)
  int* blocks = reinterpret_cast<int*>(b->img.data() + c.blk);
  int acc = 0;
  for (int k = 0; k < np; ++k) {
    const wq_plan* pl = b->plans[c.members[k]];
    blocks[k] = acc;
    if (c.d == 3) acc += int(((pl->nq[0] * pl->nq[1] + 255) / 256) * pl->n[2]);
  }
  blocks[np] = acc;
  c.first_blocks = acc;
}

hipError_t upload(wq_batch* b, hipStream_t s) {
  return hipMemcpyAsync(b->ws, b->img.data(), b->total_bytes, hipMemcpyHostToDevice, s);
}

// The launches of class k (both matrices) on stream s: the class's two
// launches over its device work queues, or (schedule wgs_per_cu = 0) the
// single-patch kernels patch after patch.
// mass_own_y: the mass uses each plan's own mass buffer for the first
// contraction, so that it may run beside the stiffness of the same plans.
hipError_t enqueue_class(wq_batch* b, size_t k, int which, hipStream_t s, bool mass_own_y = false) {
  const wq_batch::Class& c = b->classes[k];
  hipError_t e = hipSuccess;
  if (c.wgs_per_cu == 0) {
    for (size_t m = 0; m < c.members.size() && e == hipSuccess; ++m) {
      const int idx = c.members[m];
      const wq_plan* pl = b->plans[idx];
      wq::PlanView v = pl->view();
      if (mass_own_y) v.ybuf = pl->ws + pl->lay.ymass;
      e = wq::launch_assemble(v, which, b->mass[idx], b->stiff[idx], s);
    }
    return e;
  }
  const wq::BatchClassView v = b->view(c);
  for (int stiff = 0; stiff < 2 && e == hipSuccess; ++stiff) {
    if (!(which & (stiff ? WQ_STIFF : WQ_MASS)) || c.total[stiff] == 0) continue;
    const int grid = std::max(1, std::min(c.total[stiff], c.wgs_per_cu * b->n_cu));
    e = wq::launch_batch_class(v, c.p, c.d, c.prec, stiff != 0, c.first_blocks, grid, s);
  }
  return e;
}

// The launch sequence of one assembly (also what a captured graph holds):
// the work-queue counters are cleared on s, then the classes run on the
// side streams forked from s, which joins them all (one class alone, or
// only_class for the autotuner, runs on s).
hipError_t enqueue(wq_batch* b, int which, hipStream_t s, int only_class = -1) {
  hipError_t e = wq::launch_zero_counters(reinterpret_cast<int*>(b->ws + b->counters), int(2 * b->classes.size()), s);
  if (only_class >= 0 || b->classes.size() == 1) {
    for (size_t k = 0; k < b->classes.size() && e == hipSuccess; ++k)
      if (only_class < 0 || int(k) == only_class) e = enqueue_class(b, k, which, s);
    return e;
  }
  if (e == hipSuccess && b->side.empty()) e = hipErrorInvalidHandle;   // made by wq_batch_bind
  if (e == hipSuccess) e = hipEventRecord(b->ev_fork, s);
  for (size_t j = 0; j < b->side.size() && e == hipSuccess; ++j) e = hipStreamWaitEvent(b->side[j], b->ev_fork, 0);
  // units of work dealt round-robin to the side streams: a class, or, for
  // a class launched patch after patch with both matrices, its masses and
  // its stiffnesses as two units (the masses on their own buffers)
  size_t u = 0;
  for (size_t k = 0; k < b->classes.size() && e == hipSuccess; ++k) {
    const bool split = b->classes[k].wgs_per_cu == 0 && which == (WQ_MASS | WQ_STIFF);
    for (int part = 0; part < (split ? 2 : 1) && e == hipSuccess; ++part, ++u) {
      hipStream_t su = b->side[u % b->side.size()];
      const int w = split ? (part == 0 ? WQ_MASS : WQ_STIFF) : which;
      e = enqueue_class(b, k, w, su, split && part == 0);
      if (e == hipSuccess) e = hipEventRecord(b->ev_done[u], su);
    }
  }
  for (size_t j = 0; j < u && e == hipSuccess; ++j) e = hipStreamWaitEvent(s, b->ev_done[j], 0);
  return e;
}

// Make `stream` wait for the univariate stage of every member's last setup.
hipError_t join_all(wq_batch* b, hipStream_t s) {
  for (wq_plan* pl : b->plans)
    if (pl->rules_launched) {
      hipError_t e = hipStreamWaitEvent(s, pl->ev_rules, 0);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

wq_status check_ready(wq_batch* b, int which) {
  if (!b->bound) return bfail(b, WQ_ESTATE, "batch not bound");
  if (which <= 0 || (which & ~(WQ_MASS | WQ_STIFF))) return bfail(b, WQ_EINVAL, "which must be WQ_MASS, WQ_STIFF or both");
  for (size_t k = 0; k < b->plans.size(); ++k) {
    if (!b->plans[k]->setup_done) return bfail(b, WQ_ESTATE, "patch " + std::to_string(k) + " has no wq_setup");
    if (b->plans[k]->nurbs_basis)
      return bfail(b, WQ_EINVAL, "patch " + std::to_string(k) + ": rational test/trial functions (WQ_BASIS_NURBS) are not batched");
    if ((which & WQ_MASS) && !b->mass[k]) return bfail(b, WQ_EINVAL, "patch " + std::to_string(k) + ": no mass output");
    if ((which & WQ_STIFF) && !b->stiff[k]) return bfail(b, WQ_EINVAL, "patch " + std::to_string(k) + ": no stiffness output");
  }
  return WQ_OK;
}

}  // namespace

extern "C" {

wq_status wq_batch_create(int n, wq_plan* const* plans, wq_batch** out) {
  if (!out) return WQ_EINVAL;
  *out = nullptr;
  if (n <= 0 || !plans) return WQ_EINVAL;
  wq_batch* b = new (std::nothrow) wq_batch();
  if (!b) return WQ_EINVAL;
  for (int k = 0; k < n; ++k) {
    if (!plans[k]) { delete b; return WQ_EINVAL; }
    for (int j = 0; j < k; ++j)
      if (plans[j] == plans[k]) { delete b; return WQ_EINVAL; }   // a plan's buffers serve one patch at a time
    b->plans.push_back(plans[k]);
    const wq_plan* pl = plans[k];
    auto it = std::find_if(b->classes.begin(), b->classes.end(), [&](const wq_batch::Class& c) {
      return c.p == pl->p && c.d == pl->d && c.prec == pl->prec;
    });
    if (it == b->classes.end()) {
      wq_batch::Class c;
      c.p = pl->p;
      c.d = pl->d;
      c.prec = pl->prec;
      b->classes.push_back(c);
      it = b->classes.end() - 1;
    }
    it->members.push_back(k);
  }
  // workspace layout: counters, then per class its descriptor arrays
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  b->counters = take(2 * b->classes.size() * sizeof(int));
  for (wq_batch::Class& c : b->classes) {
    const size_t np = c.members.size();
    c.views = take(np * sizeof(wq::PlanView));
    c.outm = take(np * sizeof(void*));
    c.outs = take(np * sizeof(void*));
    c.itm = take((np + 1) * sizeof(int));
    c.its = take((np + 1) * sizeof(int));
    c.nsm = take(np * sizeof(int));
    c.nss = take(np * sizeof(int));
    c.blk = take((np + 1) * sizeof(int));
  }
  b->total_bytes = off;
  b->img.assign(off, 0);
  b->mass.assign(n, nullptr);
  b->stiff.assign(n, nullptr);
  *out = b;
  return WQ_OK;
}

wq_status wq_batch_sizes(const wq_batch* b, size_t* workspace_bytes, int* n_classes) {
  if (!b) return WQ_EINVAL;
  if (workspace_bytes) *workspace_bytes = b->total_bytes;
  if (n_classes) *n_classes = int(b->classes.size());
  return WQ_OK;
}

wq_status wq_batch_bind(wq_batch* b, void* workspace, size_t bytes, void* const* mass_vals,
                        void* const* stiff_vals, hipStream_t stream) {
  if (!b || !workspace) return bfail(b, WQ_EINVAL, "null workspace");
  if (bytes < b->total_bytes) return bfail(b, WQ_ENOSPACE, "batch workspace smaller than wq_batch_sizes()");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return bfail(b, WQ_ENOSPACE, "batch workspace must be 256-byte aligned");
  for (size_t k = 0; k < b->plans.size(); ++k)
    if (!b->plans[k]->bound) return bfail(b, WQ_ESTATE, "patch " + std::to_string(k) + " is not bound");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return bhip(b, e, "wq_batch_bind: device attributes");
  b->ws = static_cast<char*>(workspace);
  for (size_t k = 0; k < b->plans.size(); ++k) {
    b->mass[k] = mass_vals ? mass_vals[k] : nullptr;
    b->stiff[k] = stiff_vals ? stiff_vals[k] : nullptr;
  }
  for (wq_batch::Class& c : b->classes) {
    for (size_t k = 0; k < c.members.size(); ++k) {
      const int m = c.members[k];
      const wq::PlanView pv = b->plans[m]->view();
      std::memcpy(b->img.data() + c.views + k * sizeof(wq::PlanView), &pv, sizeof(pv));
      std::memcpy(b->img.data() + c.outm + k * sizeof(void*), &b->mass[m], sizeof(void*));
      std::memcpy(b->img.data() + c.outs + k * sizeof(void*), &b->stiff[m], sizeof(void*));
    }
    fill_schedule(b, c);
  }
  e = upload(b, stream);
  if (e != hipSuccess) return bhip(b, e, "wq_batch_bind: descriptor upload");
  // side streams and events of the concurrent classes, made here so that
  // a later graph capture only records work on them
  if (b->classes.size() > 1) e = b->make_side();
  if (e != hipSuccess) return bhip(b, e, "wq_batch_bind: side streams");
  b->bound = true;
  b->drop_graph();
  b->err.clear();
  return WQ_OK;
}

wq_status wq_batch_tune(wq_batch* b, int which, hipStream_t stream) {
  if (!b) return WQ_EINVAL;
  wq_status st = check_ready(b, which);
  if (st != WQ_OK) return st;
  hipError_t e = join_all(b, stream);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  for (size_t k = 0; k < b->classes.size() && e == hipSuccess; ++k) {
    wq_batch::Class& c = b->classes[k];
    float best = 1e30f;
    int best_t = c.seg_target, best_g = c.wgs_per_cu;
    // the persistent schedules, then one launch per patch (g = 0)
    std::vector<std::pair<int, int>> cands;
    for (int tgt : kSegTargets)
      for (int g : kWgsPerCu) cands.emplace_back(tgt, g);
    cands.emplace_back(0, 0);
    for (const auto& cand : cands) {
      const int tgt = cand.first, g = cand.second;
      c.seg_target = tgt;
      c.wgs_per_cu = g;
      fill_schedule(b, c);
      e = upload(b, stream);
      if (e == hipSuccess) e = enqueue(b, which, stream, int(k));   // warm-up
      if (e == hipSuccess) e = hipEventRecord(t0, stream);
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) e = enqueue(b, which, stream, int(k));
      if (e == hipSuccess) e = hipEventRecord(t1, stream);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (e != hipSuccess) break;
      if (ms < best) {
        best = ms;
        best_t = tgt;
        best_g = g;
      }
    }
    c.seg_target = best_t;
    c.wgs_per_cu = best_g;
    fill_schedule(b, c);
  }
  if (e == hipSuccess) e = upload(b, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (e != hipSuccess) return bhip(b, e, "wq_batch_tune");
  b->drop_graph();
  return WQ_OK;
}

wq_status wq_batch_assemble(wq_batch* b, int which, int use_graph, hipStream_t stream) {
  if (!b) return WQ_EINVAL;
  wq_status st = check_ready(b, which);
  if (st != WQ_OK) return st;
  if (use_graph && !stream) return bfail(b, WQ_EINVAL, "graph capture needs a stream other than the legacy default stream");
  hipError_t e = join_all(b, stream);
  if (e != hipSuccess) return bhip(b, e, "wq_batch_assemble: join");
  if (!use_graph) {
    e = enqueue(b, which, stream);
    return e == hipSuccess ? WQ_OK : bhip(b, e, "wq_batch_assemble");
  }
  if (!b->graph || b->graph_which != which || b->graph_stream != stream) {
    b->drop_graph();
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bhip(b, e, "wq_batch_assemble: begin capture");
    hipError_t el = enqueue(b, which, stream);
    e = hipStreamEndCapture(stream, &g);
    if (el != hipSuccess) e = el;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->graph = nullptr;
      return bhip(b, e, "wq_batch_assemble: capture");
    }
    b->graph_which = which;
    b->graph_stream = stream;
  }
  e = hipGraphLaunch(b->graph, stream);
  return e == hipSuccess ? WQ_OK : bhip(b, e, "wq_batch_assemble: graph launch");
}

wq_status wq_batch_schedule(const wq_batch* b, int k, int* info) {
  if (!b || !info || k < 0 || k >= int(b->classes.size())) return WQ_EINVAL;
  const wq_batch::Class& c = b->classes[k];
  info[0] = c.p;
  info[1] = c.d;
  info[2] = c.prec;
  info[3] = int(c.members.size());
  info[4] = c.seg_target;
  info[5] = c.wgs_per_cu;
  return WQ_OK;
}

const char* wq_batch_last_error(const wq_batch* b) { return b ? b->err.c_str() : "null batch"; }

void wq_batch_destroy(wq_batch* b) { delete b; }

}  // extern "C"
