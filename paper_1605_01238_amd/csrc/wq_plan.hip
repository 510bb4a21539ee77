// C ABI entry points: plan validation, sizes, workspace layout, and the
// ordering of the device stages.  See include/wq.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "wq_internal.h"

namespace {

// Message of the last failed wq_plan_create of this thread (no plan exists
// to carry it); returned by wq_last_error(NULL).
thread_local std::string g_create_err;

wq_status create_fail(wq_status st, const std::string& msg) {
  g_create_err = msg;
  return st;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

wq_status fail(wq_plan* plan, wq_status st, const std::string& msg) {
  if (plan) plan->err = msg;
  return st;
}

wq_status hip_fail(wq_plan* plan, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(plan, WQ_EDEVICE, m);
}

// Validates one knot vector; returns "" if fine.
std::string check_knots(const double* k, int64_t len, int p, int64_t* nel_out) {
  if (len < 2 * (p + 1) + 1) return "knot vector too short";
  for (int64_t i = 0; i < len; ++i)
    if (!std::isfinite(k[i])) return "non-finite knot";
  for (int64_t i = 0; i + 1 < len; ++i)
    if (k[i + 1] < k[i]) return "knots must be non-decreasing";
  for (int i = 1; i <= p; ++i)
    if (k[i] != k[0] || k[len - 1 - i] != k[len - 1]) return "knot vector must be open (end knots repeated p+1 times)";
  if (!(k[p + 1] > k[p]) || !(k[len - 1 - p] > k[len - 2 - p])) return "knot vector must be open (end knots repeated exactly p+1 times)";
  for (int64_t i = p + 1; i + 1 < len - p; ++i)
    if (!(k[i + 1] > k[i])) return "interior knots must be simple (maximal regularity C^{p-1})";
  int64_t nel = len - 2 * p - 1;
  if (nel < p + 2) return "need at least p+2 knot-spans per direction";
  *nel_out = nel;
  return "";
}

void compute_layout(wq_plan* pl) {
  wq::Layout& L = pl->lay;
  size_t off = 0;
  const int p = pl->p, qc = wq::qcap_of(p), ic = wq::icap_of(p);
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  for (int k = 0; k < 3; ++k) {
    const size_t n = size_t(pl->n[k]), nq = size_t(pl->nq[k]);
    L.knots[k] = take((n + p + 1) * 8);
    L.x[k] = take(nq * 8);
    L.qspan[k] = take(nq * 4);
    L.bv[k] = take(nq * (p + 1) * 8);
    L.bd[k] = take(nq * (p + 1) * 8);
    L.bw[k] = take(nq * p * 8);
    L.w[k] = take(4 * n * qc * 8);
    L.op64[k] = take(4 * n * ic * qc * 8);
    L.op32[k] = take(4 * n * ic * qc * 4);
    L.bt64[k] = take(2 * n * ic * qc * 8);
    L.bt32[k] = take(2 * n * ic * qc * 4);
    L.b0t64[k] = take(n * ic * qc * 8);
    L.b0t32[k] = take(n * ic * qc * 4);
    L.wt64[k] = take(4 * n * qc * 8);
    L.wt32[k] = take(4 * n * qc * 4);
    L.prefix[k] = take((n + 1) * 8);
    L.colt64[k] = take(nq * 6 * (p + 1) * 8);
    L.colt32[k] = take(nq * 6 * (p + 1) * 4);
  }
  const size_t elem = pl->prec == WQ_FP64 ? 8 : 4;
  L.field = take(size_t(wq::kNumChannels) * size_t(pl->nqtot) * elem);
  // first contraction (over q3) of the coefficient field: [n3][nq2][nq1][icap][8];
  // before an assembly it also holds the geometry pass intermediates
  // ([nq3][n2][n1][9] and [nq3][nq2][n1][9] doubles)
  const size_t ybytes = size_t(pl->n[2]) * size_t(pl->nq[1]) * size_t(pl->nq[0]) * ic * wq::kYChannels * elem;
  const size_t gbytes = size_t(pl->nq[2]) * size_t(pl->n[0]) * (size_t(pl->n[1]) + size_t(pl->nq[1])) * 9 * 8;
  L.ybuf = take(ybytes > gbytes ? ybytes : gbytes);
  // the mass matrix's own first-contraction buffer (one channel; a plane
  // patch or curve has no first contraction)
  L.ymass = take(pl->d == 3 ? size_t(pl->n[2]) * size_t(pl->nq[1]) * size_t(pl->nq[0]) * ic * elem : 0);
  L.ctrl = take(size_t(pl->nrows) * 3 * 8);
  L.dctrl = take(size_t(pl->nrows) * 9 * 8);
  L.wts = take(size_t(pl->nrows) * 8);
  L.flags = take(wq::kNumFlags * 4);
  L.total = off;
}

}  // namespace

wq_plan::~wq_plan() {
  if (aux) {
    (void)hipStreamSynchronize(aux);
    (void)hipStreamDestroy(aux);
  }
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_rules) (void)hipEventDestroy(ev_rules);
  if (ev_mass_fork) (void)hipEventDestroy(ev_mass_fork);
  if (ev_mass_join) (void)hipEventDestroy(ev_mass_join);
}

wq::PlanView wq_plan::view() const {
  wq::PlanView v{};
  v.p = p;
  v.prec = prec;
  v.d = d;
  for (int k = 0; k < 3; ++k) {
    wq::DirView& d = v.dir[k];
    d.n = int(n[k]);
    d.nel = int(nel[k]);
    d.nq = int(nq[k]);
    d.knots = reinterpret_cast<const double*>(ws + lay.knots[k]);
    d.x = reinterpret_cast<double*>(ws + lay.x[k]);
    d.qspan = reinterpret_cast<int32_t*>(ws + lay.qspan[k]);
    d.bv = reinterpret_cast<double*>(ws + lay.bv[k]);
    d.bd = reinterpret_cast<double*>(ws + lay.bd[k]);
    d.bw = reinterpret_cast<double*>(ws + lay.bw[k]);
    d.w = reinterpret_cast<double*>(ws + lay.w[k]);
    d.op64 = reinterpret_cast<double*>(ws + lay.op64[k]);
    d.op32 = reinterpret_cast<float*>(ws + lay.op32[k]);
    d.bt64 = reinterpret_cast<double*>(ws + lay.bt64[k]);
    d.bt32 = reinterpret_cast<float*>(ws + lay.bt32[k]);
    d.b0t64 = reinterpret_cast<double*>(ws + lay.b0t64[k]);
    d.b0t32 = reinterpret_cast<float*>(ws + lay.b0t32[k]);
    d.wt64 = reinterpret_cast<double*>(ws + lay.wt64[k]);
    d.wt32 = reinterpret_cast<float*>(ws + lay.wt32[k]);
    d.prefix = reinterpret_cast<int64_t*>(ws + lay.prefix[k]);
    d.colt64 = reinterpret_cast<double*>(ws + lay.colt64[k]);
    d.colt32 = reinterpret_cast<float*>(ws + lay.colt32[k]);
  }
  v.field = ws + lay.field;
  v.ybuf = ws + lay.ybuf;
  v.ctrl = reinterpret_cast<double*>(ws + lay.ctrl);
  v.dctrl = reinterpret_cast<double*>(ws + lay.dctrl);
  v.wts = rational ? reinterpret_cast<const double*>(ws + lay.wts) : nullptr;
  v.nurbs_basis = nurbs_basis ? 1 : 0;
  v.flags = reinterpret_cast<int32_t*>(ws + lay.flags);
  v.nqtot = nqtot;
  return v;
}

extern "C" {

const char* wq_version(void) { return "wq-gfx950 0.1"; }

wq_status wq_plan_create(int d, int p, const int64_t* n_knots, const double* const* knots,
                         int precision, wq_plan** out) {
  if (!out) return create_fail(WQ_EINVAL, "null output pointer");
  *out = nullptr;
  if (d < 1 || d > 3) return create_fail(WQ_EINVAL, "d must be 1, 2 or 3");
  if (p < WQ_MIN_P || p > WQ_MAX_P) return create_fail(WQ_EINVAL, "degree outside the compiled range");
  if (!n_knots || !knots) return create_fail(WQ_EINVAL, "null knot arrays");
  if (precision != WQ_FP64 && precision != WQ_FP32) return create_fail(WQ_EINVAL, "precision must be WQ_FP64 or WQ_FP32");
  wq_plan* pl = new (std::nothrow) wq_plan();
  if (!pl) return create_fail(WQ_EINVAL, "out of host memory");
  pl->d = d;
  pl->p = p;
  pl->prec = precision;
  int64_t nrows = 1, nnz = 1, nqtot = 1;
  // d < 3: directions d+1..3 are trivial (one function, one point; their
  // tables are constant and written by wq_bind), so the 3D kernels form the
  // rows of the lower-dimensional problem
  for (int k = d; k < 3; ++k) {
    pl->nel[k] = 0;
    pl->n[k] = 1;
    pl->nq[k] = 1;
  }
  for (int k = 0; k < d; ++k) {
    if (!knots[k] || n_knots[k] <= 0 || n_knots[k] > (int64_t(1) << 24)) {
      delete pl;
      return create_fail(WQ_EINVAL, "knot vector " + std::to_string(k) + ": null or bad length");
    }
    int64_t nel = 0;
    std::string msg = check_knots(knots[k], n_knots[k], p, &nel);
    if (!msg.empty()) {
      delete pl;
      return create_fail(WQ_EKNOTS, "knot vector " + std::to_string(k) + ": " + msg);
    }
    pl->knots[k].assign(knots[k], knots[k] + n_knots[k]);
    pl->nel[k] = nel;
    pl->n[k] = nel + p;
    pl->nq[k] = 2 * nel + 2 * p - 1;
    nrows *= pl->n[k];
    nnz *= (2 * p + 1) * pl->n[k] - p * (p + 1);   // Section 3, 1D count; tensor product
    nqtot *= pl->nq[k];
  }
  // 32-bit index limits of the kernels: column and quadrature-point indices,
  // and element offsets within one i3 plane of the first-contraction buffer
  // (solid patches only: plane patches and curves have none)
  if (nrows >= (int64_t(1) << 31) || nqtot >= (int64_t(1) << 31)) {
    delete pl;
    return create_fail(WQ_EINVAL, "patch too large: N_DOF and N_QP must stay below 2^31");
  }
  const int64_t yplane = pl->nq[0] * pl->nq[1] * wq::icap_of(p) * wq::kYChannels;
  if (d == 3 && yplane >= (int64_t(1) << 32)) {
    delete pl;
    return create_fail(WQ_EINVAL, "patch too large: n_qp1 * n_qp2 * (2p+1) * 8 must stay below 2^32");
  }
  pl->nrows = nrows;
  pl->nnz = nnz;
  pl->nqtot = nqtot;
  compute_layout(pl);
  g_create_err.clear();
  *out = pl;
  return WQ_OK;
}

wq_status wq_sizes(const wq_plan* plan, wq_sizes_t* out) {
  if (!plan || !out) return WQ_EINVAL;
  for (int k = 0; k < 3; ++k) {
    out->n[k] = plan->n[k];
    out->n_qp[k] = plan->nq[k];
  }
  out->n_rows = plan->nrows;
  out->nnz = plan->nnz;
  out->n_qp_total = plan->nqtot;
  out->workspace_bytes = plan->lay.total;
  out->value_bytes = size_t(plan->nnz) * (plan->prec == WQ_FP64 ? 8 : 4);
  return WQ_OK;
}

wq_status wq_qpoints(const wq_plan* plan, int dir, double* x) {
  if (!plan || !x || dir < 0 || dir >= plan->d) return WQ_EINVAL;
  const int p = plan->p;
  const int nel = int(plan->nel[dir]);
  const double* k = plan->knots[dir].data();
  for (int q = 0; q < plan->nq[dir]; ++q) {
    double v;
    if (q <= p) {
      v = k[p] + (q + 1) * ((k[p + 1] - k[p]) / (p + 2));
    } else if (q >= p + 2 * nel - 2) {
      const int t = q - (p + 2 * nel - 2);
      v = k[p + nel - 1] + (t + 1) * ((k[p + nel] - k[p + nel - 1]) / (p + 2));
    } else {
      const int m = q - p;
      v = (m & 1) ? k[p + (m + 1) / 2] : 0.5 * (k[p + m / 2] + k[p + m / 2 + 1]);
    }
    x[q] = v;
  }
  return WQ_OK;
}

wq_status wq_bind(wq_plan* plan, void* workspace, size_t bytes, hipStream_t stream) {
  if (!plan || !workspace) return fail(plan, WQ_EINVAL, "null workspace");
  if (bytes < plan->lay.total) return fail(plan, WQ_ENOSPACE, "workspace smaller than wq_sizes().workspace_bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(plan, WQ_ENOSPACE, "workspace must be 256-byte aligned");
  plan->ws = static_cast<char*>(workspace);
  plan->ws_bytes = bytes;
  plan->bound = true;
  plan->setup_done = false;
  for (int k = 0; k < plan->d; ++k) {
    hipError_t e = hipMemcpyAsync(plan->ws + plan->lay.knots[k], plan->knots[k].data(),
                                  plan->knots[k].size() * 8, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(plan, e, "wq_bind: knot upload");
  }
  // the trivial directions: qspan = 0, T^(0,0) = B^(0) = w^(0,0) = 1 at the
  // one point and function, every other rule and B^(1) zero
  for (int k = plan->d; k < 3; ++k) {
    const int ic = wq::icap_of(plan->p), qc = wq::qcap_of(plan->p);
    static const double one64 = 1.0;
    static const float one32 = 1.0f;
    const wq::Layout& L = plan->lay;
    char* w = plan->ws;
    hipError_t e = hipMemsetAsync(w + L.qspan[k], 0, 4, stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.op64[k], 0, size_t(4) * ic * qc * 8, stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.op32[k], 0, size_t(4) * ic * qc * 4, stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.bt64[k], 0, size_t(2) * ic * qc * 8, stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.bt32[k], 0, size_t(2) * ic * qc * 4, stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.b0t64[k], 0, size_t(ic) * qc * 8, stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.b0t32[k], 0, size_t(ic) * qc * 4, stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.wt64[k], 0, size_t(4) * qc * 8, stream);
    if (e == hipSuccess) e = hipMemsetAsync(w + L.wt32[k], 0, size_t(4) * qc * 4, stream);
    for (size_t off : {L.op64[k], L.bt64[k], L.b0t64[k], L.wt64[k]})
      if (e == hipSuccess) e = hipMemcpyAsync(w + off, &one64, 8, hipMemcpyHostToDevice, stream);
    for (size_t off : {L.op32[k], L.bt32[k], L.b0t32[k], L.wt32[k]})
      if (e == hipSuccess) e = hipMemcpyAsync(w + off, &one32, 4, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(plan, e, "wq_bind: trivial direction");
  }
  hipError_t e = hipMemsetAsync(plan->ws + plan->lay.flags, 0, wq::kNumFlags * 4, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_bind: flag reset");
  // FLAG_DETJ_FIRST / FLAG_SOLVE_FIRST start at INT_MAX (atomicMin targets).
  static const int32_t init[2] = {0x7fffffff, 0x7fffffff};
  e = hipMemcpyAsync(plan->ws + plan->lay.flags + 4 * wq::FLAG_DETJ_FIRST, &init[0], 4, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(plan->ws + plan->lay.flags + 4 * wq::FLAG_SOLVE_FIRST, &init[1], 4, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_bind: flag init");
  e = wq::launch_points(plan->view(), stream);
  if (e == hipSuccess) e = wq::launch_prefix(plan->view(), stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_bind: points kernel");
  if (!plan->aux) {
    e = hipStreamCreateWithFlags(&plan->aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ev_rules, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ev_mass_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ev_mass_join, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(plan, e, "wq_bind: stream/event creation");
  }
  plan->rules_launched = false;
  plan->err.clear();
  return WQ_OK;
}

// Make `stream` wait for the univariate stage of the last wq_setup.
static hipError_t join_rules(const wq_plan* plan, hipStream_t stream) {
  return plan->rules_launched ? hipStreamWaitEvent(stream, plan->ev_rules, 0) : hipSuccess;
}

static const char nurbs_stiff_msg[] =
    "the stiffness of rational (NURBS) test and trial functions is not formed: set up with WQ_BASIS_BSPLINE";
static wq_status setup_common(wq_plan* plan, const double* ctrl_dev, const double* coef_dev, hipStream_t stream,
                              bool rules);

wq_status wq_setup(wq_plan* plan, const double* ctrl_dev, const double* coef_dev, hipStream_t stream) {
  if (!plan) return WQ_EINVAL;
  if (!plan->bound) return fail(plan, WQ_ESTATE, "wq_setup before wq_bind");
  if (!ctrl_dev) return fail(plan, WQ_EINVAL, "null control net");
  plan->rational = false;
  plan->nurbs_basis = false;
  return setup_common(plan, ctrl_dev, coef_dev, stream, true);
}

wq_status wq_set_geometry(wq_plan* plan, const double* ctrl_dev, const double* coef_dev, hipStream_t stream) {
  if (!plan) return WQ_EINVAL;
  if (!plan->setup_done) return fail(plan, WQ_ESTATE, "wq_set_geometry before wq_setup");
  if (!ctrl_dev) return fail(plan, WQ_EINVAL, "null control net");
  plan->rational = false;
  plan->nurbs_basis = false;
  return setup_common(plan, ctrl_dev, coef_dev, stream, false);
}

wq_status wq_setup_nurbs(wq_plan* plan, const double* ctrl_dev, const double* weights_dev, const double* coef_dev,
                         int basis, hipStream_t stream) {
  if (!plan) return WQ_EINVAL;
  if (!plan->bound) return fail(plan, WQ_ESTATE, "wq_setup_nurbs before wq_bind");
  if (!ctrl_dev) return fail(plan, WQ_EINVAL, "null control net");
  if (!weights_dev) return fail(plan, WQ_EINVAL, "null weights");
  if (basis != WQ_BASIS_BSPLINE && basis != WQ_BASIS_NURBS)
    return fail(plan, WQ_EINVAL, "basis must be WQ_BASIS_BSPLINE or WQ_BASIS_NURBS");
  hipError_t e = hipMemcpyAsync(plan->ws + plan->lay.wts, weights_dev, size_t(plan->nrows) * 8,
                                hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_setup_nurbs: weights copy");
  plan->rational = true;
  plan->nurbs_basis = basis == WQ_BASIS_NURBS;
  return setup_common(plan, ctrl_dev, coef_dev, stream, true);
}

static wq_status setup_common(wq_plan* plan, const double* ctrl_dev, const double* coef_dev, hipStream_t stream,
                              bool rules = true) {
  wq::PlanView v = plan->view();
  hipError_t e;
  if (rules) {
    // univariate stage on the second stream, after everything already
    // queued on `stream` (earlier assemblies read the tables it rewrites)
    e = hipEventRecord(plan->ev_fork, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->aux, plan->ev_fork, 0);
    if (e == hipSuccess) e = wq::launch_rules(v, plan->aux);
    if (e == hipSuccess) e = hipEventRecord(plan->ev_rules, plan->aux);
    if (e != hipSuccess) return hip_fail(plan, e, "wq_setup: univariate kernel");
    plan->rules_launched = true;
  }
  if (plan->d == 3) {
    e = wq::launch_ctrl_diff(v, ctrl_dev, stream);
  } else {   // the 1D and 2D geometry kernels read the plan's copy of the net directly
    e = hipMemcpyAsync(v.ctrl, ctrl_dev, size_t(plan->nrows) * plan->d * 8, hipMemcpyDeviceToDevice, stream);
  }
  if (e != hipSuccess) return hip_fail(plan, e, "wq_setup: control-net differences");
  e = wq::launch_geometry(v, coef_dev, nullptr, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_setup: geometry kernel");
  plan->setup_done = true;
  plan->unit_coef = coef_dev == nullptr;
  return WQ_OK;
}

wq_status wq_set_coefficient(wq_plan* plan, const double* coef_dev, hipStream_t stream) {
  if (!plan) return WQ_EINVAL;
  if (!plan->setup_done) return fail(plan, WQ_ESTATE, "wq_set_coefficient before wq_setup");
  hipError_t e = wq::launch_geometry(plan->view(), coef_dev, nullptr, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_set_coefficient: geometry kernel");
  plan->unit_coef = coef_dev == nullptr;
  return WQ_OK;
}

// Request context: the coefficient field and the first-contraction buffer.
static void request_layout(const wq_plan* plan, size_t* field_off, size_t* y_off, size_t* total) {
  const size_t elem = plan->prec == WQ_FP64 ? 8 : 4;
  const size_t fbytes = size_t(wq::kNumChannels) * size_t(plan->nqtot) * elem;
  // (the strip kernel of a plane patch or curve reads the field directly)
  const size_t ybytes = plan->d == 3 ? size_t(plan->n[2]) * size_t(plan->nq[1]) * size_t(plan->nq[0]) *
                                           size_t(wq::icap_of(plan->p)) * wq::kYChannels * elem
                                     : 0;
  *field_off = 0;
  *y_off = align256(fbytes);
  *total = *y_off + align256(ybytes);
}

wq_status wq_request_bytes(const wq_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return WQ_EINVAL;
  size_t f, y;
  request_layout(plan, &f, &y, bytes);
  return WQ_OK;
}

wq_status wq_assemble_request(wq_plan* plan, void* ctx, size_t ctx_bytes, const double* coef_dev, int which,
                              void* mass, void* stiff, hipStream_t stream) {
  if (!plan) return WQ_EINVAL;
  if (!ctx) return fail(plan, WQ_EINVAL, "null request context");
  if (which <= 0 || (which & ~(WQ_MASS | WQ_STIFF))) return fail(plan, WQ_EINVAL, "which must be WQ_MASS, WQ_STIFF or both");
  if ((which & WQ_MASS) && !mass) return fail(plan, WQ_EINVAL, "null mass output");
  if ((which & WQ_STIFF) && !stiff) return fail(plan, WQ_EINVAL, "null stiffness output");
  if (!plan->setup_done) return fail(plan, WQ_ESTATE, "wq_assemble_request before wq_setup");
  if (!plan->unit_coef) return fail(plan, WQ_ESTATE, "wq_assemble_request needs the plan's field for a = 1 (set up or set with a NULL coefficient)");
  if (plan->nurbs_basis && (which & WQ_STIFF)) return fail(plan, WQ_EINVAL, nurbs_stiff_msg);
  size_t f, y, total;
  request_layout(plan, &f, &y, &total);
  if (ctx_bytes < total) return fail(plan, WQ_ENOSPACE, "request context smaller than wq_request_bytes()");
  if (reinterpret_cast<uintptr_t>(ctx) % 256 != 0) return fail(plan, WQ_ENOSPACE, "request context must be 256-byte aligned");
  hipError_t e = join_rules(plan, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_assemble_request: join");
  wq::PlanView v = plan->view();
  char* c = static_cast<char*>(ctx);
  e = wq::launch_scale_field(v, coef_dev, c + f, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_assemble_request: coefficient field");
  v.field = c + f;
  v.ybuf = c + y;
  e = wq::launch_assemble(v, which, mass, stiff, stream);
  if (e == hipSuccess && plan->nurbs_basis) e = wq::launch_nurbs_scale(v, mass, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_assemble_request: contraction kernel");
  return WQ_OK;
}

wq_status wq_qp_physical(const wq_plan* plan, double* x_dev, hipStream_t stream) {
  if (!plan || !x_dev) return WQ_EINVAL;
  if (!plan->setup_done) return WQ_ESTATE;
  hipError_t e = wq::launch_geometry(plan->view(), nullptr, x_dev, stream);
  return e == hipSuccess ? WQ_OK : WQ_EDEVICE;
}

wq_status wq_pattern(const wq_plan* plan, int64_t* row_ptr, int32_t* col_idx, hipStream_t stream) {
  if (!plan || !row_ptr || !col_idx) return WQ_EINVAL;
  if (!plan->bound) return WQ_ESTATE;
  hipError_t e = wq::launch_pattern(plan->view(), row_ptr, col_idx, stream);
  return e == hipSuccess ? WQ_OK : WQ_EDEVICE;
}

wq_status wq_assemble(wq_plan* plan, int which, void* mass, void* stiff, hipStream_t stream) {
  if (!plan) return WQ_EINVAL;
  if (which <= 0 || (which & ~(WQ_MASS | WQ_STIFF))) return fail(plan, WQ_EINVAL, "which must be WQ_MASS, WQ_STIFF or both");
  if ((which & WQ_MASS) && !mass) return fail(plan, WQ_EINVAL, "null mass output");
  if ((which & WQ_STIFF) && !stiff) return fail(plan, WQ_EINVAL, "null stiffness output");
  if (!plan->setup_done) return fail(plan, WQ_ESTATE, "wq_assemble before wq_setup");
  if (plan->nurbs_basis && (which & WQ_STIFF)) return fail(plan, WQ_EINVAL, nurbs_stiff_msg);
  hipError_t e = join_rules(plan, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_assemble: join");
  if (which == (WQ_MASS | WQ_STIFF)) {
    // both matrices: the mass on the plan's second stream with its own
    // first-contraction buffer, beside the stiffness; `stream` joins it
    wq::PlanView vm = plan->view();
    vm.ybuf = plan->ws + plan->lay.ymass;
    e = hipEventRecord(plan->ev_mass_fork, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->aux, plan->ev_mass_fork, 0);
    if (e == hipSuccess) e = wq::launch_assemble(vm, WQ_MASS, mass, nullptr, plan->aux);
    if (e == hipSuccess) e = wq::launch_assemble(plan->view(), WQ_STIFF, nullptr, stiff, stream);
    if (e == hipSuccess) e = hipEventRecord(plan->ev_mass_join, plan->aux);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream, plan->ev_mass_join, 0);
  } else {
    e = wq::launch_assemble(plan->view(), which, mass, stiff, stream);
    if (e == hipSuccess && plan->nurbs_basis) e = wq::launch_nurbs_scale(plan->view(), mass, stream);
  }
  if (e != hipSuccess) return hip_fail(plan, e, "wq_assemble: contraction kernel");
  return WQ_OK;
}

wq_status wq_assemble_static(wq_plan* plan, int which, void* mass, void* stiff, hipStream_t stream) {
  if (!plan) return WQ_EINVAL;
  if (which <= 0 || (which & ~(WQ_MASS | WQ_STIFF))) return fail(plan, WQ_EINVAL, "which must be WQ_MASS, WQ_STIFF or both");
  if ((which & WQ_MASS) && !mass) return fail(plan, WQ_EINVAL, "null mass output");
  if ((which & WQ_STIFF) && !stiff) return fail(plan, WQ_EINVAL, "null stiffness output");
  if (!plan->setup_done) return fail(plan, WQ_ESTATE, "wq_assemble_static before wq_setup");
  if (plan->nurbs_basis && (which & WQ_STIFF)) return fail(plan, WQ_EINVAL, nurbs_stiff_msg);
  const wq::PlanView v = plan->view();
  const size_t pb = wq::static_plane_bytes(v, which);
  if (pb > wq::kStaticScratchBytes) {
    char buf[200];
    std::snprintf(buf, sizeof buf, "one first-contraction plane needs %zu bytes; the static scratch holds %zu",
                  pb, wq::kStaticScratchBytes);
    return fail(plan, WQ_ENOSPACE, buf);
  }
  hipError_t e = join_rules(plan, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_assemble_static: join");
  e = wq::launch_assemble_static(v, which, mass, stiff, stream);
  if (e == hipSuccess && plan->nurbs_basis) e = wq::launch_nurbs_scale(v, mass, stream);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_assemble_static");
  return WQ_OK;
}

wq_status wq_weights(const wq_plan* plan, int dir, int pair, double* w_dev, int32_t* qs_dev,
                     int32_t* qc_dev, hipStream_t stream) {
  if (!plan || dir < 0 || dir >= plan->d || pair < 0 || pair > 3 || !w_dev) return WQ_EINVAL;
  if (!plan->setup_done) return WQ_ESTATE;
  const int p = plan->p, n = int(plan->n[dir]), qc = wq::qcap_of(p);
  const size_t bytes = size_t(n) * qc * 8;
  hipError_t e = join_rules(plan, stream);
  if (e != hipSuccess) return WQ_EDEVICE;
  e = hipMemcpyAsync(w_dev, plan->ws + plan->lay.w[dir] + size_t(pair) * bytes, bytes,
                     hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return WQ_EDEVICE;
  if (qs_dev || qc_dev) {
    e = wq::launch_qranges(plan->view(), dir, qs_dev, qc_dev, stream);
    if (e != hipSuccess) return WQ_EDEVICE;
  }
  return WQ_OK;
}

wq_status wq_field(const wq_plan* plan, void* field_dev, hipStream_t stream) {
  if (!plan || !field_dev) return WQ_EINVAL;
  if (!plan->setup_done) return WQ_ESTATE;
  const size_t bytes = size_t(wq::kNumChannels) * size_t(plan->nqtot) * (plan->prec == WQ_FP64 ? 8 : 4);
  hipError_t e = hipMemcpyAsync(field_dev, plan->ws + plan->lay.field, bytes, hipMemcpyDeviceToDevice, stream);
  return e == hipSuccess ? WQ_OK : WQ_EDEVICE;
}

wq_status wq_sync(wq_plan* plan, hipStream_t stream) {
  if (!plan) return WQ_EINVAL;
  hipError_t e = hipStreamSynchronize(stream);
  if (e == hipSuccess && plan->rules_launched) e = hipEventSynchronize(plan->ev_rules);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_sync");
  if (!plan->bound) return WQ_OK;
  int32_t f[wq::kNumFlags];
  e = hipMemcpy(f, plan->ws + plan->lay.flags, sizeof(f), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(plan, e, "wq_sync: flag read");
  wq_status st = WQ_OK;
  char buf[256];
  if (f[wq::FLAG_SOLVE_BAD] > 0) {
    std::snprintf(buf, sizeof buf, "%d weight systems broke down (first: %d)", f[wq::FLAG_SOLVE_BAD], f[wq::FLAG_SOLVE_FIRST]);
    plan->err = buf;
    st = WQ_ESINGULAR;
  }
  if (f[wq::FLAG_DETJ_BAD] > 0) {
    std::snprintf(buf, sizeof buf, "det J <= 0 at %d quadrature points (first linear index %d)", f[wq::FLAG_DETJ_BAD], f[wq::FLAG_DETJ_FIRST]);
    plan->err = buf;
    st = WQ_EGEOM;
  }
  if (st != WQ_OK) {
    const int32_t zero[4] = {0, 0x7fffffff, 0, 0x7fffffff};
    e = hipMemcpy(plan->ws + plan->lay.flags, zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(plan, e, "wq_sync: flag clear");
  }
  return st;
}

const char* wq_last_error(const wq_plan* plan) { return plan ? plan->err.c_str() : g_create_err.c_str(); }

void wq_plan_destroy(wq_plan* plan) { delete plan; }

}  // extern "C"
