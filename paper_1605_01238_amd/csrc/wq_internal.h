// Internal declarations of the weighted-quadrature library (not part of the ABI).
//
// Index conventions follow include/wq.h.  Per direction, with n_el knot-spans
// (distinct knots chi_0 < ... < chi_{n_el}), n = n_el + p basis functions and
// the quadrature points of Remark 4.1 numbered left to right:
//   q = 0..p                  : p+1 points inside the first span,
//   q = p + 2k - 1, k=1..n_el-1 : interior knot chi_k,
//   q = p + 2k,     k=1..n_el-2 : midpoint of the internal span k,
//   q = p + 2 n_el - 2 + t, t=0..p : p+1 points inside the last span.
// n_qp = 2 n_el + 2p - 1.  B_i is supported on the spans e in
// [max(0, i-p), min(n_el, i+1)); Q_i is the contiguous range of points
// strictly inside that support; I_i = [max(0, i-p), min(n-1, i+p)].
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wq.h"

namespace wq {

constexpr int kNumChannels = 7;   // det J, K11, K22, K33, K12, K13, K23
constexpr int kYChannels = 8;     // distinct (coefficient, dir-3 rule) pairs of the stiffness
constexpr int kNumFlags = 16;
// Scratch of the allocation-free assembly (a static device array per GPU).
constexpr size_t kStaticScratchBytes = WQ_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Latched device conditions (int32 counters in the workspace).
enum Flag : int {
  FLAG_DETJ_BAD = 0,      // count of quadrature points with det J <= 0 or not finite
  FLAG_DETJ_FIRST = 1,    // smallest offending linear quadrature-point index (atomicMin)
  FLAG_SOLVE_BAD = 2,     // count of weight systems that broke down
  FLAG_SOLVE_FIRST = 3,   // first offending (dir*4 + pair) * n + i
};

__host__ __device__ inline int qcap_of(int p) { return 3 * p + 1; }
__host__ __device__ inline int icap_of(int p) { return 2 * p + 1; }

__host__ __device__ inline int span_first_q(int e, int p, int nel) {
  return e == 0 ? 0 : (e <= nel - 2 ? p + 2 * e : p + 2 * nel - 2);
}
__host__ __device__ inline int span_last_q(int e, int p, int nel) {
  return e == 0 ? p : (e <= nel - 2 ? p + 2 * e : 2 * nel + 2 * p - 2);
}
// Q_i = [qs, qs + qc)
__host__ __device__ inline void q_range(int i, int p, int nel, int& qs, int& qc) {
  if (nel == 0) {   // trivial direction of a 1D or 2D problem: one point
    qs = 0;
    qc = 1;
    return;
  }
  int e0 = i - p > 0 ? i - p : 0;
  int e1 = i + 1 < nel ? i + 1 : nel;
  qs = span_first_q(e0, p, nel);
  qc = span_last_q(e1 - 1, p, nel) - qs + 1;
}
// I_i = [is, is + ic)
__host__ __device__ inline void i_range(int i, int p, int n, int& is, int& ic) {
  is = i - p > 0 ? i - p : 0;
  int ie = i + p < n - 1 ? i + p : n - 1;
  ic = ie - is + 1;
}

// Device views (passed by value to kernels).
struct DirView {
  int n, nel, nq;
  const double* knots;   // n + p + 1
  double* x;             // nq   quadrature points
  int32_t* qspan;        // nq   first nonzero function at x_q (= distinct-span index)
  double* bv;            // nq * (p+1) values of functions qspan..qspan+p at x_q
  double* bd;            // nq * (p+1) derivatives
  double* bw;            // nq * p  p N_{i,p-1}(x_q) / (xi_{i+p} - xi_i), i = qspan+1 .. qspan+p
  double* w;             // 4 * n * qcap   weights, pair = 2*beta + alpha
  // Tables of the contraction, laid out so that everything one quadrature
  // point qq of function i needs is contiguous (wide scalar loads):
  double* op64;          // [n][qcap][icap][4]  T^(o)[jj][qq] = B^(alpha)_{is+jj}(x_{qs+qq}) w^(o)_qq, o = 2*beta + alpha
  float* op32;           // same in FP32
  double* bt64;          // [n][qcap][icap][2]  B^(alpha)_{is+jj}(x_{qs+qq})
  float* bt32;
  double* b0t64;         // [n][qcap][icap]     B^(0) alone (the mass's operator, contiguous per qq)
  float* b0t32;
  double* wt64;          // [n][qcap][4]        w^(o)_qq
  float* wt32;
  int64_t* prefix;       // n + 1  prefix sums of #I_i
  // Per quadrature point q (span e = qspan[q]), for the rows i = e + s,
  // s = 0..p, whose support contains x_q: their four weights at x_q (0 if x_q
  // is not in Q_i or i >= n), then B_{e+r}(x_q) and B'_{e+r}(x_q), r = 0..p:
  // [nq][6(p+1)] = { w[s][o] (4(p+1)), b0[r] (p+1), b1[r] (p+1) }.
  double* colt64;
  float* colt32;
};

struct PlanView {
  int p;
  int prec;
  int d;                 // 3, 2 or 1: directions d+1..3 are trivial (one
                         // function, one point, nel = 0, rule w^(0,0) = 1,
                         // B^(0) = 1, every other rule and B^(1) zero)
  DirView dir[3];
  void* field;           // kNumChannels * nqtot in the plan precision
  void* ybuf;            // [n3][nq2][nq1][icap][kYChannels]: field contracted over q3 per test index i3
  double* ctrl;          // n3*n2*n1*3 (n2*n1*2 in 2D)
  double* dctrl;         // 3 * n3*n2*n1*3: C_i - C_{i - e_b} along direction b (0 where i_b = 0)
  int32_t* flags;        // kNumFlags
  int64_t nqtot;
  int y_i3;              // ybuf holds the first-contraction planes i3 >= y_i3
  const double* wts;     // NURBS weights of the net ([n3][n2][n1]), or null for a polynomial map
  int nurbs_basis;       // 1: rational test/trial functions (mass factor det J / W^2)
};

// One class (degree p, dimension d, precision) of a batch of patches, in
// the batch workspace: per patch its plan view, outputs, the prefix of its
// pencil-kernel work items and first-contraction blocks, and its runs of
// rows per pencil; two work-queue counters (mass, stiffness).
struct BatchClassView {
  const PlanView* views;
  void* const* out_mass;
  void* const* out_stiff;
  const int* items_mass;    // [np + 1]
  const int* items_stiff;   // [np + 1]
  const int* nsegs_mass;    // [np]
  const int* nsegs_stiff;   // [np]
  const int* blocks;        // [np + 1]
  int* counter;             // [2]
  int np;
};

struct Layout {
  size_t knots[3], x[3], qspan[3], bv[3], bd[3], bw[3], w[3], op64[3], op32[3], bt64[3], bt32[3], b0t64[3], b0t32[3], wt64[3], wt32[3], prefix[3], colt64[3], colt32[3];
  size_t field, ybuf, ymass, ctrl, dctrl, wts, flags, total;
};

}  // namespace wq

struct wq_plan {
  int d = 3, p = 0, prec = 0;
  int64_t n[3] = {0, 0, 0}, nel[3] = {0, 0, 0}, nq[3] = {0, 0, 0};
  std::vector<double> knots[3];
  int64_t nrows = 0, nnz = 0, nqtot = 0;
  wq::Layout lay{};
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false, setup_done = false;
  bool unit_coef = false;   // the field holds the coefficients of a = 1 (requests scale it)
  bool rational = false;    // NURBS map: weights in the workspace
  bool nurbs_basis = false; // rational test/trial functions (mass only)
  std::string err;
  // The univariate stage runs on a second stream, forked from the caller's
  // stream at wq_setup and joined by the calls that read its tables.
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_rules = nullptr;
  // wq_assemble of both matrices: the mass on `aux` (with a first-contraction
  // buffer of its own) beside the stiffness on the caller's stream
  hipEvent_t ev_mass_fork = nullptr, ev_mass_join = nullptr;
  bool rules_launched = false;
  wq::PlanView view() const;
  ~wq_plan();
};

namespace wq {
// Kernel launchers (return hipError_t of the launch).
hipError_t launch_points(const PlanView& v, hipStream_t s);
hipError_t launch_rules(const PlanView& v, hipStream_t s);
hipError_t launch_prefix(const PlanView& v, hipStream_t s);
hipError_t launch_ctrl_diff(const PlanView& v, const double* ctrl, hipStream_t s);
hipError_t launch_geometry(const PlanView& v, const double* coef, double* xphys_out, hipStream_t s);
hipError_t launch_pattern(const PlanView& v, int64_t* row_ptr, int32_t* col_idx, hipStream_t s);
hipError_t launch_qranges(const PlanView& v, int dir, int32_t* q_start, int32_t* q_count, hipStream_t s);
// field_out = the plan's field with channels K (1..6) multiplied by a(x_q).
// Row i, column j of a mass matrix with rational test/trial functions:
// value * w_i * w_j (rows in closed-form CSR order).
hipError_t launch_nurbs_scale(const PlanView& v, void* vals, hipStream_t s);
hipError_t launch_scale_field(const PlanView& v, const double* coef, void* field_out, hipStream_t s);
hipError_t launch_assemble(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s);
// The same rows with the first-contraction buffer in the library's static
// scratch, i3 plane slab by slab (no allocation of any kind; a plane patch
// or curve uses no buffer).
hipError_t launch_assemble_static(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s);
// Bytes of one first-contraction plane (one i3) for the matrices of `which`
// (0 for d <= 2: no first contraction there).
size_t static_plane_bytes(const PlanView& v, int which);
// Batched form: one class of patches (first contraction over all blocks,
// then the persistent pencil kernel with `grid` workgroups).
hipError_t launch_batch_class(const BatchClassView& b, int p, int d, int prec, bool stiff, int first_blocks,
                              int grid, hipStream_t s);
hipError_t launch_zero_counters(int* c, int n, hipStream_t s);
// Work units per run of rows for (p, d, precision, matrix) on a patch with
// n2 x n3 pencils: (pencil, j3 part) pairs of a solid patch, strips of rows
// i2 of a plane patch or curve.
int64_t push_units(int p, int d, int prec, bool stiff, int n2, int n3);
}  // namespace wq
