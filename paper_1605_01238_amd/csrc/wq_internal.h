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

// Per-span operand tables of the direction-1 contraction in the lane layout
// of the 16x16x4 matrix instructions (see the pencil kernel).  For knot-span
// e of direction 1 and k-step ks, lane l = m + 16k of the A table holds
// B^(alpha)_{e+m-p}(x_q) (0 unless 0 <= m-p <= p): the operand of the open
// row e (s = 0); row e+s uses the same values moved up by s lanes.  The point
// is q = first point of e + c with (c, alpha) = (kappa/2, kappa%2),
// kappa = 4 ks + k (the mass uses alpha = 0 only: its alpha = 1 entries
// are zero).  The weight
// tables hold, per (e, ks, s, k), the weights of row e+s at that point:
// (w^(alpha,0), w^(alpha,1)) for the stiffness, w^(0,0) for the mass.
struct LaneTables {
  int kss, ksm;           // k-steps per span (stiffness, mass)
  size_t a64, w64, am64, wm64, a32, w32, am32, wm32, total;   // byte offsets
};
__host__ __device__ inline LaneTables lane_tables(int p, int nel1) {
  LaneTables t;
  t.kss = (2 * (p + 2) + 3) / 4;
  t.ksm = t.kss;
  const size_t ne = size_t(nel1), nw = size_t(nel1) * (p + 1);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~size_t(255); return o; };
  t.a64 = take(ne * t.kss * 64 * 8);
  t.w64 = take(nw * t.kss * 4 * 2 * 8);
  t.am64 = take(ne * t.ksm * 64 * 8);
  t.wm64 = take(nw * t.ksm * 4 * 8);
  t.a32 = take(ne * t.kss * 64 * 4);
  t.w32 = take(nw * t.kss * 4 * 2 * 4);
  t.am32 = take(ne * t.ksm * 64 * 4);
  t.wm32 = take(nw * t.ksm * 4 * 4);
  t.total = off;
  return t;
}

struct PlanView {
  int p;
  int prec;
  int d;                 // 3, or 2: then direction 3 is the trivial one (one
                         // function, one point, nel = 0, operator T^(0,0) = 1)
  DirView dir[3];
  void* field;           // kNumChannels * nqtot in the plan precision
  void* ybuf;            // [n3][nq2][nq1][icap][kYChannels]: field contracted over q3 per test index i3
  char* lanes;           // per-span operand tables of direction 1 (LaneTables)
  double* ctrl;          // n3*n2*n1*3 (n2*n1*2 in 2D)
  double* dctrl;         // 3 * n3*n2*n1*3: C_i - C_{i - e_b} along direction b (0 where i_b = 0)
  int32_t* flags;        // kNumFlags
  int64_t nqtot;
};

struct Layout {
  size_t knots[3], x[3], qspan[3], bv[3], bd[3], bw[3], w[3], op64[3], op32[3], bt64[3], bt32[3], wt64[3], wt32[3], prefix[3], colt64[3], colt32[3];
  size_t field, ybuf, lanes, ctrl, dctrl, flags, total;
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
  std::string err;
  // The univariate stage runs on a second stream, forked from the caller's
  // stream at wq_setup and joined by the calls that read its tables.
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_rules = nullptr;
  bool rules_launched = false;
  wq::PlanView view() const;
  ~wq_plan();
};

namespace wq {
// Kernel launchers (return hipError_t of the launch).
hipError_t launch_points(const PlanView& v, hipStream_t s);
hipError_t launch_rules(const PlanView& v, hipStream_t s);
hipError_t launch_lanes(const PlanView& v, hipStream_t s);
hipError_t launch_prefix(const PlanView& v, hipStream_t s);
hipError_t launch_ctrl_diff(const PlanView& v, const double* ctrl, hipStream_t s);
hipError_t launch_geometry(const PlanView& v, const double* coef, double* xphys_out, hipStream_t s);
hipError_t launch_pattern(const PlanView& v, int64_t* row_ptr, int32_t* col_idx, hipStream_t s);
hipError_t launch_qranges(const PlanView& v, int dir, int32_t* q_start, int32_t* q_count, hipStream_t s);
hipError_t launch_assemble(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s);
}  // namespace wq
