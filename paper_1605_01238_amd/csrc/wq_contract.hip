// Row formation by sum factorization (Section 6, eq. sumfactorization,
// Algorithm 3) for the mass matrix, and its stiffness analogue (eq. stiff):
// the sum over the 9 pairs (l, m) of test/trial derivative directions, where
// direction k uses the rule w^(alpha_k, beta_k) with alpha_k = [k == m]
// (trial) and beta_k = [k == l] (test), applied to the coefficient c_lm.
//
// Work decomposition.  The first contraction (over q3) does not depend on
// i1 or i2, so it is done once per test index i3 for the whole (q1, q2)
// plane by k_first and kept in HBM.  A workgroup of the pencil kernel then
// owns a run of consecutive rows (i1 = r0..r1-1, i2, i3) of one pencil,
// restricted to a range of trial indices j3 ("part"); its items are the
// pairs n = (j3, j2) of that range.  The operators of direction 2 are fixed
// along the pencil, so the contraction over q2 is done once per quadrature
// column q1 and shared by all rows:
//
//   phase B (VALU, items: dir-1 group g, column q1, j3): read the channels
//            of the first contraction at every q2 of Q_i2, fold in the
//            dir-2 weights (terms that meet the same B2^(alpha) and the same
//            dir-1 rule are summed after scaling: "weight merge") and
//            contract with B2^(alpha) into G_g[q1][n], g = 2*beta + alpha
//            the dir-1 rule (4 groups for the stiffness, 1 for the mass),
//            staged in LDS.
//   phase C (matrix cores): knot-span e of direction 1 touches only the rows
//            i1 = e..e+p and, in each, only the trial functions j1 = e..e+p.
//            For the open row e+s and every item n,
//              V[e+s][d][n] += sum_(c, alpha) B^(alpha)_{e+r}(x_c) H_s[(c, alpha)][n],
//              H_s = w^(alpha,0)_{e+s}(x_c) G_(alpha,0)[c][n] + w^(alpha,1)_{e+s}(x_c) G_(alpha,1)[c][n],
//            d = r - s + p, summed over the span's points c: one 16x16x4
//            matrix product per k-step of 4 (point, alpha) pairs (interior
//            spans have 2 points: one k-step), rows d, columns n.  The p+1
//            open rows live in matrix-core accumulators; a row is stored
//            when its last span has been seen.  The span loop is unrolled
//            p+1 times so that the accumulator of each open row is a
//            compile-time choice (no data moves when the window advances).
//
// A run of rows r0..r1-1 needs the spans max(0, r0-p) .. min(n_el-1, r1-1);
// splitting a pencil into runs repeats phase B for p spans per run, which
// buys workgroups when a patch has few pencils.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <type_traits>

#include "wq_internal.h"

// Pencils are split into runs of rows until the grid holds about this many
// workgroups.
#ifndef WQ_WG_TARGET
#define WQ_WG_TARGET 2048
#endif

namespace wq {
namespace {

// Rule index o = 2*beta + alpha of the univariate tables.
enum : int { R00 = 0, R10 = 1, R01 = 2, R11 = 3 };

template <typename T> struct V2;
template <> struct V2<double> { typedef double2 type; };
template <> struct V2<float> { typedef float2 type; };
template <typename T>
using T2v = typename V2<T>::type;
template <typename T> struct V4;
template <> struct V4<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <> struct V4<float> { typedef float type __attribute__((ext_vector_type(4))); };

// D += A B for a 16x4 A and a 4x16 B (one value of each per lane: lane
// l = i + 16 k holds A[i][k] and B[k][i]).  Element r of lane l is
// D[drow<T>(l / 16, r)][l % 16]: the FP64 instruction interleaves the rows
// of D over the four lane groups, the FP32 one gives each group four
// consecutive rows.
__device__ __forceinline__ V4<double>::type mma(double a, double b, V4<double>::type c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ V4<float>::type mma(float a, float b, V4<float>::type c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T>
__device__ __forceinline__ constexpr int drow(int kq, int r) { return sizeof(T) == 8 ? kq + 4 * r : 4 * kq + r; }

// Lane i + 1 of the same 16-lane row moved to lane i (0 into lane 15 of
// each row): the A operand of open row s+1 from that of row s.
__device__ __forceinline__ float row_up(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x101, 0xf, 0xf, true));
}
__device__ __forceinline__ double row_up(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(b)), 0x101, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), 0x101, 0xf, 0xf, true);
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(unsigned(hi)) << 32) | unsigned(lo));
}

// Uniform table data read through the constant address space: scalar loads.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> to_const(const T* p) {
  return reinterpret_cast<cptr<T>>(reinterpret_cast<uintptr_t>(p));
}

template <typename T>
__device__ inline const T* op_t(const DirView& d) {
  if constexpr (sizeof(T) == 8) return reinterpret_cast<const T*>(d.op64);
  else return reinterpret_cast<const T*>(d.op32);
}
template <typename T>
__device__ inline const T* bt_t(const DirView& d) {
  if constexpr (sizeof(T) == 8) return reinterpret_cast<const T*>(d.bt64);
  else return reinterpret_cast<const T*>(d.bt32);
}
template <typename T>
__device__ inline const T* wt_t(const DirView& d) {
  if constexpr (sizeof(T) == 8) return reinterpret_cast<const T*>(d.wt64);
  else return reinterpret_cast<const T*>(d.wt32);
}

// n consecutive values (n a multiple of the vector width, 16-byte aligned)
template <typename T, int NV>
__device__ inline void store_vec(T* __restrict__ p, const T (&v)[NV]) {
  if constexpr (sizeof(T) == 8 && NV % 2 == 0) {
#pragma unroll
    for (int k = 0; k < NV / 2; ++k) reinterpret_cast<double2*>(p)[k] = double2{v[2 * k], v[2 * k + 1]};
  } else if constexpr (sizeof(T) == 4 && NV % 4 == 0) {
#pragma unroll
    for (int k = 0; k < NV / 4; ++k)
      reinterpret_cast<float4*>(p)[k] = float4{v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]};
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) p[k] = v[k];
  }
}

// Points of knot-span e of a direction, numbered as in wq_internal.h: the
// first span holds p+1 points, an interior span its left knot and its
// midpoint, the last span its left knot and p+1 points.
__host__ __device__ inline int span_q0(int e, int p) { return e == 0 ? 0 : p + 2 * e - 1; }
__host__ __device__ inline int span_np(int e, int p, int nel) { return e == 0 ? p + 1 : (e == nel - 1 ? p + 2 : 2); }

// Per-span operand tables of the direction-1 contraction (see LaneTables),
// from the column tables of direction 1: one block per (span e, open row s);
// the A tables are those of s = 0.
template <int P>
__global__ __launch_bounds__(64) void k_lanes(PlanView v) {
  const DirView d = v.dir[0];
  const LaneTables lt = lane_tables(P, d.nel);
  const int e = blockIdx.x, s = blockIdx.y, l = threadIdx.x;
  const int m = l % 16, k = l / 16;
  const int q0 = span_q0(e, P), np = span_np(e, P, d.nel);
  const int r = m - P;   // trial function e + r sits in row m of A
  constexpr int NCT = 6 * (P + 1);
  double* a64 = reinterpret_cast<double*>(v.lanes + lt.a64);
  double* w64 = reinterpret_cast<double*>(v.lanes + lt.w64);
  double* am64 = reinterpret_cast<double*>(v.lanes + lt.am64);
  double* wm64 = reinterpret_cast<double*>(v.lanes + lt.wm64);
  float* a32 = reinterpret_cast<float*>(v.lanes + lt.a32);
  float* w32 = reinterpret_cast<float*>(v.lanes + lt.w32);
  float* am32 = reinterpret_cast<float*>(v.lanes + lt.am32);
  float* wm32 = reinterpret_cast<float*>(v.lanes + lt.wm32);
  for (int ks = 0; ks < lt.kss; ++ks) {   // stiffness: kappa = (point, alpha)
    const int kap = 4 * ks + k, c = kap / 2, al = kap % 2;
    double a = 0.0, w0 = 0.0, w1 = 0.0;
    if (c < np) {
      const double* ct = d.colt64 + size_t(q0 + c) * NCT;
      if (r >= 0 && r <= P) a = ct[(4 + al) * (P + 1) + r];
      w0 = ct[s * 4 + al];        // w^(alpha,0)
      w1 = ct[s * 4 + 2 + al];    // w^(alpha,1)
    }
    const size_t ia = size_t(e) * lt.kss + ks;
    if (s == 0) {
      a64[ia * 64 + l] = a;
      a32[ia * 64 + l] = float(a);
    }
    if (m == 0) {
      const size_t iw = (ia * (P + 1) + s) * 4 + k;
      w64[iw * 2] = w0;
      w64[iw * 2 + 1] = w1;
      w32[iw * 2] = float(w0);
      w32[iw * 2 + 1] = float(w1);
    }
  }
  for (int ks = 0; ks < lt.ksm; ++ks) {   // mass: kappa = (point, alpha), alpha = 1 empty
    const int kap = 4 * ks + k, c = kap / 2, al = kap % 2;
    double a = 0.0, w = 0.0;
    if (c < np && al == 0) {
      const double* ct = d.colt64 + size_t(q0 + c) * NCT;
      if (r >= 0 && r <= P) a = ct[4 * (P + 1) + r];
      w = ct[s * 4 + R00];
    }
    const size_t ia = size_t(e) * lt.ksm + ks;
    if (s == 0) {
      am64[ia * 64 + l] = a;
      am32[ia * 64 + l] = float(a);
    }
    if (m == 0) {
      const size_t iw = (ia * (P + 1) + s) * 4 + k;
      wm64[iw] = w;
      wm32[iw] = float(w);
    }
  }
}

// First contraction, shared by all pencils with the same i3: for every
// quadrature point (q1, q2) and every trial index j3 of I_i3,
//   Y_c[j3] = sum_{q3 in Q_i3} B3^(alpha_c)_j3(x_q3) w3^(o_c)_{i3,q3} K_c(q1, q2, q3)
// for the 8 channels c = (coefficient, dir-3 rule) of the stiffness
// (K11 T^(0,0), K22 T^(0,0), K33 T^(1,1), K12 T^(0,0), K13 T^(1,0),
//  K13 T^(0,1), K23 T^(1,0), K23 T^(0,1)) or the single det J T^(0,0) of
// the mass.  Lanes run over the (q2, q1) plane, whose points are contiguous
// in the field, so every load is coalesced; the record of a point,
// [c][jj3], is stored contiguously for the pencil kernel (whose lanes run
// over j3 within one channel).  The 64 records of
// a wavefront are one contiguous stretch of Y; they pass through LDS so that
// consecutive lanes store consecutive elements (whole lines per store).
// A plane patch (PLANE: direction 3 trivial) has only j3 = 0: one slot.
template <int P, typename T, bool STIFF, bool PLANE = false>
__global__ __launch_bounds__(256) void k_first(PlanView v) {
  constexpr int IC = 2 * P + 1, QC = 3 * P + 1, NCH = STIFF ? kYChannels : 1;
  constexpr int ICY = PLANE ? 1 : IC;                     // j3 slots per record
  constexpr int REC = ICY * NCH;                          // elements per record
  constexpr int LPR = (9216 / int(sizeof(T) * REC)) < 64 ? (9216 / int(sizeof(T) * REC)) : 64;   // records per round
  __shared__ __align__(16) T stg[4][LPR * REC];
  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int64_t plane = int64_t(d1.nq) * d2.nq;
  const int tid = threadIdx.x, wv = tid / 64, ln = tid % 64;
  const int64_t l0 = int64_t(blockIdx.x) * blockDim.x + wv * 64;   // first point of the wave
  const int64_t l = l0 + ln;
  const int i3 = blockIdx.y;
  if (l0 >= plane) return;   // uniform per wave
  const bool valid = l < plane;
  int qs3, qc3;
  q_range(i3, P, d3.nel, qs3, qc3);
  if (d3.nel == 0) {   // trivial direction of a 2D problem: one point, T3^(0,0) = 1
    qs3 = 0;
    qc3 = 1;
  }
  const T* __restrict__ T3 = op_t<T>(d3) + size_t(i3) * QC * IC * 4;    // [qq3][jj3][o]
  const int64_t N = v.nqtot;
  const T* __restrict__ f = static_cast<const T*>(v.field) + (valid ? l : l0) + plane * qs3;
  T acc[ICY * NCH];
#pragma unroll
  for (int k = 0; k < ICY * NCH; ++k) acc[k] = T(0);
#pragma unroll 2
  for (int qq3 = 0; qq3 < qc3; ++qq3) {
    const T* fk = f + plane * qq3;
    const T* t = T3 + qq3 * IC * 4;   // uniform: scalar loads
    if constexpr (STIFF) {
      const T k11 = fk[1 * N], k22 = fk[2 * N], k33 = fk[3 * N];
      const T k12 = fk[4 * N], k13 = fk[5 * N], k23 = fk[6 * N];
#pragma unroll
      for (int jj = 0; jj < ICY; ++jj) {
        const T t0 = t[jj * 4 + R00], t1 = t[jj * 4 + R10], t2 = t[jj * 4 + R01], t3 = t[jj * 4 + R11];
        T* a = acc + jj;
        a[0 * ICY] += t0 * k11;
        a[1 * ICY] += t0 * k22;
        a[2 * ICY] += t3 * k33;
        a[3 * ICY] += t0 * k12;
        a[4 * ICY] += t1 * k13;
        a[5 * ICY] += t2 * k13;
        a[6 * ICY] += t1 * k23;
        a[7 * ICY] += t2 * k23;
      }
    } else {
      const T k0 = fk[0];
#pragma unroll
      for (int jj = 0; jj < ICY; ++jj) acc[jj] += t[jj * 4 + R00] * k0;
    }
  }
  // the wave's records are contiguous in Y: pass them through LDS in rounds
  // of LPR records so that consecutive lanes store consecutive elements
  const int nvalid = int(plane - l0 < 64 ? plane - l0 : 64);
  T* y = static_cast<T*>(v.ybuf) + (int64_t(i3) * plane + l0) * REC;
  T* st = stg[wv];
  for (int r0 = 0; r0 < nvalid; r0 += LPR) {
    if (ln >= r0 && ln < r0 + LPR) store_vec<T, REC>(st + (ln - r0) * REC, acc);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int n = (nvalid - r0 < LPR ? nvalid - r0 : LPR) * REC;
    for (int e = ln; e < n; e += 64) y[int64_t(r0) * REC + e] = st[e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Shape of the pencil kernel: J3P trial indices j3 per part (items: J3P x
// (2p+1) pairs (j3, j2)), NW waves of TW 16-item tiles each; chunks of CU
// quadrature columns (two "units" of two points each, see below).
template <int P, bool PLANE>
struct PenShape {
  static constexpr int IC = 2 * P + 1, QC = 3 * P + 1;
  static constexpr int J3P = PLANE ? 1 : (P >= 4 ? (IC + 1) / 2 : IC);
  static constexpr int NITEMS = J3P * IC;
  static constexpr int TW = 1;
  static constexpr int NW = ((NITEMS + 15) / 16 + TW - 1) / TW;
  static constexpr int NT = 64 * NW;
  static constexpr int NPAD = NW * TW * 16;
  static constexpr int NPART = PLANE ? 1 : (IC + J3P - 1) / J3P;
  static constexpr int UNITS = 2, CU = 2 * UNITS;   // units and columns per chunk
  static constexpr int JH = (IC + 1) / 2;           // trial indices j2 per phase-B item
  // two workgroups of NW >= 5 waves per CU need 3 waves per SIMD: the
  // register allocation is bounded for that (0: no bound)
  static constexpr int WPE = NW >= 5 ? 3 : 0;
};

// The pencil kernel.  Direction-1 work is cut into "units": two consecutive
// points of one knot-span (an interior span is one unit, a boundary span of
// p+1 or p+2 points several), i.e. one k-step of the matrix products.  A
// chunk holds UNITS units; per chunk:
//   phase A: the first-contraction records (q2, column, j3) of the chunk,
//            loaded into registers one chunk ahead, are merged with the
//            dir-2 weights into six arrays H (one for the mass) in LDS;
//   phase B: items (column, j3, group, half of the j2 range) contract H
//            with B2^(alpha) into G[column][group][(j3, j2)] in LDS;
//   phase C: per unit, the p+1 open rows take one matrix product each; a
//            row whose span is complete is stored and the accumulators move
//            down one slot.
template <int P, typename T, bool STIFF, bool PLANE>
__device__ __forceinline__ void pencil_body(PlanView v, T* __restrict__ out, int nseg) {
  using S = PenShape<P, PLANE>;
  using v4 = typename V4<T>::type;
  constexpr int IC = S::IC, QC = S::QC, NT = S::NT, NPAD = S::NPAD, TW = S::TW, J3P = S::J3P;
  constexpr int CU = S::CU, UNITS = S::UNITS, JH = S::JH;
  constexpr int NG = STIFF ? 4 : 1, NH = STIFF ? 6 : 1, NCH = STIFF ? kYChannels : 1;
  constexpr int ICY = PLANE ? 1 : IC, REC = ICY * NCH;
  __shared__ __align__(16) T hbuf[CU * NH * QC * J3P];   // [c][h][qq2][u]
  __shared__ __align__(16) T gbuf[CU * NG * NPAD];       // [c][g][(u, j2)]
  __shared__ T hzero[QC * J3P];                          // a missing B2^(1) input

  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int n1 = d1.n, n2 = d2.n, nq1 = d1.nq, nq2 = d2.nq, nel1 = d1.nel;
  const int tid = threadIdx.x, wv = tid / 64, ln = tid % 64;
  // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs; give
  // each XCD a contiguous range of work items so that the parts of a pencil
  // and neighbouring pencils, which read overlapping first-contraction
  // records, share an L2.
  const int total = gridDim.x, L = blockIdx.x;
  const int xcd = L % 8, kx = L / 8, m8 = total / 8, r8 = total % 8;
  int item = xcd * m8 + min(xcd, r8) + kx;
  const int part = item % S::NPART;
  item /= S::NPART;
  const int i2 = item % n2;
  item /= n2;
  const int seg = item % nseg, i3 = item / nseg;

  int qs2, qc2, is2, ic2, is3, ic3;
  q_range(i2, P, d2.nel, qs2, qc2);
  i_range(i2, P, n2, is2, ic2);
  i_range(i3, P, d3.n, is3, ic3);
  // the part owns the trial indices j3 in [j3a, j3a + nj3) (indices in
  // I_i3) and all j2; its values are one contiguous stretch of each row
  const int j3a = part * J3P;
  if (j3a >= ic3) return;       // uniform per workgroup
  const int nj3 = min(J3P, ic3 - j3a);

  // rows r0..r1-1 need the spans e0..e1
  const int r0 = int(int64_t(seg) * n1 / nseg), r1 = int(int64_t(seg + 1) * n1 / nseg);
  const int e0 = max(0, r0 - P), e1 = min(nel1 - 1, r1 - 1);

  const T* __restrict__ Yb = static_cast<const T*>(v.ybuf) + int64_t(i3) * nq2 * nq1 * REC;   // [q2][q1][ch][jj3]
  const cptr<T> w2 = to_const(wt_t<T>(d2) + size_t(i2) * QC * 4);        // [qq2][o]
  const cptr<T> B2 = to_const(bt_t<T>(d2) + size_t(i2) * QC * IC * 2);   // [qq2][jj2][alpha]
  const LaneTables lt = lane_tables(P, nel1);
  const T* __restrict__ LA = reinterpret_cast<const T*>(
      v.lanes + (sizeof(T) == 8 ? (STIFF ? lt.a64 : lt.am64) : (STIFF ? lt.a32 : lt.am32)));
  const T* __restrict__ LW = reinterpret_cast<const T*>(
      v.lanes + (sizeof(T) == 8 ? (STIFF ? lt.w64 : lt.wm64) : (STIFF ? lt.w32 : lt.wm32)));
  const int KS = STIFF ? lt.kss : lt.ksm;   // k-steps per span in the tables

  // CSR position of row (i1, i2, i3): closed-form prefix of the row lengths
  const int64_t Tn1 = d1.prefix[n1], Tn2 = d2.prefix[n2];
  const int64_t pencil_start = d3.prefix[i3] * Tn2 * Tn1 + int64_t(ic3) * d2.prefix[i2] * Tn1;
  const int64_t row_mult = int64_t(ic3) * ic2;

  // items beyond the part stay zero in the staging buffer
  for (int t = tid; t < CU * NG * NPAD; t += NT) gbuf[t] = T(0);
  for (int t = tid; t < QC * J3P; t += NT) hzero[t] = T(0);

  // phase-C role of this lane: column kq of A (row kq of B), item n of each
  // of its tiles; output offset of item n = (jj3, j2) within a row, in
  // units of the row's #I_i1
  const int kq = ln / 16, nl = ln % 16;
  int64_t ooff[TW];
  bool oval[TW];
#pragma unroll
  for (int tt = 0; tt < TW; ++tt) {
    const int n = (wv * TW + tt) * 16 + nl;
    const int jj3 = n / IC, j2 = n % IC;
    oval[tt] = jj3 < nj3 && j2 < ic2;
    ooff[tt] = (j3a + jj3) * ic2 + j2;
  }
  v4 acc[P + 1][TW];   // open rows e+s, s = 0..P
#pragma unroll
  for (int s = 0; s <= P; ++s)
#pragma unroll
    for (int tt = 0; tt < TW; ++tt) acc[s][tt] = v4{T(0), T(0), T(0), T(0)};

  // CSR position of the next row to be stored (rows leave in order r0, r0+1,
  // ...): start of row r0, advanced by each row's length
  int64_t rowpos = pencil_start + row_mult * d1.prefix[r0];
  // row e (slot 0) is complete: store it if it is ours (lane (kq, nl) holds
  // entries d = drow(kq, r) of its items, d = j1 - e + P), then move the
  // open rows down one slot
  auto retire = [&](int e) {
    if (e >= r0 && e < r1) {   // uniform
      const int dlo = e < P ? P - e : 0;
      const int dhi = min(2 * P, P + n1 - 1 - e);
      const int ic1 = dhi - dlo + 1;
      T* o = out + rowpos;
      rowpos += row_mult * ic1;
#pragma unroll
      for (int tt = 0; tt < TW; ++tt) {
        T* ot = o + ooff[tt] * ic1 - dlo;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int dd = drow<T>(kq, r);
          if (oval[tt] && unsigned(dd - dlo) < unsigned(ic1)) ot[dd] = acc[0][tt][r];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < P; ++s)
#pragma unroll
      for (int tt = 0; tt < TW; ++tt) acc[s][tt] = acc[s + 1][tt];
#pragma unroll
    for (int tt = 0; tt < TW; ++tt) acc[P][tt] = v4{T(0), T(0), T(0), T(0)};
  };

  // Phase A input of a chunk: records (qq2, c, u), u fastest; each lane holds
  // RPL of them (all channels) in registers.  Records of absent items read
  // the slab start, so that every lane always loads.
  constexpr int NREC = QC * CU * J3P, RPL = (NREC + NT - 1) / NT;
  T pre[RPL][NCH];
  int64_t roff[RPL];
  bool rok[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int it = tid + r * NT;
    const int u = it % J3P, c = (it / J3P) % CU, qq2 = it / (J3P * CU);
    rok[r] = it < NREC && qq2 < qc2 && u < nj3;
    roff[r] = rok[r] ? (int64_t(qs2 + qq2) * nq1 + c) * REC + j3a + u : 0;
  }
  auto fetch = [&](int qcol0, int ncols) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int c = ((tid + r * NT) / J3P) % CU;
      const T* y = Yb + (rok[r] && c < ncols ? roff[r] + int64_t(qcol0) * REC : 0);
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) pre[r][ch] = y[ch * ICY];
    }
  };
  // fold in the dir-2 weights and stage the merged arrays H in LDS
  auto merge = [&](int ncols) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int it = tid + r * NT;
      const int u = it % J3P, c = (it / J3P) % CU, qq2 = it / (J3P * CU);
      if (!rok[r] || c >= ncols) continue;
      const T* Y = pre[r];
      const T a00 = w2[qq2 * 4 + R00], a10 = w2[qq2 * 4 + R10], a01 = w2[qq2 * 4 + R01], a11 = w2[qq2 * 4 + R11];
      T* h = hbuf + (c * NH * QC + qq2) * J3P + u;
      // channels: 0 K11 T3^(0,0), 1 K22 T3^(0,0), 2 K33 T3^(1,1), 3 K12 T3^(0,0),
      //           4 K13 T3^(1,0), 5 K13 T3^(0,1), 6 K23 T3^(1,0), 7 K23 T3^(0,1)
      if constexpr (STIFF) {
        h[0 * QC * J3P] = a11 * Y[1] + a10 * Y[7];   // -> G_(0,0) through B2^(1)
        h[1 * QC * J3P] = a00 * Y[2] + a01 * Y[6];   // -> G_(0,0) through B2^(0)
        h[2 * QC * J3P] = a00 * Y[0];                // -> G_(1,1) through B2^(0)
        h[3 * QC * J3P] = a10 * Y[3];                // -> G_(0,1) through B2^(1)
        h[4 * QC * J3P] = a00 * Y[4];                // -> G_(0,1) through B2^(0)
        h[5 * QC * J3P] = a01 * Y[3] + a00 * Y[5];   // -> G_(1,0) through B2^(0)
      } else {
        h[0] = a00 * Y[0];
      }
    }
  };

  // unit cursor: span e, unit k (k-step) within e
  auto nunits = [&](int e) { return e <= e1 ? (span_np(e, P, nel1) + 1) / 2 : 0; };
  int ce = e0, ck = 0;
  // the chunk starting at the cursor: its columns (the units' points)
  auto chunk_cols = [&](int e, int k, int& qcol0, int& ncols) {
    qcol0 = e <= e1 ? span_q0(e, P) + 2 * k : 0;
    int q = qcol0;
    for (int u = 0; u < UNITS && e <= e1; ++u) {
      q = min(span_q0(e, P) + 2 * k + 2, span_q0(e, P) + span_np(e, P, nel1));
      if (++k == nunits(e)) { ++e; k = 0; }
    }
    ncols = q - qcol0;
  };
  int qcol0, ncols;
  chunk_cols(ce, ck, qcol0, ncols);
  fetch(qcol0, ncols);
  __syncthreads();

  while (ce <= e1) {
    // ---------------- phase A ----------------
    merge(ncols);
    {
      // the next chunk's records are loaded while this one goes through B and C
      int e = ce, k = ck;
      for (int u = 0; u < UNITS && e <= e1; ++u)
        if (++k == nunits(e)) { ++e; k = 0; }
      int q0n, ncn;
      chunk_cols(e, k, q0n, ncn);
      if (ncn > 0) fetch(q0n, ncn);
    }
    __syncthreads();
    // ---------------- phase B ----------------
    // items (g, c, u, half), g slowest so that a wave mostly holds one group
    {
      const int nci = ncols * nj3 * 2, ni = NG * nci;
      for (int it = tid; it < ni; it += NT) {
        const int g = it / nci, rem = it - g * nci;
        const int c = rem / (nj3 * 2), r2 = rem - c * (nj3 * 2);
        const int u = r2 >> 1, half = r2 & 1;
        int h1, h0;   // inputs through B2^(1) and B2^(0)
        if constexpr (STIFF) {
          h1 = g == 0 ? 0 : (g == 2 ? 3 : -1);   // -1: none (zeros)
          h0 = g == 0 ? 1 : (g == 1 ? 5 : (g == 2 ? 4 : 2));
        } else {
          h1 = -1;
          h0 = 0;
        }
        const int jb = half * JH;   // first j2 of the half (the second half is one short for odd 2p+1)
        T G[JH];
#pragma unroll
        for (int j = 0; j < JH; ++j) G[j] = T(0);
        const T* hb0 = hbuf + (c * NH + h0) * QC * J3P + u;
        const T* hb1 = h1 >= 0 ? hbuf + (c * NH + h1) * QC * J3P + u : hzero + u;
        const cptr<T> bb = B2 + jb * 2;
        if (h1 >= 0) {
          for (int qq2 = 0; qq2 < qc2; ++qq2) {   // uniform trip count
            const T x0 = hb0[qq2 * J3P], x1 = hb1[qq2 * J3P];
            const cptr<T> b = bb + qq2 * IC * 2;
#pragma unroll
            for (int j = 0; j < JH; ++j) {
              const int jj = jb + j < IC ? j : IC - 1 - jb;   // in the table row
              G[j] = fma(b[2 * jj + 1], x1, fma(b[2 * jj], x0, G[j]));
            }
          }
        } else {
          for (int qq2 = 0; qq2 < qc2; ++qq2) {
            const T x0 = hb0[qq2 * J3P];
            const cptr<T> b = bb + qq2 * IC * 2;
#pragma unroll
            for (int j = 0; j < JH; ++j) {
              const int jj = jb + j < IC ? j : IC - 1 - jb;
              G[j] = fma(b[2 * jj], x0, G[j]);
            }
          }
        }
        T* gp = gbuf + (c * NG + g) * NPAD + u * IC + jb;
#pragma unroll
        for (int j = 0; j < JH; ++j)
          if (jb + j < IC) gp[j] = G[j];
      }
    }
    __syncthreads();
    // ---------------- phase C ----------------
    int cb = 0;   // first column of the unit within the chunk
    for (int un = 0; un < UNITS && ce <= e1; ++un) {
      const int np = span_np(ce, P, nel1);
      const int npu = min(2, np - 2 * ck);   // points of this unit
      // B operand of lane (kq, nl): point c = kq/2 of the unit with alpha =
      // kq%2 (the mass has no alpha = 1 entries: their weights are zero)
      const int c = kq / 2, al = STIFF ? kq % 2 : 0;
      const int cc = cb + min(c, npu - 1);   // padding entries: weights and A are zero
      const T* gp = gbuf + cc * NG * NPAD + wv * TW * 16 + nl;
      T g0[TW], g1[TW];
#pragma unroll
      for (int tt = 0; tt < TW; ++tt) {
        g0[tt] = gp[al * NPAD + tt * 16];
        g1[tt] = STIFF ? gp[(2 + al) * NPAD + tt * 16] : T(0);
      }
      const size_t ia = size_t(ce) * KS + ck;
      const T* wrow = LW + (ia * (P + 1) * 4 + kq) * (STIFF ? 2 : 1);   // weights of rows ce+s
      T a = LA[ia * 64 + ln];
#pragma unroll
      for (int s = 0; s <= P; ++s) {
        if (s > 0) a = row_up(a);
        T h[TW];
        if constexpr (STIFF) {
          const T2v<T> w = *reinterpret_cast<const T2v<T>*>(wrow + s * 8);
#pragma unroll
          for (int tt = 0; tt < TW; ++tt) h[tt] = fma(w.y, g1[tt], w.x * g0[tt]);
        } else {
          const T w0 = wrow[s * 4];
#pragma unroll
          for (int tt = 0; tt < TW; ++tt) h[tt] = w0 * g0[tt];
        }
#pragma unroll
        for (int tt = 0; tt < TW; ++tt) acc[s][tt] = mma(a, h[tt], acc[s][tt]);
      }
      cb += npu;
      if (++ck == nunits(ce)) {   // span ce complete: row ce leaves
        retire(ce);
        ++ce;
        ck = 0;
      }
    }
    chunk_cols(ce, ck, qcol0, ncols);
    __syncthreads();
  }
  // a run that ends the patch: the rows still open are complete
  if (e1 == nel1 - 1) {
#pragma unroll
    for (int s = 1; s <= P; ++s) retire(e1 + s);
  }
}

template <int P, typename T, bool STIFF, bool PLANE>
__global__ __launch_bounds__((PenShape<P, PLANE>::NT)) void k_pencil(PlanView v, T* __restrict__ out, int nseg) {
  pencil_body<P, T, STIFF, PLANE>(v, out, nseg);
}
template <int P, typename T, bool STIFF, bool PLANE>
__global__ __launch_bounds__((PenShape<P, PLANE>::NT))
__attribute__((amdgpu_waves_per_eu(PenShape<P, PLANE>::WPE > 0 ? PenShape<P, PLANE>::WPE : 1)))
void k_pencil_wpe(PlanView v, T* __restrict__ out, int nseg) {
  pencil_body<P, T, STIFF, PLANE>(v, out, nseg);
}

template <int P, typename T, bool STIFF, bool PLANE>
hipError_t push_launch(const PlanView& v, void* out, hipStream_t s) {
  using Sh = PenShape<P, PLANE>;
  const int64_t wgs = int64_t(v.dir[1].n) * v.dir[2].n * Sh::NPART;
  // runs of at least 2p rows
  const int max_seg = std::max(1, v.dir[0].n / (2 * P));
  const int nseg = int(std::min<int64_t>(max_seg, std::max<int64_t>(1, (WQ_WG_TARGET + wgs - 1) / wgs)));
  const int64_t items = wgs * nseg;
  if (items <= 0 || items > INT32_MAX) return hipErrorInvalidConfiguration;
  const int64_t plane = int64_t(v.dir[0].nq) * v.dir[1].nq;
  hipLaunchKernelGGL((k_first<P, T, STIFF, PLANE>), dim3(unsigned((plane + 255) / 256), unsigned(v.dir[2].n)), dim3(256), 0, s, v);
  if constexpr (Sh::WPE > 0)
    hipLaunchKernelGGL((k_pencil_wpe<P, T, STIFF, PLANE>), dim3(unsigned(items)), dim3(Sh::NT), 0, s, v, static_cast<T*>(out), nseg);
  else
    hipLaunchKernelGGL((k_pencil<P, T, STIFF, PLANE>), dim3(unsigned(items)), dim3(Sh::NT), 0, s, v, static_cast<T*>(out), nseg);
  return hipGetLastError();
}

template <int P, typename T>
hipError_t assemble_pt(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s) {
  if (which & WQ_MASS) {
    hipError_t e = v.d == 2 ? push_launch<P, T, false, true>(v, mass, s) : push_launch<P, T, false, false>(v, mass, s);
    if (e != hipSuccess) return e;
  }
  if (which & WQ_STIFF) {
    hipError_t e = v.d == 2 ? push_launch<P, T, true, true>(v, stiff, s) : push_launch<P, T, true, false>(v, stiff, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int P>
hipError_t assemble_p(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s) {
  return v.prec == WQ_FP64 ? assemble_pt<P, double>(v, which, mass, stiff, s)
                           : assemble_pt<P, float>(v, which, mass, stiff, s);
}

template <int P>
hipError_t lanes_p(const PlanView& v, hipStream_t s) {
  hipLaunchKernelGGL(k_lanes<P>, dim3(unsigned(v.dir[0].nel), P + 1), dim3(64), 0, s, v);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_assemble(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s) {
  switch (v.p) {
    case 2: return assemble_p<2>(v, which, mass, stiff, s);
    case 3: return assemble_p<3>(v, which, mass, stiff, s);
    case 4: return assemble_p<4>(v, which, mass, stiff, s);
    case 5: return assemble_p<5>(v, which, mass, stiff, s);
    case 6: return assemble_p<6>(v, which, mass, stiff, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_lanes(const PlanView& v, hipStream_t s) {
  switch (v.p) {
    case 2: return lanes_p<2>(v, s);
    case 3: return lanes_p<3>(v, s);
    case 4: return lanes_p<4>(v, s);
    case 5: return lanes_p<5>(v, s);
    case 6: return lanes_p<6>(v, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wq
