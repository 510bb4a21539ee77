// Row formation by sum factorization (Section 6, eq. sumfactorization,
// Algorithm 3) for the mass matrix, and its stiffness analogue (eq. stiff):
// the sum over the 9 pairs (l, m) of test/trial derivative directions, where
// direction k uses the rule w^(alpha_k, beta_k) with alpha_k = [k == m]
// (trial) and beta_k = [k == l] (test), applied to the coefficient c_lm.
//
// Work decomposition.  The first contraction (over q3) does not depend on
// i1 or i2, so it is done once per test index i3 for the whole (q1, q2)
// plane by k_first and kept in HBM.  A workgroup of the pencil kernel then
// owns a run of consecutive rows (i1 = r0..r1-1, i2, i3) of one pencil -- one
// contiguous CSR segment -- restricted to a part of the trial index j3.  The
// operators of direction 2 are fixed along the pencil, so the contraction
// over q2 is done once per quadrature column q1 and shared by all rows:
//
//   phase A (items: q1, q2, j3):  read the 8 channels Y_c[j3] of the first
//            contraction (1 for the mass) and fold in the dir-2 weights:
//            terms that meet the same B2^(alpha) and the same dir-1 rule are
//            summed after scaling by their weights ("weight merge"), leaving
//            6 arrays H[q2][j3] (1 for the mass) in LDS.
//   phase B (items: q1, j3, group):  G_g[j2][j3] = sum_q2 B2^(a)[j2][q2] H,
//            one group g = 2*beta + alpha per dir-1 rule (4 for the
//            stiffness, 1 for the mass), into LDS.
//   phase C (items: j2, j3; columns q1 in order):  the column q1 lies in the
//            knot span e; it only touches the rows i1 = e..e+p (whose support
//            holds x_q1) and, in each, only the trial functions j1 = e..e+p
//            (nonzero at x_q1).  Each item keeps the p+1 open rows in
//            registers, indexed relative to e, and adds
//              B_j1(x_q1) (w^(0,0)_i1 G_(0,0) + w^(0,1)_i1 G_(0,1))
//            + B'_j1(x_q1) (w^(1,0)_i1 G_(1,0) + w^(1,1)_i1 G_(1,1)).
//            When e advances, row e is complete: it is staged in LDS and
//            stored coalesced, and the open rows shift by one.
//
// A run of rows r0..r1-1 needs the columns of the spans max(0, r0-p) ..
// min(n_el-1, r1-1); splitting a pencil into runs repeats the phases A and B
// of p spans per run, which buys workgroups when a patch has few pencils.
//
// Uniform data (operators, weights, B-spline values) is read with scalar
// loads from tables laid out contiguously per quadrature point.
//
// Plane patches and curves (d <= 2) have no first contraction: a strip
// kernel (below) reads the coefficient field directly and puts several
// rows i2 side by side in phase C.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <mutex>
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

// NW: wavefronts per workgroup; J3: trial indices j3 per workgroup (phase C
// uses IC * J3 lanes); C: quadrature columns per chunk of phases A and B
// (phase B has J3 * C * 4 items for the stiffness); WPE: waves per SIMD the
// register allocation must allow (0: no bound).  Chosen by measurement.
template <int P, typename T, bool STIFF> struct PushCfg;
#define WQ_PUSH_CFG(P_, T_, S_, NW_, J3_, C_, WPE_) \
  template <> struct PushCfg<P_, T_, S_> { static constexpr int NW = NW_, J3 = J3_, C = C_, WPE = WPE_; };
WQ_PUSH_CFG(2, double, false, 1, 5, 4, 0)
WQ_PUSH_CFG(2, double, true, 1, 5, 3, 0)
WQ_PUSH_CFG(3, double, false, 1, 7, 4, 0)
WQ_PUSH_CFG(3, double, true, 1, 7, 2, 0)
WQ_PUSH_CFG(4, double, false, 1, 5, 6, 0)
WQ_PUSH_CFG(4, double, true, 2, 9, 3, 3)
WQ_PUSH_CFG(5, double, false, 2, 11, 2, 0)
WQ_PUSH_CFG(5, double, true, 2, 11, 2, 0)
WQ_PUSH_CFG(6, double, false, 1, 4, 8, 0)
WQ_PUSH_CFG(6, double, true, 4, 13, 3, 2)
WQ_PUSH_CFG(2, float, false, 1, 5, 8, 0)
WQ_PUSH_CFG(2, float, true, 1, 5, 3, 0)
WQ_PUSH_CFG(3, float, false, 1, 7, 8, 0)
WQ_PUSH_CFG(3, float, true, 1, 7, 2, 0)
WQ_PUSH_CFG(4, float, false, 1, 5, 8, 0)
WQ_PUSH_CFG(4, float, true, 2, 9, 3, 0)
WQ_PUSH_CFG(5, float, false, 2, 11, 4, 0)
WQ_PUSH_CFG(5, float, true, 2, 11, 2, 0)
WQ_PUSH_CFG(6, float, false, 3, 13, 8, 0)
WQ_PUSH_CFG(6, float, true, 3, 13, 3, 0)
#undef WQ_PUSH_CFG

template <int P, typename T, bool STIFF>
struct Shape {
  using Cfg = PushCfg<P, T, STIFF>;
  static constexpr int IC = 2 * P + 1, QC = 3 * P + 1;
  static constexpr int NT = 64 * Cfg::NW, J3 = Cfg::J3, C = Cfg::C;
  static constexpr int NPART = (IC + J3 - 1) / J3;        // j3 parts
  static constexpr int NG = STIFF ? 4 : 1;                // dir-1 rule groups
  static constexpr int NH = STIFF ? 6 : 1;                // merged dir-2 inputs
  static constexpr int NCH = STIFF ? 8 : 1;               // dir-3 channels
  static constexpr int NCT = 6 * (P + 1);                 // column-table entries
  static constexpr size_t HBUF = size_t(C) * NH * QC * J3;
  static constexpr size_t GBUF = size_t(C) * NG * IC * J3;
  static constexpr size_t STAGE = size_t(J3) * IC * IC;
  // Banded phase B for rows away from the boundary spans (off where it
  // makes a register-bounded configuration spill).
  static constexpr bool BAND2 = Cfg::WPE < 3;
  // For the stiffness, whose H buffer is large, the row stage shares it: H
  // is dead from the end of phase B to the merge of the next chunk, which is
  // where rows are stored.
  static constexpr bool STAGE_IN_H = STIFF;
  static constexpr size_t HSBUF = STAGE_IN_H ? (HBUF > STAGE ? HBUF : STAGE) : HBUF;
  static constexpr size_t SBUF = STAGE_IN_H ? 1 : STAGE;
  static constexpr size_t LDS_BYTES = (HSBUF + GBUF + (STAGE_IN_H ? 0 : STAGE)) * sizeof(T);
  static_assert(IC * J3 <= NT, "one phase-C item per lane");
  static_assert(LDS_BYTES <= 64 * 1024, "LDS budget per workgroup");
};

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
__device__ inline const T* b0t_t(const DirView& d) {
  if constexpr (sizeof(T) == 8) return reinterpret_cast<const T*>(d.b0t64);
  else return reinterpret_cast<const T*>(d.b0t32);
}
template <typename T>
__device__ inline const T* wt_t(const DirView& d) {
  if constexpr (sizeof(T) == 8) return reinterpret_cast<const T*>(d.wt64);
  else return reinterpret_cast<const T*>(d.wt32);
}
template <typename T>
__device__ inline const T* colt_t(const DirView& d) {
  if constexpr (sizeof(T) == 8) return reinterpret_cast<const T*>(d.colt64);
  else return reinterpret_cast<const T*>(d.colt32);
}

// n consecutive values (n a multiple of the vector width, 16-byte aligned)
template <typename T, int NV>
__device__ inline void load_vec(const T* __restrict__ p, T (&out)[NV]) {
  if constexpr (sizeof(T) == 8 && NV % 2 == 0) {
#pragma unroll
    for (int k = 0; k < NV / 2; ++k) {
      const double2 x = reinterpret_cast<const double2*>(p)[k];
      out[2 * k] = x.x;
      out[2 * k + 1] = x.y;
    }
  } else if constexpr (sizeof(T) == 4 && NV % 4 == 0) {
#pragma unroll
    for (int k = 0; k < NV / 4; ++k) {
      const float4 x = reinterpret_cast<const float4*>(p)[k];
      out[4 * k] = x.x;
      out[4 * k + 1] = x.y;
      out[4 * k + 2] = x.z;
      out[4 * k + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = p[k];
  }
}
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

// First contraction, shared by all pencils with the same i3: for every
// quadrature point (q1, q2) and every trial index j3 of I_i3,
//   Y_c[j3] = sum_{q3 in Q_i3} B3^(alpha_c)_j3(x_q3) w3^(o_c)_{i3,q3} K_c(q1, q2, q3)
// for the 8 channels c = (coefficient, dir-3 rule) of the stiffness
// (K11 T^(0,0), K22 T^(0,0), K33 T^(1,1), K12 T^(0,0), K13 T^(1,0),
//  K13 T^(0,1), K23 T^(1,0), K23 T^(0,1)) or the single det J T^(0,0) of
// the mass.  Lanes run over the (q2, q1) plane, whose points are contiguous
// in the field, so every load is coalesced; the record of a point,
// [jj3][c], is stored contiguously for the pencil kernel.  The 64 records of
// a wavefront are one contiguous stretch of Y; they pass through LDS so that
// consecutive lanes store consecutive elements (whole lines per store).
template <int P, typename T, bool STIFF>
__device__ __forceinline__ void first_body(const PlanView& v, int bx, int by) {
  constexpr int IC = 2 * P + 1, QC = 3 * P + 1, NCH = STIFF ? kYChannels : 1;
  constexpr int REC = IC * NCH;                           // elements per record
  constexpr int LPR = (9216 / int(sizeof(T) * REC)) < 64 ? (9216 / int(sizeof(T) * REC)) : 64;   // records per round
  __shared__ __align__(16) T stg[4][LPR * REC];
  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int64_t plane = int64_t(d1.nq) * d2.nq;
  const int tid = threadIdx.x, wv = tid / 64, ln = tid % 64;
  const int64_t l0 = int64_t(bx) * 256 + wv * 64;   // first point of the wave
  const int64_t l = l0 + ln;
  const int i3 = v.y_i3 + by;   // Y holds the planes i3 >= y_i3
  if (l0 >= plane) return;   // uniform per wave
  const bool valid = l < plane;
  int qs3, qc3;
  q_range(i3, P, d3.nel, qs3, qc3);
  const T* __restrict__ T3 = op_t<T>(d3) + size_t(i3) * QC * IC * 4;    // [qq3][jj3][o]
  const int64_t N = v.nqtot;
  const T* __restrict__ f = static_cast<const T*>(v.field) + (valid ? l : l0) + plane * qs3;
  T acc[IC * NCH];
#pragma unroll
  for (int k = 0; k < IC * NCH; ++k) acc[k] = T(0);
  // one quadrature point qq3: the products with the nonzero operator
  // entries jj in [lo, hi]
  auto point = [&](int qq3, int lo, int hi) {
    const T* fk = f + plane * qq3;
    const T* t = T3 + qq3 * IC * 4;   // uniform: scalar loads
    if constexpr (STIFF) {
      const T k11 = fk[1 * N], k22 = fk[2 * N], k33 = fk[3 * N];
      const T k12 = fk[4 * N], k13 = fk[5 * N], k23 = fk[6 * N];
#pragma unroll
      for (int jj = 0; jj < IC; ++jj) {
        if (jj < lo || jj > hi) continue;
        const T t0 = t[jj * 4 + R00], t1 = t[jj * 4 + R10], t2 = t[jj * 4 + R01], t3 = t[jj * 4 + R11];
        T* a = acc + jj * NCH;
        a[0] += t0 * k11;
        a[1] += t0 * k22;
        a[2] += t3 * k33;
        a[3] += t0 * k12;
        a[4] += t1 * k13;
        a[5] += t2 * k13;
        a[6] += t1 * k23;
        a[7] += t2 * k23;
      }
    } else {
      const T k0 = fk[0];
#pragma unroll
      for (int jj = 0; jj < IC; ++jj)
        if (jj >= lo && jj <= hi) acc[jj] += t[jj * 4 + R00] * k0;
    }
  };
  if (i3 >= P + 1 && i3 <= d3.nel - 2) {
    // row i3 away from the boundary spans: 2P+1 points alternating span
    // midpoints and knots, the operator's nonzeros in a fixed band (the
    // same products as below without the exact zeros)
#pragma unroll
    for (int qq3 = 0; qq3 < 2 * P + 1; ++qq3) point(qq3, (qq3 + 1) / 2, qq3 / 2 + P);
  } else {
#pragma unroll 2
    for (int qq3 = 0; qq3 < qc3; ++qq3) point(qq3, 0, IC - 1);
  }
  // the wave's records are contiguous in Y: pass them through LDS in rounds
  // of LPR records so that consecutive lanes store consecutive elements
  const int nvalid = int(plane - l0 < 64 ? plane - l0 : 64);
  T* y = static_cast<T*>(v.ybuf) + (int64_t(i3 - v.y_i3) * plane + l0) * REC;
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

template <int P, typename T, bool STIFF>
__global__ __launch_bounds__(256) void k_first(PlanView v) {
  first_body<P, T, STIFF>(v, blockIdx.x, blockIdx.y);
}

template <int P, typename T, bool STIFF>
__device__ __forceinline__ void push_body(const PlanView& v, T* __restrict__ out, int nseg, int item) {
  using S = Shape<P, T, STIFF>;
  constexpr int IC = S::IC, QC = S::QC, C = S::C, NT = S::NT, J3 = S::J3;
  constexpr int NG = S::NG, NH = S::NH, NCT = S::NCT;
  __shared__ __align__(16) T hbuf[S::HSBUF];    // [C][NH][QC][J3]   (c, h, qq2, u)
  __shared__ __align__(16) T gbuf[S::GBUF];     // [C][NG][IC][J3]   (c, g, jj2, u)
  __shared__ __align__(16) T sbuf[S::SBUF];
  T* const stage = S::STAGE_IN_H ? hbuf : sbuf;  // one row: [u3][jj2][jj1]

  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int n1 = d1.n, n2 = d2.n, nq1 = d1.nq, nq2 = d2.nq, nel1 = d1.nel;
  const int tid = threadIdx.x;
  const int part = item % S::NPART;
  item /= S::NPART;
  const int i2 = item % n2;
  item /= n2;
  const int seg = item % nseg, i3 = item / nseg;

  int qs2, qc2, is2, ic2, is3, ic3;
  q_range(i2, P, d2.nel, qs2, qc2);
  // rows whose support spans are all interior: Q_i2 and I_i2 in the fixed
  // layout (2P+1 points from the midpoint of span i2-P, I_i2 from i2-P)
  const bool band2 = S::BAND2 && i2 >= P + 1 && i2 <= d2.nel - 2;
  i_range(i2, P, n2, is2, ic2);
  i_range(i3, P, d3.n, is3, ic3);
  const int j3lo = part * J3;
  const int nj3 = min(J3, ic3 - j3lo);
  if (nj3 <= 0) return;   // uniform per workgroup

  // rows r0..r1-1 need the columns of spans e0..e1
  const int r0 = int(int64_t(seg) * n1 / nseg), r1 = int(int64_t(seg + 1) * n1 / nseg);
  const int e0 = max(0, r0 - P), e1 = min(nel1 - 1, r1 - 1);
  const int qbeg = e0 == 0 ? 0 : P + 2 * e0 - 1;        // knot chi_e0 opens span e0
  const int qend = e1 == nel1 - 1 ? nq1 : P + 2 * e1 + 1;

  constexpr int NCH = S::NCH;
  const T* __restrict__ Yb = static_cast<const T*>(v.ybuf) + int64_t(i3 - v.y_i3) * nq2 * nq1 * IC * NCH;   // [q2][q1][jj3][ch]
  const T* __restrict__ w2 = wt_t<T>(d2) + size_t(i2) * QC * 4;         // [qq2][o]
  // [qq2][jj2][a] for the stiffness, [qq2][jj2] (B2^(0) alone, contiguous) for the mass
  const T* __restrict__ B2 = STIFF ? bt_t<T>(d2) + size_t(i2) * QC * IC * 2 : b0t_t<T>(d2) + size_t(i2) * QC * IC;
  constexpr int BQ = STIFF ? IC * 2 : IC, BJ = STIFF ? 2 : 1;   // strides of qq2 and jj2 in B2
  const T* __restrict__ CT = colt_t<T>(d1);                             // [q1][NCT]
  const int* __restrict__ span1 = d1.qspan;

  // CSR position of row (i1, i2, i3): closed-form prefix of the row lengths
  const int64_t Tn1 = d1.prefix[n1], Tn2 = d2.prefix[n2];
  const int64_t pencil_start = d3.prefix[i3] * Tn2 * Tn1 + int64_t(ic3) * d2.prefix[i2] * Tn1;
  const int64_t row_mult = int64_t(ic3) * ic2;

  // phase-C role of this lane: (jj2, u3)
  const int cj2 = tid % IC, cu3 = tid / IC;
  const bool cl = tid < IC * J3 && cj2 < ic2 && cu3 < nj3;
  T acc[P + 1][2 * P + 1];   // open rows e+s, s = 0..P; trial offset d = j1 - (e+s) + P
#pragma unroll
  for (int s = 0; s <= P; ++s)
#pragma unroll
    for (int d = 0; d <= 2 * P; ++d) acc[s][d] = T(0);

  // row i1 (slot 0) is complete: store it if it is ours, then shift the slots
  auto flush = [&](int i1) {
    if (i1 >= r0 && i1 < r1) {   // uniform
      const int dlo = i1 < P ? P - i1 : 0;
      const int dhi = min(2 * P, P + n1 - 1 - i1);
      const int ic1 = dhi - dlo + 1;
      const int seglen = ic1 * ic2;
      T* o = out + pencil_start + row_mult * d1.prefix[i1] + int64_t(j3lo) * seglen;
      if (cl) {
#pragma unroll
        for (int d = 0; d <= 2 * P; ++d)
          if (d >= dlo && d <= dhi) stage[(cu3 * ic2 + cj2) * ic1 + (d - dlo)] = acc[0][d];
      }
      __syncthreads();
      const int len = nj3 * seglen;
      for (int t = tid; t < len; t += NT) o[t] = stage[t];
      __syncthreads();
    }
    // the row in slot s has met the spans up to e only, whose trial
    // functions end at e+P: offsets d <= 2P - s; only that part moves
#pragma unroll
    for (int s = 0; s < P; ++s) {
#pragma unroll
      for (int d = 0; d < 2 * P - s; ++d) acc[s][d] = acc[s + 1][d];
      acc[s][2 * P - s] = T(0);
    }
#pragma unroll
    for (int d = 0; d <= P; ++d) acc[P][d] = T(0);
  };

  // dir-2 weights of row i2
  __shared__ T w2s[QC * 4];
  for (int t = tid; t < QC * 4; t += NT) w2s[t] = w2[t];

  // Phase A input of a chunk: records (u, c, qq2) of the first contraction.
  // Each lane holds RPL records in registers; the records of the next chunk
  // are loaded while the current one goes through phases B and C.
  constexpr int NREC = QC * C * J3, RPL = (NREC + NT - 1) / NT;
  T pre[RPL][NCH];
  // per record slot: offset in the slab for column 0 (records of absent
  // items point at the slab start, so that every lane always loads)
  uint32_t roff[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int it = tid + r * NT;
    const int u = it % J3, c = (it / J3) % C, qq2 = it / (J3 * C);
    roff[r] = (it < NREC && qq2 < qc2 && u < nj3) ? uint32_t(((qs2 + qq2) * nq1 + c) * IC + j3lo + u) * NCH : ~0u;
  }
  auto rec_valid = [&](int r, int col0) {
    const int c = ((tid + r * NT) / J3) % C;
    return roff[r] != ~0u && col0 + c < qend;
  };
  auto fetch = [&](int col0) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const uint32_t off = rec_valid(r, col0) ? roff[r] + uint32_t(col0 * IC * NCH) : 0u;
      load_vec<T, NCH>(Yb + off, pre[r]);
    }
  };
  // fold in the dir-2 weights and stage the merged arrays H in LDS
  auto merge = [&](int col0) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int it = tid + r * NT;
      const int u = it % J3, c = (it / J3) % C, qq2 = it / (J3 * C);
      if (!rec_valid(r, col0)) continue;
      const T* Y = pre[r];
      const T* a = w2s + qq2 * 4;
      T* h = hbuf + (size_t(c) * NH * QC + qq2) * J3 + u;
      if constexpr (STIFF) {
        h[0 * QC * J3] = a[R11] * Y[1] + a[R10] * Y[7];   // -> G_(0,0) through B2^(1)
        h[1 * QC * J3] = a[R00] * Y[2] + a[R01] * Y[6];   // -> G_(0,0) through B2^(0)
        h[2 * QC * J3] = a[R00] * Y[0];                   // -> G_(1,1) through B2^(0)
        h[3 * QC * J3] = a[R10] * Y[3];                   // -> G_(0,1) through B2^(1)
        h[4 * QC * J3] = a[R00] * Y[4];                   // -> G_(0,1) through B2^(0)
        h[5 * QC * J3] = a[R01] * Y[3] + a[R00] * Y[5];   // -> G_(1,0) through B2^(0)
      } else {
        h[0] = a[R00] * Y[0];
      }
    }
  };

  __shared__ T hzero[STIFF ? QC * J3 : 1];   // stands in for a missing B2^(1) input
  for (int t = tid; t < (STIFF ? QC * J3 : 1); t += NT) hzero[t] = T(0);

  int e_cur = e0;
  fetch(qbeg);
  __syncthreads();
  for (int col0 = qbeg; col0 < qend; col0 += C) {
    // ---------------- phase A ----------------
    merge(col0);
    if (col0 + C < qend) fetch(col0 + C);
    __syncthreads();
    // ---------------- phase B ----------------
    // item (u, c, g); group g: 0 = G_(0,0), 1 = G_(1,0), 2 = G_(0,1), 3 = G_(1,1)
    for (int it = tid; it < J3 * C * NG; it += NT) {
      const int u = it % J3, c = (it / J3) % C, g = it / (J3 * C);
      const int q1 = col0 + c;
      if (q1 >= qend || u >= nj3) continue;
      int h1, h0;   // inputs through B2^(1) and B2^(0)
      if constexpr (STIFF) {
        h1 = g == 0 ? 0 : (g == 2 ? 3 : -1);   // -1: none (zeros)
        h0 = g == 0 ? 1 : (g == 1 ? 5 : (g == 2 ? 4 : 2));
      } else {
        h1 = -1;
        h0 = 0;
      }
      T G[IC];
#pragma unroll
      for (int jj2 = 0; jj2 < IC; ++jj2) G[jj2] = T(0);
      const T* hb0 = hbuf + (size_t(c) * NH + h0) * QC * J3 + u;
      const T* hb1 = h1 >= 0 ? hbuf + (size_t(c) * NH + h1) * QC * J3 + u : hzero + u;
      if (band2) {
        // row i2 away from the boundary spans: its 2P+1 points alternate
        // span midpoints (P+1 nonzero functions) and knots (P), so the
        // nonzero part of B2 is a fixed band; the zeros are skipped
#pragma unroll
        for (int qq2 = 0; qq2 < 2 * P + 1; ++qq2) {
          const T x0 = hb0[qq2 * J3];
          const T x1 = STIFF ? hb1[qq2 * J3] : T(0);
          const T* b = B2 + qq2 * BQ;
          const int lo = (qq2 + 1) / 2, hi = qq2 / 2 + P;
#pragma unroll
          for (int jj2 = 0; jj2 < IC; ++jj2) {
            if (jj2 < lo || jj2 > hi) continue;
            if constexpr (STIFF) G[jj2] = fma(b[jj2 * 2 + 1], x1, fma(b[jj2 * 2], x0, G[jj2]));
            else G[jj2] = fma(b[jj2 * BJ], x0, G[jj2]);
          }
        }
      } else {
#pragma unroll 2
        for (int qq2 = 0; qq2 < qc2; ++qq2) {   // uniform trip count
          const T x0 = hb0[qq2 * J3];
          const T x1 = STIFF ? hb1[qq2 * J3] : T(0);
          const T* b = B2 + __builtin_amdgcn_readfirstlane(qq2 * BQ);
#pragma unroll
          for (int jj2 = 0; jj2 < IC; ++jj2) {
            if constexpr (STIFF) G[jj2] = fma(b[jj2 * 2 + 1], x1, fma(b[jj2 * 2], x0, G[jj2]));
            else G[jj2] = fma(b[jj2 * BJ], x0, G[jj2]);
          }
        }
      }
      T* gb = gbuf + (size_t(c * NG + g) * IC) * J3 + u;
#pragma unroll
      for (int jj2 = 0; jj2 < IC; ++jj2) gb[jj2 * J3] = G[jj2];
    }
    __syncthreads();
    // ---------------- phase C ----------------
    for (int c = 0; c < C; ++c) {
      const int q1 = col0 + c;
      if (q1 >= qend) break;   // uniform
      const int e = span1[q1];
      while (e_cur < e) {      // uniform; rows before e are complete
        flush(e_cur);
        ++e_cur;
      }
      if (cl) {
        const T* ct = CT + __builtin_amdgcn_readfirstlane(q1 * NCT);
        const T* gb = gbuf + (size_t(c * NG) * IC + cj2) * J3 + cu3;
        if constexpr (STIFF) {
          const T g00 = gb[0 * IC * J3], g10 = gb[1 * IC * J3], g01 = gb[2 * IC * J3], g11 = gb[3 * IC * J3];
#pragma unroll
          for (int s = 0; s <= P; ++s) {
            const T* w = ct + s * 4;
            const T H0 = w[R00] * g00 + w[R01] * g01;
            const T H1 = w[R10] * g10 + w[R11] * g11;
#pragma unroll
            for (int r = 0; r <= P; ++r)
              acc[s][r - s + P] = fma(ct[5 * (P + 1) + r], H1, fma(ct[4 * (P + 1) + r], H0, acc[s][r - s + P]));
          }
        } else {
          const T g0 = gb[0];
#pragma unroll
          for (int s = 0; s <= P; ++s) {
            const T H0 = ct[s * 4 + R00] * g0;
#pragma unroll
            for (int r = 0; r <= P; ++r) acc[s][r - s + P] = fma(ct[4 * (P + 1) + r], H0, acc[s][r - s + P]);
          }
        }
      }
    }
    __syncthreads();
  }
  // the rows still open
  for (int s = 0; s <= P; ++s) flush(e_cur + s);
}

// ---------------------------------------------------------------------------
// Plane patches and curves (d <= 2).  Direction 3 is trivial (one point,
// T3 = 1) and the field channels that involve it (K13, K23, K33) are zero,
// so the first contraction would only copy the field, and each dir-1 rule
// group of the stiffness meets exactly one input:
//   G_(0,0) = sum_q2 B2^(1) w2^(1,1) K22     G_(1,0) = sum_q2 B2^(0) w2^(0,1) K12
//   G_(0,1) = sum_q2 B2^(1) w2^(1,0) K12     G_(1,1) = sum_q2 B2^(0) w2^(0,0) K11
// (the mass: G = sum_q2 B2^(0) w2^(0,0) det J).  A pencil has a single j3
// here, so its phase C would keep 2p+1 lanes busy; instead one wave owns a
// strip of K consecutive rows i2 (at most floor(64 / (2p+1))) over a run
// of dir-1 rows.  The strip's dir-2 operators and weights are copied to LDS
// once; per chunk of C quadrature columns the field values of the strip's
// q2 window are staged in LDS (loaded during the previous chunk's phase C,
// or after it where registers are short):
//   phase AB (lanes: column c, half h, row slot): for the strip's rows,
//            UB at a time, and each operator B2^(a) in turn, the group
//            that meets B2^(a) in half h, for all j2, into LDS;
//   phase C  (lanes: j2, row u):  the push of the pencil kernel with the K
//            rows side by side (the column tables are shared by the strip).
// These are the pencil kernel's products without its exact zeros, in the
// same order.

// Columns per chunk of the strip kernel.
#ifndef WQ_PLANE_CS
#define WQ_PLANE_CS 8
#endif
#ifndef WQ_PLANE_CM
#define WQ_PLANE_CM 16
#endif
// Rows i2 per strip (at most floor(64/(2p+1)), the rows phase C has lanes
// for; fewer rows use less LDS, which buys waves per compute unit).
#ifndef WQ_PLANE_K
#define WQ_PLANE_K 4
#endif
// Column tables of a chunk staged in LDS with the field tile (1) or read
// with scalar loads per column (0).
#ifndef WQ_PLANE_CTAB
#define WQ_PLANE_CTAB 0
#endif
// Strips are split into runs of rows until the grid holds about this many
// workgroups.
#ifndef WQ_PLANE_WG_TARGET
#define WQ_PLANE_WG_TARGET 4096
#endif

template <int P, typename T, bool STIFF>
struct PlaneShape {
  static constexpr int IC = 2 * P + 1, QC = 3 * P + 1;
  static constexpr int ICP = IC + 1;                      // even row stride of the operator copy
  // the p = 6 FP64 stiffness (phase-C accumulators alone 182 VGPRs) takes
  // 2 rows and a bound of 2 waves per SIMD: with 4 rows its LDS and
  // registers left one wave per SIMD
  static constexpr bool TIGHT = P == 6 && STIFF && sizeof(T) == 8;
  static constexpr int KW = TIGHT ? 2 : WQ_PLANE_K;
  static constexpr int K = KW > 0 && KW < 64 / IC ? KW : 64 / IC;   // rows i2 per strip
  static constexpr int WPE = TIGHT ? 2 : 0;                          // waves per SIMD bound
  static constexpr int NG = STIFF ? 4 : 1;                // dir-1 rule groups
  static constexpr int NA = STIFF ? 2 : 1;                // groups per operator (halves)
  static constexpr int NB = STIFF ? 2 : 1;                // operators B2^(a) used
  static constexpr int C = STIFF ? WQ_PLANE_CS : WQ_PLANE_CM;
  static constexpr int UB = 64 / (C * NA);                // strip rows per pass of phase AB
  static constexpr int CP = C + 1;                        // odd column stride of the tile: fewer bank conflicts
  static constexpr int NCHT = STIFF ? 3 : 1;              // field channels in the tile
  // q2 points of a strip: spans max(0, i2a-p) .. min(n_el-1, i2a+K-1), at
  // most 2 per interior span and p+1 in a boundary one
  static constexpr int WMAX = 2 * K + 4 * P - 1;
  // the mass keeps a compact copy of its operator: at each point only the
  // p+1 functions that can be nonzero there (less LDS, more workgroups per
  // compute unit); for the stiffness, whose two operators are read in the
  // same loops, the full rows measured faster
  static constexpr bool COMPACT = !STIFF;
  static constexpr int PW = P + 1;                        // functions nonzero at a point
  static constexpr int PWS = (PW + 1) & ~1;               // their even row stride in the compact copy
  static constexpr size_t GBUF = size_t(NG) * C * K * IC;   // [g][c][u][jj2]: phase-C reads contiguous
  static constexpr size_t STAGE = size_t(K) * IC * IC;
  static constexpr size_t TILE = size_t(NCHT) * WMAX * CP;
  static constexpr size_t TSBUF = TILE > STAGE ? TILE : STAGE;   // the row stage shares the tile
  static constexpr size_t BS = COMPACT ? size_t(K) * NB * QC * PWS : size_t(K) * NB * QC * ICP;
  static constexpr size_t BLO = COMPACT ? size_t(K) * QC : 1;   // first function of the window (int)
  static constexpr size_t WS = size_t(K) * QC * 4;
  static constexpr int NCT = 6 * (P + 1);                 // column-table entries
  static constexpr size_t CTAB = WQ_PLANE_CTAB ? size_t(C) * NCT : 1;
  static constexpr int TPL = int((size_t(NCHT) * WMAX * C + 63) / 64);   // tile values per lane
  static constexpr int CPL = WQ_PLANE_CTAB ? int((CTAB + 63) / 64) : 0;   // column-table values per lane
  // FP64 at p >= 4: fewer live registers (the next tile is loaded after
  // phase C instead of during it, and rows are stored one strip row at a
  // time), which buys a wave per SIMD where the count crosses 128 or 256
  static constexpr bool LEAN = sizeof(T) == 8 && P >= 4;
  static constexpr size_t LDS_BYTES = (GBUF + TSBUF + BS + WS + CTAB) * sizeof(T) + BLO * sizeof(int);
  static_assert(C * NA * UB <= 64 && C * NA * 2 * UB > 64, "phase AB fills most of the wave");
  static_assert(LDS_BYTES <= 64 * 1024, "LDS budget per workgroup");
};

template <int P, typename T, bool STIFF>
__device__ __forceinline__ void plane_body(const PlanView& v, T* __restrict__ out, int nseg, int item) {
  using S = PlaneShape<P, T, STIFF>;
  constexpr int IC = S::IC, QC = S::QC, ICP = S::ICP, K = S::K, C = S::C, CP = S::CP, UB = S::UB;
  constexpr int NB = S::NB, NCHT = S::NCHT, WMAX = S::WMAX, TPL = S::TPL, CPL = S::CPL, NCT = S::NCT;
  constexpr int PW = S::PW, PWS = S::PWS;
  constexpr int GSTR = C * K * IC;   // distance between groups in the G buffer
  const DirView d1 = v.dir[0], d2 = v.dir[1];
  const int n1 = d1.n, n2 = d2.n, nq1 = d1.nq, nel1 = d1.nel;
  const int tid = threadIdx.x;
  const int nstrip = (n2 + K - 1) / K;
  const int strip = item % nstrip, seg = item / nstrip;
  const int i2a = strip * K;
  const int nu = min(K, n2 - i2a);   // rows of this strip

  // rows r0..r1-1 need the columns of spans e0..e1 (as for the pencils)
  const int r0 = int(int64_t(seg) * n1 / nseg), r1 = int(int64_t(seg + 1) * n1 / nseg);
  const int e0 = max(0, r0 - P), e1 = min(nel1 - 1, r1 - 1);
  const int qbeg = e0 == 0 ? 0 : P + 2 * e0 - 1;
  const int qend = e1 == nel1 - 1 ? nq1 : P + 2 * e1 + 1;
  // q2 window of the strip: [wq0, wq0 + nw)
  int wq0, wqc, wql, wqlc;
  q_range(i2a, P, d2.nel, wq0, wqc);
  q_range(i2a + nu - 1, P, d2.nel, wql, wqlc);
  const int nw = wql + wqlc - wq0;

  __shared__ __align__(16) T gbuf[S::GBUF];     // the groups G of a chunk, [g][c][u][jj2]
  // the field tile, [channel][q2 - wq0][c] (stride CP), is read in phase AB
  // only; in phase C it is free and holds the row stage [u][jj2][jj1]
  __shared__ __align__(16) T tsbuf[S::TSBUF];
  T* const tile = tsbuf;
  T* const stage = tsbuf;
  __shared__ __align__(16) T bs[S::BS];         // [u][a][qq2][r], jj2 = blo + r (compact), or [u][a][qq2][jj2] (stride ICP)
  __shared__ int blo[S::BLO];                   // [u][qq2]: first function of the window, relative to I_i2
  __shared__ __align__(16) T wsh[S::WS];        // [u][qq2][o]
  __shared__ __align__(16) T ctab[S::CTAB];     // column tables of the chunk, [c][NCT]
  const T* __restrict__ fld = static_cast<const T*>(v.field);
  const int64_t N = v.nqtot;
  const T* __restrict__ CT = colt_t<T>(d1);
  const int* __restrict__ span1 = d1.qspan;
  const int64_t Tn1 = d1.prefix[n1];

  // the strip's dir-2 operators (B2^(a) rows, a-major) and weights
  {
    const T* __restrict__ bsrc = bt_t<T>(d2) + size_t(i2a) * QC * IC * 2;   // [u][qq2][jj2][a]
    if constexpr (S::COMPACT) {
      // at point q the functions qspan(q) .. qspan(q) + p can be nonzero; all
      // of them lie in I_i2 when x_q lies in the support of B_i2
      for (int t = tid; t < nu * QC; t += 64) {
        const int u = t / QC, qq2 = t % QC;
        int qs2, qc2, is2, ic2;
        q_range(i2a + u, P, d2.nel, qs2, qc2);
        i_range(i2a + u, P, n2, is2, ic2);
        blo[t] = qq2 < qc2 ? d2.qspan[qs2 + qq2] - is2 : 0;
      }
      __syncthreads();
      for (int t = tid; t < nu * NB * QC * PWS; t += 64) {
        const int r = t % PWS, qq2 = (t / PWS) % QC, a = (t / (PWS * QC)) % NB, u = t / (PWS * QC * NB);
        const int jj2 = blo[u * QC + qq2] + r;
        bs[t] = r < PW && jj2 >= 0 && jj2 < IC ? bsrc[((u * QC + qq2) * IC + jj2) * 2 + a] : T(0);
      }
    } else {
      for (int t = tid; t < nu * QC * IC * 2; t += 64) {
        const int a = t % 2, jj2 = (t / 2) % IC, qq2 = (t / (2 * IC)) % QC, u = t / (2 * IC * QC);
        if (a < NB) bs[((u * NB + a) * QC + qq2) * ICP + jj2] = bsrc[t];
      }
    }
    const T* __restrict__ wsrc = wt_t<T>(d2) + size_t(i2a) * QC * 4;
    for (int t = tid; t < nu * QC * 4; t += 64) wsh[t] = wsrc[t];
  }

  // field tile and column tables of a chunk: element t = (channel, q2
  // offset, column) and (column, entry); each lane holds TPL + CPL of them
  // between the load and the store
  T tpre[TPL], cpre[CPL > 0 ? CPL : 1];
  auto tile_load = [&](int col0) {
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      const int t = tid + 64 * k;
      cpre[k] = T(0);
      if (t < C * NCT) cpre[k] = CT[int64_t(min(col0 + t / NCT, qend - 1)) * NCT + t % NCT];
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      const int t = tid + 64 * k;
      const int ch = t / (WMAX * C), w = (t / C) % WMAX, c = t % C;
      tpre[k] = T(0);
      if (ch < NCHT && w < nw) {
        const int fch = STIFF ? (ch == 0 ? 1 : (ch == 1 ? 2 : 4)) : 0;   // K11, K22, K12 / det J
        tpre[k] = fld[fch * N + int64_t(wq0 + w) * nq1 + min(col0 + c, qend - 1)];
      }
    }
  };
  auto tile_store = [&]() {
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      const int t = tid + 64 * k;
      if (t < C * NCT) ctab[t] = cpre[k];
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      const int t = tid + 64 * k;
      const int ch = t / (WMAX * C), w = (t / C) % WMAX, c = t % C;
      if (ch < NCHT) tile[(ch * WMAX + w) * CP + c] = tpre[k];
    }
  };

  // phase-C role of this lane: (jj2, u)
  const int cj2 = tid % IC, cu = tid / IC;
  int my_ic2 = 0;
  if (cu < nu) {
    int is2;
    i_range(i2a + cu, P, n2, is2, my_ic2);
  }
  const bool cl = cj2 < my_ic2;
  T acc[P + 1][2 * P + 1];   // open rows e+s, s = 0..P; trial offset d = j1 - (e+s) + P
#pragma unroll
  for (int s = 0; s <= P; ++s)
#pragma unroll
    for (int d = 0; d <= 2 * P; ++d) acc[s][d] = T(0);

  // row i1 (slot 0) of every row of the strip is complete: store the ones
  // of this run, then shift the slots
  auto flush = [&](int i1) {
    if (i1 >= r0 && i1 < r1) {   // uniform
      const int dlo = i1 < P ? P - i1 : 0;
      const int dhi = min(2 * P, P + n1 - 1 - i1);
      const int ic1 = dhi - dlo + 1;
      if (cl) {
        T* st = stage + cu * (IC * IC) + cj2 * ic1 - dlo;
#pragma unroll
        for (int d = 0; d <= 2 * P; ++d)
          if (d >= dlo && d <= dhi) st[d] = acc[0][d];
      }
      __syncthreads();
      const int64_t row1 = d1.prefix[i1];
#pragma unroll(S::LEAN ? 1 : K)
      for (int u = 0; u < K; ++u) {   // uniform: one contiguous CSR row each
        if (u < nu) {
          const int i2 = i2a + u;
          int is2, ic2;
          i_range(i2, P, n2, is2, ic2);
          T* o = out + d2.prefix[i2] * Tn1 + int64_t(ic2) * row1;
          const int len = ic2 * ic1;
#pragma unroll
          for (int k = 0; k < (IC * IC + 63) / 64; ++k) {
            const int t = tid + 64 * k;
            if (t < len) o[t] = stage[u * (IC * IC) + t];
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < P; ++s) {
#pragma unroll
      for (int d = 0; d < 2 * P - s; ++d) acc[s][d] = acc[s + 1][d];
      acc[s][2 * P - s] = T(0);
    }
#pragma unroll
    for (int d = 0; d <= P; ++d) acc[P][d] = T(0);
  };

  // phase-AB role of this lane: (column ac, half ah, row slot ab)
  const int ac = tid % C, ah = (tid / C) % S::NA, ab = tid / (C * S::NA);
  const bool al = ab < UB;

  int e_cur = e0;
  tile_load(qbeg);
  tile_store();
  __syncthreads();
  for (int col0 = qbeg; col0 < qend; col0 += C) {
    // ---------------- phase AB ----------------
    for (int u0 = 0; u0 < nu; u0 += UB) {   // uniform
      const int u = u0 + ab;
      if (al && u < nu) {
        const int i2 = i2a + u;
        int qs2, qc2;
        q_range(i2, P, d2.nel, qs2, qc2);
        // rows whose support spans are all interior: fixed point layout and
        // a fixed band of nonzeros in B2 (as in the pencil kernel)
        const bool band2 = i2 >= P + 1 && i2 <= d2.nel - 2;
        auto group = [&](auto a_) {
          constexpr int A = decltype(a_)::value;   // the operator B2^(A)
          constexpr int AI = NB == 2 ? A : 0;
          // group, tile channel and dir-2 rule of the halves 0 and 1
          constexpr int G0 = STIFF ? (A ? 0 : 1) : 0, G1 = STIFF ? (A ? 2 : 3) : 0;
          constexpr int TC0 = STIFF ? (A ? 1 : 2) : 0, TC1 = STIFF ? (A ? 2 : 0) : 0;
          constexpr int RL0 = STIFF ? (A ? R11 : R01) : R00, RL1 = STIFF ? (A ? R10 : R00) : R00;
          const T* tr = tile + ((ah ? TC1 : TC0) * WMAX + (qs2 - wq0)) * CP + ac;   // + qq2 * CP
          const T* wr = wsh + u * QC * 4 + (ah ? RL1 : RL0);                        // + qq2 * 4
          constexpr int BQ = S::COMPACT ? PWS : ICP;                                // operator copy: stride of qq2
          const T* br = bs + (u * NB + AI) * QC * BQ;
          T G[IC];
#pragma unroll
          for (int jj2 = 0; jj2 < IC; ++jj2) G[jj2] = T(0);
          if (band2) {
            // interior row: the window of point qq2 starts at (qq2 + 1) / 2
#pragma unroll
            for (int qq2 = 0; qq2 < 2 * P + 1; ++qq2) {
              const T x = wr[qq2 * 4] * tr[qq2 * CP];
              const int lo = (qq2 + 1) / 2, hi = qq2 / 2 + P;
#pragma unroll
              for (int jj2 = 0; jj2 < IC; ++jj2)
                if (jj2 >= lo && jj2 <= hi)
                  G[jj2] = fma(br[qq2 * BQ + (S::COMPACT ? jj2 - lo : jj2)], x, G[jj2]);
            }
          } else {
            for (int qq2 = 0; qq2 < qc2; ++qq2) {
              const T x = wr[qq2 * 4] * tr[qq2 * CP];
              const T* bq = br + qq2 * BQ;
              if constexpr (S::COMPACT) {
                const int lo = blo[u * QC + qq2];
#pragma unroll
                for (int jj2 = 0; jj2 < IC; ++jj2) {
                  const int r = jj2 - lo;
                  const T bv = bq[r < 0 ? 0 : (r > P ? P : r)];
                  G[jj2] = fma(r >= 0 && r <= P ? bv : T(0), x, G[jj2]);
                }
              } else {
#pragma unroll
                for (int jj2 = 0; jj2 < IC; ++jj2) G[jj2] = fma(bq[jj2], x, G[jj2]);
              }
            }
          }
          T* gb = gbuf + (((ah ? G1 : G0) * C + ac) * K + u) * IC;
#pragma unroll
          for (int jj2 = 0; jj2 < IC; ++jj2) gb[jj2] = G[jj2];
        };
        if constexpr (STIFF) {
          group(std::integral_constant<int, 1>{});
          group(std::integral_constant<int, 0>{});
        } else {
          group(std::integral_constant<int, 0>{});
        }
      }
    }
    __syncthreads();
    const bool more = col0 + C < qend;   // uniform
    if (!S::LEAN && more) tile_load(col0 + C);   // in flight during phase C
    // ---------------- phase C ----------------
    for (int c = 0; c < C; ++c) {
      const int q1c = col0 + c;
      if (q1c >= qend) break;   // uniform
      const int e = span1[q1c];
      while (e_cur < e) {       // uniform; rows before e are complete
        flush(e_cur);
        ++e_cur;
      }
      if (cl) {
        const T* ct = WQ_PLANE_CTAB ? ctab + c * NCT : CT + int64_t(__builtin_amdgcn_readfirstlane(q1c)) * NCT;
        const T* gb = gbuf + c * K * IC + tid;   // (g, c, u, jj2) = (g, c, cu, cj2)
        if constexpr (STIFF) {
          const T g00 = gb[0], g10 = gb[GSTR], g01 = gb[2 * GSTR], g11 = gb[3 * GSTR];
#pragma unroll
          for (int s = 0; s <= P; ++s) {
            const T* w = ct + s * 4;
            const T H0 = w[R00] * g00 + w[R01] * g01;
            const T H1 = w[R10] * g10 + w[R11] * g11;
#pragma unroll
            for (int r = 0; r <= P; ++r)
              acc[s][r - s + P] = fma(ct[5 * (P + 1) + r], H1, fma(ct[4 * (P + 1) + r], H0, acc[s][r - s + P]));
          }
        } else {
          const T g0 = gb[0];
#pragma unroll
          for (int s = 0; s <= P; ++s) {
            const T H0 = ct[s * 4 + R00] * g0;
#pragma unroll
            for (int r = 0; r <= P; ++r) acc[s][r - s + P] = fma(ct[4 * (P + 1) + r], H0, acc[s][r - s + P]);
          }
        }
      }
    }
    if (S::LEAN && more) tile_load(col0 + C);
    if (more) tile_store();   // after the last flush of the chunk's phase C
    __syncthreads();
  }
  // the rows still open
  for (int s = 0; s <= P; ++s) flush(e_cur + s);
}

// XCD-aware order: workgroups are dealt round-robin to the 8 XCDs; give
// each XCD a contiguous range of work items so that neighbouring pencils,
// which read overlapping coefficient blocks, share an L2.
__device__ inline int xcd_item() {
  const int total = gridDim.x, L = blockIdx.x;
  const int xcd = L % 8, kx = L / 8, m8 = total / 8, r8 = total % 8;
  return xcd * m8 + min(xcd, r8) + kx;
}

// The pencil kernel; configurations with WPE > 0 use the variant whose
// register allocation is bounded for that many waves per SIMD.
template <int P, typename T, bool STIFF>
__global__ __launch_bounds__((Shape<P, T, STIFF>::NT)) void k_push(PlanView v, T* __restrict__ out, int nseg, int item0) {
  push_body<P, T, STIFF>(v, out, nseg, item0 + xcd_item());
}
template <int P, typename T, bool STIFF>
__global__ __launch_bounds__((Shape<P, T, STIFF>::NT))
__attribute__((amdgpu_waves_per_eu(PushCfg<P, T, STIFF>::WPE))) void k_push_wpe(PlanView v, T* __restrict__ out, int nseg, int item0) {
  push_body<P, T, STIFF>(v, out, nseg, item0 + xcd_item());
}
// The strip kernel of plane patches and curves (one wave per workgroup).
template <int P, typename T, bool STIFF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(PlaneShape<P, T, STIFF>::WPE)))
void k_plane(PlanView v, T* __restrict__ out, int nseg) {
  plane_body<P, T, STIFF>(v, out, nseg, xcd_item());
}

// Work units per run of rows: (pencil, j3 part) of a solid patch, strips
// of K rows i2 of a plane patch or curve.
template <int P, typename T, bool STIFF, bool PLANE>
int64_t units_of(int n2, int n3) {
  if constexpr (PLANE) return (int64_t(n2) + PlaneShape<P, T, STIFF>::K - 1) / PlaneShape<P, T, STIFF>::K * n3;
  else return int64_t(n2) * n3 * Shape<P, T, STIFF>::NPART;
}

// ---------------------------------------------------------------------------
// Batched form: the patches of one class (degree p, dimension d, precision)
// of a batch, each with its own plan view, outputs and work list.  For
// solid patches the first contraction runs as one launch over all patches'
// blocks; the pencil (or strip) kernel as one persistent launch whose
// workgroups take (patch, work item) pairs from a device queue until it is
// exhausted.  Work items of a patch are numbered as in the single-patch
// launch, so each row is formed by the same arithmetic in the same order.

// largest k in [0, n) with off[k] <= x (off ascending, off[0] = 0)
__device__ inline int find_patch(const int* __restrict__ off, int n, int x) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (off[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int P, typename T, bool STIFF>
__global__ __launch_bounds__(256) void k_first_batch(BatchClassView b) {
  __shared__ int sk;
  if (threadIdx.x == 0) sk = find_patch(b.blocks, b.np, blockIdx.x);
  __syncthreads();
  const int k = sk;
  const PlanView v = b.views[k];
  const int64_t plane = int64_t(v.dir[0].nq) * v.dir[1].nq;
  const int nbx = int((plane + 255) / 256);
  const int local = int(blockIdx.x) - b.blocks[k];
  first_body<P, T, STIFF>(v, local % nbx, local / nbx);
}

template <int P, typename T, bool STIFF, bool PLANE>
__device__ __forceinline__ void push_batch_body(const BatchClassView& b) {
  __shared__ int s_w, s_k;
  const int* items = STIFF ? b.items_stiff : b.items_mass;
  const int* nsegs = STIFF ? b.nsegs_stiff : b.nsegs_mass;
  int* counter = b.counter + (STIFF ? 1 : 0);
  const int total = items[b.np];
  for (;;) {
    if (threadIdx.x == 0) {
      const int w = atomicAdd(counter, 1);
      s_w = w;
      s_k = w < total ? find_patch(items, b.np, w) : 0;
    }
    __syncthreads();
    const int w = s_w, k = s_k;
    if (w >= total) break;   // uniform: every workgroup leaves once the queue is empty
    const PlanView v = b.views[k];
    T* out = static_cast<T*>(STIFF ? b.out_stiff[k] : b.out_mass[k]);
    if constexpr (PLANE) plane_body<P, T, STIFF>(v, out, nsegs[k], w - items[k]);
    else push_body<P, T, STIFF>(v, out, nsegs[k], w - items[k]);
    __syncthreads();   // s_w and s_k are rewritten by the next take
  }
}
template <int P, typename T, bool STIFF, bool PLANE>
constexpr int batch_threads() { return PLANE ? 64 : Shape<P, T, STIFF>::NT; }
template <int P, typename T, bool STIFF, bool PLANE>
__global__ __launch_bounds__((batch_threads<P, T, STIFF, PLANE>())) void k_push_batch(BatchClassView b) {
  push_batch_body<P, T, STIFF, PLANE>(b);
}

__global__ void k_zero_counters(int* c, int n) {
  if (int(threadIdx.x) < n) c[threadIdx.x] = 0;
}

template <int P, typename T, bool STIFF, bool PLANE>
hipError_t batch_launch(const BatchClassView& b, int first_blocks, int grid, hipStream_t s) {
  if constexpr (!PLANE) {
    if (first_blocks > 0)
      hipLaunchKernelGGL((k_first_batch<P, T, STIFF>), dim3(unsigned(first_blocks)), dim3(256), 0, s, b);
  }
  // (the persistent loop needs more registers than one pencil: the bounds
  // of the single-patch configurations would make it spill)
  hipLaunchKernelGGL((k_push_batch<P, T, STIFF, PLANE>), dim3(unsigned(grid)), dim3(batch_threads<P, T, STIFF, PLANE>()), 0, s, b);
  return hipGetLastError();
}

template <int P, typename T>
hipError_t batch_pt(const BatchClassView& b, int d, bool stiff, int first_blocks, int grid, hipStream_t s) {
  if (stiff)
    return d <= 2 ? batch_launch<P, T, true, true>(b, first_blocks, grid, s) : batch_launch<P, T, true, false>(b, first_blocks, grid, s);
  return d <= 2 ? batch_launch<P, T, false, true>(b, first_blocks, grid, s) : batch_launch<P, T, false, false>(b, first_blocks, grid, s);
}

template <int P>
hipError_t batch_p(const BatchClassView& b, int d, int prec, bool stiff, int first_blocks, int grid, hipStream_t s) {
  return prec == WQ_FP64 ? batch_pt<P, double>(b, d, stiff, first_blocks, grid, s)
                         : batch_pt<P, float>(b, d, stiff, first_blocks, grid, s);
}

template <int P>
int64_t units_p(int d, int prec, bool stiff, int n2, int n3) {
  if (prec == WQ_FP64) {
    if (stiff) return d <= 2 ? units_of<P, double, true, true>(n2, n3) : units_of<P, double, true, false>(n2, n3);
    return d <= 2 ? units_of<P, double, false, true>(n2, n3) : units_of<P, double, false, false>(n2, n3);
  }
  if (stiff) return d <= 2 ? units_of<P, float, true, true>(n2, n3) : units_of<P, float, true, false>(n2, n3);
  return d <= 2 ? units_of<P, float, false, true>(n2, n3) : units_of<P, float, false, false>(n2, n3);
}

// The rows of the pencils with i3 in [i3a, i3b): k_first fills the Y planes
// of that slab (v.ybuf holds the planes from v.y_i3 on), k_push forms them.
// Workgroups are ordered i3 slowest, so a slab is a contiguous item range.
template <int P, typename T, bool STIFF>
hipError_t push_launch(const PlanView& v, void* out, hipStream_t s, int i3a, int i3b) {
  using Sh = Shape<P, T, STIFF>;
  const int64_t wgs = units_of<P, T, STIFF, false>(v.dir[1].n, v.dir[2].n);
  // runs of at least 2p rows
  const int max_seg = std::max(1, v.dir[0].n / (2 * P));
  const int nseg = int(std::min<int64_t>(max_seg, std::max<int64_t>(1, (WQ_WG_TARGET + wgs - 1) / wgs)));
  const int64_t items = wgs * nseg;
  if (items <= 0 || items > INT32_MAX) return hipErrorInvalidConfiguration;
  const int64_t per_i3 = items / v.dir[2].n;
  const int64_t plane = int64_t(v.dir[0].nq) * v.dir[1].nq;
  if (i3b <= i3a) return hipSuccess;
  hipLaunchKernelGGL((k_first<P, T, STIFF>), dim3(unsigned((plane + 255) / 256), unsigned(i3b - i3a)), dim3(256), 0, s, v);
  const dim3 grid(unsigned(per_i3 * (i3b - i3a)));
  const int item0 = int(per_i3 * i3a);
  if constexpr (PushCfg<P, T, STIFF>::WPE > 0)
    hipLaunchKernelGGL((k_push_wpe<P, T, STIFF>), grid, dim3(Sh::NT), 0, s, v, static_cast<T*>(out), nseg, item0);
  else
    hipLaunchKernelGGL((k_push<P, T, STIFF>), grid, dim3(Sh::NT), 0, s, v, static_cast<T*>(out), nseg, item0);
  return hipGetLastError();
}

// All rows of a plane patch or curve: the strip kernel alone (it reads the
// coefficient field directly; no first-contraction buffer).
template <int P, typename T, bool STIFF>
hipError_t plane_launch(const PlanView& v, void* out, hipStream_t s) {
  const int64_t wgs = units_of<P, T, STIFF, true>(v.dir[1].n, v.dir[2].n);
  const int max_seg = std::max(1, v.dir[0].n / (2 * P));
  const int nseg = int(std::min<int64_t>(max_seg, std::max<int64_t>(1, (WQ_PLANE_WG_TARGET + wgs - 1) / wgs)));
  const int64_t items = wgs * nseg;
  if (items <= 0 || items > INT32_MAX) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_plane<P, T, STIFF>), dim3(unsigned(items)), dim3(64), 0, s, v, static_cast<T*>(out), nseg);
  return hipGetLastError();
}

template <int P, typename T>
hipError_t assemble_pt(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s, int i3a, int i3b) {
  if (which & WQ_MASS) {
    hipError_t e = v.d <= 2 ? plane_launch<P, T, false>(v, mass, s) : push_launch<P, T, false>(v, mass, s, i3a, i3b);
    if (e != hipSuccess) return e;
  }
  if (which & WQ_STIFF) {
    hipError_t e = v.d <= 2 ? plane_launch<P, T, true>(v, stiff, s) : push_launch<P, T, true>(v, stiff, s, i3a, i3b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int P>
hipError_t assemble_p(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s, int i3a, int i3b) {
  return v.prec == WQ_FP64 ? assemble_pt<P, double>(v, which, mass, stiff, s, i3a, i3b)
                           : assemble_pt<P, float>(v, which, mass, stiff, s, i3a, i3b);
}

hipError_t assemble_slab(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s, int i3a, int i3b) {
  switch (v.p) {
    case 2: return assemble_p<2>(v, which, mass, stiff, s, i3a, i3b);
    case 3: return assemble_p<3>(v, which, mass, stiff, s, i3a, i3b);
    case 4: return assemble_p<4>(v, which, mass, stiff, s, i3a, i3b);
    case 5: return assemble_p<5>(v, which, mass, stiff, s, i3a, i3b);
    case 6: return assemble_p<6>(v, which, mass, stiff, s, i3a, i3b);
    default: return hipErrorInvalidValue;
  }
}

// Scratch of the allocation-free assembly: the first-contraction buffer Y
// for a slab of i3 planes.  Each GPU the library runs on holds its own copy
// (loaded with the code object, kept until the process ends); its address
// on a device comes from hipGetSymbolAddress, taken once per device.
static __device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

hipError_t launch_assemble(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s) {
  PlanView w = v;
  w.y_i3 = 0;
  return assemble_slab(w, which, mass, stiff, s, 0, v.dir[2].n);
}

hipError_t launch_batch_class(const BatchClassView& b, int p, int d, int prec, bool stiff, int first_blocks,
                              int grid, hipStream_t s) {
  switch (p) {
    case 2: return batch_p<2>(b, d, prec, stiff, first_blocks, grid, s);
    case 3: return batch_p<3>(b, d, prec, stiff, first_blocks, grid, s);
    case 4: return batch_p<4>(b, d, prec, stiff, first_blocks, grid, s);
    case 5: return batch_p<5>(b, d, prec, stiff, first_blocks, grid, s);
    case 6: return batch_p<6>(b, d, prec, stiff, first_blocks, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zero_counters(int* c, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, s, c, n);
  return hipGetLastError();
}

int64_t push_units(int p, int d, int prec, bool stiff, int n2, int n3) {
  switch (p) {
    case 2: return units_p<2>(d, prec, stiff, n2, n3);
    case 3: return units_p<3>(d, prec, stiff, n2, n3);
    case 4: return units_p<4>(d, prec, stiff, n2, n3);
    case 5: return units_p<5>(d, prec, stiff, n2, n3);
    case 6: return units_p<6>(d, prec, stiff, n2, n3);
    default: return 0;
  }
}

size_t static_plane_bytes(const PlanView& v, int which) {
  if (v.d <= 2) return 0;   // the strip kernel needs no first-contraction buffer
  const size_t elem = v.prec == WQ_FP64 ? 8 : 4;
  const size_t icy = size_t(icap_of(v.p));
  const size_t nch = (which & WQ_STIFF) ? size_t(kYChannels) : 1;
  return size_t(v.dir[0].nq) * size_t(v.dir[1].nq) * icy * nch * elem;
}

hipError_t launch_assemble_static(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s) {
  if (v.d <= 2) return assemble_slab(v, which, mass, stiff, s, 0, 1);   // no scratch used
  const size_t pb = static_plane_bytes(v, which);
  const int per_slab = int(std::min<size_t>(kStaticScratchBytes / pb, size_t(v.dir[2].n)));
  if (per_slab < 1) return hipErrorInvalidValue;   // refused by the caller beforehand
  void* ptr = nullptr;
  hipError_t e = scratch_on_current_device(&ptr);
  if (e != hipSuccess) return e;
  PlanView w = v;
  w.ybuf = ptr;
  for (int a = 0; a < v.dir[2].n; a += per_slab) {
    const int b = std::min(v.dir[2].n, a + per_slab);
    w.y_i3 = a;
    e = assemble_slab(w, which, mass, stiff, s, a, b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace wq
