// Row formation by sum factorization (Section 6, eq. sumfactorization,
// Algorithm 3) for the mass matrix, and its stiffness analogue (eq. stiff):
// the sum over the 9 pairs (l, m) of test/trial derivative directions, where
// direction k uses the rule w^(alpha_k, beta_k) with alpha_k = [k == m]
// (trial) and beta_k = [k == l] (test), applied to the coefficient c_lm.
//
// Work decomposition ("pencil" kernel).  A workgroup owns the rows
// (i1 = 0..n1-1, i2, i3) of one pencil; they are consecutive rows, so the
// pencil's output is one contiguous CSR segment.  For a pencil the operators
// of directions 3 and 2 are fixed, so the contractions over q3 and q2 are
// shared by all its rows and done once per quadrature column q1:
//
//   phase A (items: q1, q2):  Y_c[j3] = sum_q3 T3_c[j3][q3] K_c(q1,q2,q3) for
//            the 8 distinct (field, dir-3 rule) channels of the stiffness
//            (1 for the mass); then the dir-2 weights are folded in:
//            terms that will meet the same B2^(alpha) and the same dir-1 rule
//            are summed after scaling by their weights w2 ("weight merge"),
//            leaving 6 arrays H[q2][j3] (1 for the mass) in LDS.
//   phase B (items: q1, j3, group):  G_g[j2][j3] = sum_q2 B2^(a)[j2][q2] H,
//            one group per dir-1 rule (4 for the stiffness, 1 for the mass),
//            into an LDS ring buffer indexed by q1.
//   phase C (items: row, j2, j3, j1-part):  for each row i1, once all q1 in
//            Q_i1 are in the ring,  out[j1][j2][j3] = sum_q1
//            B1^(0)[j1][q1] (w1^(0,0) G_(0,0) + w1^(0,1) G_(0,1))
//          + B1^(1)[j1][q1] (w1^(1,0) G_(1,0) + w1^(1,1) G_(1,1)),
//            staged in LDS and stored coalesced.
//
// All univariate operators, weights and B-spline tables are read with
// wavefront-uniform addresses (scalar loads); only the coefficient field and
// the LDS intermediates are per-lane data.  The j3 range can be split across
// workgroups (SC parts) and, inside phases A/B, processed in SA sub-parts, to
// fit the FP64 ring buffer into LDS at high degree.
#include <hip/hip_runtime.h>

#include "wq_internal.h"

// Unroll factors of the quadrature loops of phases A and B/C (trade register
// pressure against loads in flight).
#ifndef WQ_UNROLL_A
#define WQ_UNROLL_A 2
#endif
#ifndef WQ_UNROLL_BC
#define WQ_UNROLL_BC 4
#endif
#define WQ_STR(x) #x
#define WQ_UNROLL(n) _Pragma(WQ_STR(unroll n))

namespace wq {
namespace {

// Rule index o = 2*beta + alpha of the univariate tables.
enum : int { R00 = 0, R10 = 1, R01 = 2, R11 = 3 };

template <int P, typename T> struct PencilCfg;
// SC: j3 parts over workgroups; SA: j3 sub-parts in phases A/B; NP1: j1 parts
// in phase C; C: q1 columns per chunk; NT: threads per workgroup.
template <> struct PencilCfg<2, double> { static constexpr int SC = 1, SA = 1, NP1 = 2, C = 16, NT = 256; };
template <> struct PencilCfg<3, double> { static constexpr int SC = 1, SA = 2, NP1 = 1, C = 12, NT = 256; };
template <> struct PencilCfg<4, double> { static constexpr int SC = 2, SA = 2, NP1 = 1, C = 8, NT = 384; };
template <> struct PencilCfg<5, double> { static constexpr int SC = 2, SA = 2, NP1 = 2, C = 8, NT = 384; };
template <> struct PencilCfg<6, double> { static constexpr int SC = 2, SA = 2, NP1 = 1, C = 8, NT = 256; };
template <> struct PencilCfg<2, float> { static constexpr int SC = 1, SA = 1, NP1 = 2, C = 16, NT = 256; };
template <> struct PencilCfg<3, float> { static constexpr int SC = 1, SA = 1, NP1 = 1, C = 16, NT = 256; };
template <> struct PencilCfg<4, float> { static constexpr int SC = 1, SA = 1, NP1 = 2, C = 16, NT = 384; };
template <> struct PencilCfg<5, float> { static constexpr int SC = 1, SA = 2, NP1 = 1, C = 12, NT = 256; };
template <> struct PencilCfg<6, float> { static constexpr int SC = 1, SA = 2, NP1 = 1, C = 8, NT = 192; };

template <int P, typename T, bool STIFF>
struct Shape {
  using Cfg = PencilCfg<P, T>;
  static constexpr int IC = 2 * P + 1, QC = 3 * P + 1;
  static constexpr int SC = Cfg::SC, SA = Cfg::SA, NP1 = Cfg::NP1, C = Cfg::C, NT = Cfg::NT;
  static constexpr int J3C = (IC + SC - 1) / SC;          // j3 per workgroup
  static constexpr int J3A = (J3C + SA - 1) / SA;         // j3 per phase-A/B sub-part
  static constexpr int J1P = (IC + NP1 - 1) / NP1;        // j1 per phase-C item
  static constexpr int ITEMS_ROW = NP1 * IC * J3C;        // phase-C items of one row
  static constexpr int WPR = (ITEMS_ROW + 63) / 64;       // wavefronts per row
  static constexpr int RB = NT / (64 * WPR);              // rows per phase-C pass
  static constexpr int W = QC + 2 * (RB - 1) + C;         // ring capacity (columns)
  static constexpr int NG = STIFF ? 4 : 1;                // dir-1 rule groups
  static constexpr int NH = STIFF ? 6 : 1;                // merged dir-2 inputs
  static constexpr int NCH = STIFF ? 8 : 1;               // dir-3 channels
  static constexpr size_t RING = size_t(W) * NG * IC * J3C;
  static constexpr size_t HBUF = size_t(C) * NH * QC * J3A;
  static constexpr size_t STAGE = size_t(RB) * IC * IC * J3C;
  static constexpr size_t LDS_BYTES = (RING + HBUF + STAGE) * sizeof(T);
  static_assert(RB >= 1, "a row must fit in one workgroup");
  static_assert(NT % 64 == 0, "whole wavefronts");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS capacity");
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
__device__ inline const T* wt_t(const DirView& d) {
  if constexpr (sizeof(T) == 8) return reinterpret_cast<const T*>(d.wt64);
  else return reinterpret_cast<const T*>(d.wt32);
}

template <int P, typename T, bool STIFF>
__global__ __launch_bounds__((Shape<P, T, STIFF>::NT)) void k_pencil(PlanView v, T* __restrict__ out) {
  using S = Shape<P, T, STIFF>;
  constexpr int IC = S::IC, QC = S::QC, C = S::C, NT = S::NT, J3C = S::J3C, J3A = S::J3A;
  constexpr int J1P = S::J1P, NG = S::NG, NH = S::NH, W = S::W, RB = S::RB, WPR = S::WPR;
  extern __shared__ __align__(16) unsigned char smem[];
  T* ring = reinterpret_cast<T*>(smem);              // [W][NG][IC][J3C]   (slot, g, jj2, u3)
  T* hbuf = ring + S::RING;                          // [C][NH][QC][J3A]   (c, h, qq2, u)
  T* stage = hbuf + S::HBUF;                         // [RB][J3C][IC][IC]  (r, u3, jj2, jj1)

  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int n1 = d1.n, n2 = d2.n, nq1 = d1.nq, nq2 = d2.nq;
  const int tid = threadIdx.x;
  const int pencil = blockIdx.x;
  const int i2 = pencil % n2, i3 = pencil / n2;
  int qs2, qc2, qs3, qc3, is2, ic2, is3, ic3;
  q_range(i2, P, d2.nel, qs2, qc2);
  q_range(i3, P, d3.nel, qs3, qc3);
  i_range(i2, P, n2, is2, ic2);
  i_range(i3, P, d3.n, is3, ic3);
  // this workgroup's j3 range [j3lo, j3lo + nj3)
  const int j3lo = blockIdx.y * J3C;
  const int nj3 = min(J3C, ic3 - j3lo);
  if (nj3 <= 0) return;   // uniform per workgroup

  const int64_t N = v.nqtot;
  const T* __restrict__ field = static_cast<const T*>(v.field);
  // pencil-constant tables (uniform addresses -> scalar loads)
  const T* __restrict__ T3 = op_t<T>(d3) + size_t(i3) * QC * IC * 4;    // [qq3][jj3][o]
  const T* __restrict__ w2 = wt_t<T>(d2) + size_t(i2) * QC * 4;         // [qq2][o]
  const T* __restrict__ B2 = bt_t<T>(d2) + size_t(i2) * QC * IC * 2;    // [qq2][jj2][a]

  // CSR position of row (i1, i2, i3): closed-form prefix of the row lengths
  const int64_t Tn1 = d1.prefix[n1], Tn2 = d2.prefix[n2];
  const int64_t pencil_start = d3.prefix[i3] * Tn2 * Tn1 + int64_t(ic3) * d2.prefix[i2] * Tn1;
  const int64_t row_mult = int64_t(ic3) * ic2;      // row start = pencil_start + row_mult * prefix1[i1]

  int next_col = 0;
  for (int row0 = 0; row0 < n1; row0 += RB) {
    const int rows = min(RB, n1 - row0);
    int qsl, qcl;
    q_range(row0 + rows - 1, P, d1.nel, qsl, qcl);
    const int need_hi = qsl + qcl - 1;                // last column the batch needs
    // ---- produce columns until the batch's window is in the ring ----
    while (next_col <= need_hi) {
      const int col0 = next_col;
      for (int sub = 0; sub < J3C; sub += J3A) {     // j3 sub-parts of phases A/B
        const int ua = sub, na = min(J3A, nj3 - sub); // u in [ua, ua + na) within this WG's range
        if (na <= 0) break;
        // ---------------- phase A ----------------
        for (int it = tid; it < C * QC; it += NT) {
          const int c = it % C, qq2 = it / C;
          const int q1 = col0 + c;
          if (q1 >= nq1 || qq2 >= qc2) continue;
          const int q2 = qs2 + qq2;
          T Y[S::NCH][J3A];
#pragma unroll
          for (int ch = 0; ch < S::NCH; ++ch)
#pragma unroll
            for (int u = 0; u < J3A; ++u) Y[ch][u] = T(0);
          const T* f = field + q1 + int64_t(nq1) * (q2 + int64_t(nq2) * qs3);
          const int64_t fstride = int64_t(nq1) * nq2;
          // field values are loaded for KB consecutive q3 before they are used,
          // so that several loads are in flight per lane
          constexpr int KB = 4;
          constexpr int NF = STIFF ? 6 : 1;
#pragma unroll 1
          for (int b0 = 0; b0 < QC; b0 += KB) {
            if (b0 < qc3) {   // uniform
              T kv[KB][NF];
#pragma unroll
              for (int kb = 0; kb < KB; ++kb) {
                const int qq3 = b0 + kb;
                if (qq3 < qc3) {
                  const T* fk = f + qq3 * fstride;
#pragma unroll
                  for (int fi = 0; fi < NF; ++fi) kv[kb][fi] = fk[(STIFF ? fi + 1 : 0) * N];
                } else {
#pragma unroll
                  for (int fi = 0; fi < NF; ++fi) kv[kb][fi] = T(0);
                }
              }
#pragma unroll
              for (int kb = 0; kb < KB; ++kb) {
                const int qq3 = b0 + kb;
                if (qq3 < qc3) {   // uniform
                  const T* t = T3 + __builtin_amdgcn_readfirstlane((qq3 * IC + j3lo + ua) * 4);
                  if constexpr (STIFF) {
                    const T k11 = kv[kb][0], k22 = kv[kb][1], k33 = kv[kb][2];
                    const T k12 = kv[kb][3], k13 = kv[kb][4], k23 = kv[kb][5];
#pragma unroll
                    for (int u = 0; u < J3A; ++u) {
                      if (j3lo + ua + u < IC) {   // uniform
                        const T t0 = t[u * 4 + R00], t1 = t[u * 4 + R10], t2 = t[u * 4 + R01], t3 = t[u * 4 + R11];
                        Y[0][u] += t0 * k11;
                        Y[1][u] += t0 * k22;
                        Y[2][u] += t3 * k33;
                        Y[3][u] += t0 * k12;
                        Y[4][u] += t1 * k13;
                        Y[5][u] += t2 * k13;
                        Y[6][u] += t1 * k23;
                        Y[7][u] += t2 * k23;
                      }
                    }
                  } else {
#pragma unroll
                    for (int u = 0; u < J3A; ++u)
                      if (j3lo + ua + u < IC) Y[0][u] += t[u * 4 + R00] * kv[kb][0];
                  }
                }
              }
            }
          }
          // fold in the dir-2 weights of this q2 (weight merge)
          T* h = hbuf + (size_t(c) * NH * QC + qq2) * J3A;
          if constexpr (STIFF) {
            const T a0 = w2[qq2 * 4 + R00], a1 = w2[qq2 * 4 + R10];
            const T a2 = w2[qq2 * 4 + R01], a3 = w2[qq2 * 4 + R11];
#pragma unroll
            for (int u = 0; u < J3A; ++u) {
              h[0 * QC * J3A + u] = a3 * Y[1][u] + a1 * Y[7][u];   // -> G_(0,0) through B2^(1)
              h[1 * QC * J3A + u] = a0 * Y[2][u] + a2 * Y[6][u];   // -> G_(0,0) through B2^(0)
              h[2 * QC * J3A + u] = a0 * Y[0][u];                  // -> G_(1,1) through B2^(0)
              h[3 * QC * J3A + u] = a1 * Y[3][u];                  // -> G_(0,1) through B2^(1)
              h[4 * QC * J3A + u] = a0 * Y[4][u];                  // -> G_(0,1) through B2^(0)
              h[5 * QC * J3A + u] = a2 * Y[3][u] + a0 * Y[5][u];   // -> G_(1,0) through B2^(0)
            }
          } else {
            const T a0 = w2[qq2 * 4 + R00];
#pragma unroll
            for (int u = 0; u < J3A; ++u) h[u] = a0 * Y[0][u];
          }
        }
        __syncthreads();
        // ---------------- phase B ----------------
        // item: (u, c, g); group g: 0 = G_(0,0), 1 = G_(1,0), 2 = G_(0,1), 3 = G_(1,1)
        for (int it = tid; it < J3A * C * NG; it += NT) {
          const int u = it % J3A, c = (it / J3A) % C, g = it / (J3A * C);
          const int q1 = col0 + c;
          if (q1 >= nq1 || u >= na) continue;
          // inputs through B2^(1) (h1) and B2^(0) (h0); -1 = none
          int h1, h0;
          if constexpr (STIFF) {
            h1 = g == 0 ? 0 : (g == 2 ? 3 : -1);
            h0 = g == 0 ? 1 : (g == 1 ? 5 : (g == 2 ? 4 : 2));
          } else {
            h1 = -1;
            h0 = 0;
          }
          T G[IC];
#pragma unroll
          for (int jj2 = 0; jj2 < IC; ++jj2) G[jj2] = T(0);
          const T* hb = hbuf + size_t(c) * NH * QC * J3A + u;
WQ_UNROLL(WQ_UNROLL_BC)
          for (int qq2 = 0; qq2 < QC; ++qq2) {
            if (qq2 < qc2) {   // uniform
              const T x0 = hb[(h0 * QC + qq2) * J3A];
              const T x1 = h1 >= 0 ? hb[(h1 * QC + qq2) * J3A] : T(0);
              const T* b = B2 + __builtin_amdgcn_readfirstlane(qq2 * IC * 2);
#pragma unroll
              for (int jj2 = 0; jj2 < IC; ++jj2) {
                if constexpr (STIFF) G[jj2] += b[jj2 * 2] * x0 + b[jj2 * 2 + 1] * x1;
                else G[jj2] += b[jj2 * 2] * x0;
              }
            }
          }
          T* r = ring + ((size_t(q1 % W) * NG + g) * IC) * J3C + ua + u;
#pragma unroll
          for (int jj2 = 0; jj2 < IC; ++jj2) r[jj2 * J3C] = G[jj2];
        }
        __syncthreads();
      }
      next_col += C;
    }
    // ---------------- phase C ----------------
    {
      const int r = __builtin_amdgcn_readfirstlane(tid / (64 * WPR));   // row of this wavefront group
      const int item = tid % (64 * WPR);
      const int i1 = row0 + r;
      if (r < rows && item < S::ITEMS_ROW) {
        const int jj2 = item % IC;
        const int u3 = (item / IC) % J3C;
        const int part = item / (IC * J3C);
        int qs1, qc1, is1, ic1;
        q_range(i1, P, d1.nel, qs1, qc1);
        i_range(i1, P, n1, is1, ic1);
        const T* __restrict__ w1 = wt_t<T>(d1) + size_t(i1) * QC * 4;        // [qq1][o]
        const T* __restrict__ B1 = bt_t<T>(d1) + size_t(i1) * QC * IC * 2;   // [qq1][jj1][a]
        T acc[J1P];
#pragma unroll
        for (int k = 0; k < J1P; ++k) acc[k] = T(0);
        if (u3 < nj3 && jj2 < ic2) {
WQ_UNROLL(WQ_UNROLL_BC)
          for (int qq1 = 0; qq1 < QC; ++qq1) {
            if (qq1 < qc1) {   // uniform per wavefront
              const int q1 = qs1 + qq1;
              const T* rg = ring + (size_t(q1 % W) * NG * IC + jj2) * J3C + u3;
              const T* wq = w1 + __builtin_amdgcn_readfirstlane(qq1 * 4);
              T H0, H1;
              if constexpr (STIFF) {
                const T g00 = rg[0 * IC * J3C], g10 = rg[1 * IC * J3C];
                const T g01 = rg[2 * IC * J3C], g11 = rg[3 * IC * J3C];
                H0 = wq[R00] * g00 + wq[R01] * g01;
                H1 = wq[R10] * g10 + wq[R11] * g11;
              } else {
                H0 = wq[R00] * rg[0];
                H1 = T(0);
              }
              const T* b = B1 + __builtin_amdgcn_readfirstlane((qq1 * IC + part * J1P) * 2);
#pragma unroll
              for (int k = 0; k < J1P; ++k) {
                if (part * J1P + k < IC) {
                  if constexpr (STIFF) acc[k] += b[2 * k] * H0 + b[2 * k + 1] * H1;
                  else acc[k] += b[2 * k] * H0;
                }
              }
            }
          }
          T* st = stage + (size_t(r) * J3C + u3) * IC * IC + jj2 * IC;
#pragma unroll
          for (int k = 0; k < J1P; ++k) {
            const int jj1 = part * J1P + k;
            if (jj1 < ic1) st[jj1] = acc[k];
          }
        }
      }
    }
    __syncthreads();
    // ---- coalesced store of the batch: each row's j3 range is contiguous ----
    for (int r = 0; r < rows; ++r) {
      const int i1 = row0 + r;
      int is1, ic1;
      i_range(i1, P, n1, is1, ic1);
      const int seg = ic1 * ic2;                      // values per j3 slice of the row
      const int64_t base = pencil_start + row_mult * d1.prefix[i1] + int64_t(j3lo) * seg;
      const int len = nj3 * seg;
      for (int t = tid; t < len; t += NT) {
        const int u3 = t / seg, rem = t % seg, jj2 = rem / ic1, jj1 = rem % ic1;
        out[base + t] = stage[((size_t(r) * J3C + u3) * IC + jj2) * IC + jj1];
      }
    }
    __syncthreads();
  }
}

template <int P, typename T, bool STIFF>
hipError_t pencil_launch(const PlanView& v, void* out, hipStream_t s) {
  using Sh = Shape<P, T, STIFF>;
  const int n2 = v.dir[1].n, n3 = v.dir[2].n;
  dim3 grid(unsigned(n2 * n3), unsigned(Sh::SC));
  static bool attr_set = false;   // dynamic LDS above the default limit must be opted into
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pencil<P, T, STIFF>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(Sh::LDS_BYTES));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_pencil<P, T, STIFF>), grid, dim3(Sh::NT), Sh::LDS_BYTES, s, v, static_cast<T*>(out));
  return hipGetLastError();
}

template <int P, typename T>
hipError_t assemble_pt(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s) {
  if (which & WQ_MASS) {
    hipError_t e = pencil_launch<P, T, false>(v, mass, s);
    if (e != hipSuccess) return e;
  }
  if (which & WQ_STIFF) {
    hipError_t e = pencil_launch<P, T, true>(v, stiff, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int P>
hipError_t assemble_p(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s) {
  return v.prec == WQ_FP64 ? assemble_pt<P, double>(v, which, mass, stiff, s)
                           : assemble_pt<P, float>(v, which, mass, stiff, s);
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

}  // namespace wq
