// Row formation by sum factorization (Section 6, eq. sumfactorization,
// Algorithm 3) for the mass matrix, and its stiffness analogue: the sum over
// the 9 pairs (l, m) of test/trial derivative directions (eq. stiff), where
// direction k uses the rule w^(alpha_k, beta_k), alpha_k = [k == m] (trial),
// beta_k = [k == l] (test), applied to the coefficient field K_lm.
//
// Per row i and term: the coefficient block C on Q_i1 x Q_i2 x Q_i3 is
// contracted with T_3 = B^(3,i3) W^(3,i3) over q3, then with T_2 over q2,
// then with T_1 over q1, giving the (#I_i1 x #I_i2 x #I_i3) row block, which
// is written to the row's CSR slot (columns in increasing order, j1 fastest).
#include <hip/hip_runtime.h>

#include "wq_internal.h"

namespace wq {
namespace {

constexpr int kThreads = 256;

__device__ inline int field_channel(int l, int m) {
  if (l == m) return 1 + l;                       // K11, K22, K33
  const int s = l + m;                            // (0,1)->K12, (0,2)->K13, (1,2)->K23
  return s == 1 ? 4 : (s == 2 ? 5 : 6);
}

template <int P, typename T>
__global__ __launch_bounds__(kThreads) void k_rows(PlanView v, int stiff, T* __restrict__ out) {
  constexpr int QC = 3 * P + 1, IC = 2 * P + 1;
  constexpr int NACC = (IC * IC * IC + kThreads - 1) / kThreads;
  extern __shared__ __align__(16) unsigned char smem[];
  T* Y = reinterpret_cast<T*>(smem);                // [QC][QC][IC]   (q1, q2, j3)
  T* Z = Y + QC * QC * IC;                          // [QC][IC][IC]   (q1, j2, j3)

  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int n1 = d1.n, n2 = d2.n;
  const int64_t row = blockIdx.x;
  const int i1 = int(row % n1), i2 = int((row / n1) % n2), i3 = int(row / (int64_t(n1) * n2));
  int qs1, qc1, qs2, qc2, qs3, qc3, is1, ic1, is2, ic2, is3, ic3;
  q_range(i1, P, d1.nel, qs1, qc1);
  q_range(i2, P, d2.nel, qs2, qc2);
  q_range(i3, P, d3.nel, qs3, qc3);
  i_range(i1, P, n1, is1, ic1);
  i_range(i2, P, n2, is2, ic2);
  i_range(i3, P, d3.n, is3, ic3);
  const int nq1 = d1.nq, nq2 = d2.nq;
  const int64_t N = v.nqtot;
  const T* field = static_cast<const T*>(v.field);
  const int tid = threadIdx.x;
  const int len = ic1 * ic2 * ic3;

  T acc[NACC];
#pragma unroll
  for (int a = 0; a < NACC; ++a) acc[a] = T(0);

  const int nterms = stiff ? 9 : 1;
  for (int term = 0; term < nterms; ++term) {
    int ch, pr1, pr2, pr3;
    if (stiff) {
      const int l = term / 3, m = term % 3;
      ch = field_channel(l, m);
      pr1 = 2 * (l == 0) + (m == 0);               // pair = 2*beta + alpha
      pr2 = 2 * (l == 1) + (m == 1);
      pr3 = 2 * (l == 2) + (m == 2);
    } else {
      ch = 0;
      pr1 = pr2 = pr3 = 0;
    }
    const T* F = field + ch * N;
    const T* T1 = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)d1.op64 : (const void*)d1.op32) +
                  (size_t(pr1) * n1 + i1) * IC * QC;
    const T* T2 = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)d2.op64 : (const void*)d2.op32) +
                  (size_t(pr2) * n2 + i2) * IC * QC;
    const T* T3 = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)d3.op64 : (const void*)d3.op32) +
                  (size_t(pr3) * d3.n + i3) * IC * QC;
    // stage 1: Y[a][b][c] = sum_z T3[c][z] F[qs1+a, qs2+b, qs3+z]
    for (int idx = tid; idx < qc1 * qc2 * ic3; idx += kThreads) {
      const int a = idx % qc1, b = (idx / qc1) % qc2, c = idx / (qc1 * qc2);
      const T* f = F + (qs1 + a) + int64_t(nq1) * ((qs2 + b) + int64_t(nq2) * qs3);
      T s = T(0);
      for (int z = 0; z < qc3; ++z) s += T3[c * QC + z] * f[int64_t(z) * nq1 * nq2];
      Y[(a * QC + b) * IC + c] = s;
    }
    __syncthreads();
    // stage 2: Z[a][j2][c] = sum_b T2[j2][b] Y[a][b][c]
    for (int idx = tid; idx < qc1 * ic2 * ic3; idx += kThreads) {
      const int a = idx % qc1, j2 = (idx / qc1) % ic2, c = idx / (qc1 * ic2);
      T s = T(0);
      for (int b = 0; b < qc2; ++b) s += T2[j2 * QC + b] * Y[(a * QC + b) * IC + c];
      Z[(a * IC + j2) * IC + c] = s;
    }
    __syncthreads();
    // stage 3: acc[t] += sum_a T1[j1][a] Z[a][j2][j3], t = j1 + ic1 (j2 + ic2 j3)
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
      const int t = tid + k * kThreads;
      if (t < len) {
        const int j1 = t % ic1, j2 = (t / ic1) % ic2, j3 = t / (ic1 * ic2);
        T s = T(0);
        for (int a = 0; a < qc1; ++a) s += T1[j1 * QC + a] * Z[(a * IC + j2) * IC + j3];
        acc[k] += s;
      }
    }
    __syncthreads();
  }
  // row start (closed form of the pattern prefix)
  const int64_t Tn1 = d1.prefix[n1], Tn2 = d2.prefix[n2];
  const int64_t start = d3.prefix[i3] * Tn2 * Tn1 + int64_t(ic3) * (d2.prefix[i2] * Tn1 + int64_t(ic2) * d1.prefix[i1]);
#pragma unroll
  for (int k = 0; k < NACC; ++k) {
    const int t = tid + k * kThreads;
    if (t < len) out[start + t] = acc[k];
  }
}

template <int P, typename T>
hipError_t rows_p(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s) {
  constexpr int QC = 3 * P + 1, IC = 2 * P + 1;
  const size_t lds = size_t(QC * QC * IC + QC * IC * IC) * sizeof(T);
  const int64_t nrows = int64_t(v.dir[0].n) * v.dir[1].n * v.dir[2].n;
  if (which & WQ_MASS) {
    hipLaunchKernelGGL((k_rows<P, T>), dim3(unsigned(nrows)), dim3(kThreads), lds, s, v, 0, static_cast<T*>(mass));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (which & WQ_STIFF) {
    hipLaunchKernelGGL((k_rows<P, T>), dim3(unsigned(nrows)), dim3(kThreads), lds, s, v, 1, static_cast<T*>(stiff));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int P>
hipError_t assemble_p(const PlanView& v, int which, void* mass, void* stiff, hipStream_t s) {
  return v.prec == WQ_FP64 ? rows_p<P, double>(v, which, mass, stiff, s) : rows_p<P, float>(v, which, mass, stiff, s);
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
