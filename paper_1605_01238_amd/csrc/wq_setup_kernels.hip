// Setup kernels: quadrature points and B-spline tables (Algorithm 1), the
// univariate weighted-quadrature rules (Algorithm 2), the geometry/coefficient
// field (Section 3, eqs. mass2 and coef_stiff), and the CSR pattern
// (Section 3, sets I_i).
#include <hip/hip_runtime.h>

#include <cmath>

#include "wq_dd.h"
#include "wq_internal.h"

namespace wq {
namespace {

// Values N[r] and first derivatives D[r] at x of the degree-P B-splines
// s-P+r, r = 0..P, nonzero on the knot span [U[s], U[s+1]) (Cox-de Boor
// triangular recursion; derivatives from the degree P-1 values).  R is
// double or dd.
// Knot difference a - b: exact in double-double, rounded in FP64.
template <typename R> __device__ inline R knot_diff(double a, double b);
template <> __device__ inline double knot_diff<double>(double a, double b) { return a - b; }
template <> __device__ inline dd knot_diff<dd>(double a, double b) { return two_sum(a, -b); }

template <int P, typename R>
__device__ inline void basis_funs(const double* __restrict__ U, int s, R x, R (&N)[P + 1], R (&D)[P + 1]) {
  R left[P + 1], right[P + 1], Nm[P + 1];
  N[0] = R{1.0};
#pragma unroll
  for (int j = 1; j <= P; ++j) {
    left[j] = x - U[s + 1 - j];
    right[j] = U[s + j] - x;
    if (j == P) {
#pragma unroll
      for (int r = 0; r < P; ++r) Nm[r] = N[r];
    }
    R saved{0.0};
#pragma unroll
    for (int r = 0; r < j; ++r) {
      const R temp = N[r] / (right[r + 1] + left[j - r]);
      N[r] = saved + right[r + 1] * temp;
      saved = left[j - r] * temp;
    }
    N[j] = saved;
  }
#pragma unroll
  for (int r = 0; r <= P; ++r) {
    const int i = s - P + r;
    R d{0.0};
    if (r >= 1) d = d + (Nm[r - 1] * double(P)) / knot_diff<R>(U[i + P], U[i]);
    if (r <= P - 1) d = d - (Nm[r] * double(P)) / knot_diff<R>(U[i + P + 1], U[i + 1]);
    D[r] = d;
  }
}

// Quadrature point q of a direction (layout of Remark 4.1, see
// wq_internal.h) in double-double, and the span e holding it (interior
// knots are assigned to the span on their right).
__device__ inline dd qp_coord(const double* __restrict__ k, int P, int nel, int q, int& e) {
  if (q <= P) {
    e = 0;
    const dd h = two_sum(k[P + 1], -k[P]);
    return (h * double(q + 1)) / double(P + 2) + k[P];
  }
  if (q >= P + 2 * nel - 2) {
    e = nel - 1;
    const int t = q - (P + 2 * nel - 2);
    const dd h = two_sum(k[P + nel], -k[P + nel - 1]);
    return (h * double(t + 1)) / double(P + 2) + k[P + nel - 1];
  }
  const int m = q - P;
  if (m & 1) {
    e = (m + 1) / 2;
    return dd_from(k[P + e]);
  }
  e = m / 2;
  const dd s = two_sum(k[P + e], k[P + e + 1]);
  return dd{0.5 * s.hi, 0.5 * s.lo};
}

__device__ inline double wave_max(double x) {
  return wave_reduce(x, [](double a, double b) { return fmax(a, b); });
}

__device__ inline double wave_sum(double x) {
  return wave_reduce(x, [](double a, double b) { return a + b; });
}

// ---------------------------------------------------------------------------
// Quadrature points and the p+1 nonzero B-spline values/derivatives there
// (FP64 tables for the geometry stage).  The tables are evaluated at the
// point in double-double and then rounded, so that they belong to the same
// point as the rules: a boundary point a + h (q+1)/(p+2) is not an FP64
// number in general, and at |x| >> h its FP64 rounding moves it by a
// fraction eps |x| / h of the span.
template <int P>
__global__ __launch_bounds__(256) void k_points(PlanView v) {
  const int dir = blockIdx.y;
  const DirView d = v.dir[dir];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= d.nq) return;
  int e;
  const dd xd = qp_coord(d.knots, P, d.nel, q, e);
  dd Nx[P + 1], Dx[P + 1], Nmx[P], Dmx[P];
  basis_funs<P, dd>(d.knots, e + P, xd, Nx, Dx);
  basis_funs<P - 1, dd>(d.knots, e + P, xd, Nmx, Dmx);   // degree p-1, functions e+1 .. e+p
  double N[P + 1], D[P + 1], Nm[P];
#pragma unroll
  for (int r = 0; r <= P; ++r) {
    N[r] = Nx[r].hi;
    D[r] = Dx[r].hi;
  }
#pragma unroll
  for (int r = 0; r < P; ++r) Nm[r] = Nmx[r].hi;
  d.x[q] = xd.hi;
  d.qspan[q] = e;
#pragma unroll
  for (int r = 0; r <= P; ++r) {
    d.bv[q * (P + 1) + r] = N[r];
    d.bd[q * (P + 1) + r] = D[r];
  }
  // column table of q: the basis part here, the weights by the rule solves
  // (entries of rows without x_q strictly inside their support stay 0)
  constexpr int NCT = 6 * (P + 1);
#pragma unroll
  for (int k = 0; k < 4 * (P + 1); ++k) {
    d.colt64[q * NCT + k] = 0.0;
    d.colt32[q * NCT + k] = 0.0f;
  }
#pragma unroll
  for (int r = 0; r <= P; ++r) {
    d.colt64[q * NCT + 4 * (P + 1) + r] = N[r];
    d.colt64[q * NCT + 5 * (P + 1) + r] = D[r];
    d.colt32[q * NCT + 4 * (P + 1) + r] = float(N[r]);
    d.colt32[q * NCT + 5 * (P + 1) + r] = float(D[r]);
  }
  // derivative of a spline: sum_i C_i B_i' = sum_i (C_i - C_{i-1}) P N_{i,P-1} / (xi_{i+P} - xi_i)
#pragma unroll
  for (int r = 0; r < P; ++r) {
    const int i = e + 1 + r;
    d.bw[q * P + r] = P * Nm[r] / (d.knots[i + P] - d.knots[i]);
  }
}

// Differenced control net along each direction b: C_i - C_{i - e_b} (exact
// inputs, so each difference is correctly rounded); zero where i_b = 0.
__global__ __launch_bounds__(256) void k_ctrl_diff(PlanView v, const double* __restrict__ src) {
  const int n1 = v.dir[0].n, n2 = v.dir[1].n, n3 = v.dir[2].n;
  const int64_t N = int64_t(n1) * n2 * n3;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= N * 3) return;
  const int64_t i = t / 3;
  const int a = int(t % 3);
  const int i1 = int(i % n1), i2 = int((i / n1) % n2), i3 = int(i / (int64_t(n1) * n2));
  const double c = src[t];
  v.ctrl[t] = c;   // the plan keeps its own copy of the net
  v.dctrl[0 * N * 3 + t] = i1 > 0 ? c - src[(i - 1) * 3 + a] : 0.0;
  v.dctrl[1 * N * 3 + t] = i2 > 0 ? c - src[(i - n1) * 3 + a] : 0.0;
  v.dctrl[2 * N * 3 + t] = i3 > 0 ? c - src[(i - int64_t(n1) * n2) * 3 + a] : 0.0;
}

// ---------------------------------------------------------------------------
// Univariate rules: one workgroup (4 wavefronts) per (direction, test index i).
// Wavefront w handles pairing w = 2*beta + alpha: the minimum-norm w with
//   sum_q w_q B_j^(alpha)(x_q) = int B_i^(beta) B_j^(alpha),  j in I_i, q in Q_i
// (Algorithm 2).  For alpha = 1 the last equation is dropped: the equations
// sum to zero because the B-splines overlapping B_i sum to one on its
// support, and the remaining ones have full rank.
//
// Precision: the systems are ill-conditioned (condition numbers up to ~1e8
// at p = 6), so their data -- points, B-spline values, Gauss nodes/weights
// and integrals -- are formed in double-double.  The minimum-norm problem is
// the KKT system  w - A^T lam = 0,  A w = b;  it is solved with a Householder
// QR of A^T (lane = quadrature point = row of A^T) in FP64 and refined
// with residuals evaluated in double-double (at least once, at most three
// times, until a step no longer matters), which yields the weights to FP64
// rounding.
// KKT steps of the minimum-norm solve at most (the first is the plain solve).
#ifndef WQ_KKT_ITERS
#define WQ_KKT_ITERS 4
#endif

template <int P>
__global__ __launch_bounds__(256) void k_rules(PlanView v) {
  constexpr int QC = 3 * P + 1, IC = 2 * P + 1, NG = P + 1, MAXG = (P + 1) * NG;
  static_assert(QC <= 64, "one wavefront per system");
  const int dir = blockIdx.y;
  const DirView d = v.dir[dir];
  const int i = blockIdx.x;
  if (i >= d.n) return;   // uniform per block
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = d.n, nel = d.nel;
  int qs, qc, is, ic;
  q_range(i, P, nel, qs, qc);
  i_range(i, P, n, is, ic);

  __shared__ dd gx[NG], gw[NG];
  __shared__ dd gval[MAXG][P + 1], gder[MAXG][P + 1], gwt[MAXG];
  __shared__ int gspan[MAXG];
  __shared__ dd A[2][IC][QC];
  __shared__ dd bvec[4][IC];
  __shared__ double Rl[4][IC][IC];

  // A^(alpha)[jj][qq] = B^(alpha)_{is+jj}(x_{qs+qq}) in double-double
  // (wave 0), while wave 1 forms the Gauss-Legendre rule.
  for (int idx = tid; idx < 2 * IC * QC; idx += 256) (&A[0][0][0])[idx] = dd{0.0, 0.0};
  __syncthreads();
  for (int qq = tid; qq < qc; qq += 256) {
    int e;
    const dd x = qp_coord(d.knots, P, nel, qs + qq, e);
    dd N[P + 1], D[P + 1];
    basis_funs<P, dd>(d.knots, e + P, x, N, D);
#pragma unroll
    for (int r = 0; r <= P; ++r) {
      const int jj = e + r - is;
      if (jj >= 0 && jj < ic) {
        A[0][jj][qq] = N[r];
        A[1][jj][qq] = D[r];
      }
    }
  }
  // Wave 1 forms the Gauss-Legendre rule and the B-splines at the Gauss
  // points of the knot-spans supporting B_i, while wave 0 builds A.
  // Nodes/weights on [-1, 1]: Newton's method on the Legendre polynomial
  // P_NG, in FP64 to convergence, then in double-double.
  const int e0 = i - P > 0 ? i - P : 0;
  const int e1 = i + 1 < nel ? i + 1 : nel;
  const int ng = (e1 - e0) * NG;
  if (wave == 1) {
    if (lane < NG) {
      const int t = lane;
      double z = cos(M_PI * (t + 0.75) / (NG + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= NG; ++k) {
          const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        const double dz = p1 / (NG * (z * p1 - p0) / (z * z - 1.0));
        z -= dz;
        if (fabs(dz) <= 1e-15) break;
      }
      dd zz = dd_from(z), dp{0.0, 0.0};
      for (int it = 0; it < 3; ++it) {
        dd p0 = dd_from(1.0), p1 = zz;
        for (int k = 2; k <= NG; ++k) {
          const dd p2 = ((zz * p1) * double(2 * k - 1) - p0 * double(k - 1)) / double(k);
          p0 = p1;
          p1 = p2;
        }
        dp = ((zz * p1 - p0) * double(NG)) / (zz * zz - 1.0);
        if (it < 2) zz = zz - p1 / dp;
      }
      gx[t] = zz;
      gw[t] = 2.0 / ((1.0 - zz * zz) * (dp * dp));
    }
    // the nodes were written by other lanes of this wavefront
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int g = lane; g < ng; g += 64) {
      const int e = e0 + g / NG, t = g % NG;
      const double a = d.knots[e + P], b = d.knots[e + P + 1];
      const dd half = two_sum(b, -a) * 0.5;
      const dd xg = two_sum(a, b) * 0.5 + half * gx[t];
      dd N[P + 1], D[P + 1];
      basis_funs<P, dd>(d.knots, e + P, xg, N, D);
#pragma unroll
      for (int r = 0; r <= P; ++r) {
        gval[g][r] = N[r];
        gder[g][r] = D[r];
      }
      gwt[g] = half * gw[t];
      gspan[g] = e;
    }
  }
  __syncthreads();
  // Exact 1D integrals (degree <= 2p per span, p+1 Gauss points), in dd:
  // one partial sum per (pairing, jj, span), then the sum over the spans.
  __shared__ dd part[4][IC][P + 1];
  for (int idx = tid; idx < 4 * IC * (P + 1); idx += 256) {
    const int sp = idx % (P + 1), jj = (idx / (P + 1)) % IC, pair = idx / ((P + 1) * IC);
    const int al = pair & 1, be = pair >> 1;
    dd s{0.0, 0.0};
    if (jj < ic && sp < e1 - e0) {
      const int j = is + jj, e = e0 + sp, ri = i - e, rj = j - e;
      if (ri >= 0 && ri <= P && rj >= 0 && rj <= P) {
#pragma unroll
        for (int t = 0; t < NG; ++t) {
          const int g = sp * NG + t;
          s += gwt[g] * (be ? gder[g][ri] : gval[g][ri]) * (al ? gder[g][rj] : gval[g][rj]);
        }
      }
    }
    part[pair][jj][sp] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < 4 * IC; idx += 256) {
    const int pair = idx / IC, jj = idx % IC;
    dd s{0.0, 0.0};
#pragma unroll
    for (int sp = 0; sp <= P; ++sp) s += part[pair][jj][sp];
    bvec[pair][jj] = s;
  }
  __syncthreads();

  // ---- minimum-norm solve, one wavefront per pairing ----
  const int pair = wave, al = pair & 1;
  const int r = ic - al;
  const bool live = lane < qc;
  double m[IC], vk[IC], vn[IC];
#pragma unroll
  for (int j = 0; j < IC; ++j) {
    m[j] = (live && j < r) ? A[al][j][lane].hi : 0.0;
    vk[j] = 0.0;
    vn[j] = 1.0;
  }
  bool broke = false;
#pragma unroll
  for (int k = 0; k < IC; ++k) {
    if (k < r) {
      const double xk = (lane >= k) ? m[k] : 0.0;
      const double nrm2 = wave_sum(xk * xk);
      const double akk = lane_f64(m[k], k);
      if (nrm2 > 0.0) {
        const double nrm = sqrt(nrm2);
        const double alpha = akk >= 0.0 ? -nrm : nrm;
        const double vv = (lane == k) ? akk - alpha : xk;
        const double vnorm2 = 2.0 * (nrm2 + fabs(akk) * nrm);
        vk[k] = vv;
        vn[k] = vnorm2;
        // columns j >= r are zero and stay zero
        double sj[IC];
#pragma unroll
        for (int j = k; j < IC; ++j) sj[j] = wave_sum(vv * m[j]);
#pragma unroll
        for (int j = k; j < IC; ++j) m[j] -= (2.0 * sj[j] / vnorm2) * vv;
      } else {
        broke = true;
      }
    }
  }
  if (lane < r) {
#pragma unroll
    for (int j = 0; j < IC; ++j) Rl[pair][lane][j] = m[j];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < IC; ++k)
    if (k < r && Rl[pair][k][k] == 0.0) broke = true;

  // KKT iterations from (w, lam) = 0; the first one is the plain solve.
  dd w{0.0, 0.0};
  dd lam[IC];
#pragma unroll
  for (int j = 0; j < IC; ++j) lam[j] = dd{0.0, 0.0};
  for (int it = 0; it < WQ_KKT_ITERS && !broke; ++it) {
    // r2 = b - A w (kept equations), r1 = A^T lam - w (this lane)
    double r2[IC];
    dd r1 = -w;
    if (it == 0) {   // from (w, lam) = 0 the residuals are b and 0
#pragma unroll
      for (int j = 0; j < IC; ++j) r2[j] = dd_to_double(bvec[pair][j]);
    } else {
      // all IC rows (zero beyond #I_i; a dropped row is computed and unused,
      // its multiplier stays 0), so the IC reductions are independent
#pragma unroll
      for (int j = 0; j < IC; ++j) {
        const dd a = live ? A[al][j][lane] : dd{0.0, 0.0};
        const dd s = dd_wave_sum(a * w);
        r2[j] = dd_to_double(bvec[pair][j] - s);
        r1 += a * lam[j];
      }
    }
    // t = (Q^T r1)[0:r]: apply H_0 .. H_{r-1}
    double u = live ? dd_to_double(r1) : 0.0;
#pragma unroll
    for (int k = 0; k < IC; ++k)
      if (k < r) u -= (2.0 * wave_sum(vk[k] * u) / vn[k]) * vk[k];
    // z = R^{-T} r2 (forward substitution); s = z - t
    double z[IC], sv[IC];
#pragma unroll
    for (int k = 0; k < IC; ++k) {
      z[k] = 0.0;
      sv[k] = 0.0;
      if (k < r) {
        double acc = r2[k];
#pragma unroll
        for (int mm = 0; mm < k; ++mm) acc -= Rl[pair][mm][k] * z[mm];
        z[k] = acc / Rl[pair][k][k];
        sv[k] = z[k] - lane_f64(u, k);
      }
    }
    // dlam = R^{-1} s (back substitution)
    double dl[IC];
#pragma unroll
    for (int k = IC - 1; k >= 0; --k) {
      dl[k] = 0.0;
      if (k < r) {
        double z = sv[k];
#pragma unroll
        for (int mm = k + 1; mm < IC; ++mm)
          if (mm < r) z -= Rl[pair][k][mm] * dl[mm];
        dl[k] = z / Rl[pair][k][k];
      }
    }
    // dw = r1 + Q [s; 0]: apply H_{r-1} .. H_0
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < IC; ++k)
      if (lane == k && k < r) g = sv[k];
#pragma unroll
    for (int k = IC - 1; k >= 0; --k)
      if (k < r) g -= (2.0 * wave_sum(vk[k] * g) / vn[k]) * vk[k];
    if (live) w = (w + r1) + g;
#pragma unroll
    for (int j = 0; j < IC; ++j)
      if (j < r) lam[j] = lam[j] + dl[j];
    // A refinement step that moved w by less than 2^-30 |w| has brought the
    // error below 2^-30 of its previous size (error ~ (kappa u)^k): the next
    // one could not change the FP64 weights.
    if (it >= 1) {
      const double upd = wave_max(live ? fabs(dd_to_double(r1) + g) : 0.0);
      const double wmax = wave_max(live ? fabs(w.hi) : 0.0);
      if (upd <= 0x1p-30 * wmax) break;
    }
  }
  const double wq = live ? dd_to_double(w) : 0.0;
  // residual of all ic equations (including a dropped one); rows beyond
  // #I_i are zero on both sides.  An FP64 sum with a bound on its rounding
  // error settles the check when the bound allows (products and the a.lo
  // terms: 2u each, the 6-level reduction: 6u, of the sum of magnitudes,
  // doubled); otherwise it is decided in double-double.
  double bmax = 0.0;
#pragma unroll
  for (int j = 0; j < IC; ++j) bmax = fmax(bmax, fabs(bvec[pair][j].hi));
  const double tol = 1e-9 * bmax + 1e-300;
  bool certain = true;
#pragma unroll
  for (int j = 0; j < IC; ++j) {
    const double ah = live ? A[al][j][lane].hi : 0.0;
    const double s = wave_sum(ah * wq);
    const double m = wave_sum(fabs(ah * wq));
    const double err = 16.0 * 0x1p-53 * m + fabs(bvec[pair][j].lo);
    if (!(fabs(s - bvec[pair][j].hi) + err <= tol)) certain = false;
  }
  double rmax = 0.0;
  if (!certain) {
#pragma unroll
    for (int j = 0; j < IC; ++j) {
      const dd a = live ? A[al][j][lane] : dd{0.0, 0.0};
      const dd s = dd_wave_sum(a * wq);
      rmax = fmax(rmax, fabs(dd_to_double(s - bvec[pair][j])));
    }
  }
  if (!(rmax <= tol) || broke) {
    if (lane == 0) {
      atomicAdd(&v.flags[FLAG_SOLVE_BAD], 1);
      atomicMin(&v.flags[FLAG_SOLVE_FIRST], (dir * 4 + pair) * n + i);
    }
  }
  // outputs (lane = local quadrature point qq; zero beyond #Q_i and #I_i)
  if (lane < qc) {   // row i is slot i - e of the column table of its point
    const int q = qs + lane, sl = i - d.qspan[q];
    d.colt64[q * (6 * (P + 1)) + sl * 4 + pair] = wq;
    d.colt32[q * (6 * (P + 1)) + sl * 4 + pair] = float(wq);
  }
  if (lane < QC) {
    d.w[(size_t(pair) * n + i) * QC + lane] = wq;
    const size_t pq = size_t(i) * QC + lane;
    d.wt64[pq * 4 + pair] = wq;
    d.wt32[pq * 4 + pair] = float(wq);
#pragma unroll
    for (int jj = 0; jj < IC; ++jj) {
      const double b = dd_to_double(A[al][jj][lane]);
      const double t = b * wq;
      d.op64[(pq * IC + jj) * 4 + pair] = t;
      d.op32[(pq * IC + jj) * 4 + pair] = float(t);
      if (pair < 2) {   // the B^(alpha) tables, alpha = pair
        d.bt64[(pq * IC + jj) * 2 + pair] = b;
        d.bt32[(pq * IC + jj) * 2 + pair] = float(b);
        if (pair == 0) {
          d.b0t64[pq * IC + jj] = b;
          d.b0t32[pq * IC + jj] = float(b);
        }
      }
    }
  }
}

// Prefix sums of the 1D row lengths #I_i (one thread per direction).
__global__ void k_prefix(PlanView v) {
  const int dir = threadIdx.x;
  if (dir >= 3) return;
  const DirView d = v.dir[dir];
  int64_t s = 0;
  d.prefix[0] = 0;
  for (int i = 0; i < d.n; ++i) {
    int is, ic;
    i_range(i, v.p, d.n, is, ic);
    s += ic;
    d.prefix[i + 1] = s;
  }
}

// Coefficient field of a request: the plan's field for a = 1 (det J and
// K = det J J^{-1} J^{-T}) with K multiplied by the diffusion coefficient
// a(x_q) (eq. coef_stiff times a); det J (eq. mass2) is copied.
template <typename T>
__global__ __launch_bounds__(256) void k_scale_field(const T* __restrict__ in, const double* __restrict__ a,
                                                     T* __restrict__ out, int64_t n) {
  const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (q >= n) return;
  const double aq = a ? a[q] : 1.0;
  out[q] = in[q];
#pragma unroll
  for (int c = 1; c < kNumChannels; ++c) out[c * n + q] = T(double(in[c * n + q]) * aq);
}

// Q_i = [q_start[i], q_start[i] + q_count[i]) of one direction (either
// output may be null).
__global__ void k_qranges(PlanView v, int dir, int32_t* __restrict__ q_start, int32_t* __restrict__ q_count) {
  const DirView d = v.dir[dir];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  int qs, qc;
  q_range(i, v.p, d.nel, qs, qc);
  if (q_start) q_start[i] = qs;
  if (q_count) q_count[i] = qc;
}

// ---------------------------------------------------------------------------
// Physical coordinates F = sum_i C_i B_i at every quadrature point (used to
// sample a coefficient given as a function of x).
template <int P>
__global__ __launch_bounds__(256) void k_xphys(PlanView v, double* __restrict__ xphys) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= v.nqtot) return;
  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int q1 = int(q % d1.nq);
  const int q2 = int((q / d1.nq) % d2.nq);
  const int q3 = int(q / (int64_t(d1.nq) * d2.nq));
  const int e1 = d1.qspan[q1], e2 = d2.qspan[q2], e3 = d3.qspan[q3];
  double v1[P + 1];
#pragma unroll
  for (int r = 0; r <= P; ++r) v1[r] = d1.bv[q1 * (P + 1) + r];
  const double* bv2 = d2.bv + q2 * (P + 1);
  const double* bv3 = d3.bv + q3 * (P + 1);
  const int n1 = d1.n, n2 = d2.n;
  double F[3] = {0, 0, 0};
#pragma unroll 1
  for (int l3 = 0; l3 <= P; ++l3) {
    double f2[3] = {0, 0, 0};
#pragma unroll 1
    for (int l2 = 0; l2 <= P; ++l2) {
      const double* c = v.ctrl + ((size_t(e3 + l3) * n2 + (e2 + l2)) * n1 + e1) * 3;
      double f1[3] = {0, 0, 0};
#pragma unroll
      for (int l1 = 0; l1 <= P; ++l1)
#pragma unroll
        for (int a = 0; a < 3; ++a) f1[a] += c[l1 * 3 + a] * v1[l1];
      const double b2 = bv2[l2];
#pragma unroll
      for (int a = 0; a < 3; ++a) f2[a] += f1[a] * b2;
    }
    const double b3 = bv3[l3];
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] += f2[a] * b3;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) xphys[q * 3 + a] = F[a];
}

// t / d for 0 <= t < 2^20, d >= 1: a float estimate within one of the
// quotient, then one correction
__device__ inline int div_small(int t, int d, float inv) {
  const int q = int(float(t) * inv);
  const int r = t - q * d;
  return r < 0 ? q - 1 : (r >= d ? q + 1 : q);
}

// ---------------------------------------------------------------------------
// CSR pattern: LW lanes per row (a wavefront for the long rows of a solid
// patch, a quarter of one for the short rows of a plane patch or curve).
// A row's columns are (j3, j2, j1) lexicographic.  Lanes write 16-byte
// groups of 4 consecutive entries (the first group starts at the first
// 16-byte boundary of the row; the few entries before it and after the last
// full group are written singly).
template <int LW>
__global__ __launch_bounds__(256) void k_pattern(PlanView v, int64_t* __restrict__ row_ptr,
                                                 int32_t* __restrict__ col_idx) {
  const int lane = threadIdx.x % LW;
  // with one row per wavefront the row and everything derived from it are uniform
  const int64_t row = int64_t(blockIdx.x) * (256 / LW) +
                      (LW == 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x / LW) : int(threadIdx.x / LW));
  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int n1 = d1.n, n2 = d2.n, n3 = d3.n;
  const int64_t nrows = int64_t(n1) * n2 * n3;
  if (row >= nrows) return;
  const int i1 = int(row % n1), i2 = int((row / n1) % n2), i3 = int(row / (int64_t(n1) * n2));
  int is1, ic1, is2, ic2, is3, ic3;
  i_range(i1, v.p, n1, is1, ic1);
  i_range(i2, v.p, n2, is2, ic2);
  i_range(i3, v.p, n3, is3, ic3);
  const int64_t T1 = d1.prefix[n1], T2 = d2.prefix[n2];
  const int64_t start = d3.prefix[i3] * T2 * T1 + int64_t(ic3) * (d2.prefix[i2] * T1 + int64_t(ic2) * d1.prefix[i1]);
  const int plane = ic1 * ic2, len = plane * ic3;
  if (lane == 0) {
    row_ptr[row] = start;
    if (row == nrows - 1) row_ptr[nrows] = start + len;
  }
  const int n12 = n1 * n2;
  const int base = is1 + n1 * is2 + n12 * is3;
  const float invp = 1.0f / float(plane), inv1 = 1.0f / float(ic1);
  // entry t of the row -> (jj3, jj2, jj1), t < (2p+1)^3
  auto split = [&](int t, int& jj3, int& jj2, int& jj1) {
    jj3 = div_small(t, plane, invp);
    const int r = t - jj3 * plane;
    jj2 = div_small(r, ic1, inv1);
    jj1 = r - jj2 * ic1;
  };
  auto col_of = [&](int t) {
    int jj3, jj2, jj1;
    split(t, jj3, jj2, jj1);
    return base + jj1 + n1 * jj2 + n12 * jj3;
  };
  const int head = min(len, int((4 - (start & 3)) & 3));   // entries before the first boundary
  const int ngroups = (len - head) >> 2;
  if (lane < head) col_idx[start + lane] = col_of(lane);
  const int tail0 = head + 4 * ngroups;
  if (lane < len - tail0) col_idx[start + tail0 + lane] = col_of(tail0 + lane);
  // 16-byte groups: lane takes groups lane, lane+LW, ...; its position moves
  // by 4 LW entries per step, (s3, s2, s1) in the row's mixed radix
  constexpr int STEP = 4 * LW;
  const int s3 = STEP / plane, s2 = (STEP - s3 * plane) / ic1, s1 = STEP - s3 * plane - s2 * ic1;
  int jj3, jj2, jj1;
  split(head + 4 * lane, jj3, jj2, jj1);
  int4* __restrict__ o = reinterpret_cast<int4*>(col_idx + start + head);
  for (int g = lane; g < ngroups; g += LW) {
    int c[4];
    int a1 = jj1, a2 = jj2, a3 = jj3;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      c[k] = base + a1 + n1 * a2 + n12 * a3;
      if (++a1 == ic1) {
        a1 = 0;
        if (++a2 == ic2) {
          a2 = 0;
          ++a3;
        }
      }
    }
    o[g] = int4{c[0], c[1], c[2], c[3]};
    jj1 += s1;
    if (jj1 >= ic1) {
      jj1 -= ic1;
      ++jj2;
    }
    jj2 += s2;
    if (jj2 >= ic2) {
      jj2 -= ic2;
      ++jj3;
    }
    jj3 += s3;
  }
}

// ---------------------------------------------------------------------------
// Geometry by sum factorization, one direction at a time (three passes over
// small intermediates instead of (p+1)^3 control points per quadrature
// point).  With D_b the control net differenced along b and the weights
// g_b(i) = p N_{i,p-1} / (xi_{i+p} - xi_i), the Jacobian columns are
//   J_:,1 = sum_i D_1[i] g_1(i1) B_2(i2) B_3(i3)
//   J_:,2 = sum_i D_2[i] B_1(i1) g_2(i2) B_3(i3)
//   J_:,3 = sum_i D_3[i] B_1(i1) B_2(i2) g_3(i3).
// Records hold the 3 nets x 3 coordinates (9 doubles).
constexpr int kGeoRec = 9;

// pass 3: X[q3][i2][i1][k, a] = sum_l3 D_k[e3 + l3][i2][i1][a] * (B_3 or g_3)
template <int P>
__global__ __launch_bounds__(256) void k_geo3(PlanView v, double* __restrict__ X) {
  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int n1 = d1.n, n2 = d2.n;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(d3.nq) * n2 * n1) return;
  const int i1 = int(t % n1), i2 = int((t / n1) % n2), q3 = int(t / (int64_t(n1) * n2));
  const int e3 = d3.qspan[q3];
  const size_t NC = size_t(n1) * n2 * d3.n * 3;
  double acc[kGeoRec];
#pragma unroll
  for (int k = 0; k < kGeoRec; ++k) acc[k] = 0.0;
#pragma unroll
  for (int l = 0; l <= P; ++l) {
    const double b = d3.bv[q3 * (P + 1) + l];
    const double g = l ? d3.bw[q3 * P + l - 1] : 0.0;
    const size_t o = ((size_t(e3 + l) * n2 + i2) * n1 + i1) * 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc[0 + a] += v.dctrl[o + a] * b;
      acc[3 + a] += v.dctrl[NC + o + a] * b;
      if (l) acc[6 + a] += v.dctrl[2 * NC + o + a] * g;
    }
  }
  double* x = X + size_t(t) * kGeoRec;
#pragma unroll
  for (int k = 0; k < kGeoRec; ++k) x[k] = acc[k];
}

// pass 2: Y[q3][q2][i1][k, a] = sum_l2 X[q3][e2 + l2][i1][k, a] * (B_2 or g_2)
template <int P>
__global__ __launch_bounds__(256) void k_geo2(PlanView v, const double* __restrict__ X, double* __restrict__ Y) {
  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int n1 = d1.n, n2 = d2.n, nq2 = d2.nq;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(d3.nq) * nq2 * n1) return;
  const int i1 = int(t % n1), q2 = int((t / n1) % nq2), q3 = int(t / (int64_t(n1) * nq2));
  const int e2 = d2.qspan[q2];
  double acc[kGeoRec];
#pragma unroll
  for (int k = 0; k < kGeoRec; ++k) acc[k] = 0.0;
#pragma unroll
  for (int l = 0; l <= P; ++l) {
    const double b = d2.bv[q2 * (P + 1) + l];
    const double g = l ? d2.bw[q2 * P + l - 1] : 0.0;
    const double* x = X + ((size_t(q3) * n2 + e2 + l) * n1 + i1) * kGeoRec;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      acc[0 + a] += x[0 + a] * b;
      if (l) acc[3 + a] += x[3 + a] * g;
      acc[6 + a] += x[6 + a] * b;
    }
  }
  double* y = Y + size_t(t) * kGeoRec;
#pragma unroll
  for (int k = 0; k < kGeoRec; ++k) y[k] = acc[k];
}

// pass 1 and the point values: J from Y, then det J and the coefficients
// (det J; K = a det J J^{-1} J^{-T} = a adj(J) adj(J)^T / det J)
template <int P, typename T>
__global__ __launch_bounds__(256) void k_geo1(PlanView v, const double* __restrict__ Y,
                                              const double* __restrict__ coef) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= v.nqtot) return;
  const DirView d1 = v.dir[0], d2 = v.dir[1];
  const int n1 = d1.n, nq1 = d1.nq;
  const int q1 = int(q % nq1);
  const int64_t line = q / nq1;   // q3 * nq2 + q2
  const int e1 = d1.qspan[q1];
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int l = 0; l <= P; ++l) {
    const double b = d1.bv[q1 * (P + 1) + l];
    const double g = l ? d1.bw[q1 * P + l - 1] : 0.0;
    const double* y = Y + (size_t(line) * n1 + e1 + l) * kGeoRec;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (l) J[a][0] += y[0 + a] * g;
      J[a][1] += y[3 + a] * b;
      J[a][2] += y[6 + a] * b;
    }
  }
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double c10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  const double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  const double c12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  const double c20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  const double c21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  const double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  if (!(det > 0.0) || !isfinite(det)) {
    atomicAdd(&v.flags[FLAG_DETJ_BAD], 1);
    atomicMin(&v.flags[FLAG_DETJ_FIRST], int(q));
  }
  const double s = (coef ? coef[q] : 1.0) / det;
  T* f = static_cast<T*>(v.field);
  const int64_t N = v.nqtot;
  f[0 * N + q] = T(det);
  f[1 * N + q] = T(s * (c00 * c00 + c10 * c10 + c20 * c20));
  f[2 * N + q] = T(s * (c01 * c01 + c11 * c11 + c21 * c21));
  f[3 * N + q] = T(s * (c02 * c02 + c12 * c12 + c22 * c22));
  f[4 * N + q] = T(s * (c00 * c01 + c10 * c11 + c20 * c21));
  f[5 * N + q] = T(s * (c00 * c02 + c10 * c12 + c20 * c22));
  f[6 * N + q] = T(s * (c01 * c02 + c11 * c12 + c21 * c22));
}

// 2D map (d = 2): F, J from the (p+1)^2 control points around each point,
// the derivative columns through differenced control points as in 3D
//   J_:,1 = sum (C_i - C_{i - e_1}) g_1(i1) B_2(i2),  J_:,2 = sum (C_i - C_{i - e_2}) B_1(i1) g_2(i2),
// then det J and K = a adj(J) adj(J)^T / det J with adj(J) = [[J11, -J01], [-J10, J00]]
// (eqs. mass2 and coef_stiff in two dimensions).  The field keeps the 3D
// channel order with K33 = K13 = K23 = 0.  With xphys, writes F instead.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_geo2d(PlanView v, const double* __restrict__ coef,
                                               double* __restrict__ xphys) {
  const int64_t qq = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (qq >= v.nqtot) return;
  const DirView d1 = v.dir[0], d2 = v.dir[1];
  const int n1 = d1.n, nq1 = d1.nq;
  const int q = int(qq), q1 = q % nq1, q2 = q / nq1;
  const int e1 = d1.qspan[q1], e2 = d2.qspan[q2];
  double b1[P + 1], b2[P + 1], g1[P + 1], g2[P + 1];
#pragma unroll
  for (int l = 0; l <= P; ++l) {
    b1[l] = d1.bv[q1 * (P + 1) + l];
    b2[l] = d2.bv[q2 * (P + 1) + l];
    g1[l] = l ? d1.bw[q1 * P + l - 1] : 0.0;
    g2[l] = l ? d2.bw[q2 * P + l - 1] : 0.0;
  }
  const double* C = v.ctrl;   // [n2][n1][2]
  double F[2] = {0.0, 0.0}, J[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
  for (int l2 = 0; l2 <= P; ++l2) {
#pragma unroll
    for (int l1 = 0; l1 <= P; ++l1) {
      const size_t o = (size_t(e2 + l2) * n1 + (e1 + l1)) * 2;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double c = C[o + a];
        F[a] += c * b1[l1] * b2[l2];
        if (l1) J[a][0] += (c - C[o - 2 + a]) * g1[l1] * b2[l2];
        if (l2) J[a][1] += (c - C[o - size_t(n1) * 2 + a]) * b1[l1] * g2[l2];
      }
    }
  }
  if (xphys) {
    xphys[size_t(q) * 2 + 0] = F[0];
    xphys[size_t(q) * 2 + 1] = F[1];
    return;
  }
  const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  if (!(det > 0.0) || !isfinite(det)) {
    atomicAdd(&v.flags[FLAG_DETJ_BAD], 1);
    atomicMin(&v.flags[FLAG_DETJ_FIRST], q);
  }
  const double s = (coef ? coef[q] : 1.0) / det;
  T* f = static_cast<T*>(v.field);
  const int64_t N = v.nqtot;
  f[0 * N + q] = T(det);
  f[1 * N + q] = T(s * (J[1][1] * J[1][1] + J[0][1] * J[0][1]));
  f[2 * N + q] = T(s * (J[1][0] * J[1][0] + J[0][0] * J[0][0]));
  f[3 * N + q] = T(0);
  f[4 * N + q] = T(-s * (J[1][1] * J[1][0] + J[0][1] * J[0][0]));
  f[5 * N + q] = T(0);
  f[6 * N + q] = T(0);
}

// 1D geometry (d = 1): F = sum_i C_i B_i, J = dF/dzeta from the differenced
// control points (as in the 2D and 3D passes), det J = J and K = a J^{-1}
// (eq. coef_stiff in one direction), stored in the 3D channel order with
// zeros in the channels of the absent directions.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_geo1d(PlanView v, const double* __restrict__ coef,
                                               double* __restrict__ xphys) {
  const int64_t qq = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (qq >= v.nqtot) return;
  const DirView d1 = v.dir[0];
  const int q = int(qq), e = d1.qspan[q];
  const double* C = v.ctrl;   // [n1]
  double F = 0.0, J = 0.0;
#pragma unroll
  for (int l = 0; l <= P; ++l) {
    F += C[e + l] * d1.bv[q * (P + 1) + l];
    if (l) J += (C[e + l] - C[e + l - 1]) * d1.bw[q * P + l - 1];
  }
  if (xphys) {
    xphys[q] = F;
    return;
  }
  if (!(J > 0.0) || !isfinite(J)) {
    atomicAdd(&v.flags[FLAG_DETJ_BAD], 1);
    atomicMin(&v.flags[FLAG_DETJ_FIRST], q);
  }
  T* f = static_cast<T*>(v.field);
  const int64_t N = v.nqtot;
  f[0 * N + q] = T(J);
  f[1 * N + q] = T((coef ? coef[q] : 1.0) / J);
#pragma unroll
  for (int c = 2; c < kNumChannels; ++c) f[c * N + q] = T(0);
}

// NURBS maps (Section 3 lets rational functions enter through the factor
// c): F = N / W with N = sum_i w_i C_i B_i and W = sum_i w_i B_i over the
// (p+1)^d functions nonzero at the point, their derivatives from the
// differenced homogeneous net (w_i C_i, w_i) as for the polynomial maps, and
// J = (dN - F dW^T) / W by the quotient rule.  The field then as for a
// polynomial map; with rational test and trial functions the mass factor is
// det J / W^2 (the values are scaled by w_i w_j after the contraction).
// One thread per point, direct sums: a set-up kernel.
template <int P, typename T, int D>
__global__ __launch_bounds__(256) void k_geo_rational(PlanView v, const double* __restrict__ coef,
                                                      double* __restrict__ xphys) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= v.nqtot) return;
  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int nq1 = d1.nq, nq2 = d2.nq, n1 = d1.n, n2 = d2.n;
  const int q1 = int(q % nq1), q2 = int((q / nq1) % nq2), q3 = int(q / (int64_t(nq1) * nq2));
  constexpr int L2 = D >= 2 ? P : 0, L3 = D == 3 ? P : 0;
  const int e1 = d1.qspan[q1], e2 = D >= 2 ? d2.qspan[q2] : 0, e3 = D == 3 ? d3.qspan[q3] : 0;
  double v1[P + 1], g1[P + 1], v2[P + 1], g2[P + 1], v3[P + 1], g3[P + 1];
#pragma unroll
  for (int l = 0; l <= P; ++l) {
    v1[l] = d1.bv[q1 * (P + 1) + l];
    g1[l] = l ? d1.bw[q1 * P + l - 1] : 0.0;
    v2[l] = D >= 2 ? d2.bv[q2 * (P + 1) + l] : 1.0;
    g2[l] = (D >= 2 && l) ? d2.bw[q2 * P + l - 1] : 0.0;
    v3[l] = D == 3 ? d3.bv[q3 * (P + 1) + l] : 1.0;
    g3[l] = (D == 3 && l) ? d3.bw[q3 * P + l - 1] : 0.0;
  }
  // homogeneous control point (w C, w) of net index idx
  auto hom = [&](int64_t idx, double (&h)[D + 1]) {
    const double w = v.wts[idx];
#pragma unroll
    for (int a = 0; a < D; ++a) h[a] = w * v.ctrl[idx * D + a];
    h[D] = w;
  };
  double Nv[D + 1] = {}, dN[D + 1][D] = {};
  for (int l3 = 0; l3 <= L3; ++l3) {
    for (int l2 = 0; l2 <= L2; ++l2) {
#pragma unroll
      for (int l1 = 0; l1 <= P; ++l1) {
        const int64_t idx = (int64_t(e3 + l3) * n2 + (e2 + l2)) * n1 + (e1 + l1);
        double h[D + 1], hm[D + 1];
        hom(idx, h);
        const double b = v1[l1] * v2[l2] * v3[l3];
#pragma unroll
        for (int a = 0; a <= D; ++a) Nv[a] += h[a] * b;
        if (l1) {
          hom(idx - 1, hm);
          const double g = g1[l1] * v2[l2] * v3[l3];
#pragma unroll
          for (int a = 0; a <= D; ++a) dN[a][0] += (h[a] - hm[a]) * g;
        }
        if (D >= 2 && l2) {
          hom(idx - n1, hm);
          const double g = v1[l1] * g2[l2] * v3[l3];
#pragma unroll
          for (int a = 0; a <= D; ++a) dN[a][D >= 2 ? 1 : 0] += (h[a] - hm[a]) * g;
        }
        if (D == 3 && l3) {
          hom(idx - int64_t(n1) * n2, hm);
          const double g = v1[l1] * v2[l2] * g3[l3];
#pragma unroll
          for (int a = 0; a <= D; ++a) dN[a][D - 1] += (h[a] - hm[a]) * g;
        }
      }
    }
  }
  const double W = Nv[D];
  double F[D], J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
#pragma unroll
  for (int a = 0; a < D; ++a) F[a] = Nv[a] / W;
  if (xphys) {
#pragma unroll
    for (int a = 0; a < D; ++a) xphys[q * D + a] = F[a];
    return;
  }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) J[a][b] = (dN[a][b] - F[a] * dN[D][b]) / W;
  // cofactors of J (the absent directions are the identity)
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double c10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  const double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  const double c12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  const double c20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  const double c21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  const double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  if (!(det > 0.0) || !(W > 0.0) || !isfinite(det)) {
    atomicAdd(&v.flags[FLAG_DETJ_BAD], 1);
    atomicMin(&v.flags[FLAG_DETJ_FIRST], int(q));
  }
  const double s = (coef ? coef[q] : 1.0) / det;
  T* f = static_cast<T*>(v.field);
  const int64_t N = v.nqtot;
  f[0 * N + q] = T(v.nurbs_basis ? det / (W * W) : det);
  f[1 * N + q] = T(s * (c00 * c00 + c10 * c10 + c20 * c20));
  f[2 * N + q] = T(D >= 2 ? s * (c01 * c01 + c11 * c11 + c21 * c21) : 0.0);
  f[3 * N + q] = T(D == 3 ? s * (c02 * c02 + c12 * c12 + c22 * c22) : 0.0);
  f[4 * N + q] = T(D >= 2 ? s * (c00 * c01 + c10 * c11 + c20 * c21) : 0.0);
  f[5 * N + q] = T(D == 3 ? s * (c00 * c02 + c10 * c12 + c20 * c22) : 0.0);
  f[6 * N + q] = T(D == 3 ? s * (c01 * c02 + c11 * c12 + c21 * c22) : 0.0);
}

// Mass of rational test/trial functions: entry (i, j) times w_i w_j.  One
// workgroup per row; the row's place and its columns in closed form (CSR
// order: j3 slowest, j1 fastest, as the pattern).
template <typename T>
__global__ __launch_bounds__(256) void k_nurbs_scale(PlanView v, T* __restrict__ vals) {
  const DirView d1 = v.dir[0], d2 = v.dir[1], d3 = v.dir[2];
  const int64_t row = blockIdx.x;
  const int n1 = d1.n, n2 = d2.n, p = v.p;
  const int i1 = int(row % n1), i2 = int((row / n1) % n2), i3 = int(row / (int64_t(n1) * n2));
  int is1, ic1, is2, ic2, is3, ic3;
  i_range(i1, p, n1, is1, ic1);
  i_range(i2, p, n2, is2, ic2);
  i_range(i3, p, d3.n, is3, ic3);
  const int64_t Tn1 = d1.prefix[n1], Tn2 = d2.prefix[n2];
  const int64_t start = d3.prefix[i3] * Tn2 * Tn1 + int64_t(ic3) * d2.prefix[i2] * Tn1 + int64_t(ic3) * ic2 * d1.prefix[i1];
  const double wi = v.wts[row];
  const int len = ic1 * ic2 * ic3;
  for (int k = threadIdx.x; k < len; k += blockDim.x) {
    const int jj1 = k % ic1, jj2 = (k / ic1) % ic2, jj3 = k / (ic1 * ic2);
    const int64_t j = (int64_t(is3 + jj3) * n2 + (is2 + jj2)) * n1 + (is1 + jj1);
    vals[start + k] = T(double(vals[start + k]) * (wi * v.wts[j]));
  }
}

template <int P>
hipError_t points_p(const PlanView& v, hipStream_t s) {
  int maxq = 0;
  for (int k = 0; k < v.d; ++k) maxq = v.dir[k].nq > maxq ? v.dir[k].nq : maxq;
  dim3 grid((maxq + 255) / 256, v.d);
  hipLaunchKernelGGL(k_points<P>, grid, dim3(256), 0, s, v);
  return hipGetLastError();
}

template <int P>
hipError_t rules_p(const PlanView& v, hipStream_t s) {
  int maxn = 0;
  for (int k = 0; k < v.d; ++k) maxn = v.dir[k].n > maxn ? v.dir[k].n : maxn;
  hipLaunchKernelGGL(k_rules<P>, dim3(maxn, v.d), dim3(256), 0, s, v);
  return hipGetLastError();
}

template <int P>
hipError_t geometry_p(const PlanView& v, const double* coef, double* xphys, hipStream_t s) {
  const unsigned blocks = unsigned((v.nqtot + 255) / 256);
  if (v.wts) {   // NURBS map
    if (v.d == 3) {
      if (v.prec == WQ_FP64) hipLaunchKernelGGL((k_geo_rational<P, double, 3>), dim3(blocks), dim3(256), 0, s, v, coef, xphys);
      else hipLaunchKernelGGL((k_geo_rational<P, float, 3>), dim3(blocks), dim3(256), 0, s, v, coef, xphys);
    } else if (v.d == 2) {
      if (v.prec == WQ_FP64) hipLaunchKernelGGL((k_geo_rational<P, double, 2>), dim3(blocks), dim3(256), 0, s, v, coef, xphys);
      else hipLaunchKernelGGL((k_geo_rational<P, float, 2>), dim3(blocks), dim3(256), 0, s, v, coef, xphys);
    } else {
      if (v.prec == WQ_FP64) hipLaunchKernelGGL((k_geo_rational<P, double, 1>), dim3(blocks), dim3(256), 0, s, v, coef, xphys);
      else hipLaunchKernelGGL((k_geo_rational<P, float, 1>), dim3(blocks), dim3(256), 0, s, v, coef, xphys);
    }
    return hipGetLastError();
  }
  if (v.d == 1) {
    if (v.prec == WQ_FP64)
      hipLaunchKernelGGL((k_geo1d<P, double>), dim3(blocks), dim3(256), 0, s, v, coef, xphys);
    else
      hipLaunchKernelGGL((k_geo1d<P, float>), dim3(blocks), dim3(256), 0, s, v, coef, xphys);
    return hipGetLastError();
  }
  if (v.d == 2) {
    if (v.prec == WQ_FP64)
      hipLaunchKernelGGL((k_geo2d<P, double>), dim3(blocks), dim3(256), 0, s, v, coef, xphys);
    else
      hipLaunchKernelGGL((k_geo2d<P, float>), dim3(blocks), dim3(256), 0, s, v, coef, xphys);
    return hipGetLastError();
  }
  if (xphys) {
    hipLaunchKernelGGL((k_xphys<P>), dim3(blocks), dim3(256), 0, s, v, xphys);
    return hipGetLastError();
  }
  // the two intermediates live in the first-contraction buffer, which is
  // rewritten by every assembly
  const DirView &d1 = v.dir[0], &d2 = v.dir[1], &d3 = v.dir[2];
  double* X = static_cast<double*>(v.ybuf);
  const int64_t nx = int64_t(d3.nq) * d2.n * d1.n, ny = int64_t(d3.nq) * d2.nq * d1.n;
  double* Y = X + nx * kGeoRec;
  hipLaunchKernelGGL((k_geo3<P>), dim3(unsigned((nx + 255) / 256)), dim3(256), 0, s, v, X);
  hipLaunchKernelGGL((k_geo2<P>), dim3(unsigned((ny + 255) / 256)), dim3(256), 0, s, v, X, Y);
  if (v.prec == WQ_FP64)
    hipLaunchKernelGGL((k_geo1<P, double>), dim3(blocks), dim3(256), 0, s, v, Y, coef);
  else
    hipLaunchKernelGGL((k_geo1<P, float>), dim3(blocks), dim3(256), 0, s, v, Y, coef);
  return hipGetLastError();
}

}  // namespace

#define WQ_DISPATCH_P(p, CALL) \
  switch (p) {                 \
    case 2: return CALL(2);    \
    case 3: return CALL(3);    \
    case 4: return CALL(4);    \
    case 5: return CALL(5);    \
    case 6: return CALL(6);    \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_points(const PlanView& v, hipStream_t s) {
#define C(P) points_p<P>(v, s)
  WQ_DISPATCH_P(v.p, C)
#undef C
}

hipError_t launch_rules(const PlanView& v, hipStream_t s) {
#define C(P) rules_p<P>(v, s)
  WQ_DISPATCH_P(v.p, C)
#undef C
}

hipError_t launch_geometry(const PlanView& v, const double* coef, double* xphys, hipStream_t s) {
#define C(P) geometry_p<P>(v, coef, xphys, s)
  WQ_DISPATCH_P(v.p, C)
#undef C
}

hipError_t launch_scale_field(const PlanView& v, const double* coef, void* field_out, hipStream_t s) {
  const unsigned blocks = unsigned((v.nqtot + 255) / 256);
  if (v.prec == WQ_FP64)
    hipLaunchKernelGGL((k_scale_field<double>), dim3(blocks), dim3(256), 0, s, static_cast<const double*>(v.field), coef,
                       static_cast<double*>(field_out), v.nqtot);
  else
    hipLaunchKernelGGL((k_scale_field<float>), dim3(blocks), dim3(256), 0, s, static_cast<const float*>(v.field), coef,
                       static_cast<float*>(field_out), v.nqtot);
  return hipGetLastError();
}

hipError_t launch_qranges(const PlanView& v, int dir, int32_t* q_start, int32_t* q_count, hipStream_t s) {
  const int n = v.dir[dir].n;
  hipLaunchKernelGGL(k_qranges, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, v, dir, q_start, q_count);
  return hipGetLastError();
}

hipError_t launch_nurbs_scale(const PlanView& v, void* vals, hipStream_t s) {
  const int64_t rows = int64_t(v.dir[0].n) * v.dir[1].n * v.dir[2].n;
  if (!v.wts || rows <= 0) return hipErrorInvalidValue;
  if (v.prec == WQ_FP64)
    hipLaunchKernelGGL(k_nurbs_scale<double>, dim3(unsigned(rows)), dim3(256), 0, s, v, static_cast<double*>(vals));
  else
    hipLaunchKernelGGL(k_nurbs_scale<float>, dim3(unsigned(rows)), dim3(256), 0, s, v, static_cast<float*>(vals));
  return hipGetLastError();
}

hipError_t launch_prefix(const PlanView& v, hipStream_t s) {
  hipLaunchKernelGGL(k_prefix, dim3(1), dim3(64), 0, s, v);
  return hipGetLastError();
}

hipError_t launch_ctrl_diff(const PlanView& v, const double* ctrl, hipStream_t s) {
  const int64_t N = int64_t(v.dir[0].n) * v.dir[1].n * v.dir[2].n * 3;
  hipLaunchKernelGGL(k_ctrl_diff, dim3(unsigned((N + 255) / 256)), dim3(256), 0, s, v, ctrl);
  return hipGetLastError();
}

hipError_t launch_pattern(const PlanView& v, int64_t* row_ptr, int32_t* col_idx, hipStream_t s) {
  const int64_t nrows = int64_t(v.dir[0].n) * v.dir[1].n * v.dir[2].n;
  if (v.d == 3)
    hipLaunchKernelGGL(k_pattern<64>, dim3(unsigned((nrows + 3) / 4)), dim3(256), 0, s, v, row_ptr, col_idx);
  else
    hipLaunchKernelGGL(k_pattern<16>, dim3(unsigned((nrows + 15) / 16)), dim3(256), 0, s, v, row_ptr, col_idx);
  return hipGetLastError();
}

}  // namespace wq
