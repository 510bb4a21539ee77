// Double-double ("dd") arithmetic for the univariate weight builder.
//
// A dd value is an unevaluated sum hi + lo with |lo| <= ulp(hi)/2, giving
// about 106 significant bits.  Error-free transformations: TwoSum (Knuth),
// FastTwoSum (Dekker, |a| >= |b|), TwoProd via fused multiply-add.  The
// add/mul/div/sqrt compositions follow the standard double-double algorithms
// of the QD library (Hida, Li and Bailey, 2001).  Floating-point contraction
// is switched off inside every routine: fusing a product into a following
// addition (e.g. hi + lo with hi = a*b into fma(a, b, lo)) would break the
// error-free transformations.
#pragma once

#include <hip/hip_runtime.h>

namespace wq {

struct dd {
  double hi, lo;
};

// ---------------------------------------------------------------------------
// Wavefront (64-lane) reductions through DPP lane moves (register to
// register, no LDS round trip).  Steps: pairs and quads within a row of 16
// (quad_perm), half-rows (row_half_mirror), rows (row_mirror), then rows 0+1
// into row 1 and 2+3 into row 3 (row_bcast:15), and rows 0..1 into rows 2..3
// (row_bcast:31); lane 63 ends with the total, read back as a uniform value.
// Lanes of rows that a step leaves out receive 0.
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ inline double lane_f64(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(int(b), lane);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

template <typename Op>
__device__ inline double wave_reduce(double x, Op op) {
  x = op(x, dpp_f64<0xB1, 0xF>(x));    // quad_perm [1,0,3,2]
  x = op(x, dpp_f64<0x4E, 0xF>(x));    // quad_perm [2,3,0,1]
  x = op(x, dpp_f64<0x141, 0xF>(x));   // row_half_mirror
  x = op(x, dpp_f64<0x140, 0xF>(x));   // row_mirror
  x = op(x, dpp_f64<0x142, 0xA>(x));   // row_bcast:15 -> rows 1, 3
  x = op(x, dpp_f64<0x143, 0xC>(x));   // row_bcast:31 -> rows 2, 3
  return lane_f64(x, 63);
}

__device__ inline dd dd_from(double a) { return dd{a, 0.0}; }

__device__ inline dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return dd{s, e};
}

__device__ inline dd fast_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  return dd{s, b - (s - a)};
}

__device__ inline dd two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return dd{p, fma(a, b, -p)};
}

__device__ inline dd operator+(dd x, dd y) {
#pragma clang fp contract(off)
  dd s = two_sum(x.hi, y.hi);
  const dd t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

__device__ inline dd operator-(dd x) { return dd{-x.hi, -x.lo}; }
__device__ inline dd operator-(dd x, dd y) { return x + (-y); }

__device__ inline dd operator+(dd x, double b) {
#pragma clang fp contract(off)
  dd s = two_sum(x.hi, b);
  s.lo += x.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ inline dd operator+(double b, dd x) { return x + b; }
__device__ inline dd operator-(dd x, double b) { return x + (-b); }
__device__ inline dd operator-(double b, dd x) { return (-x) + b; }

__device__ inline dd operator*(dd x, dd y) {
#pragma clang fp contract(off)
  dd p = two_prod(x.hi, y.hi);
  p.lo += x.hi * y.lo + x.lo * y.hi;
  return fast_two_sum(p.hi, p.lo);
}

__device__ inline dd operator*(dd x, double b) {
#pragma clang fp contract(off)
  dd p = two_prod(x.hi, b);
  p.lo += x.lo * b;
  return fast_two_sum(p.hi, p.lo);
}
__device__ inline dd operator*(double b, dd x) { return x * b; }

__device__ inline dd operator/(dd x, dd y) {
#pragma clang fp contract(off)
  const double q1 = x.hi / y.hi;
  dd r = x - y * q1;
  const double q2 = r.hi / y.hi;
  r = r - y * q2;
  const double q3 = r.hi / y.hi;
  return fast_two_sum(q1, q2) + q3;
}

__device__ inline dd operator/(dd x, double b) { return x / dd_from(b); }
__device__ inline dd operator/(double a, dd y) { return dd_from(a) / y; }

__device__ inline dd& operator+=(dd& x, dd y) { return x = x + y; }
__device__ inline dd& operator-=(dd& x, dd y) { return x = x - y; }

__device__ inline dd dd_sqrt(dd a) {
#pragma clang fp contract(off)
  if (a.hi <= 0.0) return dd{0.0, 0.0};
  const double x = sqrt(a.hi);
  // one Newton step: x + (a - x^2) / (2x)
  const dd r = a - two_prod(x, x);
  return fast_two_sum(x, r.hi / (2.0 * x));
}

__device__ inline double dd_to_double(dd a) { return a.hi + a.lo; }

// Wavefront-wide sums (64 lanes) by butterfly exchange.
// Sum over the wavefront in double-double (same DPP steps as wave_reduce).
__device__ inline dd dd_wave_sum(dd x) {
#pragma clang fp contract(off)
  x = x + dd{dpp_f64<0xB1, 0xF>(x.hi), dpp_f64<0xB1, 0xF>(x.lo)};
  x = x + dd{dpp_f64<0x4E, 0xF>(x.hi), dpp_f64<0x4E, 0xF>(x.lo)};
  x = x + dd{dpp_f64<0x141, 0xF>(x.hi), dpp_f64<0x141, 0xF>(x.lo)};
  x = x + dd{dpp_f64<0x140, 0xF>(x.hi), dpp_f64<0x140, 0xF>(x.lo)};
  x = x + dd{dpp_f64<0x142, 0xA>(x.hi), dpp_f64<0x142, 0xA>(x.lo)};
  x = x + dd{dpp_f64<0x143, 0xC>(x.hi), dpp_f64<0x143, 0xC>(x.lo)};
  return dd{lane_f64(x.hi, 63), lane_f64(x.lo, 63)};
}

}  // namespace wq
