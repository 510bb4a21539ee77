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
__device__ inline dd dd_wave_sum(dd x) {
#pragma clang fp contract(off)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    dd y{__shfl_xor(x.hi, off, 64), __shfl_xor(x.lo, off, 64)};
    x = x + y;
  }
  return x;
}

}  // namespace wq
