// Double-double arithmetic: a value is the unevaluated sum hi + lo of two doubles with
// |lo| <= ulp(hi) / 2, about 106 significant bits.  Error-free sum after Knuth (TwoSum)
// and Dekker (Fast2Sum, for |a| >= |b|); error-free product from the fused multiply-add
// (the rounding error of a*b is fma(a, b, -a*b) exactly).  Every function turns off
// floating-point contraction: a multiply fused into a later add would change the
// rounding the error terms are computed for.
#pragma once

#include <hip/hip_runtime.h>

namespace cutcell {

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd dd_from(double a) { return dd{a, 0.0}; }

__device__ __forceinline__ dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return dd{s, e};
}

__device__ __forceinline__ dd fast_two_sum(double a, double b) {   // |a| >= |b| (or a = 0)
#pragma clang fp contract(off)
  const double s = a + b;
  return dd{s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return dd{p, __builtin_fma(a, b, -p)};
}

__device__ __forceinline__ dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }

// a + b, with the low parts summed error-free as well (relative error ~ 2^-104)
__device__ __forceinline__ dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
  dd s = two_sum(a.hi, b.hi);
  const dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

// a * b (the product of the low parts, below 2^-106 relative, is dropped)
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
  dd p = two_prod(a.hi, b.hi);
  const double c = __builtin_fma(a.hi, b.lo, a.lo * b.hi);
  p.lo += c;
  return fast_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
#pragma clang fp contract(off)
  dd p = two_prod(a.hi, b);
  p.lo = __builtin_fma(a.lo, b, p.lo);
  return fast_two_sum(p.hi, p.lo);
}

// a / b by long division: three quotient digits, each from the remainder of the last
__device__ __forceinline__ dd dd_div(dd a, dd b) {
#pragma clang fp contract(off)
  const double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul_d(b, q1));
  const double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul_d(b, q2));
  const double q3 = r.hi / b.hi;
  return dd_add(fast_two_sum(q1, q2), dd_from(q3));
}

__device__ __forceinline__ bool dd_isfinite(dd a) { return isfinite(a.hi) && isfinite(a.lo); }

}  // namespace cutcell
