// Double-double arithmetic (value = hi + lo, |lo| <= ulp(hi)/2) for the fold.
//
// The unpivoted cluster elimination of Algorithm 1 forms Schur complements
// whose entries mix large (1/sigma_min of a nearly singular block) and O(1)
// parts; carrying the fold in double-double keeps the O(1) parts exact to
// FP64 level.  Built from the classic error-free transformations:
//   two_sum (Knuth): s + e == a + b exactly,
//   two_prod via fused multiply-add: p + e == a * b exactly.
// Every function body turns floating-point contraction off: hipcc contracts by
// default, and fusing the product a * b of two_prod into the sum that follows
// (s = p + e becomes fma(a, b, e)) counts the product's rounding error twice,
// leaving the result only about as accurate as plain FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace hsc {

struct dd {
  double hi, lo;
};

struct zdd {   // complex double-double, 32 bytes
  dd re, im;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return dd{s, e};
}

__device__ __forceinline__ dd quick_two_sum(double a, double b) {   // |a| >= |b|
#pragma clang fp contract(off)
  const double s = a + b;
  return dd{s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  return dd{p, fma(a, b, -p)};
}

// sum with error bounded by ~2^-104 (|x| + |y|) (the "sloppy" double-double add):
// absolute accuracy relative to the operands, which is what the fold needs.
__device__ __forceinline__ dd dd_add(dd x, dd y) {
#pragma clang fp contract(off)
  dd s = two_sum(x.hi, y.hi);
  s.lo += x.lo + y.lo;
  return quick_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_neg(dd x) { return dd{-x.hi, -x.lo}; }
__device__ __forceinline__ dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }

__device__ __forceinline__ dd dd_mul(dd x, dd y) {
#pragma clang fp contract(off)
  dd p = two_prod(x.hi, y.hi);
  p.lo = fma(x.hi, y.lo, p.lo);
  p.lo = fma(x.lo, y.hi, p.lo);
  return quick_two_sum(p.hi, p.lo);
}

__device__ __forceinline__ dd dd_from(double a) { return dd{a, 0.0}; }

// x / y: two Newton corrections of the FP64 quotient
__device__ __forceinline__ dd dd_div(dd x, dd y) {
#pragma clang fp contract(off)
  const double q1 = x.hi / y.hi;
  dd r = dd_sub(x, dd_mul(dd_from(q1), y));
  const double q2 = r.hi / y.hi;
  r = dd_sub(r, dd_mul(dd_from(q2), y));
  const double q3 = r.hi / y.hi;
  dd q = quick_two_sum(q1, q2);
  return dd_add(q, dd_from(q3));
}

__device__ __forceinline__ zdd zdd_from(double2 v) { return zdd{dd{v.x, 0.0}, dd{v.y, 0.0}}; }
__device__ __forceinline__ double2 zdd_round(zdd v) { return make_double2(v.re.hi + v.re.lo, v.im.hi + v.im.lo); }
__device__ __forceinline__ zdd zdd_zero() { return zdd{dd{0.0, 0.0}, dd{0.0, 0.0}}; }
__device__ __forceinline__ zdd zdd_add(zdd a, zdd b) { return zdd{dd_add(a.re, b.re), dd_add(a.im, b.im)}; }
__device__ __forceinline__ zdd zdd_sub(zdd a, zdd b) { return zdd{dd_sub(a.re, b.re), dd_sub(a.im, b.im)}; }
__device__ __forceinline__ zdd zdd_neg(zdd a) { return zdd{dd_neg(a.re), dd_neg(a.im)}; }

__device__ __forceinline__ zdd zdd_mul(zdd a, zdd b) {
  return zdd{dd_sub(dd_mul(a.re, b.re), dd_mul(a.im, b.im)), dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
}

// acc + a * b
__device__ __forceinline__ zdd zdd_fma(zdd acc, zdd a, zdd b) { return zdd_add(acc, zdd_mul(a, b)); }

// 1 / a = conj(a) / |a|^2, with the larger component scaled out
__device__ __forceinline__ zdd zdd_rcp(zdd a) {
  const double s = fmax(fabs(a.re.hi), fabs(a.im.hi));
  if (s == 0.0) return zdd_zero();
  const dd inv_s = dd_from(1.0 / s);   // exact only up to rounding; it cancels below
  const dd ar = dd_mul(a.re, inv_s), ai = dd_mul(a.im, inv_s);
  const dd den = dd_add(dd_mul(ar, ar), dd_mul(ai, ai));   // |a/s|^2
  const dd qr = dd_div(ar, den), qi = dd_div(dd_neg(ai), den);
  return zdd{dd_mul(qr, inv_s), dd_mul(qi, inv_s)};
}

// Lazy accumulation of a sum of double-double products (the GEMM inner loop): hi
// holds the running FP64 sum, lo collects the exact rounding errors of the hi
// additions (two_sum) and the products' low parts in plain FP64.  renorm() folds
// lo back into hi; called every few terms it keeps the result double-double
// accurate while each product-accumulate costs 12 FP64 operations instead of 18.
struct ddacc {
  double hi, lo;
};

struct zddacc {
  ddacc re, im;
};

__device__ __forceinline__ void ddacc_add_prod(ddacc& a, dd x, dd y) {
#pragma clang fp contract(off)
  const double ph = x.hi * y.hi;
  double pl = fma(x.hi, y.hi, -ph);
  pl = fma(x.hi, y.lo, pl);
  pl = fma(x.lo, y.hi, pl);
  const double s = a.hi + ph;
  const double bb = s - a.hi;
  const double e = (a.hi - (s - bb)) + (ph - bb);
  a.hi = s;
  a.lo += e + pl;
}

__device__ __forceinline__ void ddacc_renorm(ddacc& a) {
  const dd s = two_sum(a.hi, a.lo);
  a.hi = s.hi;
  a.lo = s.lo;
}

// c += a * b
__device__ __forceinline__ void zddacc_fma(zddacc& c, zdd a, zdd b) {
  ddacc_add_prod(c.re, a.re, b.re);
  ddacc_add_prod(c.re, dd_neg(a.im), b.im);
  ddacc_add_prod(c.im, a.re, b.im);
  ddacc_add_prod(c.im, a.im, b.re);
}

__device__ __forceinline__ void zddacc_renorm(zddacc& c) {
  ddacc_renorm(c.re);
  ddacc_renorm(c.im);
}

__device__ __forceinline__ zdd zddacc_value(zddacc c) { return zdd{two_sum(c.re.hi, c.re.lo), two_sum(c.im.hi, c.im.lo)}; }

__device__ __forceinline__ double zdd_cabs1(zdd a) { return fabs(a.re.hi) + fabs(a.im.hi); }

}  // namespace hsc
