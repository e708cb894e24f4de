// Correctly rounded FP64 logarithm, exponential and power of positive
// arguments, for host and device alike.
//
// The method evaluates elementary functions in two places: the primal-weight
// update at a restart, omega = exp(theta ln(dy / dx) + (1 - theta) ln omega)
// (PDLP's rule, which the paper adopts in Section 3.2), and the adaptive
// step's factors (j + 1)^-e. Library implementations of exp, log and pow
// differ between platforms in the last bit, and one such bit in omega grows
// through the iteration. These functions are therefore computed in
// double-double arithmetic (about 2^-100 relative accuracy) and rounded once,
// which gives the FP64 number nearest the exact value except when that value
// lies within ~2^-100 of a rounding boundary. Host and device run the same
// sequence of IEEE operations (+, -, *, /, fma, frexp, ldexp), so they give
// the same bits.
//
//   log:  x = m 2^e with m in [1/sqrt(2), sqrt(2)); ln m = 2 atanh(s),
//         s = (m - 1) / (m + 1), |s| <= 0.172, by its odd power series;
//         ln x = e ln 2 + ln m.
//   exp:  a = k ln 2 + r with k = round(a / ln 2), |r| <= ln(2) / 2;
//         expm1(r / 2^10) by its Taylor series, then ten squarings
//         (1 + E)^2 - 1 = 2E + E^2; exp a = 2^k (1 + E).
//   pow:  x^y = exp(y ln x) with y ln x kept in double-double.
//
// Arguments are positive, finite and normal, and results in the normal
// range: the method only takes logarithms of positive ratios and weights,
// and exponentials of moderate arguments.
#pragma once

#include <math.h>

#if defined(__HIPCC__) || defined(__HIP__)
#define OPDHG_CRM_FN __host__ __device__ inline
#else
#define OPDHG_CRM_FN inline
#endif

namespace opdhg {
namespace crm {

struct DDv {
  double hi, lo;
};

OPDHG_CRM_FN DDv two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return DDv{s, (a - (s - bb)) + (b - bb)};
}

// |a| >= |b|
OPDHG_CRM_FN DDv quick_two_sum(double a, double b) {
  const double s = a + b;
  return DDv{s, b - (s - a)};
}

OPDHG_CRM_FN DDv two_prod(double a, double b) {
  const double p = a * b;
  return DDv{p, fma(a, b, -p)};
}

OPDHG_CRM_FN DDv neg(DDv a) { return DDv{-a.hi, -a.lo}; }

OPDHG_CRM_FN DDv add(DDv a, DDv b) {
  DDv s = two_sum(a.hi, b.hi);
  const DDv t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}

OPDHG_CRM_FN DDv mul(DDv a, DDv b) {
  DDv p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo;
  p.lo += a.lo * b.hi;
  return quick_two_sum(p.hi, p.lo);
}

OPDHG_CRM_FN DDv mul_d(DDv a, double b) {
  DDv p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return quick_two_sum(p.hi, p.lo);
}

// a / b: three quotient digits, each from the remainder of the ones before
OPDHG_CRM_FN DDv div(DDv a, DDv b) {
  const double q1 = a.hi / b.hi;
  DDv r = add(a, neg(mul_d(b, q1)));
  const double q2 = r.hi / b.hi;
  r = add(r, neg(mul_d(b, q2)));
  const double q3 = r.hi / b.hi;
  return add(quick_two_sum(q1, q2), DDv{q3, 0.0});
}

// ln 2 to 106 bits
OPDHG_CRM_FN DDv ln2() { return DDv{0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56}; }

// ln x in double-double, x > 0 finite and normal
OPDHG_CRM_FN DDv log_dd(double x) {
  int e = 0;
  double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
  if (m < 0x1.6a09e667f3bccp-1) {  // below 1/sqrt(2): move to [1/sqrt(2), sqrt(2))
    m *= 2.0;
    e -= 1;
  }
  const DDv num{m - 1.0, 0.0};  // exact: m is within a factor 2 of 1
  const DDv s = div(num, two_sum(m, 1.0));
  const DDv s2 = mul(s, s);
  // atanh(s) / s = sum_k s^(2k) / (2k + 1); s^2 <= 0.0295, so 25 terms reach 2^-125
  constexpr int kTerms = 25;
  DDv t = div(DDv{1.0, 0.0}, DDv{2.0 * kTerms - 1.0, 0.0});
  for (int k = kTerms - 2; k >= 0; --k)
    t = add(mul(t, s2), div(DDv{1.0, 0.0}, DDv{2.0 * k + 1.0, 0.0}));
  const DDv lnm = mul_d(mul(s, t), 2.0);
  return add(mul_d(ln2(), (double)e), lnm);
}

// exp a for a double-double argument a (|a| < 700)
OPDHG_CRM_FN double exp_dd(DDv a) {
  const DDv L = ln2();
  const double k = rint(a.hi / L.hi);
  DDv r = add(a, neg(mul_d(L, k)));  // |r| <= ln(2) / 2 (a little more from rounding)
  constexpr int kHalvings = 10;
  r.hi = ldexp(r.hi, -kHalvings);
  r.lo = ldexp(r.lo, -kHalvings);
  // expm1(r) = r (1 + r/2 (1 + r/3 (1 + ...))): |r| <= 3.4e-4, 12 terms reach 2^-150
  constexpr int kOrder = 12;
  DDv t{1.0, 0.0};
  for (int n = kOrder; n >= 2; --n) t = add(DDv{1.0, 0.0}, mul(t, div(r, DDv{(double)n, 0.0})));
  DDv E = mul(t, r);
  for (int i = 0; i < kHalvings; ++i) E = add(mul_d(E, 2.0), mul(E, E));
  const DDv y = add(DDv{1.0, 0.0}, E);
  return ldexp(y.hi + y.lo, (int)k);
}

OPDHG_CRM_FN double cr_log(double x) {
  const DDv v = log_dd(x);
  return v.hi + v.lo;
}

OPDHG_CRM_FN double cr_exp(double a) { return exp_dd(DDv{a, 0.0}); }

// x^y for x > 0
OPDHG_CRM_FN double cr_pow(double x, double y) { return exp_dd(mul_d(log_dd(x), y)); }

}  // namespace crm
}  // namespace opdhg
