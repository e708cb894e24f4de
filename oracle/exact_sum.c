/*
 * Correctly rounded FP64 sums for the CPU oracle (test infrastructure).
 *
 * Summation keeps a list of non-overlapping partial sums that together
 * equal the exact sum of the terms seen so far (Shewchuk, "Adaptive
 * Precision Floating-Point Arithmetic and Fast Robust Geometric
 * Predicates", 1997: each new term is added to every partial with an
 * error-free two-sum, and the nonzero round-off parts are kept). The final
 * rounding is not in Shewchuk's paper: it is the step of R. Hettinger's
 * "msum" recipe (Python Cookbook recipe 393090, the method behind Python's
 * math.fsum), restated here. The partials are added from the largest down
 * until a nonzero round-off appears, and a result that lies exactly half
 * way between two FP64 numbers is moved to the correct one by the sign of
 * the next partial, which gives the FP64 number nearest the exact sum.
 *
 * A dot product adds the exact products: fma(a, b, -p) recovers the
 * round-off e of p = a * b exactly, so p + e == a * b.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define MAXP 2112 /* non-overlapping partials never exceed the 2098 bit positions of FP64 */

typedef struct {
  double p[MAXP];
  int n;
} acc_t;

static void acc_init(acc_t* a) { a->n = 0; }

static void acc_add(acc_t* a, double x) {
  int i = 0;
  for (int j = 0; j < a->n; ++j) {
    double y = a->p[j];
    if (fabs(x) < fabs(y)) {
      double t = x;
      x = y;
      y = t;
    }
    double hi = x + y;
    double lo = y - (hi - x);
    if (lo != 0.0) a->p[i++] = lo;
    x = hi;
  }
  a->p[i++] = x;
  a->n = i;
}

static double acc_round(const acc_t* a) {
  int n = a->n;
  double hi = 0.0, lo = 0.0;
  if (n > 0) {
    hi = a->p[--n];
    while (n > 0) {
      double x = hi;
      double y = a->p[--n];
      hi = x + y;
      double yr = hi - x;
      lo = y - yr;
      if (lo != 0.0) break;
    }
    if (n > 0 && ((lo < 0.0 && a->p[n - 1] < 0.0) || (lo > 0.0 && a->p[n - 1] > 0.0))) {
      double y = lo * 2.0;
      double x = hi + y;
      double yr = x - hi;
      if (y == yr) hi = x;
    }
  }
  return hi;
}

double exact_sum(int64_t n, const double* v) {
  acc_t a;
  acc_init(&a);
  for (int64_t i = 0; i < n; ++i) acc_add(&a, v[i]);
  return acc_round(&a);
}

double exact_dot(int64_t n, const double* x, const double* y) {
  acc_t a;
  acc_init(&a);
  for (int64_t i = 0; i < n; ++i) {
    const double p = x[i] * y[i];
    const double e = fma(x[i], y[i], -p);
    acc_add(&a, p);
    if (e != 0.0) acc_add(&a, e);
  }
  return acc_round(&a);
}

/* out[i] = correctly rounded sum over row i of val[k] * x[col[k]] */
void exact_spmv(int64_t m, const int64_t* row_ptr, const int64_t* col, const double* val,
                const double* x, double* out) {
  for (int64_t i = 0; i < m; ++i) {
    acc_t a;
    acc_init(&a);
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const double xv = x[col[k]];
      const double p = val[k] * xv;
      const double e = fma(val[k], xv, -p);
      acc_add(&a, p);
      if (e != 0.0) acc_add(&a, e);
    }
    out[i] = acc_round(&a);
  }
}

/* out[i] = correctly rounded sum over row i of v[k] */
void exact_row_sums(int64_t m, const int64_t* row_ptr, const double* v, double* out) {
  for (int64_t i = 0; i < m; ++i) {
    acc_t a;
    acc_init(&a);
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) acc_add(&a, v[k]);
    out[i] = acc_round(&a);
  }
}
