// Correctly rounded summation of float64 values (host and device).
//
// The canonical reduction of Section 2.3 merges the coefficients of equal
// (X, Z) keys.  Each merged coefficient here is the exact sum of its
// contributions rounded once to nearest-even, so the result does not depend
// on the order in which contributions arrive (threads, sort order, loop
// order of Algorithm 1).
//
// Method (Shewchuk, "Adaptive Precision Floating-Point Arithmetic and Fast
// Robust Geometric Predicates", 1997): the running sum is a nonoverlapping
// expansion -- components of increasing magnitude whose exact sum is the
// exact running total -- updated with GROW-EXPANSION (a chain of TWO-SUM
// error-free additions) and zero elimination.  To round it once, components
// are added from the largest down while the additions stay exact; the first
// inexact addition gives a rounded value hi and its error lo, and the
// remaining smaller components can only matter when lo is exactly half an
// ulp of hi, in which case their sign (that of the largest remaining one)
// decides whether the true sum lies beyond the half-way point.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define PBS_HD __host__ __device__
#else
#define PBS_HD
#endif

namespace pbs {

constexpr int kExpansionMax = 40;

struct ExactAcc {
  double c[kExpansionMax];
  int n;
  int overflow;  // set when more than kExpansionMax components were needed
};

// Knuth's TWO-SUM: s = fl(a + b) and e = (a + b) - s exactly, any magnitudes.
PBS_HD inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bv = s - a;
  double av = s - bv;
  e = (a - av) + (b - bv);
}

PBS_HD inline void acc_init(ExactAcc& A) {
  A.n = 0;
  A.overflow = 0;
}

// GROW-EXPANSION with zero elimination.
PBS_HD inline void acc_add(ExactAcc& A, double v) {
  double q = v;
  int m = 0;
  for (int i = 0; i < A.n; ++i) {
    double s, e;
    two_sum(q, A.c[i], s, e);
    if (e != 0.0) A.c[m++] = e;
    q = s;
  }
  if (q != 0.0) {
    if (m < kExpansionMax) {
      A.c[m++] = q;
    } else {
      A.overflow = 1;
    }
  }
  A.n = m;
}

// The expansion's exact value rounded to nearest-even; an exact zero is +0.0.
PBS_HD inline double acc_round(const ExactAcc& A) {
  int i = A.n;
  if (i == 0) return 0.0;
  double hi = A.c[--i];
  double lo = 0.0;
  while (i > 0) {
    double x = hi;
    double y = A.c[--i];
    hi = x + y;
    double y_taken = hi - x;
    lo = y - y_taken;
    if (lo != 0.0) break;
  }
  if (i > 0 && ((lo < 0.0 && A.c[i - 1] < 0.0) || (lo > 0.0 && A.c[i - 1] > 0.0))) {
    double y = lo * 2.0;
    double x = hi + y;
    double y_taken = x - hi;
    if (y == y_taken) hi = x;
  }
  return hi + 0.0;
}

}  // namespace pbs
