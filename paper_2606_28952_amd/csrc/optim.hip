// Limited-memory BFGS for the variational outer loop (host code).
//
// Search directions come from the two-loop recursion over the last `history`
// curvature pairs with the initial inverse Hessian scaled by s'y / y'y; the
// step satisfies the strong Wolfe conditions (c1 = 1e-4, c2 = 0.9), found by
// bracketing and safeguarded cubic interpolation (Nocedal and Wright,
// Numerical Optimization, Algorithms 3.5, 3.6 and 7.4).  The paper's VQE runs
// use L-BFGS with a More-Thuente line search; this bracketing search meets
// the same conditions.  Near a minimum the decrease c1 a g'd falls below the
// rounding noise of f, so the sufficient-decrease test allows f to exceed
// its bound by f_noise * max(|f|, 1) (an approximate Wolfe condition in the
// sense of Hager and Zhang); the curvature condition is kept exact.  The run
// stops when the largest gradient component is at most g_tol, when (f_tol >
// 0) an accepted step lowers f by no more than f_tol * max(|f|, |f_new|, 1),
// or after max_iter iterations.
#include <algorithm>
#include <cmath>
#include <deque>
#include <vector>

#include "pbs_internal.h"

namespace pbs {

namespace {

constexpr double kC1 = 1e-4, kC2 = 0.9;
constexpr int kMaxLineEvals = 30;

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

double inf_norm(const std::vector<double>& a) {
  double m = 0.0;
  for (double v : a) m = std::max(m, std::fabs(v));
  return m;
}

// Minimiser of the cubic through (a, fa, da) and (b, fb, db), kept inside
// the middle 80% of the interval; bisection when the cubic has no minimum.
double cubic_step(double a, double fa, double da, double b, double fb, double db) {
  const double lo = std::min(a, b), hi = std::max(a, b), w = hi - lo;
  const double d1 = da + db - 3.0 * (fa - fb) / (a - b);
  const double disc = d1 * d1 - da * db;
  double t = 0.5 * (a + b);
  if (disc >= 0.0) {
    const double d2 = std::copysign(std::sqrt(disc), b - a);
    const double den = db - da + 2.0 * d2;
    if (den != 0.0) {
      const double c = b - (b - a) * (db + d2 - d1) / den;
      if (std::isfinite(c)) t = c;
    }
  }
  return std::clamp(t, lo + 0.1 * w, hi - 0.1 * w);
}

struct Point {
  double a = 0.0, f = 0.0, d = 0.0;  // step, value, directional derivative
  std::vector<double> x, g;
};

}  // namespace

LbfgsResult lbfgs_minimize(uint32_t n, double* x0, const Objective& fg, uint32_t max_iter, uint32_t history,
                           double g_tol, double f_tol, double f_noise) {
  LbfgsResult res;
  std::vector<double> x(x0, x0 + n), g(n), d(n), q(n);
  double f = 0.0;
  fg(x.data(), &f, g.data());
  res.evals = 1;
  std::deque<std::vector<double>> S, Y;
  std::deque<double> rho;
  auto eval_at = [&](double a, Point& p) {
    p.a = a;
    p.x.resize(n);
    p.g.resize(n);
    for (uint32_t i = 0; i < n; ++i) p.x[i] = x[i] + a * d[i];
    fg(p.x.data(), &p.f, p.g.data());
    ++res.evals;
    p.d = dot(p.g, d);
  };
  res.reason = kStopIterations;
  if (inf_norm(g) <= g_tol) res.reason = kStopGradient;
  bool reset = false;
  while (res.reason == kStopIterations && res.iters < max_iter) {
    // direction: two-loop recursion
    q = g;
    std::vector<double> alpha(S.size());
    for (size_t k = S.size(); k-- > 0;) {
      alpha[k] = rho[k] * dot(S[k], q);
      for (uint32_t i = 0; i < n; ++i) q[i] -= alpha[k] * Y[k][i];
    }
    const double gamma = S.empty() ? 1.0 : dot(S.back(), Y.back()) / dot(Y.back(), Y.back());
    for (uint32_t i = 0; i < n; ++i) q[i] *= gamma;
    for (size_t k = 0; k < S.size(); ++k) {
      const double beta = rho[k] * dot(Y[k], q);
      for (uint32_t i = 0; i < n; ++i) q[i] += (alpha[k] - beta) * S[k][i];
    }
    for (uint32_t i = 0; i < n; ++i) d[i] = -q[i];
    double d0 = dot(g, d);
    if (!(d0 < 0.0)) {  // not a descent direction: restart from steepest descent
      S.clear();
      Y.clear();
      rho.clear();
      for (uint32_t i = 0; i < n; ++i) d[i] = -g[i];
      d0 = dot(g, d);
    }
    const double a0 = S.empty() ? std::min(1.0, 1.0 / std::sqrt(dot(g, g))) : 1.0;
    const double slack = f_noise * std::max(std::fabs(f), 1.0);
    auto too_high = [&](const Point& p) { return !std::isfinite(p.f) || p.f > f + kC1 * p.a * d0 + slack; };
    // strong Wolfe line search
    Point prev;
    prev.a = 0.0;
    prev.f = f;
    prev.d = d0;
    Point cur, acc;
    bool found = false, have_lo = false;
    Point lo, hi;
    double a = a0;
    int evals = 0;
    for (; evals < kMaxLineEvals && !found; ++evals) {
      eval_at(a, cur);
      if (too_high(cur) || (cur.a > a0 && cur.f >= prev.f)) {
        lo = prev;
        hi = cur;
        have_lo = true;
        break;
      }
      if (std::fabs(cur.d) <= -kC2 * d0) {
        acc = cur;
        found = true;
        break;
      }
      if (cur.d >= 0.0) {
        lo = cur;
        hi = prev;
        have_lo = true;
        break;
      }
      prev = cur;
      a *= 2.0;
    }
    if (!found && have_lo) {
      // zoom: lo satisfies sufficient decrease and has the lowest value so far
      for (++evals; evals < kMaxLineEvals; ++evals) {
        const double aj = std::isfinite(hi.f) ? cubic_step(lo.a, lo.f, lo.d, hi.a, hi.f, hi.d) : 0.5 * (lo.a + hi.a);
        Point pj;
        eval_at(aj, pj);
        if (too_high(pj) || pj.f >= lo.f) {
          hi = pj;
        } else {
          if (std::fabs(pj.d) <= -kC2 * d0) {
            acc = pj;
            found = true;
            break;
          }
          if (pj.d * (hi.a - lo.a) >= 0.0) hi = lo;
          lo = pj;
        }
        if (std::fabs(hi.a - lo.a) <= 1e-14 * std::max(1.0, lo.a)) break;
      }
      if (!found && lo.a > 0.0 && lo.f < f) {  // a decrease without the curvature condition: still a step
        acc = lo;
        found = true;
      }
    }
    if (!found) {
      if (!S.empty() && !reset) {  // retry once from steepest descent
        S.clear();
        Y.clear();
        rho.clear();
        reset = true;
        continue;
      }
      res.reason = kStopLineSearch;
      break;
    }
    reset = false;
    ++res.iters;
    std::vector<double> s(n), y(n);
    for (uint32_t i = 0; i < n; ++i) {
      s[i] = acc.x[i] - x[i];
      y[i] = acc.g[i] - g[i];
    }
    const double sy = dot(s, y);
    if (sy > 1e-12 * std::sqrt(dot(s, s) * dot(y, y))) {
      S.push_back(std::move(s));
      Y.push_back(std::move(y));
      rho.push_back(1.0 / sy);
      if (S.size() > history) {
        S.pop_front();
        Y.pop_front();
        rho.pop_front();
      }
    }
    const double f_old = f;
    x = acc.x;
    g = acc.g;
    f = acc.f;
    if (inf_norm(g) <= g_tol)
      res.reason = kStopGradient;
    else if (f_tol > 0.0 && f_old - f >= 0.0 && f_old - f <= f_tol * std::max({std::fabs(f_old), std::fabs(f), 1.0}))
      res.reason = kStopDecrease;
  }
  std::copy(x.begin(), x.end(), x0);
  res.f = f;
  res.g_inf = inf_norm(g);
  return res;
}

}  // namespace pbs

extern "C" pbs_status pbs_lbfgs_minimize(uint32_t n, double* x, pbs_objective fn, void* user, uint32_t max_iter,
                                         uint32_t history, double g_tol, double f_tol, double* f_out,
                                         uint32_t* iters, uint32_t* evals, int32_t* reason) {
  return pbs::guarded([&] {
    PBS_REQUIRE(n >= 1 && x != nullptr && fn != nullptr, PBS_ERR_ARG, "null argument or empty problem");
    PBS_REQUIRE(history >= 1 && history <= 64, PBS_ERR_RANGE, "history must be in 1..64");
    const pbs::Objective fg = [&](const double* xx, double* f, double* g) {
      PBS_REQUIRE(fn(user, n, xx, f, g) == 0, PBS_ERR_ARG, "objective reported failure");
    };
    const pbs::LbfgsResult r = pbs::lbfgs_minimize(n, x, fg, max_iter, history, g_tol, f_tol, 1e-13);
    if (f_out) *f_out = r.f;
    if (iters) *iters = r.iters;
    if (evals) *evals = r.evals;
    if (reason) *reason = r.reason;
  });
}
