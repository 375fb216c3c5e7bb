// Host-only part of the runtime (see validate.hpp).
#include "validate.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

namespace lkp {
namespace rt {

namespace {
thread_local std::string g_err;
}  // namespace

const char *last_error() { return g_err.c_str(); }

lkp_status fail(lkp_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

void clear_error() { g_err.clear(); }

lkp_status validate_desc(const lkp_problem_desc *d, LatticeConstants *lc, double *tau_out) {
  if (!d) return fail(LKP_ERR_ARG, "null problem description");
  if (d->lattice < 0 || d->lattice >= LKP_NUM_LATTICES)
    return fail(LKP_ERR_ARG, "unknown lattice %d", d->lattice);
  const VelTable T = velocity_table(d->lattice);
  if (d->dim != T.dim)
    return fail(LKP_ERR_LATTICE_ORDER, "lattice is %dD, problem dim is %d", T.dim, d->dim);
  if (d->order != 1 && d->order != 3 && d->order != 5 && d->order != 7)
    return fail(LKP_ERR_LATTICE_ORDER, "order must be 1, 3, 5 or 7 (got %d)", d->order);
  if (d->order > T.max_order)
    return fail(LKP_ERR_LATTICE_ORDER, "lattice supports order <= %d (got %d)", T.max_order,
                d->order);
  if (d->precision < LKP_F64 || d->precision > LKP_BF16DEV_IR)
    return fail(LKP_ERR_ARG, "unknown precision %d", d->precision);
  int64_t cells = 1;
  for (int a = 0; a < 3; ++a) {
    if (d->n[a] < 1) return fail(LKP_ERR_ARG, "n[%d] = %lld < 1", a, (long long)d->n[a]);
    if (a >= d->dim && d->n[a] != 1) return fail(LKP_ERR_ARG, "n[%d] must be 1 for dim %d", a, d->dim);
    if (d->n[a] >= (int64_t(1) << 29)) return fail(LKP_ERR_ARG, "grid too large (>= 2^29 cells)");
    cells *= d->n[a];  // both factors below 2^29: no overflow
    // each population plane must stay below 4 GiB in FP64 (32-bit byte offsets)
    if (cells >= (int64_t(1) << 29)) return fail(LKP_ERR_ARG, "grid too large (>= 2^29 cells)");
  }
  if (!lattice_constants(d->lattice, lc)) return fail(LKP_ERR_HIP, "lattice constant solve failed");
  double tau = d->tau_lb;
  if (d->knudsen > 0) {
    int64_t L = d->n[0];
    for (int a = 1; a < d->dim; ++a) L = std::min(L, d->n[a]);
    tau = 0.5 + d->knudsen * (double)L / std::sqrt((double)lc->cs2);
  }
  if (!(tau > 0.5) || !std::isfinite(tau))
    return fail(LKP_ERR_UNSTABLE, "tau_lb = %g must exceed 1/2", tau);
  const double thr = stability_threshold(d->lattice, d->order);
  if (!d->allow_unstable && tau < thr)
    return fail(LKP_ERR_UNSTABLE, "tau_lb = %g is below the stability limit %g for order %d", tau,
                thr, d->order);
  double u2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(d->drift[a])) return fail(LKP_ERR_ARG, "drift[%d] is not finite", a);
    if (a >= d->dim && d->drift[a] != 0.0)
      return fail(LKP_ERR_ARG, "drift[%d] must be 0 for dim %d", a, d->dim);
    u2 += d->drift[a] * d->drift[a];
  }
  if (!d->allow_unstable && !(u2 < (double)lc->cs2))
    return fail(LKP_ERR_UNSTABLE, "drift |u|^2 = %g must stay below c_s^2 = %g", u2, (double)lc->cs2);
  *tau_out = tau;
  return LKP_OK;
}

bool has_drift(const lkp_problem_desc *d) {
  return d->drift[0] != 0.0 || d->drift[1] != 0.0 || d->drift[2] != 0.0;
}

double contraction_bound(const VelTable &T, int dim, const double *phi, double omega,
                         const int64_t n[3]) {
  using C = std::complex<double>;
  const int Q = T.q;
  const double a = 1.0 - omega;
  double best = std::fabs(a);
  // Corner modes: e_j = +1 or -1 by the parity of v_j's components along the
  // axes where k = pi.  With A, B the sums of phi_j over e_j = +1 and -1, the
  // eigenvalues other than +-a solve
  //   lambda^2 - omega (A - B) lambda - (a^2 + omega a (A + B)) = 0.
  for (int mask = 1; mask < (1 << dim); ++mask) {
    bool exists = true;
    for (int ax = 0; ax < dim; ++ax)
      if (((mask >> ax) & 1) && n[ax] < 2) exists = false;
    if (!exists) continue;
    double A = 0.0, B = 0.0;
    for (int j = 0; j < Q; ++j) {
      int par = 0;
      for (int ax = 0; ax < dim; ++ax)
        if ((mask >> ax) & 1) par += T.v[j][ax];
      if (par & 1) B += phi[j];
      else A += phi[j];
    }
    const double b = omega * (A - B);
    const C r = std::sqrt(C(b * b + 4.0 * (a * a + omega * a * (A + B)), 0.0));
    best = std::max({best, std::abs((b + r) / 2.0), std::abs((b - r) / 2.0)});
  }
  // The longest wave along each axis: the root of
  //   f(lambda) = 1 + omega sum_j phi_j e_j / (a e_j - lambda) = 0
  // that continues lambda = 1 of the mass mode, by Newton's method from 1.
  // Where that root is not isolated (kinetic regime, where the corners and
  // |1 - omega| dominate) Newton does not settle and the axis is skipped.
  const double kPi = 3.14159265358979323846;
  for (int ax = 0; ax < dim; ++ax) {
    if (n[ax] < 2) continue;
    const double k = 2.0 * kPi / (double)n[ax];
    std::vector<C> e(Q);
    for (int j = 0; j < Q; ++j) e[j] = std::polar(1.0, -k * (double)T.v[j][ax]);
    C lam(1.0, 0.0);
    bool settled = false;
    for (int it = 0; it < 100; ++it) {
      C f(1.0, 0.0), fp(0.0, 0.0);
      for (int j = 0; j < Q; ++j) {
        const C den = a * e[j] - lam;
        const C t = omega * phi[j] * e[j] / den;
        f += t;
        fp += t / den;
      }
      const C step = f / fp;
      if (!std::isfinite(step.real()) || !std::isfinite(step.imag())) break;
      lam -= step;
      if (std::abs(step) < 1e-14) {
        settled = true;
        break;
      }
    }
    if (settled) best = std::max(best, std::abs(lam));
  }
  return best;
}

}  // namespace rt
}  // namespace lkp
