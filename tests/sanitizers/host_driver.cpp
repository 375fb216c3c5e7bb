// Host-side driver for the sanitizer build (AddressSanitizer + UBSan, plain
// host compiler, no GPU): the library's constant solves and the validation of
// problem descriptions, including malformed ones.  Exit status 0 and "OK" on
// success; any sanitizer report aborts the run.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "constants.hpp"
#include "lkp.h"
#include "validate.hpp"

using namespace lkp;

static int failures = 0;
#define EXPECT(cond)                                                     \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond);      \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

static lkp_problem_desc valid_desc(int lattice) {
  lkp_problem_desc d;
  std::memset(&d, 0, sizeof d);
  const VelTable T = velocity_table(lattice);
  d.dim = T.dim;
  d.lattice = lattice;
  for (int a = 0; a < 3; ++a) d.n[a] = a < T.dim ? 17 + 3 * a : 1;
  d.order = T.max_order;
  d.precision = LKP_F64;
  d.tau_lb = 1.3;
  return d;
}

int main() {
  // constants of every set at every order it supports
  for (int id = 0; id < LKP_NUM_LATTICES; ++id) {
    LatticeConstants lc;
    EXPECT(lattice_constants(id, &lc));
    long double sw = 0, sv2 = 0;
    for (int i = 0; i < lc.table.q; ++i) {
      sw += lc.w[i];
      long double v2 = 0;
      for (int a = 0; a < 3; ++a) v2 += (long double)lc.table.v[i][a] * lc.table.v[i][a];
      sv2 += lc.w[i] * v2;
    }
    EXPECT(std::fabs((double)(sw - 1)) < 1e-15);
    EXPECT(std::fabs((double)(sv2 - lc.table.dim * lc.cs2)) < 1e-14);
    for (int order : {1, 3, 5, 7}) {
      std::vector<long double> phi, chi;
      const bool ok = shape_coefficients(lc, order, &phi, &chi);
      EXPECT(ok == (order <= lc.table.max_order));
      if (!ok) continue;
      long double sp = 0, sc = 0;
      for (int i = 0; i < lc.table.q; ++i) {
        sp += phi[i];
        sc += chi[i];
      }
      EXPECT(std::fabs((double)(sp - 1)) < 1e-14 && std::fabs((double)(sc - 1)) < 1e-14);
    }
    EXPECT(stability_threshold(id, 1) == 0.5);
  }
  LatticeConstants bad;
  EXPECT(!lattice_constants(-1, &bad) && !lattice_constants(LKP_NUM_LATTICES, &bad));

  // validation: accepted and rejected descriptions
  LatticeConstants lc;
  double tau = 0;
  for (int id = 0; id < LKP_NUM_LATTICES; ++id) {
    lkp_problem_desc d = valid_desc(id);
    EXPECT(rt::validate_desc(&d, &lc, &tau) == LKP_OK && tau == 1.3);
    d.tau_lb = 0;
    d.knudsen = 0.1;
    EXPECT(rt::validate_desc(&d, &lc, &tau) == LKP_OK && tau > 0.5);
  }
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const double inf = std::numeric_limits<double>::infinity();
  struct Case {
    void (*mutate)(lkp_problem_desc *);
    lkp_status want;
  };
  const Case cases[] = {
      {[](lkp_problem_desc *d) { d->lattice = -1; }, LKP_ERR_ARG},
      {[](lkp_problem_desc *d) { d->lattice = 99; }, LKP_ERR_ARG},
      {[](lkp_problem_desc *d) { d->dim = 2; }, LKP_ERR_LATTICE_ORDER},
      {[](lkp_problem_desc *d) { d->order = 4; }, LKP_ERR_LATTICE_ORDER},
      {[](lkp_problem_desc *d) { d->order = 7; }, LKP_ERR_LATTICE_ORDER},
      {[](lkp_problem_desc *d) { d->precision = 9; }, LKP_ERR_ARG},
      {[](lkp_problem_desc *d) { d->n[1] = 0; }, LKP_ERR_ARG},
      {[](lkp_problem_desc *d) { d->n[0] = -5; }, LKP_ERR_ARG},
      {[](lkp_problem_desc *d) { d->n[0] = int64_t(1) << 40; d->n[1] = int64_t(1) << 40; }, LKP_ERR_ARG},
      {[](lkp_problem_desc *d) { d->n[0] = 1024; d->n[1] = 1024; d->n[2] = 1024; }, LKP_ERR_ARG},
      {[](lkp_problem_desc *d) { d->n[0] = INT64_MAX; }, LKP_ERR_ARG},
      {[](lkp_problem_desc *d) { d->tau_lb = 0.5; }, LKP_ERR_UNSTABLE},
      {[](lkp_problem_desc *d) { d->tau_lb = 0.6; }, LKP_ERR_UNSTABLE},
      {[](lkp_problem_desc *d) { d->tau_lb = std::numeric_limits<double>::quiet_NaN(); }, LKP_ERR_UNSTABLE},
      {[](lkp_problem_desc *d) { d->tau_lb = std::numeric_limits<double>::infinity(); }, LKP_ERR_UNSTABLE},
      {[](lkp_problem_desc *d) { d->knudsen = std::numeric_limits<double>::infinity(); }, LKP_ERR_UNSTABLE},
      {[](lkp_problem_desc *d) { d->drift[0] = std::numeric_limits<double>::quiet_NaN(); }, LKP_ERR_ARG},
      {[](lkp_problem_desc *d) { d->drift[0] = 5.0; }, LKP_ERR_UNSTABLE},
  };
  (void)nan;
  (void)inf;
  for (const Case &c : cases) {
    lkp_problem_desc d = valid_desc(D3Q111);
    c.mutate(&d);
    EXPECT(rt::validate_desc(&d, &lc, &tau) == c.want);
    EXPECT(std::strlen(rt::last_error()) > 0);
  }
  {  // a drift along an axis the set does not have
    lkp_problem_desc d = valid_desc(D2Q81);
    d.drift[2] = 0.01;
    EXPECT(rt::validate_desc(&d, &lc, &tau) == LKP_ERR_ARG);
    d.drift[2] = 0;
    d.tau_lb = 0.55;
    d.allow_unstable = 1;
    EXPECT(rt::validate_desc(&d, &lc, &tau) == LKP_OK);
  }
  EXPECT(rt::validate_desc(nullptr, &lc, &tau) == LKP_ERR_ARG);
  // the contraction bound of every set and order: a modulus in (0, 1] at a
  // stable tau_lb, on grids with odd, even and unit sides
  for (int id = 0; id < LKP_NUM_LATTICES; ++id) {
    LatticeConstants c;
    EXPECT(lattice_constants(id, &c));
    for (int order : {1, 3, 5, 7}) {
      std::vector<long double> phl, chl;
      if (!shape_coefficients(c, order, &phl, &chl)) continue;
      std::vector<double> ph(phl.begin(), phl.end());
      const double t = std::max(1.3, stability_threshold(id, order) + 0.05);
      for (int64_t side : {1, 7, 16}) {
        const int64_t n[3] = {side, c.table.dim > 1 ? side + 1 : 1, c.table.dim > 2 ? side : 1};
        const double rho = rt::contraction_bound(c.table, c.table.dim, ph.data(), 1.0 / t, n);
        EXPECT(std::isfinite(rho) && rho > 0.0 && rho <= 1.0 + 1e-12);
      }
    }
  }
  // an over-long message is truncated, not overrun
  std::vector<char> big(4000, 'x');
  big.back() = 0;
  EXPECT(rt::fail(LKP_ERR_ARG, "%s", big.data()) == LKP_ERR_ARG);
  EXPECT(std::strlen(rt::last_error()) < 512);
  rt::clear_error();
  EXPECT(rt::last_error()[0] == 0);
  if (failures) return 1;
  std::printf("OK\n");
  return 0;
}
