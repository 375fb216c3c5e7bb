// Host-side constants of each velocity set: quadrature weights, sound speed
// and the Hermite-designed equilibrium/source shapes phi_i, chi_i.
//
// Weights come from the quadrature condition (Sec. 4, Eq. quadrature in 1D,
// Eq. quad3 in 3D), which for Hermite quadrature amounts to reproducing the
// Gaussian moments  sum_i w_i v^a = prod_k (a_k - 1)!! c_s^{a_k}  (even a_k).
// All solves run in long double with partial pivoting; results are rounded
// to double once at the end.
//
// c_s^2:
//   D1Q5   1 - sqrt(2/5)                                     (Appendix A)
//   D1Q9   the value at which the degree-10 moment also holds (the Appendix
//          prints c_s = 0.86952909818721338884964163917209 under the
//          label c_s^2)
//   D1Q13  c_s = 1.1544053947399681272395977588380 as printed (Appendix A,
//          again under the label c_s^2)
//   D3Q111 the value at which all eleven cubic moment classes of degree <= 8
//          hold with ten shell weights (Table vector2 does not print it)
//   D2Q37, D2Q77, D3Q107  generated shell sets (Sec. 4's systematic
//          construction): the value at which all 9 (degree <= 8), 16 (degree
//          <= 12) resp. 11 (degree <= 8) moment classes hold with 8, 15 resp.
//          10 shell weights
//   D2Q5, D2Q9  1/3 (standard nearest-neighbour sets)
//
// phi_i / w_i and chi_i / w_i in the radial Hermite polynomials of
// r^2 = |v|^2 / c_s^2 in d dimensions (Sec. 4, Eqs. omega:eq, chi:eq,
// omega:eq3, chi:eq3; in 1D R4 = He4 and R6 = He6):
//   R2 = r^2 - d
//   R4 = r^4 - 2(d+2) r^2 + d(d+2)
//   R6 = r^6 - 3(d+4) r^4 + 3(d+2)(d+4) r^2 - d(d+2)(d+4)
//   N=1: 1, 1     N=3: 1, 1 - R2/2     N=5: 1 - R4/8, 1 - R2/2 + R4/8
//   N=7: 1 - R4/8 + R6/24, 1 - R2/2 + R4/8 - R6/48
#include "constants.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <map>

namespace lkp {
namespace {

using ld = long double;

// Solve A x = b (n x n, row-major) by Gaussian elimination with partial
// pivoting plus one step of iterative refinement. Returns false if singular.
bool solve(std::vector<ld> A, std::vector<ld> b, int n, std::vector<ld>* x) {
  const std::vector<ld> A0 = A, b0 = b;
  std::vector<int> piv(n);
  for (int i = 0; i < n; ++i) piv[i] = i;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[p * n + k])) p = i;
    if (A[p * n + k] == 0) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
      std::swap(piv[k], piv[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      const ld m = A[i * n + k] / A[k * n + k];
      A[i * n + k] = m;
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= m * A[k * n + j];
    }
  }
  auto lu_solve = [&](const std::vector<ld>& rhs) {
    std::vector<ld> y(n);
    for (int i = 0; i < n; ++i) {
      ld s = rhs[piv[i]];
      for (int j = 0; j < i; ++j) s -= A[i * n + j] * y[j];
      y[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      ld s = y[i];
      for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * y[j];
      y[i] = s / A[i * n + i];
    }
    return y;
  };
  std::vector<ld> sol = lu_solve(b0);
  std::vector<ld> r(n);
  for (int i = 0; i < n; ++i) {
    ld s = b0[i];
    for (int j = 0; j < n; ++j) s -= A0[i * n + j] * sol[j];
    r[i] = s;
  }
  const std::vector<ld> corr = lu_solve(r);
  for (int i = 0; i < n; ++i) sol[i] += corr[i];
  *x = sol;
  return true;
}

ld odd_factorial(int m) {  // (m)!! for odd m, (-1)!! = 1
  ld r = 1;
  for (int k = m; k > 1; k -= 2) r *= k;
  return r;
}

// Gaussian moment of x^a y^b z^c (variance t per axis).
ld gauss(const int* e, int d, ld t) {
  ld r = 1;
  for (int k = 0; k < d; ++k) {
    if (e[k] % 2) return 0;
    r *= odd_factorial(e[k] - 1) * std::pow(t, (ld)(e[k] / 2));
  }
  return r;
}

// 1D: per-speed weights W(|v|) for speeds {0, s_1, ...} from moments 0..K.
bool weights_1d(const int* speeds, int nshell, ld t, std::vector<ld>* W) {
  std::vector<ld> A(nshell * nshell), b(nshell);
  for (int k = 0; k < nshell; ++k) {
    for (int j = 0; j < nshell; ++j) {
      const ld s = speeds[j];
      A[k * nshell + j] = (speeds[j] == 0 ? 1 : 2) * std::pow(s, (ld)(2 * k));
    }
    const int e = 2 * k;
    b[k] = gauss(&e, 1, t);
  }
  return solve(A, b, nshell, W);
}

// Secant iteration for a root of f near [t0, t1].
template <class F>
bool secant(F f, ld t0, ld t1, ld* root) {
  ld f0 = f(t0), f1 = f(t1);
  for (int it = 0; it < 100; ++it) {
    if (f1 == f0) break;
    const ld t2 = t1 - f1 * (t1 - t0) / (f1 - f0);
    t0 = t1;
    f0 = f1;
    t1 = t2;
    f1 = f(t1);
    if (std::fabs(t1 - t0) <= 4 * std::numeric_limits<ld>::epsilon() * std::fabs(t1)) {
      *root = t1;
      return true;
    }
  }
  *root = t1;
  return std::isfinite(t1);
}

struct Base1D {
  int shells[7];
  int nshell;
};

bool base_1d(int id, Base1D* b, ld* t) {
  static const int s5[] = {0, 1, 3}, s9[] = {0, 1, 2, 3, 5}, s13[] = {0, 1, 2, 3, 4, 5, 6};
  const int* s;
  int m;
  switch (id) {
    case D1Q5: case D2Q25: s = s5; m = 3; break;
    case D1Q9: case D2Q81: s = s9; m = 5; break;
    case D1Q13: case D2Q169: s = s13; m = 7; break;
    default: return false;
  }
  for (int i = 0; i < m; ++i) b->shells[i] = s[i];
  b->nshell = m;
  if (m == 3) {
    *t = 1.0L - std::sqrt(2.0L / 5.0L);
  } else if (m == 7) {
    const ld cs = 1.1544053947399681272395977588380L;
    *t = cs * cs;
  } else {
    // degree-10 moment residual with weights from moments 0..8
    auto resid = [&](ld tt) {
      std::vector<ld> W;
      weights_1d(b->shells, m, tt, &W);
      ld mom = 0;
      for (int j = 0; j < m; ++j)
        mom += (b->shells[j] == 0 ? 1 : 2) * W[j] * std::pow((ld)b->shells[j], (ld)10);
      return mom - 945.0L * std::pow(tt, (ld)5);
    };
    if (!secant(resid, 0.75L, 0.76L, t)) return false;
  }
  return true;
}

// Shell sets (D3Q111 and the generated 2D sets): one weight per shell of
// signed permutations.  The weights and c_s^2 are fixed by the even moment
// classes x1^a1 ... xd^ad (a1 >= ... >= ad, all even) of total degree <= D,
// D the smallest degree with one class more than shells.  Dropping one class
// leaves a square system for the weights at a given t; c_s^2 is the t at which
// the dropped class holds as well, taken where every weight is positive.
bool shell_constants(const VelTable& T, ld* t_out, std::vector<ld>* w_out) {
  const int d = T.dim;
  // shell index of each velocity (key: sorted absolute components)
  std::vector<int> shell_of(T.q);
  std::map<long, int> shell_id;
  for (int i = 0; i < T.q; ++i) {
    int a[3] = {std::abs(T.v[i][0]), std::abs(T.v[i][1]), std::abs(T.v[i][2])};
    std::sort(a, a + 3);
    const long key = (a[2] * 64L + a[1]) * 64L + a[0];
    auto it = shell_id.find(key);
    if (it == shell_id.end()) it = shell_id.emplace(key, (int)shell_id.size()).first;
    shell_of[i] = it->second;
  }
  const int nsh = (int)shell_id.size();
  // even classes of the smallest degree with nsh + 1 of them
  std::vector<std::array<int, 3>> cls;
  for (int deg = 0; deg <= 24 && (int)cls.size() < nsh + 1; deg += 2) {
    cls.clear();
    for (int a0 = 0; a0 <= deg; a0 += 2)
      for (int a1 = 0; a1 <= (d >= 2 ? a0 : 0); a1 += 2)
        for (int a2 = 0; a2 <= (d >= 3 ? a1 : 0); a2 += 2)
          if (a0 + a1 + a2 <= deg) cls.push_back({a0, a1, a2});
  }
  const int nc = (int)cls.size();
  if (nc != nsh + 1) return false;
  std::vector<ld> M((size_t)nc * nsh, 0.0L);  // class moment of each shell's orbit
  for (int r = 0; r < nc; ++r)
    for (int i = 0; i < T.q; ++i) {
      ld m = 1;
      for (int a = 0; a < d; ++a) m *= std::pow((ld)T.v[i][a], (ld)cls[r][a]);
      M[(size_t)r * nsh + shell_of[i]] += m;
    }
  // drop one class, from the last, until the remaining square system is
  // solvable with a healthy pivot
  int drop = -1;
  for (int dr = nc - 1; dr >= 0 && drop < 0; --dr) {
    std::vector<ld> A, b(nsh, 1.0L);
    for (int r = 0; r < nc; ++r)
      if (r != dr)
        for (int j = 0; j < nsh; ++j) A.push_back(M[(size_t)r * nsh + j]);
    std::vector<ld> x;
    if (!solve(A, b, nsh, &x)) continue;
    bool ok = true;
    for (ld v : x) ok = ok && std::isfinite(v) && std::fabs(v) < 1e12L;
    if (ok) drop = dr;
  }
  if (drop < 0) return false;
  auto weights_at = [&](ld tt, std::vector<ld>* x) {
    std::vector<ld> A, b;
    for (int r = 0; r < nc; ++r)
      if (r != drop) {
        for (int j = 0; j < nsh; ++j) A.push_back(M[(size_t)r * nsh + j]);
        b.push_back(gauss(cls[r].data(), d, tt));
      }
    return solve(A, b, nsh, x);
  };
  auto resid = [&](ld tt) {
    std::vector<ld> x;
    if (!weights_at(tt, &x)) return (ld)NAN;
    ld m = 0;
    for (int j = 0; j < nsh; ++j) m += M[(size_t)drop * nsh + j] * x[j];
    return m - gauss(cls[drop].data(), d, tt);
  };
  // scan t for sign changes, refine each by bisection, keep the root with
  // positive weights
  const ld step = 0.005L;
  ld lo = 0.05L, flo = resid(lo);
  for (ld hi = lo + step; hi <= 3.0L; hi += step) {
    const ld fhi = resid(hi);
    if (std::isfinite(flo) && std::isfinite(fhi) && (flo == 0 || flo * fhi < 0)) {
      ld a = lo, b = hi, fa = flo;
      for (int it = 0; it < 200 && b - a > 1e-19L * b; ++it) {
        const ld m = 0.5L * (a + b), fm = resid(m);
        if (fa * fm <= 0) b = m;
        else { a = m; fa = fm; }
      }
      const ld t = 0.5L * (a + b);
      std::vector<ld> W;
      // a sign change across a pole of the reduced system is no root
      const ld scale = std::fabs(gauss(cls[drop].data(), d, t));
      if (std::fabs(resid(t)) < 1e-12L * scale && weights_at(t, &W)) {
        bool pos = true;
        for (ld w : W) pos = pos && w > 0;
        if (pos) {
          w_out->resize(T.q);
          for (int i = 0; i < T.q; ++i) (*w_out)[i] = W[shell_of[i]];
          *t_out = t;
          return true;
        }
      }
    }
    lo = hi;
    flo = fhi;
  }
  return false;
}

}  // namespace

bool lattice_constants(int id, LatticeConstants* out) {
  if (id < 0 || id >= NUM_LATTICES) return false;
  const VelTable T = velocity_table(id);
  out->table = T;
  out->w.assign(T.q, 0.0L);
  if (id == D2Q5 || id == D2Q9) {
    out->cs2 = 1.0L / 3.0L;
    for (int i = 0; i < T.q; ++i) {
      const int r2 = T.v[i][0] * T.v[i][0] + T.v[i][1] * T.v[i][1];
      if (id == D2Q5) out->w[i] = r2 == 0 ? 1.0L / 3.0L : 1.0L / 6.0L;
      else out->w[i] = r2 == 0 ? 4.0L / 9.0L : (r2 == 1 ? 1.0L / 9.0L : 1.0L / 36.0L);
    }
    return true;
  }
  if (id == D3Q111 || id == D3Q107 || id == D2Q37 || id == D2Q77)
    return shell_constants(T, &out->cs2, &out->w);
  Base1D b;
  ld t;
  if (!base_1d(id, &b, &t)) return false;
  std::vector<ld> W;
  if (!weights_1d(b.shells, b.nshell, t, &W)) return false;
  auto wof = [&](int v) {
    const int a = std::abs(v);
    for (int j = 0; j < b.nshell; ++j)
      if (b.shells[j] == a) return W[j];
    return (ld)NAN;
  };
  out->cs2 = t;
  for (int i = 0; i < T.q; ++i)
    out->w[i] = T.dim == 1 ? wof(T.v[i][0]) : wof(T.v[i][0]) * wof(T.v[i][1]);
  return true;
}

bool shape_coefficients(const LatticeConstants& c, int order, std::vector<long double>* phi,
                        std::vector<long double>* chi) {
  if (order != 1 && order != 3 && order != 5 && order != 7) return false;
  if (order > c.table.max_order) return false;
  const int q = c.table.q, d = c.table.dim;
  phi->resize(q);
  chi->resize(q);
  for (int i = 0; i < q; ++i) {
    ld v2 = 0;
    for (int a = 0; a < 3; ++a) v2 += (ld)c.table.v[i][a] * c.table.v[i][a];
    const ld r2 = v2 / c.cs2;
    const ld R2 = r2 - d;
    const ld R4 = r2 * r2 - 2.0L * (d + 2) * r2 + (ld)d * (d + 2);
    const ld R6 = r2 * r2 * r2 - 3.0L * (d + 4) * r2 * r2 + 3.0L * (d + 2) * (d + 4) * r2 -
                  (ld)d * (d + 2) * (d + 4);
    ld p = 1, x = 1;
    if (order >= 3) x = 1 - R2 / 2;
    if (order >= 5) { p -= R4 / 8; x += R4 / 8; }
    if (order >= 7) { p += R6 / 24; x -= R6 / 48; }
    (*phi)[i] = c.w[i] * p;
    (*chi)[i] = c.w[i] * x;
  }
  return true;
}

double stability_threshold(int id, int order) {
  // Smallest tau_lb accepted.  Orders 1 and 3 need tau_lb > 1/2 (positive
  // diffusivity c_s^2 (tau_lb - 1/2), Sec. 5).  The N = 5 and N = 7
  // equilibria carry negative phi_i and lose linear stability below about
  // tau_lb = 0.62 and 0.76; the limits below keep a margin above those.
  if (order <= 3) return 0.5;
  if (order == 5) return 0.65;
  (void)id;
  return 0.8;
}

}  // namespace lkp
