// Discrete velocity sets of the higher-order lattice-kinetic Poisson scheme,
// as compile-time tables usable in kernels (every index folds to a literal).
//
//   1D sets (Appendix A): D1Q5 {0,+-1,+-3} (N <= 3), D1Q9 {0,+-1,+-2,+-3,+-5}
//     (N <= 5), D1Q13 {0,+-1,...,+-6} (N <= 7).
//   2D: the paper only says the extension uses tensor Hermite polynomials
//     (Sec. 4); D2Q25, D2Q81, D2Q169 are tensor products of the 1D sets.
//     D2Q5 and D2Q9 are the standard nearest-neighbour sets.
//   3D: D3Q111 (Appendix A, Table vector2), ten shells of signed
//     permutations, N <= 5.
//   D3Q107: generated 3D set, the smallest shell set stable at N = 5.
//   Generated 2D sets (Sec. 4's construction from the quadrature conditions:
//     the smallest shell sets with positive weights reproducing every Gaussian
//     moment to the needed degree, stable at their order):
//     D2Q37 = shells (0,0) (1,0) (1,1) (2,0) (2,1) (2,2) (3,0) (3,1), N <= 5;
//     D2Q77 = shells (0,0) (1,0) (1,1) (2,0) (2,1) (2,2) (3,0) (3,1) (3,2)
//             (4,0) (4,1) (3,3) (5,0) (4,4) (5,3), N <= 7.
#pragma once

namespace lkp {

enum LatticeId : int {
  D1Q5 = 0, D1Q9, D1Q13, D2Q5, D2Q9, D2Q25, D2Q81, D2Q169, D3Q111, D2Q37, D2Q77, D3Q107,
  NUM_LATTICES
};

constexpr int MAXQ = 169;

struct VelTable {
  int v[MAXQ][3];
  int q;
  int dim;
  int max_order;
};

namespace detail {

constexpr int S5[5] = {0, 1, -1, 3, -3};
constexpr int S9[9] = {0, 1, -1, 2, -2, 3, -3, 5, -5};
constexpr int S13[13] = {0, 1, -1, 2, -2, 3, -3, 4, -4, 5, -5, 6, -6};

constexpr VelTable line(const int* s, int m, int max_order) {
  VelTable t{};
  for (int i = 0; i < m; ++i) t.v[i][0] = s[i];
  t.q = m;
  t.dim = 1;
  t.max_order = max_order;
  return t;
}

// index i = iy * m + ix, v = (s[ix], s[iy])
constexpr VelTable square(const int* s, int m, int max_order) {
  VelTable t{};
  int k = 0;
  for (int iy = 0; iy < m; ++iy)
    for (int ix = 0; ix < m; ++ix) {
      t.v[k][0] = s[ix];
      t.v[k][1] = s[iy];
      ++k;
    }
  t.q = k;
  t.dim = 2;
  t.max_order = max_order;
  return t;
}

constexpr VelTable nearest(bool diagonals) {
  VelTable t{};
  const int axis[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
  const int diag[4][2] = {{1, 1}, {-1, 1}, {1, -1}, {-1, -1}};
  int k = 1;
  for (int i = 0; i < 4; ++i) { t.v[k][0] = axis[i][0]; t.v[k][1] = axis[i][1]; ++k; }
  if (diagonals)
    for (int i = 0; i < 4; ++i) { t.v[k][0] = diag[i][0]; t.v[k][1] = diag[i][1]; ++k; }
  t.q = k;
  t.dim = 2;
  t.max_order = diagonals ? 3 : 1;
  return t;
}

// Table vector2 shell representatives, in the table's order.
constexpr int SHELLS111[10][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {3, 3, 3}, {3, 3, 0},
                                  {3, 1, 0}, {2, 2, 0}, {2, 1, 1}, {2, 0, 0}, {3, 0, 0}};

// Generated 3D set: the smallest shell set whose N = 5 scheme is stable
// (Sec. 4's construction from the quadrature conditions, with the stability
// the Appendix sets do not need to state): 107 velocities.
constexpr int SHELLS107[10][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {1, 1, 1}, {2, 0, 0},
                                  {2, 1, 0}, {2, 2, 0}, {3, 0, 0}, {3, 1, 1}, {2, 2, 2}};

// 3D set from shell representatives: each shell's signed permutations, shell
// after shell.
constexpr VelTable shells_3d(const int (*sh)[3], int nshell, int max_order) {
  VelTable t{};
  const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int k = 0;
  for (int s = 0; s < nshell; ++s) {
    const int start = k;
    for (int p = 0; p < 6; ++p)
      for (int sg = 0; sg < 8; ++sg) {
        int c[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
          const int val = sh[s][perm[p][a]];
          c[a] = ((sg >> a) & 1) ? -val : val;
        }
        bool seen = false;
        for (int j = start; j < k; ++j)
          if (t.v[j][0] == c[0] && t.v[j][1] == c[1] && t.v[j][2] == c[2]) seen = true;
        if (!seen) {
          t.v[k][0] = c[0];
          t.v[k][1] = c[1];
          t.v[k][2] = c[2];
          ++k;
        }
      }
  }
  t.q = k;
  t.dim = 3;
  t.max_order = max_order;
  return t;
}

constexpr int SHELLS37[8][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}, {3, 0}, {3, 1}};
constexpr int SHELLS77[15][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}, {3, 0}, {3, 1},
                                 {3, 2}, {4, 0}, {4, 1}, {3, 3}, {5, 0}, {4, 4}, {5, 3}};

// 2D set from shell representatives: each shell's signed permutations, shell
// after shell.
constexpr VelTable shells_2d(const int (*sh)[2], int nshell, int max_order) {
  VelTable t{};
  int k = 0;
  for (int s = 0; s < nshell; ++s) {
    const int start = k;
    for (int p = 0; p < 2; ++p)
      for (int sg = 0; sg < 4; ++sg) {
        int c0 = p ? sh[s][1] : sh[s][0], c1 = p ? sh[s][0] : sh[s][1];
        if (sg & 1) c0 = -c0;
        if (sg & 2) c1 = -c1;
        bool seen = false;
        for (int j = start; j < k; ++j)
          if (t.v[j][0] == c0 && t.v[j][1] == c1) seen = true;
        if (!seen) {
          t.v[k][0] = c0;
          t.v[k][1] = c1;
          t.v[k][2] = 0;
          ++k;
        }
      }
  }
  t.q = k;
  t.dim = 2;
  t.max_order = max_order;
  return t;
}

}  // namespace detail

constexpr VelTable velocity_table(int id) {
  switch (id) {
    case D1Q5: return detail::line(detail::S5, 5, 3);
    case D1Q9: return detail::line(detail::S9, 9, 5);
    case D1Q13: return detail::line(detail::S13, 13, 7);
    case D2Q5: return detail::nearest(false);
    case D2Q9: return detail::nearest(true);
    case D2Q25: return detail::square(detail::S5, 5, 3);
    case D2Q81: return detail::square(detail::S9, 9, 5);
    case D2Q169: return detail::square(detail::S13, 13, 7);
    case D3Q111: return detail::shells_3d(detail::SHELLS111, 10, 5);
    case D3Q107: return detail::shells_3d(detail::SHELLS107, 10, 5);
    case D2Q37: return detail::shells_2d(detail::SHELLS37, 8, 5);
    case D2Q77: return detail::shells_2d(detail::SHELLS77, 15, 7);
    default: return VelTable{};
  }
}

constexpr int max_component(const VelTable& t, int axis) {
  int m = 0;
  for (int i = 0; i < t.q; ++i) {
    const int a = t.v[i][axis] < 0 ? -t.v[i][axis] : t.v[i][axis];
    if (a > m) m = a;
  }
  return m;
}

// Orbit of a velocity under axis permutations and sign changes: the sorted
// absolute components.  Weights (tensor products of 1D weights, or D3Q111
// shell weights) and the radial Hermite factors of phi_i and chi_i are all
// constant on an orbit, so stencil weights need one value per orbit.
constexpr int orbit_key(const VelTable &t, int i) {
  int a = t.v[i][0] < 0 ? -t.v[i][0] : t.v[i][0];
  int b = t.v[i][1] < 0 ? -t.v[i][1] : t.v[i][1];
  int c = t.v[i][2] < 0 ? -t.v[i][2] : t.v[i][2];
  if (a < b) { const int x = a; a = b; b = x; }
  if (b < c) { const int x = b; b = c; c = x; }
  if (a < b) { const int x = a; a = b; b = x; }
  return (a * 16 + b) * 16 + c;
}

// Lookup tables of one set: velocity index by components (-1 where the set
// has no such velocity; components lie in [-6, 6]) and orbit index by
// velocity.  Built once per set, so kernel templates look them up in
// constant time instead of searching the table.
struct VelMaps {
  int vidx[13][13][13];
  int orbit[MAXQ];
};

constexpr VelMaps build_maps(const VelTable &t) {
  VelMaps m{};
  for (int a = 0; a < 13; ++a)
    for (int b = 0; b < 13; ++b)
      for (int c = 0; c < 13; ++c) m.vidx[a][b][c] = -1;
  int key[MAXQ] = {};
  for (int i = 0; i < t.q; ++i) {
    m.vidx[t.v[i][0] + 6][t.v[i][1] + 6][t.v[i][2] + 6] = i;
    key[i] = orbit_key(t, i);
  }
  int first[MAXQ] = {};  // key of orbit n
  int n = 0;
  for (int i = 0; i < t.q; ++i) {
    int o = -1;
    for (int j = 0; j < n; ++j)
      if (first[j] == key[i]) o = j;
    if (o < 0) {
      first[n] = key[i];
      o = n++;
    }
    m.orbit[i] = o;
  }
  return m;
}

// Number of orbits of a set (orbits are numbered by first appearance).
constexpr int num_orbits(const VelTable &t) {
  const VelMaps m = build_maps(t);
  int n = 0;
  for (int i = 0; i < t.q; ++i)
    if (m.orbit[i] + 1 > n) n = m.orbit[i] + 1;
  return n;
}

// Compile-time view of one set, for kernel templates.
template <int ID>
struct Lattice {
  static constexpr VelTable table = velocity_table(ID);
  static constexpr int Q = table.q;
  static constexpr int DIM = table.dim;
  static constexpr int VMX = max_component(table, 0);
  static constexpr int VMY = max_component(table, 1);
  static constexpr int VMZ = max_component(table, 2);
  static constexpr VelMaps maps = build_maps(table);
  // index of velocity (vx, vy, vz), -1 if absent
  static constexpr int vel(int vx, int vy, int vz) {
    return (vx < -6 || vx > 6 || vy < -6 || vy > 6 || vz < -6 || vz > 6)
               ? -1
               : maps.vidx[vx + 6][vy + 6][vz + 6];
  }
  static constexpr int orbit(int i) { return maps.orbit[i]; }
};

static_assert(velocity_table(D3Q111).q == 111, "Table vector2 lists 111 velocities");
static_assert(velocity_table(D2Q169).q == 169, "");
static_assert(velocity_table(D2Q81).q == 81, "");
static_assert(velocity_table(D2Q37).q == 37, "eight shells of 1, 4, 4, 4, 8, 4, 4, 8 velocities");
static_assert(velocity_table(D2Q77).q == 77, "fifteen shells");
static_assert(num_orbits(velocity_table(D3Q111)) == 10, "Table vector2 has ten weight classes");
static_assert(velocity_table(D3Q107).q == 107, "ten shells of 1, 6, 12, 8, 6, 24, 12, 6, 24, 8");
static_assert(num_orbits(velocity_table(D2Q169)) <= 32, "stencil weights travel in scalar registers");

}  // namespace lkp
