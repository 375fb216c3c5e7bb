// Host-side lattice constants (weights, sound speed, phi_i, chi_i).
#pragma once

#include <algorithm>
#include <limits>
#include <vector>

#include "lattices.hpp"

namespace lkp {

struct LatticeConstants {
  VelTable table;
  long double cs2;
  std::vector<long double> w;
};

// Weights and c_s^2 of set `id`; false if the solve fails.
bool lattice_constants(int id, LatticeConstants* out);

// phi_i, chi_i for expansion order N (1, 3, 5, 7 and <= the set's maximum).
bool shape_coefficients(const LatticeConstants& c, int order, std::vector<long double>* phi,
                        std::vector<long double>* chi);

// Smallest admissible tau_lb for the set and order.
double stability_threshold(int id, int order);

}  // namespace lkp
