// Host-only part of the runtime: the thread-local error message and the
// validation of a problem description.  No HIP dependency, so it also builds
// with a plain host compiler (the sanitizer build of the tests).
#pragma once

#include "constants.hpp"
#include "lkp.h"

namespace lkp {
namespace rt {

lkp_status fail(lkp_status st, const char *fmt, ...);
void clear_error();
const char *last_error();

// Check a problem description (shape, set, order, precision, tau_lb or Kn,
// stability, drift).  On success fills the set's constants and tau_lb (from
// Kn = lambda / L with lambda = c_s (tau_lb - 1/2), L the smallest box side;
// Sec. 2).  The source pointer is not examined.
lkp_status validate_desc(const lkp_problem_desc *d, LatticeConstants *lc, double *tau_out);

// Whether the description asks for the drifted (advection-diffusion) equilibrium.
bool has_drift(const lkp_problem_desc *d);

// The slowest decay the sweep allows on a periodic grid of n[0..dim-1] cells:
// the largest modulus of its one-sweep amplification over the grid's modes
// other than the mass mode (Fourier analysis of the sweep, Sec. 4 and 5: mode
// k maps the post-collision populations by (1 - omega) E + omega phi e^T,
// E = diag(e), e_j = exp(-i k.v_j)).  Taken over the modes where it peaks:
// the kinetic value |1 - omega| (the k = 0 modes other than mass), every
// corner mode (each component of k 0 or pi; a closed form, since e_j = +-1),
// and the longest wave along each axis (the root of the secular equation
// that continues the mass eigenvalue 1, by Newton's method).  phi: the Q
// equilibrium shape values.
double contraction_bound(const VelTable &T, int dim, const double *phi, double omega,
                         const int64_t n[3]);

}  // namespace rt
}  // namespace lkp
