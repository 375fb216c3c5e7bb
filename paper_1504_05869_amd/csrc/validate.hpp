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

}  // namespace rt
}  // namespace lkp
