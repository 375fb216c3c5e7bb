// lkp_residual_noalloc: the FP64 residual report of lkp_residual for a
// population state in caller-owned device buffers, with no device
// allocation: the per-block partial norms live in a file-scope device array.
// Host code plus that array; the kernels are the library's residual sweep and
// norm finish, which take the array's device address as an argument.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "constants.hpp"
#include "kernels.hpp"
#include "lkp.h"
#include "runtime.hpp"

using namespace lkp;
using namespace lkp::rt;

namespace {

// Largest grid the array serves: 2^24 cells.  The residual sweep covers at
// least 64 cells per block (P = 4), so at most 2^18 blocks of NUM_NORMS
// partials: 12 MiB per GPU, held until the process ends.
constexpr int64_t kMaxCells = int64_t(1) << 24;
constexpr size_t kMaxBlocks = size_t(kMaxCells / 64);
constexpr size_t kScratchDoubles = kMaxBlocks * NUM_NORMS;

static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` on each device, looked up once per device with
// that device current (each GPU holds its own copy of the array).
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

lkp_status scratch_for_current_device(double **out) {
  int dev = -1;
  LKP_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LKP_ERR_ARG, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    LKP_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(LKP_ERR_HIP, "no device address for the residual scratch");
    g_scratch[dev] = static_cast<double *>(p);
  }
  *out = g_scratch[dev];
  return LKP_OK;
}

}  // namespace

extern "C" lkp_status lkp_residual_noalloc(int32_t lattice, int32_t order, const int64_t n[3],
                                           double tau_lb, const double *f, const double *S,
                                           const double *phi_prev, double *phi_out, float *r_out,
                                           double *norms_out, void *stream) {
  if (!n || !f || !S || !phi_out || !norms_out)
    return fail(LKP_ERR_ARG, "lkp_residual_noalloc: null argument");
  if (lattice < 0 || lattice >= LKP_NUM_LATTICES) return fail(LKP_ERR_ARG, "unknown lattice %d", lattice);
  const VelTable T = velocity_table(lattice);
  if (order != 1 && order != 3 && order != 5 && order != 7)
    return fail(LKP_ERR_LATTICE_ORDER, "order must be 1, 3, 5 or 7 (got %d)", order);
  if (order > T.max_order)
    return fail(LKP_ERR_LATTICE_ORDER, "lattice supports order <= %d (got %d)", T.max_order, order);
  int64_t cells = 1;
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1) return fail(LKP_ERR_ARG, "n[%d] = %lld < 1", a, (long long)n[a]);
    if (a >= T.dim && n[a] != 1) return fail(LKP_ERR_ARG, "n[%d] must be 1 for a %dD set", a, T.dim);
    if (n[a] > kMaxCells)
      return fail(LKP_ERR_ARG, "lkp_residual_noalloc serves at most 2^24 cells (its scratch is fixed)");
    cells *= n[a];  // both factors at most 2^24: no overflow
    if (cells > kMaxCells)
      return fail(LKP_ERR_ARG, "lkp_residual_noalloc serves at most 2^24 cells (its scratch is fixed)");
  }
  if (!(tau_lb > 0.5) || !std::isfinite(tau_lb)) return fail(LKP_ERR_ARG, "tau_lb = %g must exceed 1/2", tau_lb);
  LatticeConstants lc;
  if (!lattice_constants(lattice, &lc)) return fail(LKP_ERR_HIP, "lattice constant solve failed");
  std::vector<long double> phi, chi;
  if (!shape_coefficients(lc, order, &phi, &chi))
    return fail(LKP_ERR_LATTICE_ORDER, "no coefficients for order %d", order);

  double *partials = nullptr;
  if (lkp_status st = scratch_for_current_device(&partials)) return st;

  // the residual sweep of lkp_residual: same split, coefficients formed the
  // same way (omega phi_i and chi_i rounded from the long-double solve)
  const int Q = T.q;
  const int P = default_split(Q, MODE_RESID);
  SweepParams p{};
  const double omega = 1.0 / tau_lb;
  p.om1 = 1.0 - omega;
  p.nx = (unsigned)n[0];
  p.ny = (unsigned)n[1];
  p.nz = (unsigned)n[2];
  p.ncells = (unsigned)cells;
  p.plane = (unsigned)cells;
  p.simple_wrap = (n[0] >= max_component(T, 0) && n[1] >= max_component(T, 1) && n[2] >= max_component(T, 2))
                      ? 1u : 0u;
  for (int i = 0; i < Q; ++i) {
    p.coef.d[i] = omega * (double)phi[i];
    p.coef.d[Q + i] = (double)chi[i];
  }
  p.fin = f;
  p.fout = r_out;
  p.src = S;
  p.phi_prev = phi_prev;
  p.phi_out = phi_out;
  p.partials = partials;
  const unsigned nblocks = (unsigned)((cells + cells_per_block(P) - 1) / cells_per_block(P));
  if ((size_t)nblocks > kMaxBlocks) return fail(LKP_ERR_ARG, "grid exceeds the residual scratch");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_sweep(lattice, MODE_RESID, P, FLAG_REDUCE, p, s);
  if (e != hipSuccess) return fail(LKP_ERR_HIP, "residual sweep launch: %s", hipGetErrorString(e));
  e = launch_finish(partials, nblocks, norms_out, s);
  if (e != hipSuccess) return fail(LKP_ERR_HIP, "norm finish launch: %s", hipGetErrorString(e));
  clear_error();
  return LKP_OK;
}
