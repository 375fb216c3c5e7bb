// C-ABI runtime of the lattice-kinetic Poisson solver (see include/lkp.h).
//
// Host side only: validation, constants, device memory, the chunked
// convergence loop (sweeps, FP64 norms, one small read-back per chunk),
// hipGraph replay of chunks, the velocity-group tuner and the FP64
// iterative-refinement controller around FP32 inner sweeps.
#include "lkp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "constants.hpp"
#include "dev_kernels.hpp"
#include "kernels.hpp"
#include "stencil.hpp"
#include "runtime.hpp"

using namespace lkp;
using namespace lkp::rt;

#define HIP_TRY LKP_HIP_TRY

namespace lkp {
namespace rt {

namespace {
// Process-wide choice of the velocity-group split per (lattice, mode, size class).
std::mutex g_tune_mu;
std::map<long, int> g_tune;
std::map<long, std::pair<int, unsigned>> g_stile;  // 3D stencil: (tile, block order)

long tune_key(int lattice, int mode, int64_t ncells) {
  int cls = 0;
  while ((int64_t(1) << (2 * cls + 12)) < ncells && cls < 12) ++cls;
  return ((long)lattice * 16 + mode) * 32 + cls;
}
}  // namespace

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int default_split(int Q, int mode) {
  const bool wide = (mode == MODE_F64 || mode == MODE_RESID);
  if (Q <= 25) return 1;
  if (mode == MODE_INNER) return inner_split(Q);
  if (wide) return Q >= 169 ? 4 : 2;
  return Q >= 169 ? 2 : 1;
}

unsigned sweep_blocks(const lkp_handle *h, int P) {
  const unsigned c = cells_per_block(P);
  return (h->ncells + c - 1) / c;
}

void set_coefficients(const lkp_handle *h, int mode, SweepParams *p) {
  const size_t n = h->c64.size();
  if (mode == MODE_F32 || mode == MODE_INNER)
    std::memcpy(p->coef.f, h->c32.data(), n * sizeof(float));
  else
    std::memcpy(p->coef.d, h->c64.data(), n * sizeof(double));
}

SweepParams base_params(const lkp_handle *h) {
  SweepParams p{};
  p.om1 = 1.0 - h->omega;
  p.nx = (unsigned)h->n[0];
  p.ny = (unsigned)h->n[1];
  p.nz = (unsigned)h->n[2];
  p.ncells = h->ncells;
  p.plane = h->ncells;
  p.simple_wrap = h->simple_wrap ? 1u : 0u;
  return p;
}

lkp_status finish_norms(lkp_handle *h, unsigned nblocks, double *dst_dev, hipStream_t s) {
  hipError_t e = launch_finish(h->partials, nblocks, dst_dev, s);
  if (e != hipSuccess) return fail(LKP_ERR_HIP, "finish launch: %s", hipGetErrorString(e));
  return LKP_OK;
}

bool interval_checks(const lkp_handle *h, const lkp_solve_opts &o) {
  return !h->scalar && !(o.tol_maxchange > 0) && o.tol_rel_l2 > 0;
}

void commit_chunk(lkp_handle *h, int k, bool pair) {
  const int64_t t0 = h->total_sweeps;
  if (k % 2) h->cur = 1 - h->cur;
  if (!pair) {
    // the change over the chunk: Phi_t written to phib[1] and copied to
    // phib[0], where the next check compares with it
    h->phi_last = 1;
    h->phi_sweep[0] = h->phi_sweep[1] = t0 + k;
  } else if (k >= 2) {
    h->phi_sweep[0] = t0 + k - 1;
    h->phi_sweep[1] = t0 + k;
    h->phi_last = 1;
  } else {
    h->phi_last = 1 - h->phi_last;
    h->phi_sweep[h->phi_last] = t0 + 1;
  }
  h->total_sweeps = t0 + k;
}

lkp_status track_check(lkp_handle *h, const double nr[NUM_NORMS], int64_t span,
                       const lkp_solve_opts &o, lkp_solve_report *rep, bool *converged) {
  *converged = false;
  Tracker &t = h->trk;
  if (nr[NORM_BAD] > 0)
    return fail(LKP_ERR_DIVERGED, "non-finite values after %lld sweeps", (long long)h->total_sweeps);
  rep->max_change = nr[NORM_MAX_DPHI];
  rep->l2_change = std::sqrt(nr[NORM_SUM_DPHI2]);
  rep->phi_l2 = std::sqrt(nr[NORM_SUM_PHI2]);
  rep->mass = nr[NORM_SUM_PHI];
  if (span < 1) return LKP_OK;
  const double l2 = rep->l2_change;
  // changes over windows of equal length shrink by the contraction to the
  // power of the sweeps between them
  if (t.l2_prev > 0 && l2 > 0 && h->total_sweeps > t.t_prev && span == t.span_prev) {
    t.rates[t.nrates % Tracker::kRates] =
        std::pow(l2 / t.l2_prev, 1.0 / (double)(h->total_sweeps - t.t_prev));
    t.nrates += 1;
    t.rate = 0.0;
    for (int j = 0; j < std::min(t.nrates, Tracker::kRates); ++j) t.rate = std::max(t.rate, t.rates[j]);
    // A slow mode carries little of the one-sweep change while faster ones
    // still decay (its share of the change is (1 - lambda) times its share of
    // the error), so the measured contraction can sit below the slowest
    // mode's for thousands of sweeps; the estimate never uses less than the
    // slowest decay the grid's modes allow.
    if (h->rho_bound < 1.0) t.rate = std::max(t.rate, h->rho_bound);
    rep->rate = t.rate;
  }
  if (l2 > 0) t.min_l2 = std::min(t.min_l2, l2);
  if (l2 > 1e10 * t.min_l2 && l2 > 1e-300)
    return fail(LKP_ERR_DIVERGED, "change grew by 1e10 (unstable tau_lb?)");
  if (o.tol_maxchange > 0 && rep->max_change < o.tol_maxchange) *converged = true;
  if (o.tol_rel_l2 > 0) {
    if (l2 == 0) {
      rep->est_rel_err = 0;
      *converged = true;
    } else if (t.rate > 0 && t.rate < 1 && rep->phi_l2 > 0) {
      // a change D over the last `span` sweeps of a geometric decay at rate r
      // leaves D r^span / (1 - r^span) to go (span = 1: d r / (1 - r))
      const double rs = std::pow(t.rate, (double)span);
      rep->est_rel_err = l2 * rs / (1 - rs) / rep->phi_l2;
      if (rep->est_rel_err <= o.tol_rel_l2) *converged = true;
    } else {
      rep->est_rel_err = INFINITY;
    }
  }
  t.l2_prev = l2;
  t.t_prev = h->total_sweeps;
  t.span_prev = span;
  return LKP_OK;
}

// ---------------------------------------------------------------- F32 + IR
//
// x (FP64 population state) is refined by corrections d that solve
// (I - T) d = r with r = T x + g - x, where T is one sweep without source and
// g = chi_i S its source term.  r is formed in FP64 arithmetic on the GPU and
// stored in FP32; d is iterated in FP32 (d <- T d + r) from d = 0; then
// x += d - phi_i mean(d) in FP64, which keeps the mass mode (the eigenvector
// phi_i of T with eigenvalue 1) at the zero of the initial state.

lkp_status ir_launch_residual(lkp_handle *h, double *dst_dev) {
  if (h->scalar) {  // R = A x + G - x on the Phi state
    StencilParams p{};
    p.nx = (unsigned)h->n[0];
    p.ny = (unsigned)h->n[1];
    p.nz = (unsigned)h->n[2];
    p.simple_wrap = h->simple_wrap ? 1u : 0u;
    p.partials = h->partials;
    p.tile = (unsigned)h->stile;
    p.remap = h->sremap;
    const VelTable T = velocity_table(h->lattice);
    const VelMaps M = build_maps(T);
    for (int i = 0; i < T.q; ++i) p.coef.d[M.orbit[i]] = h->phi[i];
    p.xin = h->f[0];
    p.xout = h->r32;
    p.src = h->S;
    hipError_t e = launch_stencil(h->lattice, SMODE_RESID, FLAG_REDUCE, p, h->stream);
    if (e != hipSuccess) return fail(LKP_ERR_HIP, "residual stencil launch: %s", hipGetErrorString(e));
    h->total_sweeps += 1;
    return finish_norms(h, stencil_blocks(h->lattice, p.nx, p.ny, p.nz, h->stile), dst_dev, h->stream);
  }
  const int P = default_split(h->Q, MODE_RESID);
  SweepParams p = base_params(h);
  p.fin = h->f[0];
  p.fout = h->r32;
  p.src = h->S;
  set_coefficients(h, MODE_RESID, &p);
  p.phi_prev = nullptr;
  p.phi_out = h->phib[1];
  p.partials = h->partials;
  hipError_t e = launch_sweep(h->lattice, MODE_RESID, P, FLAG_REDUCE, p, h->stream);
  if (e != hipSuccess) return fail(LKP_ERR_HIP, "residual sweep launch: %s", hipGetErrorString(e));
  h->total_sweeps += 1;  // one FP64 sweep of x
  h->phi_last = 1;
  h->phi_sweep[1] = h->total_sweeps;  // Phi of the refined state
  return finish_norms(h, sweep_blocks(h, P), dst_dev, h->stream);
}

lkp_status ir_begin_inner(lkp_handle *h, const lkp_solve_opts &o) {
  IrState &s = h->ir;
  if (s.phase == IR_START) s.rnorm = h->g_norm;  // residual of x = 0
  const size_t QN = (size_t)(h->scalar ? 1 : h->Q) * h->ncells;
  if (h->bf16dev()) {
    LKP_HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(h->dn[0]), 0u, (QN + 1) / 2, h->stream));
    LKP_HIP_TRY(launch_fill_f32(h->dphi[0], 0.0f, h->ncells, h->stream));
  } else {
    LKP_HIP_TRY(launch_fill_f32(h->d32[0], 0.0f, QN, h->stream));
  }
  s.dc = 0;
  s.est_in = -1.0;
  // Inner accuracy: as asked, or just enough to close the remaining gap
  // (30 % margin), never below the FP32 sweep's own floor (~1e-7 relative).
  if (o.ir_inner_tol > 0) {
    s.inner_tol = o.ir_inner_tol;
  } else {
    const double want = s.est > 0 ? 0.3 * o.tol_rel_l2 / s.est : 1e-1;
    s.inner_tol = std::min(1e-1, std::max(1e-7, want));
  }
  s.l2_prev = -1;
  s.best_l2 = 1e300;
  s.stall = 0;
  s.t_in = 0;
  s.t_prev = 0;
  s.phase = IR_INNER;
  return LKP_OK;
}

lkp_status ir_after_residual(lkp_handle *h, const double nr[NUM_NORMS], const lkp_solve_opts &o,
                             lkp_solve_report *rep, bool *converged) {
  IrState &s = h->ir;
  *converged = false;
  s.rnorm = std::sqrt(nr[NORM_SUM_R2]);
  const double phi_l2 = std::sqrt(nr[NORM_SUM_PHI2]);
  rep->phi_l2 = phi_l2;
  rep->mass = nr[NORM_SUM_PHI];
  rep->outer = s.outer;
  if (nr[NORM_BAD] > 0) return fail(LKP_ERR_DIVERGED, "non-finite residual");
  if (s.corr_prev >= 0 && s.rnorm_prev > 0 && phi_l2 > 0) {
    // the last correction scaled by how much the residual shrank since it,
    // and never less than what that correction's inner solve estimated it
    // left undone (the residual shrinks faster than the error when the error
    // left is in slow modes)
    rep->est_rel_err = std::max(s.corr_prev * (s.rnorm / s.rnorm_prev), s.left) / phi_l2;
    s.est = rep->est_rel_err;
    if (rep->est_rel_err <= o.tol_rel_l2) *converged = true;
  }
  if (s.rnorm == 0) {
    rep->est_rel_err = 0;
    *converged = true;
  }
  if (*converged) {
    s.phase = IR_DONE;
    return LKP_OK;
  }
  const int max_outer = o.max_outer > 0 ? o.max_outer : 20;
  if (s.outer >= max_outer) return fail(LKP_ERR_NOT_CONVERGED, "refinement: %d outer steps", s.outer);
  return ir_begin_inner(h, o);
}

int ir_inner_mode(const lkp_handle *h) { return h->ir.first ? MODE_F32 : MODE_INNER; }

void ir_reset(lkp_handle *h) {
  const IrState old = h->ir;
  h->ir = IrState();
  if (h->x_nonzero) {  // resume: refine the current x, starting from its residual
    h->ir.phase = IR_RESID;
    h->ir.first = false;
    // the last correction and the residual before it: the first residual of
    // the resumed solve already gives an error estimate
    h->ir.corr_prev = old.corr_prev;
    h->ir.left = old.left;
    h->ir.rnorm_prev = old.rnorm_prev;
    h->ir.est = old.est;
  }
}

SweepParams ir_inner_params(lkp_handle *h, int P) {
  SweepParams p = base_params(h);
  const int mode = ir_inner_mode(h);
  p.fin = h->d32[h->ir.dc];
  p.fout = h->d32[1 - h->ir.dc];
  p.src = mode == MODE_F32 ? (const void *)h->S32 : (const void *)h->r32;
  set_coefficients(h, mode, &p);
  p.partials = h->partials;
  (void)P;
  return p;
}

lkp_status ir_apply_correction(lkp_handle *h, lkp_solve_report *rep, bool truncated = false);

lkp_status ir_after_inner(lkp_handle *h, const double nr[NUM_NORMS], int K,
                          const lkp_solve_opts &o, lkp_solve_report *rep) {
  IrState &s = h->ir;
  if (nr[NORM_BAD] > 0) return fail(LKP_ERR_DIVERGED, "non-finite inner sweep");
  s.t_in += K;
  const double l2 = std::sqrt(nr[NORM_SUM_DPHI2]);
  s.corr = std::sqrt(nr[NORM_SUM_PHI2]);
  if (s.l2_prev > 0 && l2 > 0) {
    const double r = std::pow(l2 / s.l2_prev, 1.0 / (double)(s.t_in - s.t_prev));
    if (r < 1) s.rate = r;
  }
  // Stagnation at the FP32 rounding floor: the change stops shrinking at
  // (half) the contraction rate measured while it still converged.
  const bool no_progress =
      s.l2_prev > 0 && (s.rate > 0 ? l2 >= s.l2_prev * std::pow(s.rate, 0.5 * K) : l2 >= s.l2_prev);
  s.stall = (no_progress && s.t_in >= 4 * (int64_t)K) ? s.stall + 1 : 0;
  s.best_l2 = std::min(s.best_l2, l2);
  s.l2_prev = l2;
  s.t_prev = s.t_in;
  // the contraction of the correction's error: the measured one, never below
  // the slowest decay the grid's modes allow (as for the plain sweep)
  const double rho = (s.rate > 0 && h->rho_bound < 1) ? std::max(s.rate, h->rho_bound) : s.rate;
  rep->rate = rho;
  const double est = (rho > 0 && rho < 1) ? l2 * rho / (1 - rho) : 1e300;
  s.est_in = est < 1e300 ? est : -1.0;
  // FP32 sweeps cannot bring the correction closer than about u32 / (1 - rho)
  // of its size (rounding of each sweep, amplified by the contraction the
  // solve shows); stop there rather than sweep on without gaining accuracy.
  // BF16 deviation storage has no such simple floor (its rounding is
  // relative to the deviation, not the population): there the stall rule
  // decides.
  const double floor32 =
      (!h->bf16dev() && s.rate > 0 && s.rate < 1) ? 2.0 * 5.96e-8 / (1 - s.rate) : 0.0;
  const double goal = std::max(s.inner_tol, floor32);
  const bool met = s.corr == 0 || est <= goal * s.corr;
  if (!(met || s.stall >= 2)) return LKP_OK;
  // what the correction leaves undone, by its own estimate; a solve stopped
  // for stalling has no meaningful one (its change is rounding noise)
  s.left = s.corr == 0 ? 0.0 : (met ? std::max(est, floor32 * s.corr) : -1.0);
  return ir_apply_correction(h, rep);
}

// x += d - phi_i mean(d), FP64 (scalar state: x += d - mean(d)); next: residual.
// Also used when max_sweeps ends an inner solve early (truncated): the partial
// correction (a truncated sum of the contraction's powers applied to r) still
// lowers the error, and a later solve resumes from the updated x.
lkp_status ir_apply_correction(lkp_handle *h, lkp_solve_report *rep, bool truncated) {
  IrState &s = h->ir;
  const int q = h->scalar ? 1 : h->Q;
  const size_t QN = (size_t)q * h->ncells;
  unsigned nb = 0;
  if (h->bf16dev()) {  // d_i = phi_i Phi + n_i
    LKP_HIP_TRY(launch_dev_sum(h->dn[s.dc], h->dphi[s.dc], (unsigned)q, h->ncells, h->partials,
                               (unsigned)h->partial_cap, &nb, h->stream));
    LKP_HIP_TRY(launch_finish(h->partials, nb, h->norms_dev, h->stream));
    LKP_HIP_TRY(launch_ir_update_dev((double *)h->f[0], h->dn[s.dc], h->dphi[s.dc], h->phi_dev,
                                     h->norms_dev, (unsigned)q, h->ncells, h->stream));
  } else {
    LKP_HIP_TRY(launch_sum_f32(h->d32[s.dc], QN, h->partials, (unsigned)h->partial_cap, &nb, h->stream,
                               h->inplace ? h->opp_dev : nullptr, h->ncells));
    LKP_HIP_TRY(launch_finish(h->partials, nb, h->norms_dev, h->stream));
    // in place the corrections sit in the swapped layout (even chunks: dc == 0)
    LKP_HIP_TRY(launch_ir_update((double *)h->f[0], h->d32[s.dc], h->phi_dev, h->norms_dev, q,
                                 h->ncells, h->stream, h->inplace ? h->opp_dev : nullptr));
  }
  s.outer += 1;
  s.first = false;
  h->x_nonzero = true;
  // The next residual's estimate is this correction scaled by the residual's
  // shrink.  After K sweeps at contraction rho the partial correction is about
  // (1 - rho^K) of the full one, so a truncated correction stands for
  // |d| / (1 - rho^K); with no rate measured yet it gives no estimate.
  // What a truncated correction leaves undone is its inner solve's latest
  // estimate (which never uses less than the slowest decay the grid allows).
  if (!truncated) {
    s.corr_prev = s.corr;
  } else if (s.rate > 0 && s.rate < 1 && s.t_in > 0) {
    const double got = 1.0 - std::pow(s.rate, (double)s.t_in);
    s.corr_prev = got > 0 ? s.corr / got : -1.0;
    s.left = s.est_in >= 0 ? s.est_in : (got > 0 ? s.corr_prev - s.corr : -1.0);
  } else {
    s.corr_prev = -1.0;
    s.left = -1.0;
  }
  s.rnorm_prev = s.rnorm;
  s.phase = IR_RESID;
  rep->outer = s.outer;
  return LKP_OK;
}

// Pick the velocity-group split by timing each built candidate on the
// handle's own buffers.  Sweeps read f[cur] and write f[1-cur] without
// swapping, so the state is unchanged.
lkp_status tune_split(lkp_handle *h) {
  if (h->tuned) return LKP_OK;
  h->tuned = true;
  if (h->bf16dev()) {  // one deviation-sweep variant per lattice
    h->split = dev_split(h->lattice);
    return LKP_OK;
  }
  const int mode = h->precision == LKP_F32_IR ? MODE_INNER : h->mode();
  const long key = tune_key(h->lattice, mode, h->ncells);
  // LKP_SPLIT forces a split when that variant is built (tests, experiments)
  if (const char *env = std::getenv("LKP_SPLIT")) {
    const int P = std::atoi(env);
    if (sweep_variant_available(h->lattice, mode, P)) {
      h->split = P;
      return LKP_OK;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      h->split = it->second;
      return LKP_OK;
    }
  }
  const char *off = std::getenv("LKP_AUTOTUNE");
  // in place, a timing sweep would change the state: no tuning
  if ((off && std::atoi(off) == 0) || h->ncells < 4096 || h->inplace) {
    h->split = default_split(h->Q, mode);
    return LKP_OK;
  }
  // refinement: the correction sweep (FP32 d -> the idle correction buffer,
  // residual source; contents do not matter for timing), at splits built for
  // the FP32 first solve as well
  const bool ir = h->precision == LKP_F32_IR;
  auto sweep_once = [&](int P) -> lkp_status {
    SweepParams p = base_params(h);
    p.fin = ir ? (const void *)h->d32[0] : h->f[h->cur];
    p.fout = ir ? (void *)h->d32[1] : h->f[1 - h->cur];
    p.src = ir ? (const void *)h->r32 : h->S;
    set_coefficients(h, mode, &p);
    hipError_t e = launch_sweep(h->lattice, mode, P, 0, p, h->stream);
    if (e != hipSuccess) return fail(LKP_ERR_HIP, "tuning sweep: %s", hipGetErrorString(e));
    return LKP_OK;
  };
  hipEvent_t e0, e1;
  LKP_HIP_TRY(hipEventCreate(&e0));
  LKP_HIP_TRY(hipEventCreate(&e1));
  float best = 1e30f;
  int bestP = default_split(h->Q, mode);
  const int saved = h->split;
  for (int P : {1, 2, 4}) {
    if (!sweep_variant_available(h->lattice, mode, P)) continue;
    if (ir && !sweep_variant_available(h->lattice, MODE_F32, P)) continue;
    h->split = P;
    if (lkp_status st = sweep_once(P)) {
      h->split = saved;
      return st;
    }
    LKP_HIP_TRY(hipEventRecord(e0, h->stream));
    for (int r = 0; r < 3; ++r)
      if (lkp_status st = sweep_once(P)) return st;
    LKP_HIP_TRY(hipEventRecord(e1, h->stream));
    LKP_HIP_TRY(hipEventSynchronize(e1));
    float ms = 0;
    LKP_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      bestP = P;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->split = bestP;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = bestP;
  return LKP_OK;
}

}  // namespace rt
}  // namespace lkp

namespace {

// Device memory of a handle: hipMalloc'd and owned by the handle, or carved
// from a caller-provided workspace (256-byte aligned pieces); count_only
// walks the same plan to measure it (lkp_footprint_bytes).
struct DevAlloc {
  char *base = nullptr;  // workspace, or null
  size_t cap = 0;
  size_t used = 0;
  bool count_only = false;

  lkp_status get(lkp_handle *h, void **p, size_t bytes) {
    const size_t off = (used + 255) & ~size_t(255);
    used = off + bytes;
    if (count_only) {
      *p = reinterpret_cast<void *>(uintptr_t(256));  // placeholder, never used
      return LKP_OK;
    }
    if (base) {
      if (used > cap)
        return fail(LKP_ERR_ARG, "workspace of %zu bytes is too small (lkp_footprint_bytes: at least %zu)",
                    cap, used);
      *p = base + off;
      return LKP_OK;
    }
    HIP_TRY(hipMalloc(p, bytes));
    h->owned.push_back(*p);
    return LKP_OK;
  }
  // Give back memory needed only while the handle is created (owned mode).
  void drop(lkp_handle *h, void *p) {
    if (base || count_only || !p) return;
    auto it = std::find(h->owned.begin(), h->owned.end(), p);
    if (it != h->owned.end()) {
      (void)hipFree(p);
      h->owned.erase(it);
    }
  }
};

template <class T>
lkp_status dget(DevAlloc &A, lkp_handle *h, T **p, size_t bytes) {
  void *v = nullptr;
  lkp_status st = A.get(h, &v, bytes);
  *p = static_cast<T *>(v);
  return st;
}

unsigned partial_blocks(const lkp_handle *h);

// Every device buffer of a handle, in one fixed order.  Create-time
// temporaries of the stencil form (the FP64 source, and for FP32 its
// stencil G) come back in tmp_S / tmp_G.
lkp_status plan_state(lkp_handle *h, DevAlloc &A, double **tmp_S, double **tmp_G) {
  const size_t n = h->ncells, Q = h->Q;
  *tmp_S = *tmp_G = nullptr;
  if (lkp_status st = dget(A, h, &h->norms_dev, NUM_NORMS * sizeof(double))) return st;
  if (h->scalar) {
    const size_t nb = partial_blocks(h);
    if (lkp_status st = dget(A, h, &h->partials, nb * NUM_NORMS * sizeof(double))) return st;
    h->partial_cap = nb;
    if (lkp_status st = dget(A, h, tmp_S, n * 8)) return st;
    if (lkp_status st = dget(A, h, tmp_G, n * 8)) return st;
    const size_t fb = h->precision == LKP_F32 ? 4 : 8;
    if (lkp_status st = dget(A, h, &h->f[0], n * fb)) return st;
    if (h->precision != LKP_F32_IR)
      if (lkp_status st = dget(A, h, &h->f[1], n * fb)) return st;
    if (h->precision == LKP_F32) {
      if (lkp_status st = dget(A, h, &h->S, n * 4)) return st;
    } else {
      h->S = *tmp_G;  // the stencil of the source is the state's G
      *tmp_G = nullptr;
    }
    if (h->precision == LKP_F32_IR) {
      if (lkp_status st = dget(A, h, &h->r32, n * 4)) return st;
      if (lkp_status st = dget(A, h, &h->d32[0], n * 4)) return st;
      if (lkp_status st = dget(A, h, &h->d32[1], n * 4)) return st;
      if (lkp_status st = dget(A, h, &h->S32, n * 4)) return st;
      if (lkp_status st = dget(A, h, &h->phi_dev, sizeof(double))) return st;
    }
    return LKP_OK;
  }
  // partial norms for the finest block split (P = 4: 64 cells per block)
  const size_t nb = sweep_blocks(h, 4) + 8;
  if (lkp_status st = dget(A, h, &h->partials, nb * NUM_NORMS * sizeof(double))) return st;
  h->partial_cap = nb;
  if (h->precision == LKP_F64 || h->precision == LKP_F32) {
    const size_t fb = h->precision == LKP_F64 ? 8 : 4;
    if (lkp_status st = dget(A, h, &h->f[0], Q * n * fb)) return st;
    if (h->inplace) h->f[1] = h->f[0];
    else if (lkp_status st = dget(A, h, &h->f[1], Q * n * fb)) return st;
    if (lkp_status st = dget(A, h, &h->S, n * fb)) return st;
  } else {
    if (lkp_status st = dget(A, h, &h->f[0], Q * n * 8)) return st;  // x, the FP64 refined state
    h->f[1] = nullptr;
    if (lkp_status st = dget(A, h, &h->r32, Q * n * 4)) return st;
    if (h->bf16dev()) {
      const size_t words = (Q * n + 1) / 2;  // BF16 planes, cleared as 32-bit words
      for (int k = 0; k < 2; ++k) {
        if (lkp_status st = dget(A, h, &h->dn[k], words * 4)) return st;
        if (lkp_status st = dget(A, h, &h->dphi[k], n * 4)) return st;
      }
    } else {
      if (lkp_status st = dget(A, h, &h->d32[0], Q * n * 4)) return st;
      if (h->inplace) {
        h->d32[1] = h->d32[0];
        if (lkp_status st = dget(A, h, &h->opp_dev, Q * sizeof(int))) return st;
      } else if (lkp_status st = dget(A, h, &h->d32[1], Q * n * 4)) {
        return st;
      }
    }
    if (lkp_status st = dget(A, h, &h->S, n * 8)) return st;
    if (lkp_status st = dget(A, h, &h->S32, n * 4)) return st;
    if (lkp_status st = dget(A, h, &h->phi_dev, Q * sizeof(double))) return st;
  }
  if (lkp_status st = dget(A, h, &h->phib[0], n * 8)) return st;
  if (lkp_status st = dget(A, h, &h->phib[1], n * 8)) return st;
  return LKP_OK;
}

// One population sweep of the handle's own state (F64 / F32) from buffer
// `in` to buffer `out` with `flags`.
// In place, buffer index `in` is the layout phase: 0 = swapped, 1 = pushed.
int aa_of(const lkp_handle *h, int in) { return h->inplace ? (in == 0 ? 1 : 2) : 0; }

lkp_status enqueue_sweep(lkp_handle *h, hipStream_t s, int in, int out, int flags,
                         const double *phi_prev, double *phi_out, bool dry = false) {
  SweepParams p = base_params(h);
  p.fin = h->f[in];
  p.fout = dry ? nullptr : h->f[out];
  p.src = h->S;
  set_coefficients(h, h->mode(), &p);
  p.phi_prev = phi_prev;
  p.phi_out = phi_out;
  p.partials = h->partials;
  hipError_t e = launch_sweep(h->lattice, h->mode(), h->split, flags, p, s, aa_of(h, in));
  if (e != hipSuccess) return fail(LKP_ERR_HIP, "sweep launch: %s", hipGetErrorString(e));
  return LKP_OK;
}

lkp_status read_back(lkp_handle *h, double out[NUM_NORMS]) {
  HIP_TRY(hipMemcpyAsync(h->norms_host, h->norms_dev, NUM_NORMS * sizeof(double),
                         hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  std::memcpy(out, h->norms_host, NUM_NORMS * sizeof(double));
  return LKP_OK;
}

lkp_status read_norms(lkp_handle *h, unsigned nblocks, double out[NUM_NORMS]) {
  if (lkp_status st = finish_norms(h, nblocks, h->norms_dev, h->stream)) return st;
  HIP_TRY(hipMemcpyAsync(h->norms_host, h->norms_dev, NUM_NORMS * sizeof(double),
                         hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  std::memcpy(out, h->norms_host, NUM_NORMS * sizeof(double));
  return LKP_OK;
}

StencilParams stencil_params(const lkp_handle *h);
void stencil_weights(const lkp_handle *h, bool fp32, StencilParams *p);

// One omega = 1 sweep number t (1-based) of the Phi state: sweep 1 starts
// from f* = 0, so its Phi is exactly 0; later sweeps apply the stencil.
lkp_status scalar_sweep(lkp_handle *h, hipStream_t s, int64_t t, int in, int out, int flags) {
  const size_t n = h->ncells;
  const bool fp32 = h->precision == LKP_F32;
  if (t == 1) {
    if (fp32) HIP_TRY(launch_fill_f32((float *)h->f[out], 0.0f, n, s));
    else HIP_TRY(launch_fill_f64((double *)h->f[out], 0.0, n, s));
    return LKP_OK;
  }
  StencilParams p = stencil_params(h);
  stencil_weights(h, fp32, &p);
  p.xin = h->f[in];
  p.xout = h->f[out];
  p.src = h->S;
  HIP_TRY(launch_stencil(h->lattice, fp32 ? SMODE_F32 : SMODE_F64, flags, p, s));
  return LKP_OK;
}

unsigned scalar_blocks(const lkp_handle *h) {
  return stencil_blocks(h->lattice, (unsigned)h->n[0], (unsigned)h->n[1], (unsigned)h->n[2], h->stile);
}

// Enqueue a chunk of k >= 1 sweeps whose last sweep reduces norms: with
// `pair` against the Phi of the sweep before it (for k = 1 the Phi stored
// last), else against the Phi of the previous check in phib[0], writing
// phib[1] and copying it to phib[0].  Updates cur.
lkp_status enqueue_chunk(lkp_handle *h, hipStream_t s, int k, bool pair) {
  int cur = h->cur;
  if (h->scalar) {
    for (int j = 0; j < k; ++j) {
      const int flags = j == k - 1 ? FLAG_REDUCE : 0;
      if (lkp_status st = scalar_sweep(h, s, h->total_sweeps + j + 1, cur, 1 - cur, flags)) return st;
      cur = 1 - cur;
    }
    return LKP_OK;
  }
  const bool two = k >= 2 && pair;
  for (int j = 0; j < k - (two ? 2 : 1); ++j) {
    if (lkp_status st = enqueue_sweep(h, s, cur, 1 - cur, 0, nullptr, nullptr)) return st;
    cur = 1 - cur;
  }
  if (!pair) {
    if (lkp_status st = enqueue_sweep(h, s, cur, 1 - cur, FLAG_REDUCE, h->phib[0], h->phib[1]))
      return st;
    HIP_TRY(launch_copy_f64(h->phib[1], h->phib[0], h->ncells, s));
    cur = 1 - cur;
  } else if (two) {
    if (lkp_status st = enqueue_sweep(h, s, cur, 1 - cur, FLAG_PHI, nullptr, h->phib[0])) return st;
    cur = 1 - cur;
    if (lkp_status st = enqueue_sweep(h, s, cur, 1 - cur, FLAG_REDUCE, h->phib[0], h->phib[1]))
      return st;
    cur = 1 - cur;
  } else {
    const int a = h->phi_last, b = 1 - h->phi_last;
    if (lkp_status st = enqueue_sweep(h, s, cur, 1 - cur, FLAG_REDUCE, h->phib[a], h->phib[b]))
      return st;
    cur = 1 - cur;
  }
  return LKP_OK;
}

lkp_status run_chunk(lkp_handle *h, int k, bool use_graph, bool pair) {
  if (h->scalar && h->total_sweeps == 0) use_graph = false;  // sweep 1 is a fill
  if (use_graph && k >= 2) {
    // the split is part of the key: a graph launches one split's kernels and
    // its norm finish covers that split's blocks
    const long key = (((long)k * 2 + h->cur) * 2 + (pair ? 1 : 0)) * 8 + h->split;
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
      if (!h->capture) HIP_TRY(hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking));
      HIP_TRY(hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal));
      lkp_status st = enqueue_chunk(h, h->capture, k, pair);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(h->capture, &g);
      if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(LKP_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(LKP_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
      it = h->graphs.emplace(key, ex).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, h->stream));
  } else {
    if (lkp_status st = enqueue_chunk(h, h->stream, k, pair)) return st;
  }
  commit_chunk(h, k, pair || h->scalar);
  return LKP_OK;
}

void drop_graphs(lkp_handle *h) {
  for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  h->graphs.clear();
}

lkp_status upload_coefficients(lkp_handle *h) {
  const int Q = h->Q;
  h->c64.assign(2 * Q, 0.0);
  h->c32.assign(2 * Q, 0.0f);
  for (int i = 0; i < Q; ++i) {
    h->c64[i] = h->omega * h->phi[i];
    h->c64[Q + i] = h->chi[i];
    h->c32[i] = (float)h->c64[i];
    h->c32[Q + i] = (float)h->chi[i];
  }
  if (h->refined() && !h->scalar)
    HIP_TRY(hipMemcpy(h->phi_dev, h->phi.data(), Q * sizeof(double), hipMemcpyHostToDevice));
  return LKP_OK;
}

void release(lkp_handle *h) {
  drop_graphs(h);
  for (void *p : h->owned) (void)hipFree(p);  // a caller's workspace is not ours to free
  h->owned.clear();
  if (h->norms_host) (void)hipHostFree(h->norms_host);
  if (h->capture) (void)hipStreamDestroy(h->capture);
}

// Geometry and coefficients of a BF16 deviation-storage sweep (buffers unset).
DevParams dev_params(const lkp_handle *h) {
  DevParams p{};
  p.om1 = (float)(1.0 - h->omega);
  p.nx = (unsigned)h->n[0];
  p.ny = (unsigned)h->n[1];
  p.nz = (unsigned)h->n[2];
  p.ncells = h->ncells;
  p.plane = h->ncells;
  p.simple_wrap = h->simple_wrap ? 1u : 0u;
  p.partials = h->partials;
  for (int i = 0; i < h->Q; ++i) {
    p.phi[i] = (float)h->phi[i];
    p.chi[i] = (float)h->chi[i];
  }
  return p;
}

StencilParams stencil_params(const lkp_handle *h) {
  StencilParams p{};
  p.nx = (unsigned)h->n[0];
  p.ny = (unsigned)h->n[1];
  p.nz = (unsigned)h->n[2];
  p.simple_wrap = h->simple_wrap ? 1u : 0u;
  p.partials = h->partials;
  p.tile = (unsigned)h->stile;
  p.remap = h->sremap;
  return p;
}

// Pick the 3D stencil's tile variant and block order by timing each
// candidate on the handle's own buffers (a few sweeps from the current Phi
// into the idle buffer: the state is unchanged).  The variants of one family
// (velocity by velocity, separable, or plane sums) give the same bits; the
// families differ by rounding.  A variant a grid does not take (the
// LDS-staged plane sums on rows of a ragged 16-byte length) is refused before
// it launches and passed over.  Cached per process and (set, mode, size
// class); LKP_STENCIL_TILE / LKP_STENCIL_REMAP force a choice, LKP_AUTOTUNE=0
// and grids below 2^18 cells keep the default (the smallest plane-sum tile).
lkp_status tune_stencil(lkp_handle *h) {
  if (h->dim != 3) return LKP_OK;
  h->stile = kStencilDefault3;
  h->sremap = 0;
  const char *ft = std::getenv("LKP_STENCIL_TILE");
  const char *fr = std::getenv("LKP_STENCIL_REMAP");
  if (ft || fr) {
    if (ft) h->stile = std::max(0, std::min(kStencilTiles3 - 1, std::atoi(ft)));
    if (fr) h->sremap = (unsigned)std::max(0, std::atoi(fr));
    return LKP_OK;
  }
  const char *off = std::getenv("LKP_AUTOTUNE");
  if ((off && std::atoi(off) == 0) || h->ncells < (1u << 18)) return LKP_OK;
  const bool fp32 = h->precision != LKP_F64;
  const long key = tune_key(h->lattice, 16 + (fp32 ? 1 : 0), h->ncells);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_stile.find(key);
    if (it != g_stile.end()) {
      h->stile = it->second.first;
      h->sremap = it->second.second;
      return LKP_OK;
    }
  }
  StencilParams p = stencil_params(h);
  stencil_weights(h, fp32, &p);
  if (h->precision == LKP_F32_IR) {
    p.xin = h->d32[0];
    p.xout = h->d32[1];
    p.src = h->S32;
  } else {
    p.xin = h->f[h->cur];
    p.xout = h->f[1 - h->cur];
    p.src = h->S;
  }
  const int smode = fp32 ? SMODE_F32 : SMODE_F64;
  hipEvent_t e0, e1;
  LKP_HIP_TRY(hipEventCreate(&e0));
  LKP_HIP_TRY(hipEventCreate(&e1));
  // two passes over the candidates, each timed on its own and kept at its
  // slower pass: a candidate timed while the GPU is still cool (clocks not
  // yet settled under load) must not win by that alone
  constexpr unsigned kRemaps[3] = {0u, 4u, 16u};
  float worst[kStencilTiles3][3] = {};
  for (int pass = 0; pass < 2; ++pass)
    for (int t = 0; t < kStencilTiles3; ++t)
      for (int ri = 0; ri < 3; ++ri) {
        p.tile = (unsigned)t;
        p.remap = kRemaps[ri];
        if (launch_stencil(h->lattice, smode, 0, p, h->stream) == hipErrorInvalidValue) {
          worst[t][ri] = 1e30f;  // a variant this set does not take (returned before launching)
          continue;
        }
        LKP_HIP_TRY(hipEventRecord(e0, h->stream));
        for (int k = 0; k < 5; ++k) LKP_HIP_TRY(launch_stencil(h->lattice, smode, 0, p, h->stream));
        LKP_HIP_TRY(hipEventRecord(e1, h->stream));
        LKP_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0;
        LKP_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        worst[t][ri] = std::max(worst[t][ri], ms);
      }
  float best = 1e30f;
  int bt = 0;
  unsigned br = 0;
  for (int t = 0; t < kStencilTiles3; ++t)
    for (int ri = 0; ri < 3; ++ri)
      if (worst[t][ri] < best) {
        best = worst[t][ri];
        bt = t;
        br = kRemaps[ri];
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->stile = bt;
  h->sremap = br;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_stile[key] = {bt, br};
  return LKP_OK;
}

// Per-orbit stencil weights from per-velocity values (equal on an orbit).
void orbit_weights(const lkp_handle *h, const std::vector<double> &per_velocity, bool fp32,
                   StencilParams *p) {
  const VelTable T = velocity_table(h->lattice);
  const VelMaps M = build_maps(T);
  for (int i = 0; i < T.q; ++i) {
    const int o = M.orbit[i];
    if (fp32) p->coef.f[o] = (float)per_velocity[i];
    else p->coef.d[o] = per_velocity[i];
  }
}

// phi_i (omega = 1) as stencil weights in the given precision
void stencil_weights(const lkp_handle *h, bool fp32, StencilParams *p) {
  orbit_weights(h, h->phi, fp32, p);
}

unsigned partial_blocks(int lattice, const int64_t n[3]) {
  const unsigned ncells = (unsigned)(n[0] * n[1] * n[2]);
  const unsigned a = (ncells + cells_per_block(4) - 1) / cells_per_block(4);
  const unsigned b = stencil_blocks_max(lattice, (unsigned)n[0], (unsigned)n[1], (unsigned)n[2]);
  return std::max(a, b) + 8;
}

unsigned partial_blocks(const lkp_handle *h) { return partial_blocks(h->lattice, h->n); }

// Fill a stencil-form handle whose device memory was just planned.
lkp_status create_scalar(lkp_handle *h, DevAlloc &A, double *S_dev, double *G_dev,
                         const std::vector<double> &S) {
  {  // phi_i and chi_i must be equal on every orbit for per-orbit stencil weights
    const VelTable T = velocity_table(h->lattice);
    const VelMaps M = build_maps(T);
    std::vector<int> rep(num_orbits(T), -1);
    for (int i = 0; i < T.q; ++i) {
      const int o = M.orbit[i];
      if (rep[o] < 0) rep[o] = i;
      else if (h->phi[i] != h->phi[rep[o]] || h->chi[i] != h->chi[rep[o]])
        return fail(LKP_ERR_HIP, "coefficients differ within a velocity orbit");
    }
  }
  const size_t n = h->ncells;
  h->S_host = S;
  if (lkp_status st = upload_coefficients(h)) return st;
  // G = sum_i chi_i S(x - v_i), once, with the FP64 stencil
  double *G = G_dev ? G_dev : (double *)h->S;
  HIP_TRY(hipMemcpy(S_dev, S.data(), n * 8, hipMemcpyHostToDevice));
  StencilParams p = stencil_params(h);
  orbit_weights(h, h->chi, false, &p);
  p.xin = S_dev;
  p.xout = G;
  p.src = nullptr;
  HIP_TRY(launch_stencil(h->lattice, SMODE_F64, 0, p, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  A.drop(h, S_dev);
  if (h->precision == LKP_F32) {
    HIP_TRY(launch_f64_to_f32(G, (float *)h->S, n, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    A.drop(h, G_dev);
    HIP_TRY(launch_fill_f32((float *)h->f[0], 0.0f, n, h->stream));
  } else {
    HIP_TRY(launch_fill_f64((double *)h->f[0], 0.0, n, h->stream));
  }
  if (h->precision == LKP_F32_IR) {
    HIP_TRY(launch_f64_to_f32((const double *)h->S, h->S32, n, h->stream));
    // residual of x = 0 is G
    std::vector<double> Gh(n);
    HIP_TRY(hipMemcpy(Gh.data(), h->S, n * 8, hipMemcpyDeviceToHost));
    long double g2 = 0;
    for (double v : Gh) g2 += (long double)v * v;
    h->g_norm = (double)std::sqrt(g2);
    const double one = 1.0;
    HIP_TRY(hipMemcpy(h->phi_dev, &one, sizeof(double), hipMemcpyHostToDevice));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->split = 1;
  h->tuned = true;
  return tune_stencil(h);
}

// Host-side set-up of a handle from a description: validation, constants,
// the stencil / in-place choice (no device memory, no source).
lkp_status init_handle(const lkp_problem_desc *d, lkp_handle *h) {
  LatticeConstants lc;
  double tau;
  if (lkp_status st = validate_desc(d, &lc, &tau)) return st;
  h->lattice = d->lattice;
  h->order = d->order;
  h->dim = d->dim;
  h->precision = d->precision;
  h->Q = lc.table.q;
  for (int a = 0; a < 3; ++a) h->n[a] = d->n[a];
  h->ncells = (unsigned)(d->n[0] * d->n[1] * d->n[2]);
  h->tau_lb = tau;
  h->omega = 1.0 / tau;
  h->cs2 = (double)lc.cs2;
  h->stream = (hipStream_t)d->stream;
  std::vector<long double> phi, chi;
  if (!shape_coefficients(lc, d->order, &phi, &chi))
    return fail(LKP_ERR_LATTICE_ORDER, "no coefficients for order %d", d->order);
  h->drift = has_drift(d);
  if (h->drift) {
    // advection-diffusion: the equilibrium of the Gaussian moved by u, to
    // second order in u (first moment u, second moment c_s^2 delta + u u)
    const long double c2 = lc.cs2;
    long double u2 = 0;
    for (int a = 0; a < 3; ++a) u2 += (long double)d->drift[a] * d->drift[a];
    for (int i = 0; i < h->Q; ++i) {
      long double vu = 0;
      for (int a = 0; a < 3; ++a) vu += (long double)lc.table.v[i][a] * d->drift[a];
      phi[i] += lc.w[i] * (vu / c2 + (vu * vu - c2 * u2) / (2 * c2 * c2));
    }
  }
  h->w.resize(h->Q);
  h->phi.resize(h->Q);
  h->chi.resize(h->Q);
  for (int i = 0; i < h->Q; ++i) {
    h->w[i] = (double)lc.w[i];
    h->phi[i] = (double)phi[i];
    h->chi[i] = (double)chi[i];
  }
  h->rho_bound = contraction_bound(lc.table, h->dim, h->phi.data(), h->omega, h->n);
  h->simple_wrap = h->n[0] >= max_component(lc.table, 0) && h->n[1] >= max_component(lc.table, 1) &&
                   h->n[2] >= max_component(lc.table, 2);
  // omega = 1 exactly: run the scalar stencil form unless populations are asked
  // for (or a drift makes phi_i differ within a velocity orbit)
  h->scalar = (h->omega == 1.0) && !(d->flags & LKP_FLAG_POPULATION_SWEEP) && !h->drift;
  if (h->scalar && h->bf16dev())
    return fail(LKP_ERR_UNSUPPORTED,
                "BF16DEV_IR at tau_lb = 1: the stencil form keeps no populations (the deviation "
                "is exactly chi_i S); set LKP_FLAG_POPULATION_SWEEP or use F32_IR");
  h->inplace = !h->scalar && (d->flags & LKP_FLAG_IN_PLACE) != 0;
  if (h->inplace && h->bf16dev())
    return fail(LKP_ERR_UNSUPPORTED, "LKP_FLAG_IN_PLACE is not available for BF16DEV_IR");
  return LKP_OK;
}

// Bytes the description's device memory takes (the allocation plan walked
// without allocating); 0 if the description is invalid.
int64_t plan_bytes(const lkp_problem_desc *d) {
  lkp_handle h;
  if (init_handle(d, &h) != LKP_OK) return 0;
  DevAlloc A;
  A.count_only = true;
  double *ts = nullptr, *tg = nullptr;
  if (plan_state(&h, A, &ts, &tg) != LKP_OK) return 0;
  return (int64_t)A.used;
}

lkp_status create_impl(const lkp_problem_desc *d, lkp_handle *h) {
  if (lkp_status st = init_handle(d, h)) return st;
  // source: host copy, mean check, scaling S = s c_s^2 (tau_lb - 1/2)
  if (!d->source) return fail(LKP_ERR_ARG, "null source");
  const size_t n = h->ncells;
  std::vector<double> s(n);
  if (d->source_on_device)
    HIP_TRY(hipMemcpy(s.data(), d->source, n * sizeof(double), hipMemcpyDeviceToHost));
  else
    std::memcpy(s.data(), d->source, n * sizeof(double));
  long double sum = 0, amax = 0;
  for (double v : s) {
    if (!std::isfinite(v)) return fail(LKP_ERR_ARG, "source has non-finite values");
    sum += v;
    amax = std::max(amax, (long double)std::fabs(v));
  }
  const double mean = (double)(sum / (long double)n);
  if (std::fabs(mean) > 1e-12 * (double)amax && n > 1) {
    if (!d->subtract_mean)
      return fail(LKP_ERR_SOURCE_MEAN,
                  "source mean %g is not zero: a periodic Poisson problem needs a zero-mean "
                  "source (set subtract_mean to remove it)", mean);
  }
  const bool remove = d->subtract_mean != 0;
  const double scale = h->cs2 * (h->tau_lb - 0.5);
  std::vector<double> S(n);
  for (size_t c = 0; c < n; ++c) S[c] = (remove ? s[c] - mean : s[c]) * scale;

  // device memory: the caller's workspace, or owned allocations
  if (d->workspace && d->workspace_bytes <= 0) return fail(LKP_ERR_ARG, "workspace without a size");
  if (!d->workspace && d->workspace_bytes != 0) return fail(LKP_ERR_ARG, "workspace size without a workspace");
  DevAlloc A;
  A.base = static_cast<char *>(d->workspace);
  A.cap = d->workspace ? (size_t)d->workspace_bytes : 0;
  if (A.base && (reinterpret_cast<uintptr_t>(A.base) & 255))
    return fail(LKP_ERR_ARG, "workspace must be 256-byte aligned");
  double *tmp_S = nullptr, *tmp_G = nullptr;
  if (lkp_status st = plan_state(h, A, &tmp_S, &tmp_G)) return st;
  h->footprint = (int64_t)A.used;  // the plan's size, owned or in the workspace
  h->external = A.base != nullptr;
  HIP_TRY(hipHostMalloc(&h->norms_host, NUM_NORMS * sizeof(double), hipHostMallocDefault));
  if (h->scalar) return create_scalar(h, A, tmp_S, tmp_G, S);

  const size_t Q = h->Q;
  if (h->precision == LKP_F64) {
    HIP_TRY(hipMemcpy(h->S, S.data(), n * 8, hipMemcpyHostToDevice));
  } else if (h->precision == LKP_F32) {
    std::vector<float> S32(n);
    for (size_t c = 0; c < n; ++c) S32[c] = (float)S[c];
    HIP_TRY(hipMemcpy(h->S, S32.data(), n * 4, hipMemcpyHostToDevice));
  } else {
    if (h->inplace && !h->bf16dev()) {
      const VelTable T = velocity_table(h->lattice);
      const VelMaps M = build_maps(T);
      std::vector<int> opp(Q);
      for (size_t i = 0; i < Q; ++i) opp[i] = M.vidx[6 - T.v[i][0]][6 - T.v[i][1]][6 - T.v[i][2]];
      HIP_TRY(hipMemcpy(h->opp_dev, opp.data(), Q * sizeof(int), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(h->S, S.data(), n * 8, hipMemcpyHostToDevice));
    std::vector<float> S32(n);
    long double s2 = 0, c2 = 0;
    for (size_t c = 0; c < n; ++c) {
      S32[c] = (float)S[c];
      s2 += (long double)S[c] * S[c];
    }
    for (int i = 0; i < h->Q; ++i) c2 += (long double)h->chi[i] * h->chi[i];
    h->g_norm = (double)std::sqrt(s2 * c2);
    HIP_TRY(hipMemcpy(h->S32, S32.data(), n * 4, hipMemcpyHostToDevice));
  }
  if (lkp_status st = upload_coefficients(h)) return st;

  // initial state f* = 0 (fill kernels, not memset), Phi buffers = 0
  if (h->precision == LKP_F32) {
    HIP_TRY(launch_fill_f32((float *)h->f[0], 0.0f, Q * n, h->stream));
  } else {
    HIP_TRY(launch_fill_f64((double *)h->f[0], 0.0, Q * n, h->stream));
  }
  HIP_TRY(launch_fill_f64(h->phib[0], 0.0, n, h->stream));
  HIP_TRY(launch_fill_f64(h->phib[1], 0.0, n, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->split = h->bf16dev() ? dev_split(h->lattice)
                          : default_split(h->Q, h->precision == LKP_F32_IR ? MODE_INNER : h->mode());
  return LKP_OK;
}

// In-place layouts <-> the pull layout f*_i(y) (host copies, FP64).
//   phase 0 (swapped): f*_i(y) at plane opp(i), cell y
//   phase 1 (pushed):  f*_i(y) at plane i, cell y + v_i
void inplace_to_pull(const lkp_handle *h, int phase, const std::vector<double> &raw,
                     std::vector<double> &out) {
  const VelTable T = velocity_table(h->lattice);
  const VelMaps M = build_maps(T);
  const int64_t nx = h->n[0], ny = h->n[1], nz = h->n[2], n = h->ncells;
  out.assign(raw.size(), 0.0);
  for (int i = 0; i < h->Q; ++i) {
    const int oi = M.vidx[6 - T.v[i][0]][6 - T.v[i][1]][6 - T.v[i][2]];
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
          const int64_t c = (z * ny + y) * nx + x;
          if (phase == 0) {
            out[(size_t)i * n + c] = raw[(size_t)oi * n + c];
          } else {
            const int64_t xs = ((x + T.v[i][0]) % nx + nx) % nx, ys = ((y + T.v[i][1]) % ny + ny) % ny,
                          zs = ((z + T.v[i][2]) % nz + nz) % nz;
            out[(size_t)i * n + c] = raw[(size_t)i * n + (zs * ny + ys) * nx + xs];
          }
        }
  }
}

void pull_to_swapped(const lkp_handle *h, const std::vector<double> &in, std::vector<double> &raw) {
  const VelTable T = velocity_table(h->lattice);
  const VelMaps M = build_maps(T);
  const size_t n = h->ncells;
  raw.assign(in.size(), 0.0);
  for (int i = 0; i < h->Q; ++i) {
    const int oi = M.vidx[6 - T.v[i][0]][6 - T.v[i][1]][6 - T.v[i][2]];
    std::memcpy(&raw[(size_t)oi * n], &in[(size_t)i * n], n * sizeof(double));
  }
}

}  // namespace

// ================================================================== C ABI

extern "C" {

const char *lkp_last_error(void) { return lkp::rt::last_error(); }

lkp_status lkp_contraction_bound(const lkp_problem_desc *d, double *rho) {
  if (!rho) return fail(LKP_ERR_ARG, "null output pointer");
  lkp_handle h;
  if (lkp_status st = init_handle(d, &h)) return st;
  *rho = h.rho_bound;
  clear_error();
  return LKP_OK;
}

int64_t lkp_footprint_bytes(const lkp_problem_desc *d) {
  const std::string keep = lkp::rt::last_error();
  const int64_t b = plan_bytes(d);
  if (b == 0) lkp::rt::fail(LKP_OK, "%s", keep.c_str());
  return b;
}

lkp_status lkp_create(const lkp_problem_desc *d, lkp_handle **out) {
  if (!out) return fail(LKP_ERR_ARG, "null output handle pointer");
  *out = nullptr;
  lkp_handle *h = new lkp_handle();
  lkp_status st = create_impl(d, h);
  if (st != LKP_OK) {
    release(h);
    delete h;
    return st;
  }
  *out = h;
  clear_error();
  return LKP_OK;
}

lkp_status lkp_destroy(lkp_handle *h) {
  if (!h) return LKP_OK;
  if (h->group) lkp_group_remove(h->group, h);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  release(h);
  delete h;
  return LKP_OK;
}

lkp_status lkp_step(lkp_handle *h, int64_t sweeps) {
  if (!h || sweeps < 0) return fail(LKP_ERR_ARG, "lkp_step: bad arguments");
  if (sweeps == 0) return LKP_OK;
  if (h->bf16dev()) {  // plain sweeps with BF16 deviation storage, no refinement
    if (h->group) return fail(LKP_ERR_STATE, "lkp_step: the handle is resident in a group");
    if (!h->dev_plain) {  // start from rest
      const size_t QN = (size_t)h->Q * h->ncells;
      HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(h->dn[0]), 0u, (QN + 1) / 2, h->stream));
      HIP_TRY(launch_fill_f32(h->dphi[0], 0.0f, h->ncells, h->stream));
      h->dev_cur = 0;
      h->dev_plain = true;
    }
    for (int64_t j = 0; j < sweeps; ++j) {
      DevParams p = dev_params(h);
      p.nin = h->dn[h->dev_cur];
      p.nout = h->dn[1 - h->dev_cur];
      p.phin = h->dphi[h->dev_cur];
      p.phout = h->dphi[1 - h->dev_cur];
      p.src = h->S32;
      hipError_t e = launch_dev(h->lattice, false, 0, p, h->stream);
      if (e != hipSuccess) return fail(LKP_ERR_HIP, "deviation sweep launch: %s", hipGetErrorString(e));
      h->dev_cur = 1 - h->dev_cur;
    }
    h->total_sweeps += sweeps;
    return LKP_OK;
  }
  if (h->refined())
    return fail(LKP_ERR_UNSUPPORTED, "lkp_step drives the plain sweep; refinement handles use lkp_solve");
  if (h->group) return fail(LKP_ERR_STATE, "lkp_step: the handle is resident in a group");
  if (h->scalar) {
    int cur = h->cur;
    for (int64_t j = 0; j < sweeps; ++j) {
      if (lkp_status st = scalar_sweep(h, h->stream, h->total_sweeps + j + 1, cur, 1 - cur, 0)) return st;
      cur = 1 - cur;
    }
    h->cur = cur;
    h->total_sweeps += sweeps;
    HIP_TRY(hipGetLastError());
    return LKP_OK;
  }
  if (lkp_status st = tune_split(h)) return st;
  int cur = h->cur;
  for (int64_t j = 0; j < sweeps - 1; ++j) {
    if (lkp_status st = enqueue_sweep(h, h->stream, cur, 1 - cur, 0, nullptr, nullptr)) return st;
    cur = 1 - cur;
  }
  const int b = 1 - h->phi_last;
  if (lkp_status st = enqueue_sweep(h, h->stream, cur, 1 - cur, FLAG_PHI, nullptr, h->phib[b]))
    return st;
  cur = 1 - cur;
  h->cur = cur;
  h->total_sweeps += sweeps;
  h->phi_last = b;
  h->phi_sweep[b] = h->total_sweeps;
  HIP_TRY(hipGetLastError());
  return LKP_OK;
}

lkp_status lkp_solve(lkp_handle *h, const lkp_solve_opts *o, lkp_solve_report *rep_out) {
  if (!h || !o) return fail(LKP_ERR_ARG, "lkp_solve: null argument");
  if (o->check_every < 1 || o->max_sweeps < 1)
    return fail(LKP_ERR_ARG, "lkp_solve: check_every and max_sweeps must be >= 1");
  if (!(o->tol_rel_l2 > 0) && !(o->tol_maxchange > 0))
    return fail(LKP_ERR_ARG, "lkp_solve: give tol_rel_l2 or tol_maxchange");
  if (h->group) return fail(LKP_ERR_STATE, "lkp_solve: the handle is resident in a group");
  lkp_solve_report rep{};
  const double t_start = now_s();
  const int64_t start = h->total_sweeps;
  lkp_status result = LKP_OK;
  if (lkp_status st = tune_split(h)) return st;
  // the convergence history of the plain sweep carries over from an earlier
  // call on the same state, so a resumed solve measures its contraction
  // across the calls (it is reset when the state is set or a group admits
  // the handle)

  if (h->refined()) {
    if (!(o->tol_rel_l2 > 0)) return fail(LKP_ERR_ARG, "refinement (F32_IR, BF16DEV_IR) needs tol_rel_l2");
    h->dev_plain = false;
    // a resumed solve starts a fresh refinement from the current x
    ir_reset(h);
    int K = std::max(2, o->check_every);
    if (h->inplace) K += K & 1;  // corrections end each chunk in the swapped layout
    bool converged = false;
    while (!converged) {
      double nr[NUM_NORMS];
      if (h->ir.phase == IR_START)
        if (lkp_status st = ir_begin_inner(h, *o)) return st;
      if (h->ir.phase == IR_RESID) {
        if (lkp_status st = ir_launch_residual(h, h->norms_dev)) return st;
        if (lkp_status st = read_back(h, nr)) return st;
        result = ir_after_residual(h, nr, *o, &rep, &converged);
        if (result || converged) break;
      }
      if (h->total_sweeps - start >= o->max_sweeps) {
        if (h->ir.phase == IR_INNER && h->ir.t_in > 0)  // keep the inner work done so far
          if (lkp_status st = ir_apply_correction(h, &rep, true)) return st;
        result = fail(LKP_ERR_NOT_CONVERGED, "refinement: max_sweeps reached");
        break;
      }
      // one chunk of K inner FP32 sweeps, norms on the last two
      const int P = h->split;
      if (h->scalar) {
        for (int j = 0; j < K; ++j) {
          StencilParams p = stencil_params(h);
          stencil_weights(h, true, &p);
          p.xin = h->d32[h->ir.dc];
          p.xout = h->d32[1 - h->ir.dc];
          p.src = h->ir.first ? (const void *)h->S32 : (const void *)h->r32;
          HIP_TRY(launch_stencil(h->lattice, SMODE_F32, j == K - 1 ? FLAG_REDUCE : 0, p, h->stream));
          h->ir.dc = 1 - h->ir.dc;
        }
        h->total_sweeps += K;
        if (lkp_status st = finish_norms(h, scalar_blocks(h), h->norms_dev, h->stream)) return st;
        if (lkp_status st = read_back(h, nr)) return st;
        result = ir_after_inner(h, nr, K, *o, &rep);
        if (result) break;
        continue;
      }
      if (h->bf16dev()) {  // BF16 deviation-storage inner sweeps
        for (int j = 0; j < K; ++j) {
          DevParams p = dev_params(h);
          p.nin = h->dn[h->ir.dc];
          p.nout = h->dn[1 - h->ir.dc];
          p.phin = h->dphi[h->ir.dc];
          p.phout = h->dphi[1 - h->ir.dc];
          const bool inner = !h->ir.first;
          p.src = inner ? h->r32 : h->S32;
          hipError_t e = launch_dev(h->lattice, inner, j == K - 1 ? FLAG_REDUCE : 0, p, h->stream);
          if (e != hipSuccess) return fail(LKP_ERR_HIP, "deviation sweep launch: %s", hipGetErrorString(e));
          h->ir.dc = 1 - h->ir.dc;
        }
        h->total_sweeps += K;
        if (lkp_status st = finish_norms(h, dev_blocks(h->lattice, h->ncells), h->norms_dev, h->stream))
          return st;
        if (lkp_status st = read_back(h, nr)) return st;
        result = ir_after_inner(h, nr, K, *o, &rep);
        if (result) break;
        continue;
      }
      for (int j = 0; j < K; ++j) {
        SweepParams p = ir_inner_params(h, P);
        int flags = 0;
        if (j == K - 2) { flags = FLAG_PHI; p.phi_out = h->phib[0]; }
        if (j == K - 1) { flags = FLAG_REDUCE; p.phi_prev = h->phib[0]; p.phi_out = h->phib[1]; }
        hipError_t e = launch_sweep(h->lattice, ir_inner_mode(h), P, flags, p, h->stream,
                                    aa_of(h, h->ir.dc));
        if (e != hipSuccess) return fail(LKP_ERR_HIP, "inner sweep launch: %s", hipGetErrorString(e));
        h->ir.dc = 1 - h->ir.dc;
      }
      h->total_sweeps += K;
      if (lkp_status st = finish_norms(h, sweep_blocks(h, P), h->norms_dev, h->stream)) return st;
      if (lkp_status st = read_back(h, nr)) return st;
      result = ir_after_inner(h, nr, K, *o, &rep);
      if (result) break;
    }
  } else {
    bool converged = false;
    while (!converged) {
      const int64_t done = h->total_sweeps - start;
      if (done >= o->max_sweeps) {
        result = fail(LKP_ERR_NOT_CONVERGED, "no convergence in %lld sweeps",
                      (long long)o->max_sweeps);
        break;
      }
      const int k = (int)std::min<int64_t>(o->check_every, o->max_sweeps - done);
      // The last sweep's change compares with the Phi of the sweep before it
      // (pair), or, with a relative-L2 tolerance alone, with the Phi stored
      // before the chunk (the change over the whole interval): a slow mode
      // whose one-sweep change hides under faster ones still shows over many
      // sweeps.  span: the sweeps between the two, 0 if no valid Phi exists.
      const bool pair = !interval_checks(h, *o);
      const int a = h->phi_last;
      int64_t span = 0;
      if (pair) {
        span = k >= 2 ? (h->total_sweeps + k >= 2 ? 1 : 0)
                      : (h->phi_sweep[a] == h->total_sweeps && h->total_sweeps >= 1 ? 1 : 0);
      } else if (h->phi_sweep[0] >= 0) {
        span = h->total_sweeps + k - h->phi_sweep[0];
      }
      if (lkp_status st = run_chunk(h, k, o->use_graph != 0, pair)) return st;
      double nr[NUM_NORMS];
      if (h->scalar) {
        if (h->total_sweeps < 2) continue;  // the only sweep was the first (Phi = 0)
        if (lkp_status st = read_norms(h, scalar_blocks(h), nr)) return st;
        result = track_check(h, nr, 1, *o, &rep, &converged);
      } else {
        if (lkp_status st = read_norms(h, sweep_blocks(h, h->split), nr)) return st;
        result = track_check(h, nr, span, *o, &rep, &converged);
      }
      if (result) break;
    }
  }
  rep.wall_s = now_s() - t_start;
  rep.sweeps = h->total_sweeps - start;
  rep.total_sweeps = h->total_sweeps;
  rep.outer = h->refined() ? h->ir.outer : 0;
  rep.glups = rep.wall_s > 0 ? 1e-9 * (double)h->ncells * (double)rep.sweeps / rep.wall_s : 0;
  rep.status = result;
  if (rep_out) *rep_out = rep;
  if (result == LKP_OK) clear_error();
  return result;
}

lkp_status lkp_residual(lkp_handle *h, lkp_residual_report *r) {
  if (!h || !r) return fail(LKP_ERR_ARG, "lkp_residual: null argument");
  std::memset(r, 0, sizeof *r);
  r->sweeps = h->total_sweeps;
  if (h->scalar) {
    if (h->total_sweeps < 1) return fail(LKP_ERR_STATE, "lkp_residual needs at least one sweep");
    const bool fp32 = h->precision == LKP_F32;
    const int x = h->precision == LKP_F32_IR ? 0 : h->cur;
    StencilParams p = stencil_params(h);
    stencil_weights(h, fp32, &p);
    p.xin = h->f[x];
    p.xout = h->precision == LKP_F32_IR ? (void *)h->r32 : h->f[1 - h->cur];
    p.src = h->S;
    HIP_TRY(launch_stencil(h->lattice, fp32 ? SMODE_F32 : SMODE_RESID, FLAG_REDUCE, p, h->stream));
    double nr[NUM_NORMS];
    if (lkp_status st = read_norms(h, scalar_blocks(h), nr)) return st;
    double phi2 = 0;
    for (double v : h->phi) phi2 += v * v;
    r->max_change = nr[NORM_MAX_DPHI];
    r->l2_change = std::sqrt(nr[NORM_SUM_DPHI2]);
    // populations are phi_i Phi + chi_i S, so their residual is phi_i (Phi' - Phi)
    r->pop_residual_l2 = fp32 ? NAN : std::sqrt(phi2) * r->l2_change;
    r->phi_l2 = std::sqrt(nr[NORM_SUM_PHI2]);
    r->mass = nr[NORM_SUM_PHI];
    return LKP_OK;
  }
  const int last = h->phi_last;
  if (h->total_sweeps < 1 || h->phi_sweep[last] != h->total_sweeps)
    return fail(LKP_ERR_STATE, "lkp_residual needs the Phi of the last sweep (run a sweep first)");
  const int scratch = 1 - last;
  double nr[NUM_NORMS];
  if (h->precision == LKP_F64 || h->refined()) {
    // FP64 residual of the FP64 state; r goes to idle storage
    const int P = default_split(h->Q, MODE_RESID);
    SweepParams p = base_params(h);
    const bool f64 = h->precision == LKP_F64;
    p.fin = f64 ? h->f[h->cur] : h->f[0];
    // r goes to the idle buffer; in place there is none and only the norms are kept
    p.fout = f64 ? (h->inplace ? nullptr : h->f[1 - h->cur]) : (void *)h->r32;
    p.src = h->S;
    set_coefficients(h, MODE_RESID, &p);
    p.phi_prev = h->phib[last];
    p.phi_out = h->phib[scratch];
    p.partials = h->partials;
    hipError_t e = launch_sweep(h->lattice, MODE_RESID, P, FLAG_REDUCE, p, h->stream,
                                f64 ? aa_of(h, h->cur) : 0);
    if (e != hipSuccess) return fail(LKP_ERR_HIP, "residual launch: %s", hipGetErrorString(e));
    if (lkp_status st = read_norms(h, sweep_blocks(h, P), nr)) return st;
    r->pop_residual_l2 = std::sqrt(nr[NORM_SUM_R2]);
  } else {
    if (lkp_status st = enqueue_sweep(h, h->stream, h->cur, 1 - h->cur, FLAG_REDUCE, h->phib[last],
                                      h->phib[scratch], h->inplace))
      return st;
    if (lkp_status st = read_norms(h, sweep_blocks(h, h->split), nr)) return st;
    r->pop_residual_l2 = NAN;
  }
  h->phi_sweep[scratch] = -1;
  r->max_change = nr[NORM_MAX_DPHI];
  r->l2_change = std::sqrt(nr[NORM_SUM_DPHI2]);
  r->phi_l2 = std::sqrt(nr[NORM_SUM_PHI2]);
  r->mass = nr[NORM_SUM_PHI];
  return LKP_OK;
}

lkp_status lkp_get_phi(lkp_handle *h, double *dst, int32_t dst_is_device) {
  if (!h || !dst) return fail(LKP_ERR_ARG, "lkp_get_phi: null argument");
  if (h->scalar) {
    if (h->total_sweeps < 1) return fail(LKP_ERR_STATE, "no Phi before the first sweep");
    const size_t n = h->ncells;
    const void *src = h->precision == LKP_F32_IR ? h->f[0] : h->f[h->cur];
    if (h->precision == LKP_F32) {
      double *tmp = dst;
      if (!dst_is_device) HIP_TRY(hipMalloc(&tmp, n * 8));
      HIP_TRY(launch_f32_to_f64((const float *)src, tmp, n, h->stream));
      if (!dst_is_device) {
        HIP_TRY(hipMemcpyAsync(dst, tmp, n * 8, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(hipFree(tmp));
      }
    } else {
      HIP_TRY(hipMemcpyAsync(dst, src, n * 8, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             h->stream));
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LKP_OK;
  }
  if (h->dev_plain) {  // Phi of the plain deviation sweeps (FP32 storage)
    const size_t n = h->ncells;
    double *tmp = dst;
    if (!dst_is_device) HIP_TRY(hipMalloc(&tmp, n * 8));
    HIP_TRY(launch_f32_to_f64(h->dphi[h->dev_cur], tmp, n, h->stream));
    if (!dst_is_device) {
      HIP_TRY(hipMemcpyAsync(dst, tmp, n * 8, hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
      HIP_TRY(hipFree(tmp));
    } else {
      HIP_TRY(hipStreamSynchronize(h->stream));
    }
    return LKP_OK;
  }
  const int last = h->phi_last;
  if (h->phi_sweep[last] != h->total_sweeps || h->total_sweeps < 1)
    return fail(LKP_ERR_STATE, "no Phi for the current state (run a sweep first)");
  HIP_TRY(hipMemcpyAsync(dst, h->phib[last], (size_t)h->ncells * 8,
                         dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LKP_OK;
}

lkp_status lkp_get_populations(lkp_handle *h, double *dst, int32_t dst_is_device) {
  if (!h || !dst) return fail(LKP_ERR_ARG, "lkp_get_populations: null argument");
  if (h->scalar) {  // f*_i = phi_i Phi + chi_i S after any sweep, 0 before the first
    const size_t n = h->ncells, Q = h->Q;
    std::vector<double> phi(n, 0.0), f(Q * n, 0.0);
    if (h->total_sweeps >= 1) {
      if (lkp_status st = lkp_get_phi(h, phi.data(), 0)) return st;
      for (size_t i = 0; i < Q; ++i)
        for (size_t c = 0; c < n; ++c) f[i * n + c] = h->phi[i] * phi[c] + h->chi[i] * h->S_host[c];
    }
    HIP_TRY(hipMemcpy(dst, f.data(), Q * n * 8, dst_is_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
    return LKP_OK;
  }
  const size_t QN = (size_t)h->Q * h->ncells;
  if (h->inplace && !h->refined()) {  // one buffer in one of two layouts: remap to the pull layout
    std::vector<double> raw(QN), out;
    double *tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, QN * 8));
    if (h->precision == LKP_F32) HIP_TRY(launch_f32_to_f64((const float *)h->f[0], tmp, QN, h->stream));
    else HIP_TRY(hipMemcpyAsync(tmp, h->f[0], QN * 8, hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(raw.data(), tmp, QN * 8, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipFree(tmp));
    inplace_to_pull(h, h->cur, raw, out);
    HIP_TRY(hipMemcpy(dst, out.data(), QN * 8, dst_is_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
    return LKP_OK;
  }
  if (h->precision == LKP_F32) {
    double *tmp = dst;
    if (!dst_is_device) HIP_TRY(hipMalloc(&tmp, QN * 8));
    HIP_TRY(launch_f32_to_f64((const float *)h->f[h->cur], tmp, QN, h->stream));
    if (!dst_is_device) {
      HIP_TRY(hipMemcpyAsync(dst, tmp, QN * 8, hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
      HIP_TRY(hipFree(tmp));
    }
  } else {
    const void *srcp = h->precision == LKP_F64 ? h->f[h->cur] : h->f[0];
    HIP_TRY(hipMemcpyAsync(dst, srcp, QN * 8,
                           dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LKP_OK;
}

lkp_status lkp_set_populations(lkp_handle *h, const double *src, int32_t src_is_device) {
  if (!h || !src) return fail(LKP_ERR_ARG, "lkp_set_populations: null argument");
  if (h->scalar)
    return fail(LKP_ERR_UNSUPPORTED, "the tau_lb = 1 stencil form keeps Phi only; create the handle "
                                     "with LKP_FLAG_POPULATION_SWEEP to set populations");
  const size_t QN = (size_t)h->Q * h->ncells;
  if (h->inplace && !h->refined()) {  // store in the swapped layout (phase 0)
    std::vector<double> in(QN), raw;
    HIP_TRY(hipMemcpy(in.data(), src, QN * 8, src_is_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    pull_to_swapped(h, in, raw);
    double *tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, QN * 8));
    HIP_TRY(hipMemcpyAsync(tmp, raw.data(), QN * 8, hipMemcpyHostToDevice, h->stream));
    if (h->precision == LKP_F32) HIP_TRY(launch_f64_to_f32(tmp, (float *)h->f[0], QN, h->stream));
    else HIP_TRY(hipMemcpyAsync(h->f[0], tmp, QN * 8, hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipFree(tmp));
    h->cur = 0;
    h->phi_sweep[0] = h->phi_sweep[1] = -1;
    h->trk = Tracker();
    return LKP_OK;
  }
  const hipMemcpyKind kind = src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (h->precision == LKP_F32) {
    double *tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, QN * 8));
    HIP_TRY(hipMemcpyAsync(tmp, src, QN * 8, kind, h->stream));
    HIP_TRY(launch_f64_to_f32(tmp, (float *)h->f[h->cur], QN, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipFree(tmp));
  } else {
    void *dstp = h->precision == LKP_F64 ? h->f[h->cur] : h->f[0];
    HIP_TRY(hipMemcpyAsync(dstp, src, QN * 8, kind, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  if (h->refined()) h->x_nonzero = true;  // a later solve refines this state
  h->phi_sweep[0] = h->phi_sweep[1] = -1;
  h->trk = Tracker();
  return LKP_OK;
}

lkp_status lkp_set_equilibrium(lkp_handle *h, const double *phi0, int32_t phi0_is_device) {
  if (!h || !phi0) return fail(LKP_ERR_ARG, "lkp_set_equilibrium: null argument");
  if (h->scalar)
    return fail(LKP_ERR_UNSUPPORTED, "the tau_lb = 1 stencil form keeps Phi only; create the handle "
                                     "with LKP_FLAG_POPULATION_SWEEP to start from an equilibrium");
  const size_t n = h->ncells;
  // a host field is staged through the handle's own Phi buffer (its contents
  // are invalidated below anyway): no allocation
  const double *p0 = phi0;
  if (!phi0_is_device) {
    HIP_TRY(hipMemcpyAsync(h->phib[0], phi0, n * 8, hipMemcpyHostToDevice, h->stream));
    p0 = h->phib[0];
  }
  // written straight into the state, in its precision and layout: plane j of
  // the swapped in-place layout holds velocity opp(j)
  const bool swapped = h->inplace && !h->refined();
  EqCoef cf{};
  if (swapped) {
    const VelTable T = velocity_table(h->lattice);
    const VelMaps M = build_maps(T);
    for (int i = 0; i < h->Q; ++i) cf.c[M.vidx[6 - T.v[i][0]][6 - T.v[i][1]][6 - T.v[i][2]]] = h->phi[i];
  } else {
    for (int i = 0; i < h->Q; ++i) cf.c[i] = h->phi[i];
  }
  const bool fp32 = h->precision == LKP_F32;
  void *out = h->refined() ? h->f[0] : h->f[swapped ? 0 : h->cur];
  HIP_TRY(launch_equilibrium(p0, cf, out, fp32, n, h->Q, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (swapped) h->cur = 0;
  if (h->refined()) h->x_nonzero = true;  // a later solve refines this state
  h->phi_sweep[0] = h->phi_sweep[1] = -1;
  h->trk = Tracker();
  clear_error();
  return LKP_OK;
}

lkp_status lkp_lattice_info(int32_t lattice, int32_t order, int32_t *Q, int32_t *dim, int32_t *v,
                            double *w, double *phi, double *chi, double *cs2) {
  if (lattice < 0 || lattice >= LKP_NUM_LATTICES) return fail(LKP_ERR_ARG, "unknown lattice");
  LatticeConstants lc;
  if (!lattice_constants(lattice, &lc)) return fail(LKP_ERR_HIP, "lattice constant solve failed");
  std::vector<long double> ph, ch;
  if ((phi || chi) && !shape_coefficients(lc, order, &ph, &ch))
    return fail(LKP_ERR_LATTICE_ORDER, "order %d not available on this lattice", order);
  const int q = lc.table.q;
  if (Q) *Q = q;
  if (dim) *dim = lc.table.dim;
  if (cs2) *cs2 = (double)lc.cs2;
  for (int i = 0; i < q; ++i) {
    if (v)
      for (int a = 0; a < 3; ++a) v[3 * i + a] = lc.table.v[i][a];
    if (w) w[i] = (double)lc.w[i];
    if (phi) phi[i] = (double)ph[i];
    if (chi) chi[i] = (double)ch[i];
  }
  return LKP_OK;
}

lkp_status lkp_get_coefficients(lkp_handle *h, double *phi, double *chi) {
  if (!h) return fail(LKP_ERR_ARG, "lkp_get_coefficients: null handle");
  for (int i = 0; i < h->Q; ++i) {
    if (phi) phi[i] = h->phi[i];
    if (chi) chi[i] = h->chi[i];
  }
  clear_error();
  return LKP_OK;
}

lkp_status lkp_get_info(lkp_handle *h, lkp_handle_info *info) {
  if (!h || !info) return fail(LKP_ERR_ARG, "lkp_get_info: null argument");
  info->lattice = h->lattice;
  info->order = h->order;
  info->dim = h->dim;
  info->Q = h->Q;
  info->precision = h->precision;
  info->velocity_groups = h->split;
  info->scalar_stencil = h->scalar ? 1 : 0;
  info->in_place = h->inplace ? 1 : 0;
  info->stencil_tile = h->scalar && h->dim == 3 ? h->stile : -1;
  info->stencil_remap = h->scalar && h->dim == 3 ? (int32_t)h->sremap : -1;
  for (int a = 0; a < 3; ++a) info->n[a] = h->n[a];
  info->tau_lb = h->tau_lb;
  info->omega = h->omega;
  info->cs2 = h->cs2;
  info->total_sweeps = h->total_sweeps;
  info->footprint_bytes = h->footprint;
  return LKP_OK;
}

lkp_status lkp_sync(lkp_handle *h) {
  if (!h) return fail(LKP_ERR_ARG, "lkp_sync: null handle");
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LKP_OK;
}

}  // extern "C"
