// Internal runtime shared by the single-problem ABI (lkp.cpp) and the
// batched serving ABI (group.cpp).  Host code only.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "lkp.h"
#include "validate.hpp"

namespace lkp {
namespace rt {

double now_s();

#define LKP_HIP_TRY(expr)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return ::lkp::rt::fail(e_ == hipErrorOutOfMemory ? LKP_ERR_OOM : LKP_ERR_HIP,           \
                             "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)

// Convergence bookkeeping of one problem across checks (Sec. 5: the answer is
// the steady state; the host estimates the distance to it from the one-sweep
// change and the measured contraction per sweep).
// The contraction used for the estimate is the largest of the last four
// measured between checks: where slow modes oscillate or are still emerging,
// a single measurement can be well below the asymptotic rate, and the
// estimate (1 / (1 - rho)) would stop early.
struct Tracker {
  static constexpr int kRates = 4;
  double l2_prev = -1.0;
  double min_l2 = 1e300;
  double rate = 0.0;            // contraction used for the estimate
  double rates[kRates] = {0, 0, 0, 0};  // last measured per-sweep contractions
  int nrates = 0;
  int64_t t_prev = -1;
  int64_t span_prev = 0;        // sweeps between the two Phi the previous check compared
};

// Iterative-refinement controller state of one F32_IR problem.
// IR_START: the first solve (from x = 0) has the plain source chi_i S, so it
// runs the plain FP32 sweep; later corrections solve with the population
// residual r as source (MODE_INNER).  A refinement resumed on a state that is
// not zero starts at IR_RESID with first = false.
enum IrPhase : int { IR_START = 0, IR_RESID = 1, IR_INNER = 2, IR_DONE = 3 };
struct IrState {
  int phase = IR_START;
  bool first = true;          // the next inner solve is the first solve from x = 0
  int outer = 0;
  double rnorm = -1.0, rnorm_prev = -1.0;
  double corr = 0.0, corr_prev = -1.0;
  double left = -1.0;         // the last correction's own estimate of its remaining error (Phi norm)
  double est_in = -1.0;       // the running inner solve's latest such estimate
  double est = 1.0;           // estimated relative error of x (1 for x = 0)
  double inner_tol = 1e-4;    // relative accuracy the current inner solve aims at
  int dc = 0;                 // current inner correction buffer
  double l2_prev = -1.0, best_l2 = 1e300, rate = 0.0;
  int stall = 0;
  int64_t t_in = 0, t_prev = 0;
};

}  // namespace rt
}  // namespace lkp

struct lkp_handle {
  int lattice = 0, order = 0, dim = 0, precision = 0, Q = 0;
  int64_t n[3] = {1, 1, 1};
  unsigned ncells = 0;
  double tau_lb = 0, omega = 0, cs2 = 0;
  double rho_bound = 0;      // slowest decay the grid's modes allow (rt::contraction_bound)
  std::vector<double> w, phi, chi;
  bool drift = false;       // advection-diffusion handle (nonzero drift in phi_i)
  std::vector<double> c64;  // [omega phi_i]_Q, [chi_i]_Q (FP64 sweeps, residual)
  std::vector<float> c32;   // the same rounded to FP32 (FP32 and IR inner sweeps)
  hipStream_t stream = nullptr;
  hipStream_t capture = nullptr;  // private stream used only to record graphs
  bool simple_wrap = true;

  // population state: F64 -> f[] double; F32 -> f[] float; F32_IR -> f[0] = x
  // (double) with d32[] the FP32 corrections and r32 the FP32 residual
  void *f[2] = {nullptr, nullptr};
  int cur = 0;
  void *S = nullptr;          // scaled source in the sweep precision (double for IR)
  float *S32 = nullptr;       // IR: the scaled source rounded to FP32 (first solve)
  double g_norm = 0.0;        // IR: ||chi_i S||_2, the residual of x = 0
  // omega = 1: the state is Phi alone and a sweep is the stencil
  // Phi' = sum_i phi_i Phi(x - v_i) + G.  f[0], f[1] (n values each) hold Phi,
  // S holds G (not S), r32 / d32 / S32 are n-sized (IR: R, D, G in FP32).
  bool scalar = false;
  std::vector<double> S_host;  // the scaled source S (to rebuild populations)
  double *phi_dev = nullptr;  // phi_i on the device (IR mass projection)
  float *r32 = nullptr;
  float *d32[2] = {nullptr, nullptr};
  // BF16DEV_IR: the correction as phi_i Phi + n_i (n_i BF16 planes, Phi FP32)
  uint16_t *dn[2] = {nullptr, nullptr};
  float *dphi[2] = {nullptr, nullptr};
  bool inplace = false;     // LKP_FLAG_IN_PLACE: f[1] == f[0] (d32[1] == d32[0] for F32_IR)
  bool x_nonzero = false;   // refinement: x has been updated or set (not the zero state)
  int *opp_dev = nullptr;   // in place + F32_IR: opposite-velocity map for the update
  int dev_cur = 0;          // current (dn, dphi) of plain deviation sweeps (lkp_step)
  bool dev_plain = false;   // Phi comes from plain deviation sweeps (lkp_step since the last solve)
  double *phib[2] = {nullptr, nullptr};
  int64_t phi_sweep[2] = {-1, -1};
  int phi_last = 1;
  double *partials = nullptr;
  size_t partial_cap = 0;
  double *norms_dev = nullptr;
  double *norms_host = nullptr;  // pinned
  int64_t total_sweeps = 0;
  int64_t footprint = 0;     // device bytes of the state (the allocation plan's size)
  bool external = false;     // the state lives in a caller's workspace
  std::vector<void *> owned; // device allocations the handle frees
  int split = 1;
  bool tuned = false;
  int stile = 0;            // 3D stencil form: tile variant and block order (tune_stencil)
  unsigned sremap = 0;
  int solo_split = 1;       // the handle's own split while a group imposes its own
  bool solo_tuned = false;
  std::map<long, hipGraphExec_t> graphs;

  // convergence state (kept across lkp_solve calls; reset when the state is
  // set and at lkp_group_add)
  lkp::rt::Tracker trk;
  lkp::rt::IrState ir;

  // serving: the group this handle is resident in, its stopping options and
  // progress since it was added
  struct lkp_group *group = nullptr;
  lkp_solve_opts gopts{};
  lkp_solve_report grep{};
  int gstate = 0;  // lkp_member_state
  int64_t g_sweeps = 0;

  int mode() const { return precision == LKP_F64 ? lkp::MODE_F64 : lkp::MODE_F32; }
  // FP64 refinement of the population state (FP32 or BF16-deviation inner sweeps)
  bool refined() const { return precision == LKP_F32_IR || precision == LKP_BF16DEV_IR; }
  bool bf16dev() const { return precision == LKP_BF16DEV_IR; }
};

namespace lkp {
namespace rt {

int default_split(int Q, int mode);
unsigned sweep_blocks(const lkp_handle *h, int P);
void set_coefficients(const lkp_handle *h, int mode, SweepParams *p);
SweepParams base_params(const lkp_handle *h);
lkp_status tune_split(lkp_handle *h);
lkp_status finish_norms(lkp_handle *h, unsigned nblocks, double *dst_dev, hipStream_t s);

// Bookkeeping after a chunk of k sweeps: the last two stored / reduced Phi
// (pair), or only the last reduced against the Phi stored before the chunk.
void commit_chunk(lkp_handle *h, int k, bool pair = true);

// Whether a plain solve compares Phi across the whole check interval (the
// K-sweep change) rather than across its last sweep: with a relative-L2
// tolerance alone, on the population state.
bool interval_checks(const lkp_handle *h, const lkp_solve_opts &o);

// Evaluate one check of the plain (F64 / F32) iteration.  span: the sweeps
// between the two Phi the reduced change compares (0: no valid comparison).
// Sets *converged; returns an error status on divergence.
lkp_status track_check(lkp_handle *h, const double nr[NUM_NORMS], int64_t span,
                       const lkp_solve_opts &o, lkp_solve_report *rep, bool *converged);

// F32_IR controller, split so that single and batched drivers share it.
lkp_status ir_launch_residual(lkp_handle *h, double *dst_dev);  // RESID sweep + finish
lkp_status ir_after_residual(lkp_handle *h, const double nr[NUM_NORMS], const lkp_solve_opts &o,
                             lkp_solve_report *rep, bool *converged);
lkp_status ir_begin_inner(lkp_handle *h, const lkp_solve_opts &o);  // d = 0, tolerance
int ir_inner_mode(const lkp_handle *h);             // MODE_F32 (first solve) or MODE_INNER
void ir_reset(lkp_handle *h);                       // fresh controller for the current x
SweepParams ir_inner_params(lkp_handle *h, int P);  // inner sweep d[dc] -> d[1-dc]
lkp_status ir_after_inner(lkp_handle *h, const double nr[NUM_NORMS], int K,
                          const lkp_solve_opts &o, lkp_solve_report *rep);

}  // namespace rt
}  // namespace lkp
