// Launch interface of the gfx950 kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "lattices.hpp"

namespace lkp {

// Precision modes of the fused sweep.
enum SweepMode : int {
  MODE_F64 = 0,    // FP64 in, FP64 out, source chi_i S(x)
  MODE_F32 = 1,    // FP32 in, FP32 out, source chi_i S(x) (S in FP32); FP64 moment sum
  MODE_RESID = 2,  // FP64 in, FP32 out r_i = (T x + g)_i - x_i, FP64 arithmetic
  MODE_INNER = 3,  // FP32 in, FP32 out, population-space source r_i(x) (Q FP32 planes)
  NUM_MODES = 4
};

// Extra work of one sweep.
enum SweepFlags : int {
  FLAG_PHI = 1,     // store Phi (FP64)
  FLAG_REDUCE = 2,  // also per-block partial norms (implies FLAG_PHI)
};

// Partial-norm slots, per block and in the finished result.
enum NormSlot : int {
  NORM_MAX_DPHI = 0,  // max |Phi - Phi_prev|
  NORM_SUM_DPHI2 = 1, // sum (Phi - Phi_prev)^2
  NORM_SUM_PHI2 = 2,  // sum Phi^2
  NORM_SUM_PHI = 3,   // sum Phi
  NORM_BAD = 4,       // count of non-finite Phi / residual values
  NORM_SUM_R2 = 5,    // sum over populations of r_i^2 (MODE_RESID)
  NUM_NORMS = 6
};

struct SweepParams {
  const void *fin;        // Q planes, input precision of the mode
  void *fout;             // Q planes, output precision of the mode
  const void *src;        // S (n values) or r (Q planes) in the mode's source precision
  double om1;             // 1 - omega
  const double *phi_prev; // previous sweep's Phi (FLAG_REDUCE; may be null)
  double *phi_out;        // this sweep's Phi (FLAG_PHI)
  double *partials;       // NUM_NORMS per block (FLAG_REDUCE)
  unsigned nx, ny, nz;
  unsigned ncells;        // nx * ny * nz (< 2^29)
  unsigned plane;         // elements between consecutive population planes (>= ncells)
  unsigned simple_wrap;   // 1 when every axis is at least its largest |v| component
  unsigned nblocks;       // grid size (set by the launcher)
  // [omega phi_i]_Q then [chi_i]_Q in the mode's compute precision, passed by
  // value so the kernel reads them from the constant argument segment
  union {
    double d[2 * MAXQ];
    float f[2 * MAXQ];
  } coef;
};
static_assert(sizeof(SweepParams) <= 4096, "kernel arguments are limited to 4 KiB");

// One problem of a batched launch (same fields as SweepParams, no coefficients).
struct BatchMember {
  const void *fin;
  void *fout;
  const void *src;
  double om1;             // 1 - omega
  double omega;           // omega phi_i is formed in the kernel from the class-wide phi_i
  const double *phi_prev;
  double *phi_out;
  double *partials;
  unsigned nx, ny, nz;
  unsigned ncells;
  unsigned plane;         // elements between consecutive population planes
  unsigned simple_wrap;
  unsigned nblocks;       // this member's blocks
  unsigned block_begin;   // first global block of this member
};

// Members per batched launch: the table and the class-wide phi_i, chi_i
// (FP64) must fit the 4 KiB kernel-argument segment.
constexpr int batch_capacity(int q) {
  const int m = (4000 - 16 * q - 16) / (int)sizeof(BatchMember);
  return m > 32 ? 32 : m;
}

template <int Q>
struct BatchParams {
  unsigned nmembers;
  unsigned nblocks;  // total over members
  BatchMember m[batch_capacity(Q)];
  double phi[Q];
  double chi[Q];
};
static_assert(sizeof(BatchParams<169>) <= 4096, "batched launch arguments exceed 4 KiB");
static_assert(sizeof(BatchParams<111>) <= 4096, "batched launch arguments exceed 4 KiB");
static_assert(sizeof(BatchParams<5>) <= 4096, "batched launch arguments exceed 4 KiB");
static_assert(sizeof(BatchParams<77>) <= 4096, "batched launch arguments exceed 4 KiB");
static_assert(sizeof(BatchParams<107>) <= 4096, "batched launch arguments exceed 4 KiB");

// Cells one block covers for a velocity-group split P (256 threads = 4 waves;
// P waves share one 64-cell column and each holds Q/P populations).
inline unsigned cells_per_block(int P) { return 256u / (unsigned)P; }

// Default split of the refinement's correction sweep (MODE_INNER), measured
// fastest on MI355X: 1 up to 81 velocities, 2 for 107 and 111, 4 for 169.  FP32 first
// solves of a refinement use the same split as the corrections, so every split
// built for MODE_INNER is built for MODE_F32 too; the runtime times the
// candidates.
constexpr int inner_split(int q) { return q >= 169 ? 4 : (q >= 100 ? 2 : 1); }

// Velocity-group splits compiled per (lattice, mode): small sets P = 1; for
// the large ones the candidates the tuner chooses between.
constexpr bool sweep_variant_built(int lattice, int mode, int P) {
  const int q = velocity_table(lattice).q;
  const bool wide = (mode == MODE_F64 || mode == MODE_RESID);
  if (q <= 25) return P == 1;
  if (mode == MODE_RESID) return P == (q >= 169 ? 4 : 2);
  if (mode == MODE_INNER) return q >= 169 ? (P == 2 || P == 4) : (P == 1 || P == 2);
  if (wide) {
    if (q <= 81) return P == 1 || P == 2;
    return P == 2 || P == 4;
  }
  if (q >= 169) return P == 1 || P == 2 || P == 4;
  return P == 1 || P == 2;
}

// Whether a (lattice, mode, P) variant is compiled.
bool sweep_variant_available(int lattice, int mode, int P);

// Per-lattice entry points, one translation unit each (sweep_<lattice>.hip).
template <int LID>
hipError_t launch_lattice_tu(int mode, int P, int aa, int flags, SweepParams p, hipStream_t s);

template <int LID>
hipError_t launch_batch_tu(int mode, int P, int flags, const void *bp, hipStream_t s);

// Enqueue one batched sweep over bp (a BatchParams<Q> of the lattice, with
// nmembers, nblocks and every member's block_begin / nblocks filled).
hipError_t launch_sweep_batch(int lattice, int mode, int P, int flags, const void *bp, hipStream_t s);

// Enqueue one sweep; fills p.nblocks.  aa is the storage layout of the input
// state: 0 pull (two buffers), 1 swapped, 2 pushed (in place, single buffer;
// see sweep_block).  Returns hipErrorInvalidValue for an unbuilt variant.
hipError_t launch_sweep(int lattice, int mode, int P, int flags, SweepParams p, hipStream_t s,
                        int aa = 0);

// Deterministic finish of per-block partials into out[NUM_NORMS] (device).
hipError_t launch_finish(const double *partials, unsigned nblocks, double *out, hipStream_t s);

// Elementwise helpers.
hipError_t launch_f64_to_f32(const double *in, float *out, size_t n, hipStream_t s);

// Per-plane coefficients of an equilibrium state, passed by value.
struct EqCoef {
  double c[MAXQ];
};
// out plane j (n cells) = coef.c[j] * phi0 for j < q, as FP32 (fp32) or FP64;
// phi0 and out are device pointers.
hipError_t launch_equilibrium(const double *phi0, const EqCoef &coef, void *out, bool fp32, size_t n,
                              int q, hipStream_t s);
hipError_t launch_f32_to_f64(const float *in, double *out, size_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s);
// dst = src, n doubles (a kernel, so that a captured graph holds no copy node)
hipError_t launch_copy_f64(const double *src, double *dst, size_t n, hipStream_t s);
hipError_t launch_fill_f32(float *p, float v, size_t n, hipStream_t s);
// partials[NUM_NORMS * blocks] (blocks <= max_blocks, the buffer's capacity):
// slot NORM_SUM_PHI gets the sum of d over all n values, taken in the pull
// order (with opp non-null, d is in the swapped layout with planes of `plane`
// values and is read through opp, so the sum rounds as for the pull layout).
hipError_t launch_sum_f32(const float *d, size_t n, double *partials, unsigned max_blocks,
                          unsigned *nblocks_out, hipStream_t s, const int *opp = nullptr,
                          unsigned plane = 0);
// x_i(c) += d_i(c) - phi_i * mean, mean = sums[NORM_SUM_PHI] / ncells  (mass-mode projection).
// opp (device, Q entries) non-null: d is in the swapped layout, d_i(c) at plane opp[i].
hipError_t launch_ir_update(double *x, const float *d, const double *phi, const double *sums,
                            unsigned Q, unsigned ncells, hipStream_t s, const int *opp = nullptr);

}  // namespace lkp
