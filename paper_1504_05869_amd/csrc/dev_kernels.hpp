// Launch interface of the BF16 deviation-storage sweep (host side).
//
// The post-collision populations are stored as a moment and a deviation,
//     f*_i(x) = phi_i Phi(x) + n_i(x),
// with Phi (the moment of the populations streamed into x, FP32) and n_i in
// BF16.  Near equilibrium n_i is much smaller than f*_i, so BF16 rounding of
// n_i costs less than rounding f*_i itself.  Pulling f_i(x) = f*_i(x - v_i)
// needs Phi at the Q upstream cells as well as n_i there.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lattices.hpp"

namespace lkp {

struct DevParams {
  const uint16_t *nin;  // Q BF16 planes: n_i of the previous sweep
  uint16_t *nout;       // Q BF16 planes: n_i of this sweep
  const float *phin;    // Phi of the previous sweep (n values)
  float *phout;         // Phi of this sweep (n values)
  const float *src;     // S (n values; source chi_i S) or r (Q planes; source r_i)
  double *partials;     // NUM_NORMS per block (FLAG_REDUCE)
  float om1;            // 1 - omega
  unsigned nx, ny, nz;
  unsigned ncells;      // < 2^29
  unsigned plane;       // elements between consecutive n planes (>= ncells)
  unsigned simple_wrap; // every axis at least its largest |v| component
  unsigned nblocks;     // set by the launcher
  float phi[MAXQ];      // phi_i (not scaled by omega)
  float chi[MAXQ];      // chi_i
};
static_assert(sizeof(DevParams) <= 4096, "kernel arguments are limited to 4 KiB");

// Velocity-group split of the deviation sweep (one variant per lattice).
// Measured on D2Q81 at 1024^2: P = 2 runs 2.4x faster than P = 1 (81 values
// per lane limit the waves in flight) and 1.6x faster than P = 4.
constexpr int dev_split(int lattice) {
  return velocity_table(lattice).q >= 169 ? 4 : (velocity_table(lattice).q >= 37 ? 2 : 1);
}

// Blocks of one deviation sweep over ncells cells.
constexpr unsigned dev_blocks(int lattice, unsigned ncells) {
  const unsigned cells = 256u / (unsigned)dev_split(lattice);
  return (ncells + cells - 1) / cells;
}

template <int LID>
hipError_t launch_dev_tu(bool inner, int flags, DevParams p, hipStream_t s);

// One deviation sweep; inner = source r_i (Q FP32 planes) instead of chi_i S.
// FLAG_REDUCE adds the block norms of Phi - Phi_prev (Phi_prev = phin).
hipError_t launch_dev(int lattice, bool inner, int flags, DevParams p, hipStream_t s);

// partials[NUM_NORMS * blocks]: slot NORM_SUM_PHI gets sum_x (Phi(x) + sum_i n_i(x)),
// the total mass of the stored populations.
hipError_t launch_dev_sum(const uint16_t *n, const float *phi, unsigned Q, unsigned ncells,
                          double *partials, unsigned max_blocks, unsigned *nblocks_out,
                          hipStream_t s);

// x_i(c) += phi_i Phi(c) + n_i(c) - phi_i mean, mean = sums[NORM_SUM_PHI] / ncells.
hipError_t launch_ir_update_dev(double *x, const uint16_t *n, const float *phi_field,
                                const double *phi, const double *sums, unsigned Q,
                                unsigned ncells, hipStream_t s);

// Zero n_words 32-bit words (BF16 planes are cleared two values at a time).
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n_words, hipStream_t s);

}  // namespace lkp
