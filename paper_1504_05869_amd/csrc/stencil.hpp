// Launch interface of the omega = 1 stencil-form kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace lkp {

// ---- omega = 1: the sweep as a scalar stencil on Phi --------------------
enum StencilMode : int {
  SMODE_F64 = 0,   // FP64 in/out, FP64 source field
  SMODE_F32 = 1,   // FP32 in/out, FP32 source field
  SMODE_RESID = 2  // FP64 in, FP32 out R = A X + G - X (FP64 arithmetic)
};

struct StencilParams {
  const void *xin;   // Phi (n values)
  void *xout;        // next Phi (or R in SMODE_RESID)
  const void *src;   // additive field (G, or R for correction solves); may be null
  double *partials;  // NUM_NORMS per block (FLAG_REDUCE)
  unsigned nx, ny, nz;
  unsigned simple_wrap;
  unsigned tile;     // 3D tile variant (stencil_tile_shape); 1D / 2D: 0
  unsigned remap;    // 3D block order: 0 hardware, R > 0 runs of R blocks per XCD
  unsigned gbx, gby; // 3D: blocks along x and y (set by the launcher)
  union {            // stencil weights per velocity orbit (phi, or chi to form G)
    double d[MAXQ];
    float f[MAXQ];
  } coef;
};

// Output cells of one stencil block (256 threads): 1D 256; 2D 64 x 16;
// 3D 64 x (4 CY or 8 CY) x BZ, the block marching through its BZ z-planes,
// with (CY, BZ) one of the built tile variants.  Within a family the
// accumulation order of every output cell is the same in every variant
// (input planes in z order, then a fixed order over the in-plane offsets),
// so its variants give the same bits.
struct StencilShape {
  unsigned tx, ty, tz;
};
// Three families of 3D variants, each rounding its own way (within a family
// every variant gives the same bits):
//   0..5   velocity by velocity;
//   6..9   separable: sums over +-x offsets first (shared through LDS), then
//          over +-y, then weights per (x, y, z) offset magnitude, less than
//          half the arithmetic (sets of whole shells);
//   10..19 plane sums: a thread owns two adjacent x cells, forms the x sums
//          in registers from 2-element LDS reads, and accumulates one sum per
//          |z offset| per input plane (sets of whole shells); the block tile
//          is 64 x 8 CY instead of 64 x 4 CY.  10..15 stage each plane
//          through registers one plane ahead; 16..19 load NB planes straight
//          into LDS (kStencilNB; nx a multiple of 16 bytes' elements).
enum StencilForm : int { STENCIL_BY_VELOCITY = 0, STENCIL_SEPARABLE = 1, STENCIL_PLANE_SUM = 2 };
constexpr int kStencilTiles3 = 20;
constexpr int kStencilCY[kStencilTiles3] = {2, 2, 2, 4, 4, 1, 2, 2, 1, 4, 1, 1, 2, 2, 2, 1, 2, 2, 1, 1};
constexpr int kStencilBZ[kStencilTiles3] = {32, 16, 8, 16, 8, 16, 32, 16, 16, 16,
                                            16, 32, 64, 16, 32, 64, 32, 64, 32, 64};
constexpr int kStencilForm[kStencilTiles3] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};
constexpr int kStencilNB[kStencilTiles3] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 3, 3, 3, 3};
// Variant of grids too small to time (the plane-sum form's smallest tile).
constexpr int kStencilDefault3 = 10;
constexpr StencilShape stencil_tile_shape(int dim, int tile) {
  return dim == 1 ? StencilShape{256, 1, 1}
                  : (dim == 2 ? StencilShape{64, 16, 1}
                              : StencilShape{64, (kStencilForm[tile] == STENCIL_PLANE_SUM ? 8u : 4u) *
                                                     (unsigned)kStencilCY[tile],
                                             (unsigned)kStencilBZ[tile]});
}
// Number of tile variants built for a dimension.
constexpr int stencil_tiles(int dim) { return dim == 3 ? kStencilTiles3 : 1; }

template <int LID, int SM>
hipError_t launch_stencil_mode_tu(int flags, const StencilParams &p, hipStream_t s);
template <int LID>
hipError_t launch_stencil_tu(int smode, int flags, const StencilParams &p, hipStream_t s);

// One stencil sweep Phi' = sum_i c_i Phi(x - v_i) [+ src]; FLAG_REDUCE adds
// the block norms of Phi' - Phi (or of R).
hipError_t launch_stencil(int lattice, int smode, int flags, const StencilParams &p, hipStream_t s);

// Blocks of a stencil launch on an nx x ny x nz grid with a tile variant;
// stencil_blocks_max: the most over the variants (partial-norm capacity).
unsigned stencil_blocks(int lattice, unsigned nx, unsigned ny, unsigned nz, int tile);
unsigned stencil_blocks_max(int lattice, unsigned nx, unsigned ny, unsigned nz);

}  // namespace lkp
