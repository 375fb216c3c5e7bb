// Dispatch of the fused sweep to its per-lattice translation units, and the
// small utility kernels (norm finish, conversions, fills, IR update).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"
#include "stencil.hpp"
#include "lattices.hpp"

namespace lkp {
namespace {

using namespace dev;

__global__ void __launch_bounds__(256) k_finish(const double *__restrict__ partials, unsigned nb,
                                                double *__restrict__ out) {
  double v[NUM_NORMS] = {0, 0, 0, 0, 0, 0};
  for (unsigned b = threadIdx.x; b < nb; b += 256) {
    const double *q = partials + (size_t)b * NUM_NORMS;
    v[0] = fmax(v[0], q[0]);
#pragma unroll
    for (int k = 1; k < NUM_NORMS; ++k) v[k] += q[k];
  }
  block_norms(v, out);
}

__global__ void k_f64_to_f32(const double *__restrict__ in, float *__restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// Plane j of the state gets coef[j] * phi0 (FP64 product, stored in T).
template <typename T>
__global__ void __launch_bounds__(256) k_equilibrium(const double *__restrict__ phi0, EqCoef cf,
                                                     T *__restrict__ out, size_t n) {
  const double c = cf.c[blockIdx.y];
  T *__restrict__ o = out + (size_t)blockIdx.y * n;
  for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (size_t)gridDim.x * blockDim.x)
    o[x] = (T)(c * phi0[x]);
}

__global__ void k_f32_to_f64(const float *__restrict__ in, double *__restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, T v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <class T>
__global__ void k_copy(const T *__restrict__ src, T *__restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void __launch_bounds__(256) k_sum_f32(const float *__restrict__ d, size_t n,
                                                 double *__restrict__ partials,
                                                 const int *__restrict__ opp, unsigned plane) {
  double v[NUM_NORMS] = {0, 0, 0, 0, 0, 0};
  for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) {
    // swapped layout: element k of the pull order sits in plane opp[k / plane]
    const size_t src = opp ? (size_t)opp[k / plane] * plane + k % plane : k;
    v[NORM_SUM_PHI] += (double)d[src];
  }
  block_norms(v, partials + (size_t)blockIdx.x * NUM_NORMS);
}

__global__ void __launch_bounds__(256) k_ir_update(double *__restrict__ x, const float *__restrict__ d,
                                                   const double *__restrict__ phi,
                                                   const double *__restrict__ sums, unsigned Q,
                                                   unsigned ncells,
                                                   const int *__restrict__ opp) {
  const double mean = sums[NORM_SUM_PHI] / (double)ncells;
  const size_t n = (size_t)Q * ncells;
  for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) {
    const unsigned i = (unsigned)(k / ncells);
    // swapped layout (in place): d_i(c) sits in plane opp[i]
    const size_t src = opp ? (size_t)opp[i] * ncells + (k - (size_t)i * ncells) : k;
    x[k] += (double)d[src] - phi[i] * mean;
  }
}

unsigned grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b ? b : 1);
}

}  // namespace

bool sweep_variant_available(int lattice, int mode, int P) {
  if (lattice < 0 || lattice >= NUM_LATTICES || mode < 0 || mode >= NUM_MODES) return false;
  return sweep_variant_built(lattice, mode, P);
}

hipError_t launch_sweep(int lattice, int mode, int P, int flags, SweepParams p, hipStream_t s, int aa) {
  if (!sweep_variant_available(lattice, mode, P)) return hipErrorInvalidValue;
  const unsigned cells = cells_per_block(P);
  p.nblocks = (p.ncells + cells - 1) / cells;
  switch (lattice) {
    case D1Q5: return launch_lattice_tu<D1Q5>(mode, P, aa, flags, p, s);
    case D1Q9: return launch_lattice_tu<D1Q9>(mode, P, aa, flags, p, s);
    case D1Q13: return launch_lattice_tu<D1Q13>(mode, P, aa, flags, p, s);
    case D2Q5: return launch_lattice_tu<D2Q5>(mode, P, aa, flags, p, s);
    case D2Q9: return launch_lattice_tu<D2Q9>(mode, P, aa, flags, p, s);
    case D2Q25: return launch_lattice_tu<D2Q25>(mode, P, aa, flags, p, s);
    case D2Q81: return launch_lattice_tu<D2Q81>(mode, P, aa, flags, p, s);
    case D2Q169: return launch_lattice_tu<D2Q169>(mode, P, aa, flags, p, s);
    case D3Q111: return launch_lattice_tu<D3Q111>(mode, P, aa, flags, p, s);
    case D2Q37: return launch_lattice_tu<D2Q37>(mode, P, aa, flags, p, s);
    case D2Q77: return launch_lattice_tu<D2Q77>(mode, P, aa, flags, p, s);
    case D3Q107: return launch_lattice_tu<D3Q107>(mode, P, aa, flags, p, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_batch(int lattice, int mode, int P, int flags, const void *bp, hipStream_t s) {
  if (!sweep_variant_available(lattice, mode, P) || mode == MODE_RESID) return hipErrorInvalidValue;
  switch (lattice) {
    case D1Q5: return launch_batch_tu<D1Q5>(mode, P, flags, bp, s);
    case D1Q9: return launch_batch_tu<D1Q9>(mode, P, flags, bp, s);
    case D1Q13: return launch_batch_tu<D1Q13>(mode, P, flags, bp, s);
    case D2Q5: return launch_batch_tu<D2Q5>(mode, P, flags, bp, s);
    case D2Q9: return launch_batch_tu<D2Q9>(mode, P, flags, bp, s);
    case D2Q25: return launch_batch_tu<D2Q25>(mode, P, flags, bp, s);
    case D2Q81: return launch_batch_tu<D2Q81>(mode, P, flags, bp, s);
    case D2Q169: return launch_batch_tu<D2Q169>(mode, P, flags, bp, s);
    case D3Q111: return launch_batch_tu<D3Q111>(mode, P, flags, bp, s);
    case D2Q37: return launch_batch_tu<D2Q37>(mode, P, flags, bp, s);
    case D2Q77: return launch_batch_tu<D2Q77>(mode, P, flags, bp, s);
    case D3Q107: return launch_batch_tu<D3Q107>(mode, P, flags, bp, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stencil(int lattice, int smode, int flags, const StencilParams &p, hipStream_t s) {
  switch (lattice) {
    case D1Q5: return launch_stencil_tu<D1Q5>(smode, flags, p, s);
    case D1Q9: return launch_stencil_tu<D1Q9>(smode, flags, p, s);
    case D1Q13: return launch_stencil_tu<D1Q13>(smode, flags, p, s);
    case D2Q5: return launch_stencil_tu<D2Q5>(smode, flags, p, s);
    case D2Q9: return launch_stencil_tu<D2Q9>(smode, flags, p, s);
    case D2Q25: return launch_stencil_tu<D2Q25>(smode, flags, p, s);
    case D2Q81: return launch_stencil_tu<D2Q81>(smode, flags, p, s);
    case D2Q169: return launch_stencil_tu<D2Q169>(smode, flags, p, s);
    case D3Q111: return launch_stencil_tu<D3Q111>(smode, flags, p, s);
    case D2Q37: return launch_stencil_tu<D2Q37>(smode, flags, p, s);
    case D2Q77: return launch_stencil_tu<D2Q77>(smode, flags, p, s);
    case D3Q107: return launch_stencil_tu<D3Q107>(smode, flags, p, s);
  }
  return hipErrorInvalidValue;
}

unsigned stencil_blocks(int lattice, unsigned nx, unsigned ny, unsigned nz, int tile) {
  const StencilShape sh = stencil_tile_shape(velocity_table(lattice).dim, tile);
  return ((nx + sh.tx - 1) / sh.tx) * ((ny + sh.ty - 1) / sh.ty) * ((nz + sh.tz - 1) / sh.tz);
}

unsigned stencil_blocks_max(int lattice, unsigned nx, unsigned ny, unsigned nz) {
  unsigned m = 0;
  for (int t = 0; t < stencil_tiles(velocity_table(lattice).dim); ++t)
    m = std::max(m, stencil_blocks(lattice, nx, ny, nz, t));
  return m;
}

hipError_t launch_finish(const double *partials, unsigned nblocks, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, partials, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double *in, float *out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_equilibrium(const double *phi0, const EqCoef &coef, void *out, bool fp32, size_t n,
                              int q, hipStream_t s) {
  if (q < 1 || q > MAXQ) return hipErrorInvalidValue;
  const unsigned gx = (unsigned)std::min<size_t>((n + 255) / 256, 1024);
  const dim3 grid(gx ? gx : 1, (unsigned)q);
  if (fp32)
    hipLaunchKernelGGL(k_equilibrium<float>, grid, dim3(256), 0, s, phi0, coef, (float *)out, n);
  else
    hipLaunchKernelGGL(k_equilibrium<double>, grid, dim3(256), 0, s, phi0, coef, (double *)out, n);
  return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float *in, double *out, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_copy_f64(const double *src, double *dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy<double>, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float v, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_sum_f32(const float *d, size_t n, double *partials, unsigned max_blocks,
                          unsigned *nblocks_out, hipStream_t s, const int *opp, unsigned plane) {
  unsigned nb = grid_for(n) > 4096 ? 4096 : grid_for(n);
  if (nb > max_blocks) nb = max_blocks;
  if (nb == 0 || (opp && plane == 0)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sum_f32, dim3(nb), dim3(256), 0, s, d, n, partials, opp, plane);
  *nblocks_out = nb;
  return hipGetLastError();
}

hipError_t launch_ir_update(double *x, const float *d, const double *phi, const double *sums,
                            unsigned Q, unsigned ncells, hipStream_t s, const int *opp) {
  const size_t n = (size_t)Q * ncells;
  hipLaunchKernelGGL(k_ir_update, dim3(grid_for(n)), dim3(256), 0, s, x, d, phi, sums, Q, ncells,
                     opp);
  return hipGetLastError();
}

}  // namespace lkp
