// Dispatch of the BF16 deviation-storage sweep, and its mass sum and
// refinement update.
#include <hip/hip_runtime.h>

#include "dev_kernels.hpp"
#include "device_common.hpp"
#include "kernels.hpp"

namespace lkp {
namespace {

using namespace dev;

__device__ __forceinline__ double bf16_value(uint16_t b) {
  return (double)__uint_as_float((unsigned)b << 16);
}

__global__ void __launch_bounds__(256) k_dev_sum(const uint16_t *__restrict__ n,
                                                 const float *__restrict__ phi, unsigned Q,
                                                 unsigned ncells, double *__restrict__ partials) {
  double v[NUM_NORMS] = {0, 0, 0, 0, 0, 0};
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < ncells; c += (size_t)gridDim.x * 256) {
    double m = (double)phi[c];
    for (unsigned i = 0; i < Q; ++i) m += bf16_value(n[(size_t)i * ncells + c]);
    v[NORM_SUM_PHI] += m;
  }
  block_norms(v, partials + (size_t)blockIdx.x * NUM_NORMS);
}

__global__ void k_ir_update_dev(double *__restrict__ x, const uint16_t *__restrict__ n,
                                const float *__restrict__ phi_field, const double *__restrict__ phi,
                                const double *__restrict__ sums, unsigned Q, unsigned ncells) {
  const double mean = sums[NORM_SUM_PHI] / (double)ncells;
  const size_t total = (size_t)Q * ncells;
  for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (size_t)gridDim.x * 256) {
    const unsigned i = (unsigned)(k / ncells);
    const size_t c = k - (size_t)i * ncells;
    x[k] += (phi[i] * (double)phi_field[c] + bf16_value(n[k])) - phi[i] * mean;
  }
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

unsigned grid_of(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b ? b : 1);
}

}  // namespace

hipError_t launch_dev(int lattice, bool inner, int flags, DevParams p, hipStream_t s) {
  switch (lattice) {
    case D1Q5: return launch_dev_tu<D1Q5>(inner, flags, p, s);
    case D1Q9: return launch_dev_tu<D1Q9>(inner, flags, p, s);
    case D1Q13: return launch_dev_tu<D1Q13>(inner, flags, p, s);
    case D2Q5: return launch_dev_tu<D2Q5>(inner, flags, p, s);
    case D2Q9: return launch_dev_tu<D2Q9>(inner, flags, p, s);
    case D2Q25: return launch_dev_tu<D2Q25>(inner, flags, p, s);
    case D2Q81: return launch_dev_tu<D2Q81>(inner, flags, p, s);
    case D2Q169: return launch_dev_tu<D2Q169>(inner, flags, p, s);
    case D3Q111: return launch_dev_tu<D3Q111>(inner, flags, p, s);
    case D2Q37: return launch_dev_tu<D2Q37>(inner, flags, p, s);
    case D2Q77: return launch_dev_tu<D2Q77>(inner, flags, p, s);
    case D3Q107: return launch_dev_tu<D3Q107>(inner, flags, p, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_dev_sum(const uint16_t *n, const float *phi, unsigned Q, unsigned ncells,
                          double *partials, unsigned max_blocks, unsigned *nblocks_out,
                          hipStream_t s) {
  unsigned nb = grid_of(ncells) > 4096 ? 4096 : grid_of(ncells);
  if (nb > max_blocks) nb = max_blocks;
  if (nb == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dev_sum, dim3(nb), dim3(256), 0, s, n, phi, Q, ncells, partials);
  *nblocks_out = nb;
  return hipGetLastError();
}

hipError_t launch_ir_update_dev(double *x, const uint16_t *n, const float *phi_field,
                                const double *phi, const double *sums, unsigned Q,
                                unsigned ncells, hipStream_t s) {
  const size_t total = (size_t)Q * ncells;
  hipLaunchKernelGGL(k_ir_update_dev, dim3(grid_of(total)), dim3(256), 0, s, x, n, phi_field, phi,
                     sums, Q, ncells);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n_words, hipStream_t s) {
  if (n_words == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_of(n_words)), dim3(256), 0, s, p, v, n_words);
  return hipGetLastError();
}

}  // namespace lkp
