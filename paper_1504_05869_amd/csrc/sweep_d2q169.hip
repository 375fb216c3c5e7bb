// Fused sweep kernels for D2Q169 (all precision modes and velocity splits).
#include "stencil_impl.hpp"
#include "sweep_impl.hpp"

namespace lkp {
template hipError_t launch_lattice_tu<D2Q169>(int, int, int, SweepParams, hipStream_t);
template hipError_t launch_batch_tu<D2Q169>(int, int, int, const void *, hipStream_t);
template hipError_t launch_stencil_tu<D2Q169>(int, int, const StencilParams &, hipStream_t);
}  // namespace lkp
