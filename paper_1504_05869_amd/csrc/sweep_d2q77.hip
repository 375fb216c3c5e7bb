// Fused sweep kernels for D2Q77 (all precision modes and velocity splits,
// the tau_lb = 1 stencil form and the BF16 deviation-storage sweep).
#include "dev_impl.hpp"
#include "stencil_impl.hpp"
#include "sweep_impl.hpp"

namespace lkp {
template hipError_t launch_lattice_tu<D2Q77>(int, int, int, int, SweepParams, hipStream_t);
template hipError_t launch_batch_tu<D2Q77>(int, int, int, const void *, hipStream_t);
template hipError_t launch_stencil_tu<D2Q77>(int, int, const StencilParams &, hipStream_t);
template hipError_t launch_dev_tu<D2Q77>(bool, int, DevParams, hipStream_t);
}  // namespace lkp
