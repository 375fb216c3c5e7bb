// Kernels of one velocity set, compiled once per part so that the large sets
// build in parallel: LKP_TU_LATTICE names the set (a LatticeId), LKP_TU_MODE
// the part.  Part -1 holds the dispatch over precision modes and the BF16
// deviation-storage sweep; parts 0..3 hold the fused population sweep of one
// precision mode (SweepMode), single-problem and batched; parts 10..12 the
// tau_lb = 1 stencil form of one StencilMode (10 + mode).
#include "dev_impl.hpp"
#include "stencil_impl.hpp"
#include "sweep_impl.hpp"

#ifndef LKP_TU_LATTICE
#error "define LKP_TU_LATTICE (a LatticeId) for this translation unit"
#endif
#ifndef LKP_TU_MODE
#error "define LKP_TU_MODE (-1 or a SweepMode) for this translation unit"
#endif

namespace lkp {

constexpr int kTuLattice = LKP_TU_LATTICE;

#if LKP_TU_MODE < 0
// compiled in the per-mode parts
extern template hipError_t launch_mode_tu<kTuLattice, MODE_F64>(int, int, int, SweepParams, hipStream_t);
extern template hipError_t launch_mode_tu<kTuLattice, MODE_F32>(int, int, int, SweepParams, hipStream_t);
extern template hipError_t launch_mode_tu<kTuLattice, MODE_RESID>(int, int, int, SweepParams, hipStream_t);
extern template hipError_t launch_mode_tu<kTuLattice, MODE_INNER>(int, int, int, SweepParams, hipStream_t);
extern template hipError_t launch_batch_mode_tu<kTuLattice, MODE_F64>(int, int, const void *, hipStream_t);
extern template hipError_t launch_batch_mode_tu<kTuLattice, MODE_F32>(int, int, const void *, hipStream_t);
extern template hipError_t launch_batch_mode_tu<kTuLattice, MODE_INNER>(int, int, const void *, hipStream_t);

extern template hipError_t launch_stencil_mode_tu<kTuLattice, SMODE_F64>(int, const StencilParams &, hipStream_t);
extern template hipError_t launch_stencil_mode_tu<kTuLattice, SMODE_F32>(int, const StencilParams &, hipStream_t);
extern template hipError_t launch_stencil_mode_tu<kTuLattice, SMODE_RESID>(int, const StencilParams &, hipStream_t);

template hipError_t launch_lattice_tu<kTuLattice>(int, int, int, int, SweepParams, hipStream_t);
template hipError_t launch_batch_tu<kTuLattice>(int, int, int, const void *, hipStream_t);
template hipError_t launch_stencil_tu<kTuLattice>(int, int, const StencilParams &, hipStream_t);
template hipError_t launch_dev_tu<kTuLattice>(bool, int, DevParams, hipStream_t);
#elif LKP_TU_MODE >= 10
template hipError_t launch_stencil_mode_tu<kTuLattice, LKP_TU_MODE - 10>(int, const StencilParams &, hipStream_t);
#else
template hipError_t launch_mode_tu<kTuLattice, LKP_TU_MODE>(int, int, int, SweepParams, hipStream_t);
#if LKP_TU_MODE != 2  // MODE_RESID: residual sweeps are never batched
template hipError_t launch_batch_mode_tu<kTuLattice, LKP_TU_MODE>(int, int, const void *, hipStream_t);
#endif
#endif

}  // namespace lkp
