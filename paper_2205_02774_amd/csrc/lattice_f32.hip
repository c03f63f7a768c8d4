// FP32-store statistics kernels without a body force (one cell per lane):
// D3Q19 regularized, the kernel of the FP32 channel steps (two z waves of
// whole rows per block), and the D3Q15 regularized and D3Q19 plain-BGK
// variants.  They are the kernel of lattice_step.h, instantiated in a unit of
// their own so that the build can compile them with the AMDGPU machine
// scheduler set for instruction-level parallelism (max-ilp).  Measured on
// MI355X at 512x128x256: D3Q19 regularized 0.4563 against 0.4594 ms per
// launch (three alternating runs of 1000 steps), D3Q15 0.3643 against 0.3668,
// D3Q19 BGK 0.4580 against 0.4653; the same strategy slowed the 16-bit
// launches, the FP32 launch with a body force and FP32 D3Q27, which keep the
// default schedule.
#include "lattice_step.h"

namespace stglbm {

template <int QN, bool REG>
hipError_t launch_f32_stats(const StepParams& p, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
  step_kernel<CodecF32, QN, REG, 1, true, false><<<grid, block, lds, s>>>(p);
  return hipGetLastError();
}

template hipError_t launch_f32_stats<19, true>(const StepParams&, dim3, dim3, size_t, hipStream_t);
template hipError_t launch_f32_stats<15, true>(const StepParams&, dim3, dim3, size_t, hipStream_t);
template hipError_t launch_f32_stats<19, false>(const StepParams&, dim3, dim3, size_t, hipStream_t);

}  // namespace stglbm
