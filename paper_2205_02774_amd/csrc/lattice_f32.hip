// The FP32-store D3Q19 regularized stream-collide kernel of the statistics
// launches without a body force (one cell per lane, two z waves of whole rows
// per block): the kernel of the FP32 channel steps.  It is the kernel of
// lattice_step.h, instantiated in a unit of its own so that the build can
// compile it with the AMDGPU machine scheduler set for instruction-level
// parallelism (max-ilp): measured on MI355X at 512x128x256, 0.4552 against
// 0.4596 ms per launch (three alternating runs of 1000 steps), while the same
// strategy slowed the 16-bit launches and the FP32 launch with a body force.
#include "lattice_step.h"

namespace stglbm {

hipError_t launch_f32_d3q19_stats(const StepParams& p, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
  step_kernel<CodecF32, 19, true, 1, true, false><<<grid, block, lds, s>>>(p);
  return hipGetLastError();
}

}  // namespace stglbm
