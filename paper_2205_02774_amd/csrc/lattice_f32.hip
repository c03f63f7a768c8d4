// FP32-store statistics kernels without a body force (one cell per lane),
// instantiated in a unit of their own so that the build can compile them
// with the AMDGPU machine scheduler set for instruction-level parallelism
// (max-ilp): the D3Q15 regularized and D3Q19 plain-BGK variants, which it
// makes faster (512x128x256, 500 steps after 2000: D3Q15 0.3643 against
// 0.3668 ms per launch, BGK 0.4580 against 0.4653), and a second build of the
// channel's D3Q19 regularized kernel.  That one is 1 % faster in long runs
// (0.4551 against 0.4588 ms over 200 launches) but slower over its first ten
// or so launches in a process (0.4580 against 0.4559 ms over launches 6-25),
// so the default-schedule build stays the default and this one is chosen by
// the STGLBM_F32_ILP tuning override.  The 16-bit kernels, the kernels with a
// body force and FP32 D3Q27 measured slower with max-ilp.
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
