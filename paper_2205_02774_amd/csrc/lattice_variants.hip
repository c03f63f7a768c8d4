// Velocity-set and collision variants of the stream-collide pass (one cell
// per lane): D3Q15 and D3Q27 with the regularized operator, and the plain BGK
// bulk operator on all three sets.  The kernel is the one in lattice_step.h;
// only the instantiations live here, so they compile in parallel with the
// main configuration.
#include "lattice_step.h"

namespace stglbm {
namespace {

template <class Codec>
hipError_t launch_variant_codec(const StepParams& p, bool stats, hipStream_t s) {
  if (p.vec != 1) return hipErrorInvalidValue;
  const bool reg = p.collision == 0;
  switch (p.q) {
    case 15: return reg ? launch_step_v<Codec, 15, true, 1>(p, stats, s) : launch_step_v<Codec, 15, false, 1>(p, stats, s);
    case 19: return reg ? hipErrorInvalidValue : launch_step_v<Codec, 19, false, 1>(p, stats, s);   // regularized: main unit
    case 27: return reg ? launch_step_v<Codec, 27, true, 1>(p, stats, s) : launch_step_v<Codec, 27, false, 1>(p, stats, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_step_variant(const StepParams& p, int store, bool stats, hipStream_t s) {
  switch (store) {
    case 0: return launch_variant_codec<CodecF32>(p, stats, s);
    case 1: return launch_variant_codec<CodecF16>(p, stats, s);
    case 2: return launch_variant_codec<CodecBF16>(p, stats, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace stglbm
