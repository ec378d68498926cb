// Instantiations of the fused RK stage for float state, 2 electronic states.
#include "stage_kernel.hpp"

namespace qhfpe {
hipError_t launch_stage_f32_ns2(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s) {
  return launch_stage<float, 2>(np, cpt, a, nblocks, s);
}
}  // namespace qhfpe
