// Instantiations of the fused RK stage for float state, 2 electronic states.
#include "stage_kernel.hpp"
#include "stage_wave.hpp"

namespace qhfpe {
hipError_t launch_stage_f32_ns2(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s) {
  return launch_stage<float, 2>(np, cpt, a, nblocks, s);
}
hipError_t launch_stage_wave_f32(int np, const StageArgs& a, int nblocks, hipStream_t s) {
  return launch_stage_wave<float>(np, a, nblocks, s);
}
}  // namespace qhfpe
