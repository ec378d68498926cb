// Instantiations of the fused RK stage for double state, 2 electronic states.
#include "stage_kernel.hpp"
#include "stage_wave.hpp"

namespace qhfpe {
hipError_t launch_stage_f64_ns2(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s) {
  return launch_stage<double, 2>(np, cpt, a, nblocks, s);
}
hipError_t launch_stage_wave_f64(int np, const StageArgs& a, int nblocks, hipStream_t s) {
  return launch_stage_wave<double>(np, a, nblocks, s);
}
}  // namespace qhfpe
