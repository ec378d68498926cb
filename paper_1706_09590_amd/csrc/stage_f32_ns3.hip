// Instantiations of the fused RK stage for float state, 3 electronic states (workgroup and wave variants).
#include "stage_kernel.hpp"
#include "stage_wave3.hpp"

namespace qhfpe {
hipError_t launch_stage_f32_ns3(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s) {
  return launch_stage<float, 3>(np, cpt, a, nblocks, s);
}
hipError_t launch_stage_wave3_f32(int np, const StageArgs& a, int nblocks, hipStream_t s) {
  return launch_stage_wave3<float>(np, a, nblocks, s);
}
}  // namespace qhfpe
