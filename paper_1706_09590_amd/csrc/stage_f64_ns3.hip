// Instantiations of the fused RK stage for double state, 3 electronic states (workgroup and wave variants).
#include "stage_kernel.hpp"
#include "stage_wave3.hpp"

namespace qhfpe {
hipError_t launch_stage_f64_ns3(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s) {
  return launch_stage<double, 3>(np, cpt, a, nblocks, s);
}
hipError_t launch_stage_wave3_f64(int np, const StageArgs& a, int nblocks, hipStream_t s) {
  return launch_stage_wave3<double>(np, a, nblocks, s);
}
}  // namespace qhfpe
