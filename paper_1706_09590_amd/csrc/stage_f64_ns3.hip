// Instantiations of the fused RK stage for double state, 3 electronic states.
#include "stage_kernel.hpp"

namespace qhfpe {
hipError_t launch_stage_f64_ns3(int np, int cpt, const StageArgs& a, int nblocks, hipStream_t s) {
  return launch_stage<double, 3>(np, cpt, a, nblocks, s);
}
}  // namespace qhfpe
