// 4 time steps per launch of the worm-LBM with the heat flux of flux-window
// steps accumulated in the launch (Sec. 2.2 Eq. q_corr): the kernel template
// of fused_kernel.hpp for one lattice, periodic edges or walls.
#include "fused_kernel.hpp"

namespace wlbm {

hipError_t launch_fused_flux4(const FusedArgs& a, bool per_cell, hipStream_t s) {
  if (a.x_edge == kPeriodic && a.y_edge == kPeriodic)
    return launch_fused_qk<false, 4, true>(a, per_cell, s);
  return launch_fused_qk<true, 4, true>(a, per_cell, s);
}

}  // namespace wlbm
