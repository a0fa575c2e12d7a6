// 2 time steps per launch of many lattices at once with the heat flux of
// flux-window steps accumulated in the launch (Sec. 2.2 Eq. q_corr): the
// batch kernel of fused_kernel.hpp.
#include "fused_kernel.hpp"

namespace wlbm {

hipError_t launch_fused_batch_flux2(const FusedBatchArgs& b, int q, bool per_cell,
                                    hipStream_t s) {
  return launch_fused_batch_qk<2, true>(b, q, per_cell, s);
}

}  // namespace wlbm
