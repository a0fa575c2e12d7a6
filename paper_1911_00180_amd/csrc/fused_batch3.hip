// 3 time steps per launch of many lattices at once (batches; the in-plane
// film sweeps of Sec. 3.5): the batch kernel of fused_kernel.hpp.
#include "fused_kernel.hpp"

namespace wlbm {

hipError_t launch_fused_batch_walls3(const FusedBatchArgs& b, int q, bool per_cell,
                                     hipStream_t s) {
  return launch_fused_batch_qk<3, false>(b, q, per_cell, s);
}

}  // namespace wlbm
