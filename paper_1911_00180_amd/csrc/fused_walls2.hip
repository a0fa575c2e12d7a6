// 2 time steps per launch of the worm-LBM for lattices with blackbody or
// adiabatic diffuse edges (Sec. 2.6): the kernel template of fused_kernel.hpp
// with its wall conditions compiled in.
#include "fused_kernel.hpp"

namespace wlbm {

hipError_t launch_fused_walls2(const FusedArgs& a, bool per_cell, hipStream_t s) {
  return launch_fused_qk<true, 2, false>(a, per_cell, s);
}

int fused_blocks_per_cu_walls2(int q, bool per_cell) {
  return blocks_per_cu_qk<true, 2>(q, per_cell);
}

}  // namespace wlbm
