// Several time steps of the worm-LBM per launch (temporal blocking) for
// gfx950: the kernel for lattices with both edges periodic, the launch
// dispatch, the ghost-frame refresh and the block-height candidates.  The
// kernel template is in fused_kernel.hpp; fused_walls.hip instantiates it for
// lattices with walls.
#include "fused_kernel.hpp"

namespace wlbm {
namespace {

// Ghost frame written by another producer (k_step writes the first ghost
// column and row only): every ghost cell of planes 0 .. nplanes-1 - columns
// -kGhost .. -1 and nx .. nx+kGhost-1 of rows 0 .. ny-1 if px, rows -1 and ny
// of columns -kGhost .. nx+kGhost-1 (or 0 .. nx-1 without px) if py - copies
// the cell it wraps to.
__global__ __launch_bounds__(kBlock) void k_fill_ghosts(float* base, long long plane, int nplanes,
                                                       int nx, int ny, int pitch, int px,
                                                       int py) {
  const int gc = px ? kGhost : 0;
  const long long ncol = 2LL * gc * ny, nrow = py ? 2LL * (nx + 2 * gc) : 0;
  const long long nper = ncol + nrow;
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= nper * nplanes) return;
  const int p = int(t / nper);
  const long long g = t - (long long)p * nper;
  int gx, gy;
  if (g < ncol) {
    const int k = int(g / ny);
    gy = int(g - (long long)k * ny);
    gx = k < gc ? k - gc : nx + k - gc;
  } else {
    const long long h = g - ncol;
    const int k = int(h / (nx + 2 * gc));
    gx = int(h - (long long)k * (nx + 2 * gc)) - gc;
    gy = k == 0 ? -1 : ny;
  }
  float* pl = base + (long long)p * plane;
  pl[cell(gx, gy, pitch)] = pl[cell(wrap_index(gx, nx), wrap_index(gy, ny), pitch)];
}

}  // namespace

hipError_t fill_ghosts(float* base, long long plane, int nplanes, int nx, int ny, int pitch,
                       bool px, bool py, hipStream_t s) {
  const long long gc = px ? kGhost : 0;
  const long long n = (2LL * gc * ny + (py ? 2LL * (nx + 2 * gc) : 0)) * nplanes;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_ghosts, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     base, plane, nplanes, nx, ny, pitch, px ? 1 : 0, py ? 1 : 0);
  return hipGetLastError();
}

int fused_strips_x(int nx, int k) {
  const int w = k == 4 ? kStrip<4> : (k == 3 ? kStrip<3> : kStrip<2>);
  return (nx + w - 1) / w;
}

// Candidate block heights for k steps per launch: R + 2 (k - 1) a multiple
// of 3, R up to 62, and no taller than needed to cover ny in one block row.
// Taller blocks re-read fewer halo rows but give fewer blocks, and how the
// last round of resident blocks fills the GPU depends on the lattice.
int fused_row_candidates(int ny, int k, int* cand, int max_cand) {
  int n = 0;
  // R + 2 (k - 1) = 0 (mod 3)
  const int r0 = k == 2 ? 4 : (k == 3 ? 5 : 6);
  for (int r = r0; r <= 62 && n < max_cand; r += 3) {
    cand[n++] = r;
    if (r >= ny) break;
  }
  return n;
}

// Waves per block: one per 8 directions up to q = 128, one per 16 for q = 192
// and 256 (those at most two steps per launch).
bool fused_supported(int q, int nx, int ny) {
  return nx >= 2 * kGhost && ny >= 2 && q % kMaxGroupPlanes == 0 &&
         (q <= 128 || q == 192 || q == 256);
}

int fused_blocks_per_cu(int q, int k, bool per_cell, bool walls) {
  if (walls) {
    switch (k) {
      case 2: return fused_blocks_per_cu_walls2(q, per_cell);
      case 3: return fused_blocks_per_cu_walls3(q, per_cell);
      case 4: return fused_blocks_per_cu_walls4(q, per_cell);
      default: return 0;
    }
  }
  switch (k) {
    case 2: return blocks_per_cu_qk<false, 2>(q, per_cell);
    case 3: return blocks_per_cu_qk<false, 3>(q, per_cell);
    case 4: return blocks_per_cu_qk<false, 4>(q, per_cell);
    default: return 0;
  }
}

hipError_t launch_fused(const FusedArgs& a, int k, bool per_cell, bool flux, hipStream_t s) {
  if (flux) {
    switch (k) {
      case 2: return launch_fused_flux2(a, per_cell, s);
      case 3: return launch_fused_flux3(a, per_cell, s);
      case 4: return launch_fused_flux4(a, per_cell, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (a.x_edge == kPeriodic && a.y_edge == kPeriodic) {
    switch (k) {
      case 2: return launch_fused_qk<false, 2, false>(a, per_cell, s);
      case 3: return launch_fused_qk<false, 3, false>(a, per_cell, s);
      case 4: return launch_fused_qk<false, 4, false>(a, per_cell, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (k) {
    case 2: return launch_fused_walls2(a, per_cell, s);
    case 3: return launch_fused_walls3(a, per_cell, s);
    case 4: return launch_fused_walls4(a, per_cell, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fused_batch(const FusedBatchArgs& b, int q, int k, bool per_cell, bool flux,
                              hipStream_t s) {
  if (flux) {
    switch (k) {
      case 2: return launch_fused_batch_flux2(b, q, per_cell, s);
      case 3: return launch_fused_batch_flux3(b, q, per_cell, s);
      case 4: return launch_fused_batch_flux4(b, q, per_cell, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (k) {
    case 2: return launch_fused_batch_walls2(b, q, per_cell, s);
    case 3: return launch_fused_batch_walls3(b, q, per_cell, s);
    case 4: return launch_fused_batch_walls4(b, q, per_cell, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wlbm
