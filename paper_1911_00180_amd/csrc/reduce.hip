// Float64 reductions of the worm-LBM diagnostics for gfx950: the totals of
// energy and heat flux over the lattice (Sec. 2.2 Eq. lbm-energy-density:
// T = sum_i e_i; Eq. q_corr: q = sum_i e_i s_i) and the heat flux summed over
// a range of columns (the in-plane flux of a film, Sec. 3.5).
//
// Each thread accumulates its cells in float64; a wave then adds its 64
// lanes with DPP row shifts (a fixed tree inside each row of 16 lanes, then
// the four row sums in row order), the waves of a block add their sums in
// wave order through LDS (one barrier), and one block adds the block sums
// the same way.  The order is fixed, so results do not depend on timing.
#include "device.hpp"
#include "kernel_common.hpp"

namespace wlbm {
namespace {

// v from the lane CTRL names (DPP row shift inside rows of 16 lanes); lanes
// with no source lane in their row read zero (bound control).
template <int CTRL>
__device__ __forceinline__ double dpp_from(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(b)), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, (uint64_t(uint32_t(hi)) << 32) | uint64_t(uint32_t(lo)));
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_readlane(int(uint32_t(b)), lane);
  const int hi = __builtin_amdgcn_readlane(int(uint32_t(b >> 32)), lane);
  return __builtin_bit_cast(double, (uint64_t(uint32_t(hi)) << 32) | uint64_t(uint32_t(lo)));
}

// Sum over the 64 lanes of a wave, the same value in every lane.  After the
// shifts by 1, 2, 4 and 8 lanes (DPP row_shr) lane 15 of each row holds the
// sum of its row; the rows are then added in order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_from<0x111>(v);
  v += dpp_from<0x112>(v);
  v += dpp_from<0x114>(v);
  v += dpp_from<0x118>(v);
  return ((read_lane(v, 15) + read_lane(v, 31)) + read_lane(v, 47)) + read_lane(v, 63);
}

constexpr int kWaves = kBlock / 64;

// Block sums of three values into out[0..2] (thread 0 writes): wave sums,
// then the waves in order.
__device__ __forceinline__ void block_sum3(double a, double b, double c, double* out) {
  __shared__ double sh[3][kWaves];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][wave] = a;
    sh[1][wave] = b;
    sh[2][wave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double s = sh[k][0];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) s += sh[k][w];
      r[k] = s;
    }
    out[0] = r[0];
    out[1] = r[1];
    out[2] = r[2];
  }
}

// Per block: sum of E (= T, the linear gray model) and of q over the
// block's cells (grid-strided), in float64.
__global__ __launch_bounds__(kBlock) void k_totals_partial(const Geometry g, const float* e,
                                                          const float* E, const float* sxtab,
                                                          const float* sytab,
                                                          double* partials) {
  const long long ncell = (long long)g.nx * g.ny;
  double se = 0.0, sqx = 0.0, sqy = 0.0;
  for (long long c = (long long)blockIdx.x * kBlock + threadIdx.x; c < ncell;
       c += (long long)gridDim.x * kBlock) {
    const long long o = cell(int(c % g.nx), int(c / g.nx), g.pitch);
    se += double(E[o]);
    double ax = 0.0, ay = 0.0;
    for (int i = 0; i < g.q; ++i) {
      const double v = e[(long long)i * g.plane + o];
      ax += v * double(sxtab[i]);
      ay += v * double(sytab[i]);
    }
    sqx += ax;
    sqy += ay;
  }
  block_sum3(se, sqx, sqy, partials + 3 * blockIdx.x);
}

// One block: the nb block partials, each of the three in block order.
__global__ __launch_bounds__(kBlock) void k_totals_final(const double* partials, int nb,
                                                        double* out) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    a += partials[3 * k];
    b += partials[3 * k + 1];
    c += partials[3 * k + 2];
  }
  block_sum3(a, b, c, out);
}

// Sums of the heat flux over the columns x0 <= x < x1 (all rows), in
// float64: from the flux-window sums (window mode) or from the populations.
__global__ __launch_bounds__(kBlock) void k_flux_sum_partial(const Geometry g, const float* e,
                                                            const float* sxtab,
                                                            const float* sytab,
                                                            const double* qsx, const double* qsy,
                                                            int window, int x0, int x1,
                                                            double* partials) {
  const int w = x1 - x0;
  const long long n = (long long)w * g.ny;
  double sx = 0.0, sy = 0.0;
  for (long long c = (long long)blockIdx.x * kBlock + threadIdx.x; c < n;
       c += (long long)gridDim.x * kBlock) {
    const int x = x0 + int(c % w);
    const int y = int(c / w);
    if (window) {
      const long long o = (long long)y * g.nx + x;
      sx += qsx[o];
      sy += qsy[o];
    } else {
      const long long o = cell(x, y, g.pitch);
      double ax = 0.0, ay = 0.0;
      for (int i = 0; i < g.q; ++i) {
        const double v = e[(long long)i * g.plane + o];
        ax += v * double(sxtab[i]);
        ay += v * double(sytab[i]);
      }
      sx += ax;
      sy += ay;
    }
  }
  block_sum3(sx, sy, 0.0, partials + 3 * blockIdx.x);
}

}  // namespace

hipError_t launch_totals(const Geometry& g, const float* e, const float* E, const float* sxtab,
                         const float* sytab, double* partials, int max_blocks, double* out,
                         hipStream_t s) {
  const long long need = ((long long)g.nx * g.ny + kBlock - 1) / kBlock;
  const int nb = int(need < max_blocks ? need : max_blocks);
  hipLaunchKernelGGL(k_totals_partial, dim3(nb), dim3(kBlock), 0, s, g, e, E, sxtab, sytab,
                     partials);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(kBlock), 0, s, partials, nb, out);
  return hipGetLastError();
}

hipError_t launch_flux_sum(const Geometry& g, const float* e, const float* sxtab,
                           const float* sytab, const double* qsx, const double* qsy, int window,
                           int x0, int x1, double* partials, int max_blocks, double* out,
                           hipStream_t s) {
  const long long need = ((long long)(x1 - x0) * g.ny + kBlock - 1) / kBlock;
  const int nb = int(need < max_blocks ? need : max_blocks);
  hipLaunchKernelGGL(k_flux_sum_partial, dim3(nb), dim3(kBlock), 0, s, g, e, sxtab, sytab, qsx,
                     qsy, window, x0, x1, partials);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(kBlock), 0, s, partials, nb, out);
  return hipGetLastError();
}

}  // namespace wlbm
