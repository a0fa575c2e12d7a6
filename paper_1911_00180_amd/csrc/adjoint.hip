// Reverse-mode (adjoint) kernels of the worm-LBM for gfx950 (MI355X).
//
// For a fixed relaxation field one time step is affine in the populations,
// e^m = A_m e^{m-1} + b_m (Sec. 2.3, Eq. algorithm: every cell x sends the
// DDED (1 - W(x)) e_i(x) to x + h_i, with h_i the pending worm move on a hop
// and 0 on a TAS pause, and the EED W(x) w_i E(x) to x + s_i; blackbody wall
// cells are then overwritten, Sec. 2.6).  The adjoint populations
// lam^{m-1} = dL/de^{m-1} therefore follow the transposed recursion
//     mu_j(z) = (1 - W(z)) lam_j(z + h_j) + W(z) G(z),
//     G(z)    = sum_i w_i lam_i(z + s_i),
// with lam read as zero outside the domain and at overwritten (blackbody)
// cells, whose adjoint feeds the wall temperature instead.  The gradient with
// respect to the relaxation weight of cell z collects, per step,
//     dL/dW(z) += E(z) G(z) - sum_j e_j(z) lam_j(z + h_j),
// evaluated as  - sum_j (e_j - w_j E) lam_j(z + h_j)
//               + E sum_{j paused} w_j (lam_j(z + s_j) - lam_j(z)),
// which is the same sum with the cancelling equilibrium parts taken out, so
// the FP32 rounding stays relative to the result.
//
// G is gathered from eight partial sums H_c(y) = sum_{i: s_i = u_c} w_i
// lam_i(y), one plane per D2Q8 move u_c, written by the producer of lam
// (the previous reverse step) with the moves of the step it will be used on:
// G(z) = sum_c H_c(z + u_c) reads each partial once.  Per update the kernel
// reads lam once (plus lam at z + s_j for the few paused directions) and the
// forward state once, and writes lam once.
#include "device.hpp"
#include "kernel_common.hpp"

namespace wlbm {
namespace {

// Plane index 0..7 of the partial sum of a D2Q8 move (dx, dy) != (0, 0).
__device__ __forceinline__ int move_class(int dx, int dy) {
  const int c = (dx + 1) * 3 + (dy + 1);
  return c - (c > 4 ? 1 : 0);
}

__device__ __forceinline__ bool wall_cell(int x, int y, int nx, int ny, int x_edge, int y_edge) {
  return (x_edge == kBlackbody && (x == 0 || x == nx - 1)) ||
         (y_edge == kBlackbody && (y == 0 || y == ny - 1));
}

__device__ __forceinline__ void add_class(float (&h)[8], int c, float w, float v) {
  switch (c) {
    case 0: h[0] = fmaf(w, v, h[0]); break;
    case 1: h[1] = fmaf(w, v, h[1]); break;
    case 2: h[2] = fmaf(w, v, h[2]); break;
    case 3: h[3] = fmaf(w, v, h[3]); break;
    case 4: h[4] = fmaf(w, v, h[4]); break;
    case 5: h[5] = fmaf(w, v, h[5]); break;
    case 6: h[6] = fmaf(w, v, h[6]); break;
    default: h[7] = fmaf(w, v, h[7]); break;
  }
}

constexpr int kAdjRed = 10;  // values per cell reduced across waves

template <int NW, bool WF, bool EDGE, bool GHOST = false>
__device__ __forceinline__ void adj_sweep(const AdjArgs& a, float* sRed, int x0, int y0) {
  using T = TileShape<NW>;
  constexpr int D = T::D;
  const WLBM_CONST uint32_t* codes = scalar_ptr(a.codes);
  const WLBM_CONST uint32_t* codes_next = scalar_ptr(a.codes_next);
  const WLBM_CONST float* wtab = scalar_ptr(a.wtab);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row = wave / NW;
  const int part = wave % NW;
  const int x = x0 + lane;
  const int y = y0 + row;
  const bool ok = !EDGE || (x < a.nx && y < a.ny);
  const int pitch = a.pitch;
  const long long plane = a.plane;
  const uint32_t plane_bytes = uint32_t(plane * 4);
  const int halo = pitch + 1;
  const uint32_t boff = uint32_t(cell(ok ? x : 0, ok ? y : 0, pitch) * 4);
  const bool px = a.x_edge == kPeriodic;
  const bool py = a.y_edge == kPeriodic;
  const bool ghost = (EDGE || GHOST) && ok && has_ghost(x, y, a.nx, a.ny, px, py);
  const bool wall = EDGE && ok && wall_cell(x, y, a.nx, a.ny, a.x_edge, a.y_edge);

  // G(z) from the eight move-class partial sums, in a fixed order
  const rsrc_t rh = make_rsrc(a.H_in - halo, uint32_t((8 * plane + 2 * halo) * 4));
  float G = 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int cc = c + (c >= 4 ? 1 : 0);
    const int dx = cc / 3 - 1;
    const int dy = cc % 3 - 1;
    G += buf_load(rh, boff, uint32_t((c * plane + halo + dy * pitch + dx) * 4));
  }
  const float Wz = WF ? buf_load(make_rsrc(a.Wf, plane_bytes), boff, 0) : a.W;
  const float Ep = buf_load(make_rsrc(a.E_prev, plane_bytes), boff, 0);

  float acc_neq = 0.f, acc_pause = 0.f, wsum = 0.f;
  float h[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int share = a.q / NW;
  // GHOST tiles (both edges periodic, no ragged lanes): byte offsets of this
  // cell's ghost copies, stored only where the lane has them
  const bool gxl = GHOST && (x == 0 || x == a.nx - 1);
  const bool gyl = GHOST && (y == 0 || y == a.ny - 1);
  const uint32_t gbx = boff + uint32_t((x == 0 ? a.nx : -a.nx) * 4);
  const uint32_t gby = boff + uint32_t((y == 0 ? a.ny : -a.ny) * pitch * 4);
  const uint32_t gbxy = gby + uint32_t((x == 0 ? a.nx : -a.nx) * 4);
  // lam at z + h_j, the forward state and (paused directions) lam at z + s_j
  // of the batch of directions i0 .. i0 + D - 1
  auto load = [&](int i0, float (&lh)[D], float (&ep)[D], float (&ls)[D]) {
    uint32_t words[D / 4];
#pragma unroll
    for (int k = 0; k < D / 4; ++k) words[k] = codes[(i0 >> 2) + k];
    const rsrc_t rl =
        make_rsrc(a.lam_in + (long long)i0 * plane - halo, uint32_t((D * plane + 2 * halo) * 4));
    const rsrc_t re = make_rsrc(a.e_prev + (long long)i0 * plane, uint32_t(D * plane * 4));
#pragma unroll
    for (int d = 0; d < D; ++d) {
      int dx, dy;
      bool hop;
      decode((words[d >> 2] >> (8 * (d & 3))) & 0xffu, dx, dy, hop);
      const int sh = dy * pitch + dx;
      lh[d] = buf_load(rl, boff, uint32_t((d * plane + halo + (hop ? sh : 0)) * 4));
      ep[d] = buf_load(re, boff, uint32_t(d * plane_bytes));
      ls[d] = hop ? 0.f : buf_load(rl, boff, uint32_t((d * plane + halo + sh) * 4));
    }
  };
  auto process = [&](int i0, const float (&lh)[D], const float (&ep)[D], const float (&ls)[D]) {
    uint32_t words[D / 4], nwords[D / 4];
#pragma unroll
    for (int k = 0; k < D / 4; ++k) {
      words[k] = codes[(i0 >> 2) + k];
      nwords[k] = codes_next[(i0 >> 2) + k];
    }
    const rsrc_t ro = make_rsrc(a.lam_out + (long long)i0 * plane, uint32_t(D * plane * 4));
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int i = i0 + d;
      int dx, dy, ndx, ndy;
      bool hop, nhop;
      decode((words[d >> 2] >> (8 * (d & 3))) & 0xffu, dx, dy, hop);
      decode((nwords[d >> 2] >> (8 * (d & 3))) & 0xffu, ndx, ndy, nhop);
      const float wi = wtab[i];
      const float l = lh[d];
      float mu = fmaf(Wz, G - l, l);
      acc_neq = fmaf(fmaf(-wi, Ep, ep[d]), l, acc_neq);
      if (!hop) acc_pause = fmaf(wi, ls[d] - l, acc_pause);
      if constexpr (EDGE) {
        if (wall) {
          wsum = fmaf(wi, mu, wsum);
          mu = 0.f;
        }
      }
      add_class(h, move_class(ndx, ndy), wi, mu);
      if constexpr (EDGE) {
        if (!ok) continue;
        if (ghost) {
          store_ghosted(a.lam_out + (long long)i * plane, x, y, mu, a.nx, a.ny, pitch, px, py);
          continue;
        }
      }
      buf_store_stream(mu, ro, boff, uint32_t(d * plane_bytes));
      if constexpr (GHOST) {
        if (gxl) buf_store_stream(mu, ro, gbx, uint32_t(d * plane_bytes));
        if (gyl) buf_store_stream(mu, ro, gby, uint32_t(d * plane_bytes));
        if (gxl && gyl) buf_store_stream(mu, ro, gbxy, uint32_t(d * plane_bytes));
      }
    }
  };
  for (int i0 = part * share; i0 < (part + 1) * share; i0 += D) {
    float lh[D], ep[D], ls[D];
    load(i0, lh, ep, ls);
    process(i0, lh, ep, ls);
  }
  float gw = fmaf(Ep, acc_pause, -acc_neq);

  if constexpr (NW > 1) {
    // partial sums of the NW waves of a row, added in a fixed order
    constexpr int n = T::TY * 64;
    const int slot = (part * T::TY + row) * 64 + lane;
    sRed[slot] = gw;
    sRed[NW * n + slot] = wsum;
#pragma unroll
    for (int c = 0; c < 8; ++c) sRed[(2 + c) * NW * n + slot] = h[c];
    __syncthreads();
    if (part != 0) return;
    const int base = row * 64 + lane;
#pragma unroll
    for (int k = 1; k < NW; ++k) {
      gw += sRed[k * n + base];
      wsum += sRed[NW * n + k * n + base];
#pragma unroll
      for (int c = 0; c < 8; ++c) h[c] += sRed[(2 + c) * NW * n + k * n + base];
    }
  }
  if (!ok) return;
  const long long o = (long long)y * a.nx + x;
  a.gW[o] += double(gw);
  if (wall) a.gB[o] += double(wsum);
  if (ghost) {
#pragma unroll
    for (int c = 0; c < 8; ++c)
      store_ghosted(a.H_out + c * plane, x, y, h[c], a.nx, a.ny, pitch, px, py);
  } else {
    const rsrc_t rH = make_rsrc(a.H_out, uint32_t(8 * plane * 4));
#pragma unroll
    for (int c = 0; c < 8; ++c) buf_store(h[c], rH, boff, uint32_t(c * plane_bytes));
  }
}

template <int NW, bool WF>
__global__ __launch_bounds__(kBlock) void k_adjoint(const AdjArgs a) {
  using T = TileShape<NW>;
  __shared__ float sRed[NW > 1 ? kAdjRed * kBlock : 1];
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = t % a.tiles_x;
  const int ty = t / a.tiles_x;
  const int x0 = tx * T::TX;
  const int y0 = ty * T::TY;
  const bool edge = x0 == 0 || x0 + T::TX >= a.nx || y0 == 0 || y0 + T::TY >= a.ny;
  // on a lattice with both edges periodic, an edge tile that holds no
  // ragged lane only adds the ghost copies to the interior path
  const bool pghost = edge && a.x_edge == kPeriodic && a.y_edge == kPeriodic &&
                      x0 + T::TX <= a.nx && y0 + T::TY <= a.ny;
  if (pghost)
    adj_sweep<NW, WF, false, true>(a, sRed, x0, y0);
  else if (edge)
    adj_sweep<NW, WF, true>(a, sRed, x0, y0);
  else
    adj_sweep<NW, WF, false>(a, sRed, x0, y0);
}

template <int NW>
hipError_t launch_adj_nw(const AdjArgs& a, bool wf, hipStream_t s) {
  if (wf)
    hipLaunchKernelGGL((k_adjoint<NW, true>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_adjoint<NW, false>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// Seeds dL/dT at probe cells: T = sum_i e_i, so every direction of the cell
// receives the value.  One thread per (probe, plane): planes j < q are the
// directions, q .. q+7 the partial sums, q+8 the wall accumulator.  A cell
// listed several times is handled by the threads of its first listing, which
// add up the values of all its listings in order, so the result does not
// depend on timing.
__global__ __launch_bounds__(kBlock) void k_adj_seed(const AdjSeedArgs a) {
  const int planes = a.q + 9;
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (long long)a.n * planes) return;
  const int p = int(t / planes);
  const int j = int(t - (long long)p * planes);
  const int x = a.cells[2 * p];
  const int y = a.cells[2 * p + 1];
  if (x < 0 || x >= a.nx || y < 0 || y >= a.ny) {
    if (j == 0) *a.flag = 1;
    return;
  }
  for (int r = 0; r < p; ++r)
    if (a.cells[2 * r] == x && a.cells[2 * r + 1] == y) return;
  float v = a.vals[p];
  for (int r = p + 1; r < a.n; ++r)
    if (a.cells[2 * r] == x && a.cells[2 * r + 1] == y) v += a.vals[r];
  const bool px = a.x_edge == kPeriodic, py = a.y_edge == kPeriodic;
  const bool wall = wall_cell(x, y, a.nx, a.ny, a.x_edge, a.y_edge);
  const long long o = cell(x, y, a.pitch);
  if (j < a.q) {
    if (wall) return;
    float* pl = a.lam + (long long)j * a.plane;
    store_ghosted(pl, x, y, pl[o] + v, a.nx, a.ny, a.pitch, px, py);
  } else if (j < a.q + 8) {
    if (wall) return;
    const int c = j - a.q;
    float* pl = a.H + (long long)c * a.plane;
    store_ghosted(pl, x, y, fmaf(v, a.wcls[c], pl[o]), a.nx, a.ny, a.pitch, px, py);
  } else if (wall) {
    a.gB[(long long)y * a.nx + x] += double(v) * a.wall_w;
  }
}

// dL/dMFP per cell: dL/dW_corr (accumulated) times dW_corr/dW =
// f (1 - 2W + 2 W Lambda_corr) (Eq. W-correction) times dW/dMFP = -W^2.
__global__ __launch_bounds__(kBlock) void k_adj_grad_mfp(const Geometry g, const double* gW,
                                                        const float* Wraw, double W_uniform,
                                                        double lam, double f, int corr,
                                                        float* out) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= (long long)g.nx * g.ny) return;
  const double W = Wraw ? double(Wraw[c]) : W_uniform;
  const double dwc = corr ? f * (1.0 - 2.0 * W + 2.0 * W * lam) : 1.0;
  out[c] = float(gW[c] * dwc * (-W * W));
}

// dL/dT0 = sum_i w_i lam_i^0 (e_i^0 = w_i T0), accumulated in float64.
__global__ __launch_bounds__(kBlock) void k_adj_grad_t0(const Geometry g, const float* lam,
                                                       const float* wtab, float* out) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= (long long)g.nx * g.ny) return;
  const long long o = cell(int(c % g.nx), int(c / g.nx), g.pitch);
  double s = 0.0;
  for (int i = 0; i < g.q; ++i) s += double(wtab[i]) * double(lam[(long long)i * g.plane + o]);
  out[c] = float(s);
}

// Wall-temperature gradients: sums of the per-cell wall accumulator over the
// cells each wall sets (the x walls own the corners), one block, fixed order.
__global__ __launch_bounds__(kBlock) void k_adj_walls(const Geometry g, const double* gB,
                                                     double* out) {
  __shared__ double sh[4 * kBlock];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  const int nx = g.nx, ny = g.ny;
  if (g.x_edge == kBlackbody) {
    for (int y = threadIdx.x; y < ny; y += kBlock) {
      s[0] += gB[(long long)y * nx];
      if (nx > 1) s[1] += gB[(long long)y * nx + nx - 1];
    }
  }
  if (g.y_edge == kBlackbody) {
    const int xa = g.x_edge == kBlackbody ? 1 : 0;
    const int xb = g.x_edge == kBlackbody ? nx - 1 : nx;
    for (int x = xa + threadIdx.x; x < xb; x += kBlock) {
      s[2] += gB[x];
      if (ny > 1) s[3] += gB[(long long)(ny - 1) * nx + x];
    }
  }
  for (int k = 0; k < 4; ++k) sh[k * kBlock + threadIdx.x] = s[k];
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int k = 0; k < 4; ++k) sh[k * kBlock + threadIdx.x] += sh[k * kBlock + threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = sh[threadIdx.x * kBlock];
}

// T = E at probe cells; NaN for a cell outside the lattice.
__global__ __launch_bounds__(kBlock) void k_read_probes(const Geometry g, const float* E,
                                                       const int32_t* cells, int n, float* out) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const int x = cells[2 * p], y = cells[2 * p + 1];
  out[p] = (x >= 0 && x < g.nx && y >= 0 && y < g.ny) ? E[cell(x, y, g.pitch)]
                                                      : __builtin_nanf("");
}

unsigned cell_blocks_adj(const Geometry& g) {
  return unsigned(((long long)g.nx * g.ny + kBlock - 1) / kBlock);
}

}  // namespace

hipError_t launch_adjoint(const AdjArgs& a, int split, bool per_cell, hipStream_t s) {
  switch (split) {
    case 1: return launch_adj_nw<1>(a, per_cell, s);
    case 2: return launch_adj_nw<2>(a, per_cell, s);
    case 4: return launch_adj_nw<4>(a, per_cell, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adj_seed(const AdjSeedArgs& a, hipStream_t s) {
  const long long threads = (long long)a.n * (a.q + 9);
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_seed, dim3(unsigned((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, a);
  return hipGetLastError();
}

hipError_t launch_adj_grad_mfp(const Geometry& g, const double* gW, const float* Wraw,
                               double W_uniform, double lam, double f, int corr, float* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_adj_grad_mfp, dim3(cell_blocks_adj(g)), dim3(kBlock), 0, s, g, gW, Wraw,
                     W_uniform, lam, f, corr, out);
  return hipGetLastError();
}

hipError_t launch_adj_grad_t0(const Geometry& g, const float* lam, const float* wtab, float* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_adj_grad_t0, dim3(cell_blocks_adj(g)), dim3(kBlock), 0, s, g, lam, wtab,
                     out);
  return hipGetLastError();
}

hipError_t launch_adj_walls(const Geometry& g, const double* gB, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_walls, dim3(1), dim3(kBlock), 0, s, g, gB, out);
  return hipGetLastError();
}

hipError_t launch_read_probes(const Geometry& g, const float* E, const int32_t* cells, int n,
                              float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_read_probes, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g, E,
                     cells, n, out);
  return hipGetLastError();
}

}  // namespace wlbm
