// Device helpers shared by the forward and adjoint kernels of the worm-LBM:
// padded cell addressing, buffer-resource loads and stores, scalar-cache
// table reads, ghost-copy stores of periodic edges, blackbody walls,
// schedule-code decoding and the tile shape.  Included by .hip files only.
#pragma once

#include "device.hpp"

namespace wlbm {
namespace {

// Workgroups are dispatched to the eight XCDs round-robin.  Remap the block
// index so that each XCD walks one contiguous range of tiles: neighbouring
// tiles, which share the cache lines of x-shifted rows and the E halo, then
// run close in time on the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int per = n >> 3;
  if (b < (per << 3)) return (b & 7) * per + (b >> 3);
  return b;
}

__device__ __forceinline__ long long cell(int x, int y, int pitch) {
  return (long long)(y + 1) * pitch + kXOff + x;
}

// Buffer resources: the plane base lives in scalar registers, each lane adds
// a 32-bit byte offset.  This keeps one VGPR per cell for addressing (the
// compiler cannot turn per-direction plane strides into 64-bit per-lane
// pointers) and every access is range-checked by the hardware.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const float* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, (int)bytes,
                                           kRsrcWord3);
}
// The b32 builtins move 32-bit words; reinterpret (never convert) them.
__device__ __forceinline__ float buf_load(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store(float v, rsrc_t r, uint32_t voff, uint32_t soff = 0) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}
// Population stores are streamed: nothing reads them again in this step, so
// they carry the non-temporal hint (cache-policy bit 1, "nt" on gfx950),
// which measurably raises the write throughput of the step.
constexpr int kStreamStore = 2;
__device__ __forceinline__ void buf_store_stream(float v, rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff,
                                        kStreamStore);
}

// Barrier for data exchanged through LDS only: waits for this wave's LDS
// accesses, not for its global loads and stores (a full __syncthreads()
// would also wait for every store in flight).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Tables that every lane reads at the same index (schedule codes, weights,
// unit vectors) are read through the scalar cache.
#define WLBM_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const WLBM_CONST T* scalar_ptr(const T* p) {
  return (const WLBM_CONST T*)p;
}

// Whether cell (x, y) has ghost copies (periodic edges: one ghost column and
// one ghost row each side).
__device__ __forceinline__ bool has_ghost(int x, int y, int nx, int ny, bool px, bool py) {
  return (px && (x == 0 || x == nx - 1)) || (py && (y == 0 || y == ny - 1));
}

__device__ __forceinline__ int wrap_index(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Store a cell value and, for periodic edges, its ghost copies: column nx
// holds column 0, column -1 holds column nx - 1, likewise for rows, corners
// both.  (The further ghost columns each side, which the multi-step kernels
// read, are refreshed by k_fill_ghosts.)
__device__ __forceinline__ void store_ghosted(float* __restrict__ plane, int x, int y, float v,
                                              int nx, int ny, int pitch, bool px, bool py) {
  plane[cell(x, y, pitch)] = v;
  int gx[2], gy[2], ngx = 0, ngy = 0;
  if (px) {
    if (x == 0) gx[ngx++] = nx;
    if (x == nx - 1) gx[ngx++] = -1;
  }
  if (py) {
    if (y == 0) gy[ngy++] = ny;
    if (y == ny - 1) gy[ngy++] = -1;
  }
  for (int a = 0; a < ngx; ++a) plane[cell(gx[a], y, pitch)] = v;
  for (int b = 0; b < ngy; ++b) plane[cell(x, gy[b], pitch)] = v;
  for (int a = 0; a < ngx; ++a)
    for (int b = 0; b < ngy; ++b) plane[cell(gx[a], gy[b], pitch)] = v;
}

// Blackbody walls (Sec. 2.6, Eq. isotropic): the DDEDs of a wall cell are
// w_i T_wall.  y walls first, then x walls, so the x walls win at corners.
__device__ __forceinline__ float blackbody(float v, float wi, int x, int y, int nx, int ny,
                                           int x_edge, int y_edge, float txl, float txh,
                                           float tyl, float tyh) {
  if (y_edge == kBlackbody) {
    if (y == ny - 1)
      v = wi * tyh;
    else if (y == 0)
      v = wi * tyl;
  }
  if (x_edge == kBlackbody) {
    if (x == nx - 1)
      v = wi * txh;
    else if (x == 0)
      v = wi * txl;
  }
  return v;
}

__device__ __forceinline__ void decode(uint32_t code, int& dx, int& dy, bool& hop) {
  dx = int(code & 3u) - 1;
  dy = int((code >> 2) & 3u) - 1;
  hop = (code >> 4) & 1u;
}

// The inflow of a diffuse-wall node is summed per batch of 8 directions; the
// batch sums are grouped into kNodeParts consecutive ranges of
// node_part_batches(q / 8) batches, each range added in order, and the range
// sums added in order.  (The single-step kernel gives each range to its own
// thread; the multi-step kernels add the same terms in the same order.)
constexpr int kNodeParts = 3;
__device__ __forceinline__ int node_part_batches(int nb) {
  return (nb + kNodeParts - 1) / kNodeParts;
}

// One kernel block is four waves.  Its tile is 64 cells wide (one wave) and
// 4 / NW rows tall; the Q directions of each cell are split over NW waves,
// each taking Q / NW of them in batches of D.  Splitting keeps every wave
// short-lived, so the grid holds many waves and the drain at the end of a
// launch is short; the NW partial sums of E' are added in LDS in a fixed
// order, so results do not depend on timing.
template <int NW>
struct TileShape {
  static constexpr int TX = 64;          // tile width in cells (one wave)
  static constexpr int TY = 4 / NW;      // tile height in cells
  static constexpr int LP = TX + 2;      // LDS row pitch (one halo column each side)
  static constexpr int LH = TY + 2;      // LDS rows (one halo row each side)
  static constexpr int D = kMaxGroupPlanes;  // directions per load batch
  static_assert(NW == 1 || NW == 2 || NW == 4, "direction split of 1, 2 or 4 waves");
};

}  // namespace
}  // namespace wlbm
