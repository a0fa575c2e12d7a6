// HIP kernels of the worm-LBM for gfx950 (MI355X).
//
// The hot kernel k_step advances one time step for every cell and direction:
// BGK relaxation of the directional energy densities e_i towards w_i E, with
// E = sum_i e_i and the corrected relaxation weight, and streaming along each
// direction's worm path with TAS pauses (arXiv:1911.00180, Sec. 2.2 Eq.
// lbm-energy, Sec. 2.3 Eq. algorithm, Sec. 2.5), followed by the wall
// conditions of Sec. 2.6.
//
// It is written in pull form: the thread that owns cell y gathers, for each
// direction i with pending worm move s_i (and DDED shift h_i = s_i on a hop,
// 0 on a pause),
//     out_i(y) = (1 - W(y - h_i)) e_i(y - h_i) + W(y - s_i) w_i E(y - s_i)
// and at the same time sums E'(y) = sum_i out_i(y) for the next step, so each
// population is read once and written once per step (the path is HBM-bound;
// there is no contraction and no MFMA).  E of the previous step is staged in
// LDS with a one-cell halo; the schedule row is read through the scalar cache.
#include "device.hpp"
#include "kernel_common.hpp"

#include <cmath>

namespace wlbm {
namespace {

// Boundary node of a diffuse wall (Sec. 2.6, Eq. adiabatic-diffuse): the node
// at column X behind the lo (wall 0, row -1) or hi (wall 1, row ny) wall
// absorbs the diffuse share 1 - p of what streams into it on this step and
// re-emits it isotropically, as inward DDEDs w_i T_g.  A direction with an
// inward pending move delivers w_i T_g on a hop and w_i W_g T_g (its EED
// part) on a pause; T_g is chosen so that the node emits exactly what it
// absorbed.  The node below/above a blackbody column belongs to the blackbody
// wall, and nodes outside a blackbody edge emit nothing: for those,
// node_fixed sets T_g and W_g T_g and returns true; otherwise it wraps X of a
// periodic edge and returns false.
template <bool WF>
__device__ __forceinline__ bool node_fixed(const StepArgs& a, int wall, int& X, float& tg,
                                           float& wtg) {
  const int yrow = wall == 0 ? 0 : a.ny - 1;
  if (a.x_edge == kBlackbody) {
    if (X < 0 || X >= a.nx) {
      tg = wtg = 0.f;
      return true;
    }
    if (X == 0 || X == a.nx - 1) {
      const float Wg = WF ? a.Wf[cell(X, yrow, a.pitch)] : a.W;
      tg = (1.f - a.spec) * ((X == a.nx - 1) ? a.t_x_hi : a.t_x_lo);
      wtg = Wg * tg;
      return true;
    }
  } else {
    X = ((X % a.nx) + a.nx) % a.nx;
  }
  return false;
}

// What batches b0 .. b1-1 of 8 directions stream into the node at (wrapped)
// column X on this step: for every direction whose pending move leaves the
// lattice through the node's wall, the packet that the pull form delivers to a
// cell at the node's position (the DDED of the wall-row cell X - dx on a hop,
// its EED on every step).  Each batch is summed in direction order and the
// batch sums in batch order, so the multi-step kernels, which hold the
// directions of a cell in other waves, can add the same terms in the same
// order.
template <bool WF>
__device__ float node_inflow(const StepArgs& a, int wall, int X, int b0, int b1) {
  const int yrow = wall == 0 ? 0 : a.ny - 1;
  const int out_dy = wall == 0 ? -1 : 1;
  float S = 0.f;
  for (int b = b0; b < b1; ++b) {
    float R = 0.f;
    for (int i = b * kMaxGroupPlanes; i < (b + 1) * kMaxGroupPlanes; ++i) {
      const uint32_t code = (a.codes[i >> 2] >> (8 * (i & 3))) & 0xffu;
      int dx, dy;
      bool hop;
      decode(code, dx, dy, hop);
      if (dy != out_dy) continue;
      // source cell of the packet; for a periodic x edge the ghost columns
      // hold the wrapped values, for a blackbody edge X - dx stays inside
      const long long o = cell(X - dx, yrow, a.pitch);
      const float e = hop ? a.e_in[(long long)i * a.plane + o] : 0.f;
      float out;
      if constexpr (!WF) {
        out = fmaf(a.W, fmaf(a.wtab[i], a.E_in[o], -e), e);
      } else {
        const float Ws = a.Wf[o];
        out = e + fmaf(a.wtab[i], a.E_in[o] * Ws, -(Ws * e));
      }
      R += out;
    }
    S += R;
  }
  return S;
}

// T_g and W_g T_g of the node at (wrapped) column X from its inflow R.
template <bool WF>
__device__ __forceinline__ void node_emit(const StepArgs& a, int wall, int X, float R, float& tg,
                                          float& wtg) {
  const int yrow = wall == 0 ? 0 : a.ny - 1;
  const float Wg = WF ? a.Wf[cell(X, yrow, a.pitch)] : a.W;
  const float hs = wall == 0 ? a.in_lo_hop : a.in_hi_hop;
  const float as = wall == 0 ? a.in_lo_all : a.in_hi_all;
  const float C = fmaf(Wg, as - hs, hs);
  tg = (1.f - a.spec) * R / C;
  wtg = Wg * tg;
}

// For each move code c = dx + 1 | (dy + 1) << 2 | hop << 4: the byte offset,
// from a cell's own entry in the LDS tile of E (rows of TileShape::LP = 66
// floats), of the entry at (x - dx, y - dy), and of W where the pulled
// population was (the same on a hop, 0 on a pause).
struct StepCodeTab {
  int32_t eoff[32];
  int32_t woff[32];
};
constexpr StepCodeTab make_step_code_tab() {
  StepCodeTab t{};
  for (int c = 0; c < 32; ++c) {
    const int dx = (c & 3) - 1, dy = ((c >> 2) & 3) - 1;
    const bool hop = (c >> 4) & 1;
    t.eoff[c] = -4 * (dy * 66 + dx);
    t.woff[c] = hop ? t.eoff[c] : 0;
  }
  return t;
}
__constant__ StepCodeTab kStepCode = make_step_code_tab();

// Load the populations of directions i0 .. i0+D-1 that stream into the cell
// at byte offset boff: the DDED of direction i comes from the cell one
// pending worm move back on a hop and from the cell itself on a pause.  One
// buffer descriptor covers the batch (direction d is d planes further on)
// plus one row and column either side, so the shifted offset stays positive.
//
// TAB: the host has uploaded, per step and direction, that load's byte offset
// (pulls: (1 - hy) pitch 4 + 4 (1 - hx) + (i mod 8) plane 4, the offset below)
// and the byte offset of the direction's entry in the selection table of the
// multi-step kernels (sels: its move code times kSelEntryBytes), so the
// kernel reads offsets instead of decoding codes in scalar code.
template <int D, bool TAB>
__device__ __forceinline__ void load_batch(const StepArgs& a, int i0, uint32_t boff,
                                           float (&v)[D]) {
  const WLBM_CONST uint32_t* codes = scalar_ptr(a.codes);
  const int pitch = a.pitch;
  const long long plane = a.plane;
  const uint32_t win_bytes = uint32_t((D * plane + 2 * (pitch + 1)) * 4);
  const uint32_t plane_bytes = uint32_t(plane * 4);
  const rsrc_t rs = make_rsrc(a.e_in + (long long)i0 * plane - (pitch + 1), win_bytes);
  if constexpr (TAB) {
    const WLBM_CONST uint32_t* pulls = scalar_ptr(a.pulls);
#pragma unroll
    for (int d = 0; d < D; ++d) v[d] = buf_load(rs, boff, pulls[i0 + d]);
    return;
  }
  uint32_t words[D / 4];
#pragma unroll
  for (int k = 0; k < D / 4; ++k) words[k] = codes[(i0 >> 2) + k];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    int dx, dy;
    bool hop;
    decode((words[d >> 2] >> (8 * (d & 3))) & 0xffu, dx, dy, hop);
    const int sh = hop ? dy * pitch + dx : 0;
    v[d] = buf_load(rs, boff, uint32_t(d * plane_bytes + (pitch + 1 - sh) * 4));
  }
}

// The sweep of one wave over its share of the directions for one cell per
// lane.  XWALL tiles (blackbody x edges) touch only an x edge, hold no
// ragged lanes and no y-edge rows: they run the interior path plus the
// blackbody overwrite.  GHOST tiles (both edges periodic, no ragged lanes)
// run the interior path plus the stores of the periodic ghost copies (one
// tile in eight at 1024 x 1024, Q = 64 is on an x edge: 548 -> 591 G updates/s with
// this path).  EDGE tiles touch a domain edge or are ragged: they mask cells
// outside the lattice, apply the wall conditions and write the ghost copies
// of periodic edges.  Interior tiles need none of that: every source cell of
// a pull lies inside the padded arrays, with no wrap arithmetic.
// E' = sum_i out_i is added in a fixed order that does not depend on the
// direction split: each batch of D = 8 directions is summed in direction
// order, then the batch sums are added in batch order (sBat holds them when
// several waves share a cell).  The heat flux of flux-window steps is summed
// the same way (each batch's fma chain over its directions, then the batches
// in order).  The multi-step kernels add in the same order.
template <int NW, bool WF, bool FLUX, bool TAB, bool EDGE, bool XWALL = false, bool GHOST = false>
__device__ __forceinline__ void sweep(const StepArgs& a, const float* sE, const float* sW,
                                      const float* sTg, const float* sWTg,
                                      float* sBat, int x0, int y0, uint32_t boff,
                                      const float (&v0)[TileShape<NW>::D],
                                      const float (&v1)[TileShape<NW>::D]) {
  using T = TileShape<NW>;
  constexpr int D = T::D;
  const WLBM_CONST uint32_t* codes = scalar_ptr(a.codes);
  const WLBM_CONST float* wtab = scalar_ptr(a.wtab);
  const WLBM_CONST float* sxtab = scalar_ptr(a.sxtab);
  const WLBM_CONST float* sytab = scalar_ptr(a.sytab);
  const int lane = threadIdx.x & 63;
  // wave-uniform values, kept in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row = wave / NW;       // cell row of this wave inside the tile
  const int part = wave % NW;      // which share of the directions
  const int x = x0 + lane;
  const int y = y0 + row;
  const bool px = a.x_edge == kPeriodic;
  const bool py = a.y_edge == kPeriodic;
  const int pitch = a.pitch;
  const long long plane = a.plane;
  const uint32_t plane_bytes = uint32_t(plane * 4);
  const uint32_t batch_bytes = uint32_t(D * plane * 4);

  const bool ok = !EDGE || (x < a.nx && y < a.ny);
  const int lc = (row + 1) * T::LP + lane + 1;
  const bool ghost = (EDGE || GHOST) && ok && has_ghost(x, y, a.nx, a.ny, px, py);
  // GHOST tiles (both edges periodic, no ragged lanes): byte offsets of this
  // cell's ghost copies in its plane (column nx for 0, -1 for nx - 1; rows
  // likewise), stored only where the lane has them
  const bool gxl = GHOST && (x == 0 || x == a.nx - 1);
  const bool gyl = GHOST && (y == 0 || y == a.ny - 1);
  const uint32_t gbx = boff + uint32_t((x == 0 ? a.nx : -a.nx) * 4);
  const uint32_t gby = boff + uint32_t((y == 0 ? a.ny : -a.ny) * pitch * 4);
  const uint32_t gbxy = gby + uint32_t((x == 0 ? a.nx : -a.nx) * 4);

  float Eacc = 0.f, qx = 0.f, qy = 0.f;
  const int share = a.q / NW;
  constexpr int nrow = T::TY * 64;           // cells of the tile
  // tiles other than EDGE tiles need no move components: with TAB they take
  // the LDS offsets of E and W from the code table
  constexpr bool kTab = TAB && !EDGE;
  const WLBM_CONST uint32_t* sels = scalar_ptr(a.sels);
  const char* sEc = reinterpret_cast<const char*>(sE + lc);
  const char* sWc = reinterpret_cast<const char*>(sW + lc);
  const int nbat = a.q / D;
  auto relax_batch = [&](int i0, const float (&v)[D]) {
    float bsum = 0.f, bqx = 0.f, bqy = 0.f;
    uint32_t words[D / 4];
    if constexpr (!kTab) {
#pragma unroll
      for (int k = 0; k < D / 4; ++k) words[k] = codes[(i0 >> 2) + k];
    }
    const rsrc_t ro = make_rsrc(a.e_out + (long long)i0 * plane, batch_bytes);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int i = i0 + d;
      int dx = 0, dy = 0;
      bool hop = false;
      int32_t eoff, woff;
      if constexpr (kTab) {
        const uint32_t c = sels[i] / kSelEntryBytes;
        eoff = kStepCode.eoff[c];
        woff = kStepCode.woff[c];
      } else {
        decode((words[d >> 2] >> (8 * (d & 3))) & 0xffu, dx, dy, hop);
        eoff = -4 * (dy * T::LP + dx);
        woff = hop ? eoff : 0;
      }
      const float wi = wtab[i];
      const float e = v[d];
      const float Es = *reinterpret_cast<const float*>(sEc + eoff);
      float out;
      if constexpr (!WF) {
        // e + W (w_i E - e): the rounding error stays relative to the
        // (small) change, so a nearly ballistic run does not drift
        out = fmaf(a.W, fmaf(wi, Es, -e), e);
      } else {
        // sE holds W E; sW holds W of each cell
        const float Wh = *reinterpret_cast<const float*>(sWc + woff);
        out = e + fmaf(wi, Es, -(Wh * e));
      }
      if constexpr (XWALL) {
        out = blackbody(out, wi, x, y, a.nx, a.ny, a.x_edge, a.y_edge, a.t_x_lo, a.t_x_hi,
                        a.t_y_lo, a.t_y_hi);
        buf_store_stream(out, ro, boff, d * plane_bytes);
      } else if constexpr (EDGE) {
        if (!ok) continue;
        if (a.y_edge == kDiffuse) {
          if (y == 0 && dy == 1) out = fmaf(wi, (hop ? sTg : sWTg)[lane + 1 - dx], out);
          if (y == a.ny - 1 && dy == -1)
            out = fmaf(wi, (hop ? sTg : sWTg)[T::LP + lane + 1 - dx], out);
          // specular share (Eq. adiabatic-specular): the packet that the
          // mirror direction m sends across the wall from (x - dx_m, y),
          // when its own pending move points out through that wall, is
          // reflected there and ends the step here, in direction i
          if (a.spec > 0.f && (y == 0 || y == a.ny - 1)) {
            const int m = scalar_ptr(a.mtab)[i];
            int mdx, mdy;
            bool mhop;
            decode((codes[m >> 2] >> (8 * (m & 3))) & 0xffu, mdx, mdy, mhop);
            if ((y == 0 && mdy == -1) || (y == a.ny - 1 && mdy == 1)) {
              const float em = a.e_in[(long long)m * plane + cell(x - mdx, y, pitch)];
              const int lsrc = lc - mdx;
              const float Ws = WF ? sW[lsrc] : a.W;
              const float WEs = WF ? sE[lsrc] : a.W * sE[lsrc];
              const float pk = fmaf(wtab[m], WEs, mhop ? fmaf(-Ws, em, em) : 0.f);
              out = fmaf(a.spec, pk, out);
            }
          }
        }
        out = blackbody(out, wi, x, y, a.nx, a.ny, a.x_edge, a.y_edge, a.t_x_lo, a.t_x_hi,
                        a.t_y_lo, a.t_y_hi);
        if (ghost)
          store_ghosted(a.e_out + (long long)i * plane, x, y, out, a.nx, a.ny, pitch, px, py);
        else
          buf_store_stream(out, ro, boff, d * plane_bytes);
      } else {
        buf_store_stream(out, ro, boff, d * plane_bytes);
        if constexpr (GHOST) {
          if (gxl) buf_store_stream(out, ro, gbx, d * plane_bytes);
          if (gyl) buf_store_stream(out, ro, gby, d * plane_bytes);
          if (gxl && gyl) buf_store_stream(out, ro, gbxy, d * plane_bytes);
        }
      }
      bsum += out;
      if constexpr (FLUX) {
        bqx = fmaf(out, sxtab[i], bqx);
        bqy = fmaf(out, sytab[i], bqy);
      }
    }
    if constexpr (NW == 1) {
      Eacc += bsum;
      if constexpr (FLUX) {
        qx += bqx;
        qy += bqy;
      }
    } else {
      sBat[(i0 / D) * nrow + row * 64 + lane] = bsum;
      if constexpr (FLUX) {
        sBat[(nbat + i0 / D) * nrow + row * 64 + lane] = bqx;
        sBat[(2 * nbat + i0 / D) * nrow + row * 64 + lane] = bqy;
      }
    }
  };
  // the first two batches were loaded before the E tile was staged; each
  // later batch is loaded while the one before it is relaxed
  relax_batch(part * share, v0);
  const int i_end = (part + 1) * share;
  float vc[D];
#pragma unroll
  for (int d = 0; d < D; ++d) vc[d] = v1[d];
  for (int i0 = part * share + D; i0 < i_end; i0 += D) {
    float vn[D];
    const bool more = i0 + D < i_end;
    if (more) load_batch<D, TAB>(a, i0 + D, boff, vn);
    relax_batch(i0, vc);
    if (more) {
#pragma unroll
      for (int d = 0; d < D; ++d) vc[d] = vn[d];
    }
  }

  if constexpr (NW > 1) {
    // batch sums of E' and of the flux in batch order
    constexpr int n = nrow;
    lds_barrier();
    if (part != 0) return;
    const int base = row * 64 + lane;
    for (int k = 0; k < nbat; ++k) Eacc += sBat[k * n + base];
    if constexpr (FLUX) {
      for (int k = 0; k < nbat; ++k) {
        qx += sBat[(nbat + k) * n + base];
        qy += sBat[(2 * nbat + k) * n + base];
      }
    }
  }
  if (!ok) return;
  if (ghost)
    store_ghosted(a.E_out, x, y, Eacc, a.nx, a.ny, pitch, px, py);
  else
    buf_store(Eacc, make_rsrc(a.E_out, plane_bytes), boff);
  if constexpr (FLUX) {
    const long long o = (long long)y * a.nx + x;
    if (a.q_first) {
      a.qsx[o] = double(qx);
      a.qsy[o] = double(qy);
    } else {
      a.qsx[o] += double(qx);
      a.qsy[o] += double(qy);
    }
  }
}


// LDS of one block of the step kernel.
template <int NW, bool WF, bool FLUX>
struct StepShared {
  using T = TileShape<NW>;
  float sE[T::LH * T::LP];
  float sW[WF ? T::LH * T::LP : 1];
  float sTg[2 * T::LP];
  float sWTg[2 * T::LP];
  float sInflow[2 * T::LP * kNodeParts];   // partial inflows of diffuse-wall nodes
};

// One block's tile t of one time step of lattice a.
template <int NW, bool WF, bool FLUX, bool TAB>
__device__ __forceinline__ void step_tile(const StepArgs& a, int t,
                                          StepShared<NW, WF, FLUX>& sh) {
  using T = TileShape<NW>;
  float* sE = sh.sE;
  float* sW = sh.sW;
  float* sTg = sh.sTg;
  float* sWTg = sh.sWTg;
  // when NW > 1: [q / 8][tile cells] batch sums of E', then (FLUX) of q_x, q_y
  extern __shared__ float sBat[];
  const int tx = t % a.tiles_x;
  const int ty = t / a.tiles_x;
  const int x0 = tx * T::TX;
  const int y0 = ty * T::TY;

  // This thread's cell, and the first two batches of its directions, loaded
  // before the E tile so that the memory round trips overlap.  Lanes outside
  // a ragged lattice read a valid cell and store nothing.
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cx = x0 + (threadIdx.x & 63);
  const int cy = y0 + wave / NW;
  const bool inside = cx < a.nx && cy < a.ny;
  const uint32_t boff = uint32_t(cell(inside ? cx : 0, inside ? cy : 0, a.pitch) * 4);
  float v0[T::D], v1[T::D] = {};
  const int i_first = (wave % NW) * (a.q / NW);
  load_batch<T::D, TAB>(a, i_first, boff, v0);
  if (a.q / NW > T::D) load_batch<T::D, TAB>(a, i_first + T::D, boff, v1);

  // Stage E (per-cell mode: W E) and W of the tile plus a one-cell halo.
  // Ghost rows/columns give the wrapped values of periodic edges and zero
  // beyond walls; cells past the ragged end of the lattice read as zero.
  for (int k = threadIdx.x; k < T::LH * T::LP; k += kBlock) {
    const int rr = k / T::LP;
    const int cc = k - rr * T::LP;
    const int gx = x0 - 1 + cc;
    const int gy = y0 - 1 + rr;
    float ev = 0.f, wv = 0.f;
    if (gx <= a.nx && gy <= a.ny) {
      const long long o = cell(gx, gy, a.pitch);
      ev = a.E_in[o];
      if constexpr (WF) {
        wv = a.Wf[o];
        ev *= wv;
      }
    }
    sE[k] = ev;
    if constexpr (WF) sW[k] = wv;
  }
  const bool edge = x0 == 0 || x0 + T::TX >= a.nx || y0 == 0 || y0 + T::TY >= a.ny;
  // only a blackbody x edge, every lane inside and no row on a y edge
  const bool xwall = edge && a.x_edge == kBlackbody && x0 + T::TX <= a.nx && y0 > 0 &&
                     y0 + T::TY < a.ny;
  if (edge && !xwall && a.y_edge == kDiffuse) {
    // The inflow of each node of the tile's wall rows (and halo) is summed
    // by kNodeParts threads over consecutive ranges of 8-direction batches,
    // then the parts are added in order (node_inflow, node_part_batches).
    const bool lo = y0 == 0;
    const bool hi = a.ny - 1 < y0 + T::TY;
    const int nb = a.q / kMaxGroupPlanes;
    const int per = node_part_batches(nb);
    for (int k = threadIdx.x; k < 2 * T::LP * kNodeParts; k += kBlock) {
      const int node = k / kNodeParts, part = k - node * kNodeParts;
      const int wall = node / T::LP;
      if (wall == 0 ? !lo : !hi) continue;
      int X = x0 - 1 + (node - wall * T::LP);
      float tg, wtg;
      if (node_fixed<WF>(a, wall, X, tg, wtg)) continue;
      const int b0 = min(nb, part * per), b1 = min(nb, b0 + per);
      sh.sInflow[k] = node_inflow<WF>(a, wall, X, b0, b1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 2 * T::LP; k += kBlock) {
      const int wall = k / T::LP;
      if (wall == 0 ? !lo : !hi) continue;
      int X = x0 - 1 + (k - wall * T::LP);
      float tg, wtg;
      if (!node_fixed<WF>(a, wall, X, tg, wtg)) {
        float R = sh.sInflow[k * kNodeParts];
#pragma unroll
        for (int p = 1; p < kNodeParts; ++p) R += sh.sInflow[k * kNodeParts + p];
        node_emit<WF>(a, wall, X, R, tg, wtg);
      }
      sTg[k] = tg;
      sWTg[k] = wtg;
    }
  }
  __syncthreads();
  // on a lattice with both edges periodic, a tile on the edge that holds no
  // ragged lane only adds the ghost copies to the interior path
  const bool pghost = edge && a.x_edge == kPeriodic && a.y_edge == kPeriodic &&
                      x0 + T::TX <= a.nx && y0 + T::TY <= a.ny;
  if (xwall)
    sweep<NW, WF, FLUX, TAB, false, true>(a, sE, sW, sTg, sWTg, sBat, x0, y0, boff, v0, v1);
  else if (pghost)
    sweep<NW, WF, FLUX, TAB, false, false, true>(a, sE, sW, sTg, sWTg, sBat, x0, y0, boff, v0,
                                            v1);
  else if (edge)
    sweep<NW, WF, FLUX, TAB, true>(a, sE, sW, sTg, sWTg, sBat, x0, y0, boff, v0, v1);
  else
    sweep<NW, WF, FLUX, TAB, false>(a, sE, sW, sTg, sWTg, sBat, x0, y0, boff, v0, v1);
}

template <int NW, bool WF, bool FLUX>
__global__ __launch_bounds__(kBlock) void k_step(
    const StepArgs a) {
  __shared__ StepShared<NW, WF, FLUX> sh;
  step_tile<NW, WF, FLUX, true>(a, xcd_tile(blockIdx.x, gridDim.x), sh);
}

// One time step of several lattices in one launch.  The tiles of lattice j
// are blocks first[j] .. first[j+1]-1 of the (XCD-remapped) grid; each block
// reads its lattice's arguments for the current buffer parity from the table
// through the scalar cache and runs the same tile code as k_step.  GROUPED:
// the lattices have several direction sets, each block takes the schedule
// row of its lattice's ring.
template <int NW, bool WF, bool FLUX, bool GROUPED>
__global__ __launch_bounds__(kBlock) void k_step_batch(
    const BatchStepArgs b) {
  __shared__ StepShared<NW, WF, FLUX> sh;
  const int g = xcd_tile(blockIdx.x, gridDim.x);
  const WLBM_CONST int* first = scalar_ptr(b.first);
  int j = 0;
  while (j + 1 < b.n && g >= first[j + 1]) ++j;
  j = __builtin_amdgcn_readfirstlane(j);
  StepArgs a = b.lats[2 * j + b.parity];
  const WLBM_CONST float* ins;
  if constexpr (GROUPED) {
    a.codes = scalar_ptr(b.ring_codes)[j] + size_t(b.row) * size_t(a.q >> 2);
    ins = scalar_ptr(scalar_ptr(b.ring_ins)[j]) + 4 * b.row;
  } else {
    a.codes = b.codes;
    ins = scalar_ptr(b.ins);
  }
  a.in_lo_hop = ins[0];
  a.in_lo_all = ins[1];
  a.in_hi_hop = ins[2];
  a.in_hi_all = ins[3];
  a.q_first = b.q_first;
  step_tile<NW, WF, FLUX, false>(a, g - first[j], sh);
}

template <int NW, bool WF, bool FLUX>
hipError_t launch_tmpl(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_step<NW, WF, FLUX>), dim3(a.ntiles), dim3(kBlock),
                     step_batch_lds_bytes(a.q, NW) * (FLUX ? 3 : 1), s, a);
  return hipGetLastError();
}

template <int NW>
hipError_t launch_nw(const StepArgs& a, bool wf, bool fl, hipStream_t s) {
  if (wf) return fl ? launch_tmpl<NW, true, true>(a, s) : launch_tmpl<NW, true, false>(a, s);
  return fl ? launch_tmpl<NW, false, true>(a, s) : launch_tmpl<NW, false, false>(a, s);
}

// ---------------------------------------------------------------------------
// Set-up, readout and reduction kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_init_temperature(const Geometry g, const float* T0,
                                                            float* e, float* E,
                                                            const float* wtab, Walls w) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= (long long)g.nx * g.ny) return;
  const int x = int(c % g.nx);
  const int y = int(c / g.nx);
  const bool px = g.x_edge == kPeriodic, py = g.y_edge == kPeriodic;
  const float T = T0[c];
  float sum = 0.f;
  for (int i = 0; i < g.q; ++i) {
    const float wi = wtab[i];
    const float v = blackbody(wi * T, wi, x, y, g.nx, g.ny, g.x_edge, g.y_edge, w.x_lo, w.x_hi,
                              w.y_lo, w.y_hi);
    store_ghosted(e + (long long)i * g.plane, x, y, v, g.nx, g.ny, g.pitch, px, py);
    sum += v;
  }
  store_ghosted(E, x, y, sum, g.nx, g.ny, g.pitch, px, py);
}

__global__ __launch_bounds__(kBlock) void k_init_populations(const Geometry g, const float* src,
                                                            float* e, float* E,
                                                            const float* wtab, Walls w) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long ncell = (long long)g.nx * g.ny;
  if (c >= ncell) return;
  const int x = int(c % g.nx);
  const int y = int(c / g.nx);
  const bool px = g.x_edge == kPeriodic, py = g.y_edge == kPeriodic;
  float sum = 0.f;
  for (int i = 0; i < g.q; ++i) {
    const float v = blackbody(src[(long long)i * ncell + c], wtab[i], x, y, g.nx, g.ny,
                              g.x_edge, g.y_edge, w.x_lo, w.x_hi, w.y_lo, w.y_hi);
    store_ghosted(e + (long long)i * g.plane, x, y, v, g.nx, g.ny, g.pitch, px, py);
    sum += v;
  }
  store_ghosted(E, x, y, sum, g.nx, g.ny, g.pitch, px, py);
}

// Internal sources (Sec. 2.6, Eq. isotropic and Eq. anisotropic): the DDEDs
// of source cell s are overwritten by vals[s][0..q-1], E by their sum (in
// direction order), with the ghost copies of periodic edges.  Cells are
// distinct and inside the lattice (checked by the host).
__global__ __launch_bounds__(kBlock) void k_apply_sources(const Geometry g, float* e, float* E,
                                                         const int32_t* cells,
                                                         const float* vals, int n) {
  const int s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= n) return;
  const int x = cells[2 * s], y = cells[2 * s + 1];
  const bool px = g.x_edge == kPeriodic, py = g.y_edge == kPeriodic;
  float sum = 0.f;
  for (int i = 0; i < g.q; ++i) {
    const float v = vals[(long long)s * g.q + i];
    store_ghosted(e + (long long)i * g.plane, x, y, v, g.nx, g.ny, g.pitch, px, py);
    sum += v;
  }
  store_ghosted(E, x, y, sum, g.nx, g.ny, g.pitch, px, py);
}

__global__ __launch_bounds__(kBlock) void k_read_populations(const Geometry g, const float* e,
                                                            float* dst) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long ncell = (long long)g.nx * g.ny;
  if (c >= ncell) return;
  const int i = blockIdx.y;
  const int x = int(c % g.nx);
  const int y = int(c / g.nx);
  dst[(long long)i * ncell + c] = e[(long long)i * g.plane + cell(x, y, g.pitch)];
}

__global__ __launch_bounds__(kBlock) void k_read_field(const Geometry g, const float* f,
                                                      float* dst) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= (long long)g.nx * g.ny) return;
  dst[c] = f[cell(int(c % g.nx), int(c / g.nx), g.pitch)];
}

__global__ __launch_bounds__(kBlock) void k_axpy_field(const Geometry g, float a, const float* f,
                                                      float* dst) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= (long long)g.nx * g.ny) return;
  dst[c] = fmaf(a, f[cell(int(c % g.nx), int(c / g.nx), g.pitch)], dst[c]);
}

__global__ __launch_bounds__(kBlock) void k_read_flux(const Geometry g, const float* e,
                                                     const float* sxtab, const float* sytab,
                                                     float* qx, float* qy) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= (long long)g.nx * g.ny) return;
  const long long o = cell(int(c % g.nx), int(c / g.nx), g.pitch);
  float ax = 0.f, ay = 0.f;
  for (int i = 0; i < g.q; ++i) {
    const float v = e[(long long)i * g.plane + o];
    ax = fmaf(v, sxtab[i], ax);
    ay = fmaf(v, sytab[i], ay);
  }
  qx[c] = ax;
  qy[c] = ay;
}

__global__ __launch_bounds__(kBlock) void k_scale_pair(int n, const double* ax, const double* ay,
                                                      double s, float* bx, float* by) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  bx[c] = float(ax[c] * s);
  by[c] = float(ay[c] * s);
}

__device__ __forceinline__ double corrected(double mfp, double lam, double f, int corr) {
  const double W = isinf(mfp) ? 0.0 : 1.0 / mfp;
  if (!corr) return W;
  return f * ((1.0 - W) * W + W * (W * lam));
}

__global__ __launch_bounds__(kBlock) void k_check_mfp(const Geometry g, const float* mfp,
                                                     double lam, double f, int corr, int* flag) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= (long long)g.nx * g.ny) return;
  const double m = mfp[c];
  bool bad = !(m > 0.0);
  if (!bad) {
    const double wc = corrected(m, lam, f, corr);
    bad = !(wc <= 1.0) || !isfinite(wc);
  }
  if (bad) *flag = 1;
}

__global__ __launch_bounds__(kBlock) void k_write_wfield(const Geometry g, const float* mfp,
                                                        double lam, double f, int corr,
                                                        float* Wf, float* Wraw) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= (long long)g.nx * g.ny) return;
  const int x = int(c % g.nx);
  const int y = int(c / g.nx);
  const double m = mfp[c];
  store_ghosted(Wf, x, y, float(corrected(m, lam, f, corr)), g.nx, g.ny, g.pitch,
                g.x_edge == kPeriodic, g.y_edge == kPeriodic);
  Wraw[c] = float(isinf(m) ? 0.0 : 1.0 / m);
}

unsigned cell_blocks(const Geometry& g) {
  return unsigned(((long long)g.nx * g.ny + kBlock - 1) / kBlock);
}

}  // namespace

size_t step_batch_lds_bytes(int q, int split) {
  if (split <= 1) return 0;
  return size_t(q / kMaxGroupPlanes) * (4 / split) * 64 * sizeof(float);
}

int tiles_x_for(int nx) { return (nx + 63) / 64; }
int tiles_y_for(int ny, int split) {
  const int ty = 4 / split;
  return (ny + ty - 1) / ty;
}

template <int NW, bool WF, bool FLUX, bool GROUPED>
hipError_t launch_batch_tmpl(const BatchStepArgs& b, hipStream_t s) {
  hipLaunchKernelGGL((k_step_batch<NW, WF, FLUX, GROUPED>), dim3(b.nblocks), dim3(kBlock),
                     step_batch_lds_bytes(b.q, NW) * (FLUX ? 3 : 1), s, b);
  return hipGetLastError();
}

template <int NW, bool GROUPED>
hipError_t launch_batch_wf(const BatchStepArgs& b, bool wf, bool fl, hipStream_t s) {
  if (wf)
    return fl ? launch_batch_tmpl<NW, true, true, GROUPED>(b, s)
              : launch_batch_tmpl<NW, true, false, GROUPED>(b, s);
  return fl ? launch_batch_tmpl<NW, false, true, GROUPED>(b, s)
            : launch_batch_tmpl<NW, false, false, GROUPED>(b, s);
}

template <int NW>
hipError_t launch_batch_nw(const BatchStepArgs& b, bool wf, bool fl, bool grouped,
                           hipStream_t s) {
  return grouped ? launch_batch_wf<NW, true>(b, wf, fl, s) : launch_batch_wf<NW, false>(b, wf, fl, s);
}

hipError_t launch_step(const StepArgs& a, int split, bool per_cell, bool flux, hipStream_t s) {
  switch (split) {
    case 1: return launch_nw<1>(a, per_cell, flux, s);
    case 2: return launch_nw<2>(a, per_cell, flux, s);
    case 4: return launch_nw<4>(a, per_cell, flux, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step_batch(const BatchStepArgs& b, int split, bool per_cell, bool flux,
                             bool grouped, hipStream_t s) {
  switch (split) {
    case 1: return launch_batch_nw<1>(b, per_cell, flux, grouped, s);
    case 2: return launch_batch_nw<2>(b, per_cell, flux, grouped, s);
    case 4: return launch_batch_nw<4>(b, per_cell, flux, grouped, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init_temperature(const Geometry& g, const float* T0, float* e, float* E,
                                   const float* wtab, Walls walls, hipStream_t s) {
  hipLaunchKernelGGL(k_init_temperature, dim3(cell_blocks(g)), dim3(kBlock), 0, s, g, T0, e, E,
                     wtab, walls);
  return hipGetLastError();
}

hipError_t launch_init_populations(const Geometry& g, const float* src, float* e, float* E,
                                   const float* wtab, Walls walls, hipStream_t s) {
  hipLaunchKernelGGL(k_init_populations, dim3(cell_blocks(g)), dim3(kBlock), 0, s, g, src, e, E,
                     wtab, walls);
  return hipGetLastError();
}

hipError_t launch_apply_sources(const Geometry& g, float* e, float* E, const int32_t* cells,
                                const float* vals, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply_sources, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g, e,
                     E, cells, vals, n);
  return hipGetLastError();
}

hipError_t launch_read_populations(const Geometry& g, const float* e, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_read_populations, dim3(cell_blocks(g), g.q), dim3(kBlock), 0, s, g, e,
                     dst);
  return hipGetLastError();
}

hipError_t launch_read_field(const Geometry& g, const float* f, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_read_field, dim3(cell_blocks(g)), dim3(kBlock), 0, s, g, f, dst);
  return hipGetLastError();
}

hipError_t launch_axpy_field(const Geometry& g, float a, const float* f, float* dst,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_field, dim3(cell_blocks(g)), dim3(kBlock), 0, s, g, a, f, dst);
  return hipGetLastError();
}

hipError_t launch_read_flux(const Geometry& g, const float* e, const float* sxtab,
                            const float* sytab, float* qx, float* qy, hipStream_t s) {
  hipLaunchKernelGGL(k_read_flux, dim3(cell_blocks(g)), dim3(kBlock), 0, s, g, e, sxtab, sytab,
                     qx, qy);
  return hipGetLastError();
}

hipError_t launch_scale_pair(int n, const double* ax, const double* ay, double scale, float* bx,
                             float* by, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_pair, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, ax, ay,
                     scale, bx, by);
  return hipGetLastError();
}

hipError_t launch_check_mfp(const Geometry& g, const float* mfp, double lam, double f, int corr,
                            int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_mfp, dim3(cell_blocks(g)), dim3(kBlock), 0, s, g, mfp, lam, f, corr,
                     flag);
  return hipGetLastError();
}

hipError_t launch_write_wfield(const Geometry& g, const float* mfp, double lam, double f,
                               int corr, float* Wf, float* Wraw, hipStream_t s) {
  hipLaunchKernelGGL(k_write_wfield, dim3(cell_blocks(g)), dim3(kBlock), 0, s, g, mfp, lam, f,
                     corr, Wf, Wraw);
  return hipGetLastError();
}

}  // namespace wlbm
