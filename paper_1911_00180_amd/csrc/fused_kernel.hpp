// Several time steps of the worm-LBM per launch (temporal blocking) for
// gfx950: the kernel template, included by fused.hip (lattices with both
// edges periodic) and fused_walls{2,3,4}.hip (lattices with blackbody or
// diffuse edges, one file per number of steps per launch so that they
// compile in parallel).
//
// One launch of k_stepk<..., K, WALLS> advances a lattice by steps n+1 ..
// n+K, K = 2, 3 or 4 (Sec. 2.3 Eq. algorithm, pull form as in k_step): each
// population is read from HBM once and written once per K steps, instead of
// once per step.
//
// A block owns a strip of kStrip columns and a.rows rows of the output.  Its
// NW waves cover the same 64 columns x0-K .. x0+63-K (x0-2K .. x0+63-2K with
// walls, kLane0), one per lane, and take
// SH directions each (8, or 16; see launch_fused_qk).  Rows are pipelined: at
// iteration t the waves compute level 1 (step n+1) of row r = y0-(K-1)+t from
// the step-n populations in HBM, then level l of row r-(l-1) for l = 2 .. K
// from level l-1, whose rows r-l .. r-l+2 are held in registers, a ring of
// three rows per level; level K is the output.  The one-cell shifts in x of
// the pulled populations are lane shifts of a whole wave (DPP wave_shr /
// wave_shl), so level l is valid on lanes l .. 63-l; E, which every
// direction reads at its own move, is read from the block's LDS ring of E
// rows at a shifted address.  E of each row of each level is summed over the
// waves in LDS in k_step's order (8-direction batch sums in batch order), and
// every update uses k_step's arithmetic, so one launch gives the same bits as
// K k_step launches.  Every wave adds the same batch sums in the same order
// and writes the row it has summed into the ring: the waves write the same
// bits to the same words, so a wave reads back what it has written itself
// and the ring needs no barrier of its own (a slot is overwritten only after
// the barrier that follows the last reads of its old row).
//
// Edges.  A periodic axis reads the ghost frame (kGhost columns, one row),
// which must hold the wrapped values on entry (the caller refreshes it with
// k_fill_ghosts after other producers) and which the kernel writes for its
// output; step-n rows wrap by comparison as they advance.  With WALLS the
// kernel also takes blackbody x and y edges and adiabatic diffuse y walls
// (Sec. 2.6), with the same bits as k_step:
// * rows beyond a non-periodic y edge are zero at every level (as the zero
//   ghost rows k_step reads), and their loads are clamped into the lattice;
//   columns beyond a blackbody x edge only feed the wall column, which is
//   overwritten;
// * blackbody cells are overwritten with w_i T at every level (Eq.
//   isotropic; y walls first, x walls win at corners);
// * at a diffuse wall row each level first computes the wall's boundary
//   nodes (Eq. adiabatic-diffuse): the inflow of node X is the sum of the
//   packets that the pull form delivers to a cell at the node's position,
//   from the wall row of the previous level, for the directions whose move
//   leaves through the wall (summed per 8-direction batch, the batches
//   grouped as k_step groups them); the node re-emits it as w_i T_g into the
//   inward directions of the wall row.
//
// Flux windows.  k_stepk_flux and k_stepk_batch_flux (the same code with
// FLUX set) also add the heat flux q = sum_i e_i s_i (Sec. 2.2 Eq. q_corr)
// of the launch's flux-window steps to the window's float64 per-cell sums,
// in k_step's order, so a window gives the same sums with any number of
// steps per launch.
//
// Scalar work per direction is kept to loads: the host writes, per step and
// direction, the byte offset of the direction's entry in the selection table
// and, for the first step, the offset of its pulled population, so the kernel
// decodes no schedule codes in the bulk (scalar instruction issue limits this
// kernel as much as vector issue does); wall rows decode the codes.
#pragma once

#include "device.hpp"
#include "kernel_common.hpp"

namespace wlbm {
namespace {

// Output columns per block (lanes K .. K + kStrip - 1) for K steps per
// launch: 48, a multiple of 16, so that every block's output rows are whole
// 64-byte write segments (x = 0 starts a 128-byte line).  With 60 or 56
// columns most rows end in partial segments on both sides, and those partial
// writes cost more than the idle lanes (1024 x 1024, Q = 64: four steps per
// launch 1627 G updates/s with 48 columns against 1490 with 56; three steps
// 1333 against 1209; two steps 998 against 846).
template <int K>
constexpr int kStrip = 48;
// Lane of a block's first output column.  A cell depends on cells at most one
// column away per step, so level l is valid on lanes l .. 63 - l and the
// strip starts at lane K; along a diffuse wall a cell also receives what
// its boundary node X - dx absorbed from wall cells X - dx - dx', two
// columns away per step, so the kernels with walls start at lane 2K (the
// 48-column strip then fits for K <= 4; with periodic x edges the kGhost
// ghost columns cover 2K <= 4, so such lattices run at most two steps per
// launch).
template <int K, bool WALLS>
constexpr int kLane0 = WALLS ? 2 * K : K;
// Ghost columns written on each side by every multi-step launch of a lattice
// with periodic x (the most any K reads), so that launches of different K
// can follow each other.
constexpr int kGhost = 4;

// Value held by lane l - 1 (the cell at x - 1), lane l + 1 (x + 1); lanes
// with no such neighbour (0, resp. 63) read zero (bound control), which no
// result uses.
__device__ __forceinline__ float from_lower_lane(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_upper_lane(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               0x130, 0xF, 0xF, true));
}
// The value at column x - dx for a wave-uniform dx in {-1, 0, 1}.
__device__ __forceinline__ float shift_by(float v, int dx) {
  if (dx > 0) return from_lower_lane(v);
  if (dx < 0) return from_upper_lane(v);
  return v;
}
// Selections by a direction's move are wave-uniform.  Rather than comparing
// and selecting on the decoded move in scalar code for every direction and
// row, the kernel loads the entry of the move's code from this table (one
// scalar load per direction, at a byte offset the host writes per step and
// direction) and selects with bitwise operations.  Entry c, for code
// c = dx + 1 | (dy + 1) << 2 | hop << 4 with (hx, hy) the move on a hop and
// (0, 0) on a pause: the lane masks of hy = -1, hy = 0, hx > 0 and hx < 0,
// then, for each iteration slot S, the byte offset of E at (x - dx, rho - dy)
// in the block's LDS ring of E rows, from the lane's own entry in slot 0
// (rows rho - 1, rho, rho + 1 are in slots S, S + 2, S + 1 mod 3).
enum SelWord : int { kHyLo, kHyMid, kHxPos, kHxNeg, kEOff0, kEOff1, kEOff2, kSelWords = 8 };
// Row length (floats) of one E row in LDS: 64 lanes and one pad either side
// for the lane shifts.
constexpr int kERow = 66;
struct CodeSel {
  uint32_t m[32][kSelWords];
};
constexpr CodeSel make_code_sel() {
  CodeSel t{};
  for (int c = 0; c < 32; ++c) {
    const int dx = (c & 3) - 1, dy = ((c >> 2) & 3) - 1;
    const bool hop = (c >> 4) & 1;
    const int hx = hop ? dx : 0, hy = hop ? dy : 0;
    auto m = [](bool b) { return b ? 0xffffffffu : 0u; };
    t.m[c][kHyLo] = m(hy == -1);
    t.m[c][kHyMid] = m(hy == 0);
    t.m[c][kHxPos] = m(hx > 0);
    t.m[c][kHxNeg] = m(hx < 0);
    for (int S = 0; S < 3; ++S) {
      const int slot = dy == -1 ? S : (dy == 0 ? (S + 2) % 3 : (S + 1) % 3);
      t.m[c][kEOff0 + S] = uint32_t(4 * (slot * kERow - dx));
    }
  }
  return t;
}
__constant__ CodeSel kCodeSel = make_code_sel();
static_assert(kSelWords * 4 == kSelEntryBytes, "selection entry size");

// The selection masks of a direction whose entry in the launch's table of
// selection offsets is `off` (bytes into the table: its code times the
// entry size).
__device__ __forceinline__ const WLBM_CONST uint32_t* sel_at(const WLBM_CONST uint32_t* tab,
                                                             uint32_t off) {
  return reinterpret_cast<const WLBM_CONST uint32_t*>(reinterpret_cast<const WLBM_CONST char*>(tab) +
                                                      off);
}
__device__ __forceinline__ float bsel(uint32_t m, float a, float b) {
  return __builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, a) & m) |
                                       (__builtin_bit_cast(uint32_t, b) & ~m));
}
// a where m_lo, b where m_mid, else c
__device__ __forceinline__ float pick3m(float a, float b, float c, uint32_t m_lo, uint32_t m_mid) {
  return bsel(m_lo, a, bsel(m_mid, b, c));
}
// The value at column x - dx (dx uniform, given by its masks).  Both shifts
// are computed and one is selected, so that no branch surrounds the
// (convergent) lane shifts.
__device__ __forceinline__ float at_minus(float v, uint32_t m_pos, uint32_t m_neg) {
  const float lo = from_lower_lane(v), up = from_upper_lane(v);
  return bsel(m_pos, lo, bsel(m_neg, up, v));
}
// A scalar-cache pointer that the optimizer cannot see through: loads through
// it are re-issued in every row instead of being hoisted out of the row loop
// and kept (spilled) in scalar registers with everything derived from them.
template <class T>
__device__ __forceinline__ const WLBM_CONST T* row_ptr(const T* p) {
  __asm__ volatile("" : "+s"(p));
  return scalar_ptr(p);
}

template <int SH, int K>
struct Ring {
  float X[K - 1][3][SH];   // levels 1 .. K-1: populations of this wave's directions
  float E[K - 1][3];       // E of those rows (per-cell mode: W E) at this lane's column
  float W[K - 1][3];       // W of those rows at this lane's column (per-cell mode)
  float En[3];             // step n E (per-cell mode: W E), rows by slot
  float Wn[3];             // step n W (per-cell mode)
  float V[SH];             // step n populations pulled into the next level-1 row
  uint32_t rb[3];          // byte offsets of the step-n rows, by slot
  int wn;                  // newest step-n row loaded: wrapped (periodic y), else absolute
};

// Per-lane and per-block facts about the edges (WALLS kernels).
struct EdgeCtx {
  int x;              // this lane's column
  bool blk_xbb;       // some lane of the block is a blackbody x column
  uint32_t xbb;       // all ones where this lane's column is a blackbody x column
  float xbb_t;        // its wall temperature
  bool x_in;          // this lane's column lies inside the lattice
};

// Per-row wall facts at one level (WALLS kernels): row rho outside a
// non-periodic y edge, a blackbody y row (and its temperature), a diffuse
// wall row (wall 0: lo, row 0; wall 1: hi, row ny - 1).
struct RowWalls {
  bool outside;
  bool ybb;
  float ybb_t;
  int diffuse;        // -1: not a diffuse wall row, else the wall
};
__device__ __forceinline__ RowWalls row_walls(const FusedArgs& a, int rho) {
  RowWalls w;
  w.outside = a.y_edge != kPeriodic && (rho < 0 || rho >= a.ny);
  w.ybb = a.y_edge == kBlackbody && (rho == 0 || rho == a.ny - 1);
  w.ybb_t = rho == 0 ? a.t_y_lo : a.t_y_hi;
  w.diffuse = a.y_edge != kDiffuse ? -1 : (rho == 0 ? 0 : (rho == a.ny - 1 ? 1 : -1));
  return w;
}

__device__ __forceinline__ void decode_at(const WLBM_CONST uint32_t* codes, int i, int& dx,
                                          int& dy, bool& hop) {
  decode((codes[i >> 2] >> (8 * (i & 3))) & 0xffu, dx, dy, hop);
}

// T_g and W_g T_g of the boundary nodes behind diffuse wall `wall` at each
// lane's column for the step of level L (codes, ins), from row rho of the
// previous level: src holds this wave's populations of that row at its own
// lane, eRow that row's E in the LDS ring (per-cell mode: W E), Wrow
// the row's W at its own lane (per-cell mode).  Each wave sums its batches of
// the packets leaving through the wall into sR; after an LDS barrier every
// wave adds all batches in k_step's grouping (node_part_batches).  sR is the
// level's E batch-sum buffer of the other row parity, last read for the
// previous row: a barrier first lets every wave finish those reads.
template <int NW, int SH, bool WF>
__device__ __forceinline__ void wall_nodes(const FusedArgs& a, const EdgeCtx& ec,
                                           const WLBM_CONST uint32_t* codes,
                                           const WLBM_CONST float* ins, int wall, const float (&src)[SH], const float* eRow,
                                           float Wrow, float* sR, int lane, int part, float& tg,
                                           float& wtg) {
  constexpr int NB = NW * SH / kMaxGroupPlanes;
  const WLBM_CONST float* wtab = scalar_ptr(a.wtab);
  const int out_dy = wall == 0 ? -1 : 1;
  lds_barrier();
#pragma unroll
  for (int b0 = 0; b0 < SH; b0 += kMaxGroupPlanes) {
    float R = 0.f;
#pragma unroll
    for (int d = 0; d < kMaxGroupPlanes; ++d) {
      const int i = part * SH + b0 + d;
      int dx, dy;
      bool hop;
      decode_at(codes, i, dx, dy, hop);
      if (dy != out_dy) continue;
      const float sv = shift_by(src[b0 + d], dx);
      const float e = hop ? sv : 0.f;
      const float Es = eRow[1 + lane - dx];
      float o;
      if constexpr (!WF) {
        o = fmaf(a.W, fmaf(wtab[i], Es, -e), e);
      } else {
        const float Ws = shift_by(Wrow, dx);
        o = e + fmaf(wtab[i], Es, -(Ws * e));
      }
      R += o;
    }
    sR[((part * SH + b0) / kMaxGroupPlanes) * 64 + lane] = R;
  }
  lds_barrier();
  const int per = node_part_batches(NB);
  float S[kNodeParts];
#pragma unroll
  for (int p = 0; p < kNodeParts; ++p) {
    float s = 0.f;
    const int b1 = min(NB, (p + 1) * per);
    for (int b = p * per; b < b1; ++b) s += sR[b * 64 + lane];
    S[p] = s;
  }
  float R = S[0];
#pragma unroll
  for (int p = 1; p < kNodeParts; ++p) R += S[p];
  const float Wg = WF ? Wrow : a.W;
  const float hs = ins[2 * wall], as = ins[2 * wall + 1];
  const float C = fmaf(Wg, as - hs, hs);
  tg = R / C;
  if (a.x_edge == kBlackbody) {
    // nodes behind a blackbody column belong to that wall; none beyond it
    if (!ec.x_in) tg = 0.f;
    if (ec.xbb) tg = ec.xbb_t;
  }
  wtg = Wg * tg;
}

// Issue the loads of level-1 row r: the step-n populations each of this
// wave's directions pulls (row r - hy, column x - hx) into g.V, and step-n E
// (and W) of row r + 1 into ring slot SN.  Nothing waits for them here.
// With three or four steps per launch the wave issues them at raised priority
// so that they leave early (four steps at 1024 x 1024, Q = 64: +2 %; with
// two steps raising it cost 2 %).  Rows beyond a non-periodic y edge load a
// row inside (their results are replaced by zero) and their E and W read 0.
template <int SH, int K, bool WF, int SN, bool WALLS>
__device__ __forceinline__ void issue_row(const FusedArgs& a, Ring<SH, K>& g, int i_begin,
                                          uint32_t lcol) {
  if constexpr (K >= 3) __builtin_amdgcn_s_setprio(3);
  const WLBM_CONST uint32_t* pulls = row_ptr(a.pulls);
  const long long plane = a.plane;
  const uint32_t plane_bytes = uint32_t(plane * 4);
  int row;
  bool valid = true;
  if (!WALLS || a.y_edge == kPeriodic) {
    // the rows advance by one per call: wrap the newest index by comparison
    g.wn = g.wn + 1 == a.ny ? 0 : g.wn + 1;
    row = g.wn;
  } else {
    g.wn += 1;
    row = min(max(g.wn, 0), a.ny - 1);
    valid = g.wn >= 0 && g.wn < a.ny;
  }
  g.rb[SN] = uint32_t((row + 1) * a.pitch * 4);
  const uint32_t rb_m = g.rb[SN], rb_0 = g.rb[(SN + 2) % 3];
  {
    const float Ev = buf_load(make_rsrc(a.E_in, plane_bytes), lcol, rb_m);
    if constexpr (WF) {
      const float Wv = buf_load(make_rsrc(a.Wf, plane_bytes), lcol, rb_m);
      g.Wn[SN] = valid ? Wv : 0.f;
      g.En[SN] = valid ? Ev * Wv : 0.f;
    } else {
      g.En[SN] = valid ? Ev : 0.f;
    }
  }
#pragma unroll
  for (int b0 = 0; b0 < SH; b0 += kMaxGroupPlanes) {
    const int i0 = i_begin + b0;
    // one row and one float before the batch: a pull's row r - hy and
    // column x - hx then sit at the non-negative offset in its table entry
    // (wrapped row r; rows -1 and ny are the ghost rows)
    const rsrc_t rs = make_rsrc(a.e_in + (long long)i0 * plane - 1 - a.pitch,
                                uint32_t((kMaxGroupPlanes * plane + a.pitch + 2) * 4));
#pragma unroll
    for (int d = 0; d < kMaxGroupPlanes; ++d)
      g.V[b0 + d] = buf_load(rs, lcol, rb_0 + pulls[i0 + d]);
  }
  if constexpr (K >= 3) __builtin_amdgcn_s_setprio(0);
}

// Per-row constants: schedule, weight and selection-table pointers opaque to
// the optimizer (re-read from the scalar cache each row rather than hoisted
// and spilled), and the plane size in bytes, likewise.
struct RowCtx {
  const WLBM_CONST float* wtab;
  const WLBM_CONST uint32_t* tab;
  uint32_t plane_bytes;
};
__device__ __forceinline__ RowCtx row_ctx(const FusedArgs& a) {
  RowCtx c;
  c.wtab = row_ptr(a.wtab);
  c.tab = row_ptr(&kCodeSel.m[0][0]);
  c.plane_bytes = uint32_t(a.plane * 4);
  __asm__ volatile("" : "+s"(c.plane_bytes));
  return c;
}

// The wall conditions of one updated population at a wall row or column
// (WALLS kernels): the diffuse node's emission into inward directions, then
// the blackbody overwrite (mask bbm, temperature bbt), as k_step applies
// them.
__device__ __forceinline__ float wall_update(float out, float wi, const RowWalls& rw,
                                             const WLBM_CONST uint32_t* codes, int i, float tg,
                                             float wtg, bool bb, uint32_t bbm, float bbt) {
  if (rw.diffuse >= 0) {
    int dx, dy;
    bool hop;
    decode_at(codes, i, dx, dy, hop);
    if (dy == (rw.diffuse == 0 ? 1 : -1)) out = fmaf(wi, shift_by(hop ? tg : wtg, dx), out);
  }
  if (bb) out = bsel(bbm, wi * bbt, out);
  return out;
}

// Blackbody mask and temperature of a row (WALLS kernels): x walls win at
// corners.
__device__ __forceinline__ bool row_bb(const EdgeCtx& ec, const RowWalls& rw, uint32_t& bbm,
                                       float& bbt) {
  bbm = ec.xbb | (rw.ybb ? 0xffffffffu : 0u);
  bbt = ec.xbb ? ec.xbb_t : rw.ybb_t;
  return ec.blk_xbb || rw.ybb;
}

// Heat flux of flux-window steps (FLUX kernels): each wave sums, per batch
// of 8 directions, q = sum_i out_i s_i as an fma chain in direction order
// into sQ (x then y, per level and row parity, as the E batch sums).  After
// the level's barrier the first wave adds the x batches in batch order, as
// k_step does, and the second wave the y batches (the first wave both if the
// block has one), for the cells the block outputs (rows y0 .. y0 + rows - 1
// of its strip), and keeps the step's sums in the block's ring sF until the
// row's last level; there the wave adds the launch's window steps, in step
// order, to the row's float64 window sums (fetched one output row ahead, so
// that the wave does not wait for HBM) and stores them.  Same bits as
// k_step's read-add-write per step.
struct FluxCtx {
  float* sQ;       // batch sums [level][row parity][x, y][batch][lane]
  float* sF;       // step sums [row mod K][level][x, y][lane]
  int x;           // this lane's column
  bool out_lane;   // the lane outputs a column of the lattice
  double p[2];     // window sums of the next output row: x, y (a wave that
                   // has one component keeps it in p[0])
};
template <int NB>
__device__ __forceinline__ float* flux_sums(const FluxCtx& fc, int L, int t) {
  return fc.sQ + (2 * (L - 1) + (t & 1)) * 2 * NB * 64;
}
// One component's batch sums of a row in batch order (as the E sums).
template <int NB>
__device__ __forceinline__ float flux_batch_sum(const float* q, int lane) {
  float v = 0.f;
#pragma unroll
  for (int k = 0; k < NB; ++k) v += q[k * 64 + lane];
  return v;
}
// Level L < K of row rho, component c (0: x, 1: y): the step's sum into the
// ring.
template <int NB, int K>
__device__ __forceinline__ void flux_level_c(const FusedArgs& a, const FluxCtx& fc, int L, int t,
                                             int rho, int y0, int lane, int c) {
  if (!((a.flux_levels >> (L - 1)) & 1u)) return;
  if (!fc.out_lane || rho < y0 || rho >= y0 + a.rows || rho >= a.ny) return;
  fc.sF[((rho % K) * K + (L - 1)) * 128 + c * 64 + lane] =
      flux_batch_sum<NB>(flux_sums<NB>(fc, L, t) + c * NB * 64, lane);
}
// The output level K of row ro, component c: the launch's window steps added
// to the row's sum in step order; then the next row's sum is fetched.
template <int NW, int NB, int K>
__device__ __forceinline__ void flux_out_c(const FusedArgs& a, FluxCtx& fc, int t, int ro, int y0,
                                           int lane, int c) {
  const uint32_t lv = a.flux_levels;
  if (lv == 0) return;
  double* sums = c == 0 ? a.qsx : a.qsy;
  if (fc.out_lane && ro < a.ny) {
    double acc = fc.p[NW == 1 ? c : 0];
    const float* f = fc.sF + (ro % K) * K * 128 + c * 64 + lane;
#pragma unroll
    for (int m = 1; m < K; ++m) {
      if ((lv >> (m - 1)) & 1u) {
        const double v = double(f[(m - 1) * 128]);
        acc = m == a.flux_first ? v : acc + v;
      }
    }
    if ((lv >> (K - 1)) & 1u) {
      const double v = double(flux_batch_sum<NB>(flux_sums<NB>(fc, K, t) + c * NB * 64, lane));
      acc = K == a.flux_first ? v : acc + v;
    }
    sums[(long long)ro * a.nx + fc.x] = acc;
  }
  const int rn = ro + 1;
  if (a.flux_first == 0 && fc.out_lane && rn < y0 + a.rows && rn < a.ny)
    fc.p[NW == 1 ? c : 0] = sums[(long long)rn * a.nx + fc.x];
}
// The flux work of a level's first waves (after the level's barrier).
template <int NW, int NB, int K>
__device__ __forceinline__ void flux_level(const FusedArgs& a, const FluxCtx& fc, int L, int t,
                                           int rho, int y0, int lane, int part) {
  if (part == 0) flux_level_c<NB, K>(a, fc, L, t, rho, y0, lane, 0);
  if (part == (NW == 1 ? 0 : 1)) flux_level_c<NB, K>(a, fc, L, t, rho, y0, lane, 1);
}
template <int NW, int NB, int K>
__device__ __forceinline__ void flux_out(const FusedArgs& a, FluxCtx& fc, int t, int ro, int y0,
                                         int lane, int part) {
  if (part == 0) flux_out_c<NW, NB, K>(a, fc, t, ro, y0, lane, 0);
  if (part == (NW == 1 ? 0 : 1)) flux_out_c<NW, NB, K>(a, fc, t, ro, y0, lane, 1);
}

// Level 1 at iteration t (row r = y0 - (K-1) + t, ring slot S = t mod 3)
// from the step-n loads; then the loads of the next row are issued, and E of
// row r is summed.  Step-n slots: rows r-1, r, r+1 are S, S+1, S+2 (mod 3).
template <int NW, int SH, int K, bool WF, int S, bool WALLS, bool FLUX>
__device__ __forceinline__ void level1(const FusedArgs& a, Ring<SH, K>& g, float* sP, float* eR,
                                       const EdgeCtx& ec, int t, int y0, int lane, int part,
                                       uint32_t lcol, const FluxCtx& fc) {
  constexpr int S1 = (S + 1) % 3, S2 = (S + 2) % 3;
  constexpr int NB = NW * SH / kMaxGroupPlanes;   // batches of 8 directions
  const RowCtx c = row_ctx(a);
  const WLBM_CONST uint32_t* sels = row_ptr(a.sels[0]);
  const int i_begin = part * SH;
  float* p1 = sP + (t & 1) * NB * 64;
  // step-n E of row r + 1 (loaded during the previous iteration) into the
  // LDS ring; rows r - 1 and r are there already
  eR[S2 * kERow + 1 + lane] = g.En[S2];
  __builtin_amdgcn_wave_barrier();
  const float* eLane0 = eR + 1 + lane;
  RowWalls rw{};
  float tg = 0.f, wtg = 0.f;
  uint32_t bbm = 0;
  float bbt = 0.f;
  bool bb = false;
  const WLBM_CONST uint32_t* codes = nullptr;
  if constexpr (WALLS) {
    const int r = y0 - (K - 1) + t;
    rw = row_walls(a, r);
    bb = row_bb(ec, rw, bbm, bbt);
    codes = row_ptr(a.codes);
    if (rw.diffuse >= 0) {
      // the wall row r of step n, at this lane's column: the packets that
      // leave through the wall come from it (one load per such direction)
      const int out_dy = rw.diffuse == 0 ? -1 : 1;
      const uint32_t rowb = g.rb[S1] + uint32_t(a.pitch) * 4u;
      float src[SH];
#pragma unroll
      for (int b0 = 0; b0 < SH; b0 += kMaxGroupPlanes) {
        const int i0 = i_begin + b0;
        const rsrc_t rs = make_rsrc(a.e_in + (long long)i0 * a.plane - 1 - a.pitch,
                                    uint32_t((kMaxGroupPlanes * a.plane + a.pitch + 2) * 4));
#pragma unroll
        for (int d = 0; d < kMaxGroupPlanes; ++d) {
          int dx, dy;
          bool hop;
          decode_at(codes, i0 + d, dx, dy, hop);
          src[b0 + d] = (dy == out_dy && hop)
                            ? buf_load(rs, lcol, rowb + 4u + uint32_t(d) * c.plane_bytes)
                            : 0.f;
        }
      }
      wall_nodes<NW, SH, WF>(a, ec, codes, row_ptr(a.ins), rw.diffuse, src, eR + S1 * kERow,
                             g.Wn[S1], sP + ((t + 1) & 1) * NB * 64, lane, part, tg, wtg);
    }
  }
  float* q1 = FLUX ? flux_sums<NB>(fc, 1, t) : nullptr;
  // s_x,i and s_y,i, re-read each row as the other per-direction tables
  const WLBM_CONST float* sx = FLUX ? row_ptr(a.sxtab) : nullptr;
  const WLBM_CONST float* sy = FLUX ? row_ptr(a.sytab) : nullptr;
#pragma unroll
  for (int b0 = 0; b0 < SH; b0 += kMaxGroupPlanes) {
    const int i0 = i_begin + b0;
    float bsum = 0.f, bqx = 0.f, bqy = 0.f;
#pragma unroll
    for (int d = 0; d < kMaxGroupPlanes; ++d) {
      const int i = i0 + d;
      const WLBM_CONST uint32_t* m = sel_at(c.tab, sels[i0 + d]);
      const float wi = c.wtab[i];
      const float e = g.V[b0 + d];
      // source rows r - dy: dy = -1 -> slot S2, 0 -> S1, 1 -> S
      const float Es = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(eLane0) +
                                                       int(m[kEOff0 + S2]));
      float out;
      if constexpr (!WF) {
        out = fmaf(a.W, fmaf(wi, Es, -e), e);
      } else {
        // W where the pulled population was: moved by (hx, hy)
        const float Wh = at_minus(pick3m(g.Wn[S2], g.Wn[S1], g.Wn[S], m[kHyLo], m[kHyMid]),
                                  m[kHxPos], m[kHxNeg]);
        out = e + fmaf(wi, Es, -(Wh * e));
      }
      if constexpr (WALLS) out = wall_update(out, wi, rw, codes, i, tg, wtg, bb, bbm, bbt);
      g.X[0][S][b0 + d] = out;
      bsum += out;
      if constexpr (FLUX) {
        bqx = fmaf(out, sx[i], bqx);
        bqy = fmaf(out, sy[i], bqy);
      }
    }
    p1[(i0 / kMaxGroupPlanes) * 64 + lane] = bsum;
    if constexpr (FLUX) {
      q1[(i0 / kMaxGroupPlanes) * 64 + lane] = bqx;
      q1[(NB + i0 / kMaxGroupPlanes) * 64 + lane] = bqy;
    }
  }
  // W of this row for the next level, before slot S is refilled
  if constexpr (WF) g.W[0][S] = g.Wn[S1];
  const float Wrow = WF ? g.Wn[S1] : 1.f;
  // loads of the next level-1 row (its step-n row r + 2 goes to slot S)
  if (t + 1 < a.rows + 2 * (K - 1)) issue_row<SH, K, WF, S, WALLS>(a, g, i_begin, lcol);
  // E of row r: the batch sums in batch order, as k_step adds them
  lds_barrier();
  float E = 0.f;
#pragma unroll
  for (int k = 0; k < NB; ++k) E += p1[k * 64 + lane];
  g.E[0][S] = WF ? E * Wrow : E;
  if constexpr (FLUX) {
    flux_level<NW, NB, K>(a, fc, 1, t, y0 - (K - 1) + t, y0, lane, part);
  }
  if constexpr (WALLS) {
    if (rw.outside) {
#pragma unroll
      for (int j = 0; j < SH; ++j) g.X[0][S][j] = 0.f;
      g.E[0][S] = 0.f;
      if constexpr (WF) g.W[0][S] = 0.f;
    }
  }
  // the row into the LDS ring, read with lane shifts by the next level
  eR[(3 + S) * kERow + 1 + lane] = g.E[0][S];
  __builtin_amdgcn_wave_barrier();
}

// The relaxation of level L (2 .. K) at one cell from level L-1: rows
// rho-1 .. rho+1 of level L-1 are in slots S1, S2, S (computed at iterations
// t-2, t-1, t).
template <int SH, int K, bool WF, int L, int S>
__device__ __forceinline__ float relax_up(const FusedArgs& a, const Ring<SH, K>& g,
                                          const WLBM_CONST uint32_t* m, float wi, int j,
                                          const float* eLane) {
  constexpr int S1 = (S + 1) % 3, S2 = (S + 2) % 3;
  constexpr int P = L - 2;   // ring index of level L-1
  // source rows rho - dy: dy = -1 -> slot S, 0 -> S2, 1 -> S1
  const float e = at_minus(pick3m(g.X[P][S][j], g.X[P][S2][j], g.X[P][S1][j], m[kHyLo],
                                  m[kHyMid]),
                           m[kHxPos], m[kHxNeg]);
  const float Es = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(eLane) +
                                                   int(m[kEOff0 + S]));
  if constexpr (!WF) {
    return fmaf(a.W, fmaf(wi, Es, -e), e);
  } else {
    const float Wh = at_minus(pick3m(g.W[P][S], g.W[P][S2], g.W[P][S1], m[kHyLo], m[kHyMid]),
                              m[kHxPos], m[kHxNeg]);
    return e + fmaf(wi, Es, -(Wh * e));
  }
}

// The wall facts of row rho at level L (2 .. K) and, at a diffuse wall row,
// its nodes from row rho of level L-1 (ring slot S2).
template <int NW, int SH, int K, bool WF, int L, int S>
__device__ __forceinline__ void walls_up(const FusedArgs& a, const Ring<SH, K>& g,
                                         const float* eR, float* sR, const EdgeCtx& ec, int rho,
                                         int lane, int part, RowWalls& rw, float& tg, float& wtg,
                                         bool& bb, uint32_t& bbm, float& bbt,
                                         const WLBM_CONST uint32_t*& codes) {
  constexpr int S2 = (S + 2) % 3;
  rw = row_walls(a, rho);
  bb = row_bb(ec, rw, bbm, bbt);
  codes = row_ptr(a.codes) + (L - 1) * (a.q >> 2);
  if (rw.diffuse >= 0)
    wall_nodes<NW, SH, WF>(a, ec, codes, row_ptr(a.ins) + 4 * (L - 1), rw.diffuse, g.X[L - 2][S2],
                           eR + (L - 1) * 3 * kERow + S2 * kERow, WF ? g.W[L - 2][S2] : 1.f, sR,
                           lane, part, tg, wtg);
}

// An intermediate level L (2 .. K-1) at iteration t: row r - (L-1) into ring
// slot S of level L, and its E.
template <int NW, int SH, int K, bool WF, int L, int S, bool WALLS, bool FLUX>
__device__ __forceinline__ void level_mid(const FusedArgs& a, Ring<SH, K>& g, float* sP,
                                          float* eR, const EdgeCtx& ec, int t, int y0, int lane,
                                          int part, const FluxCtx& fc) {
  constexpr int S2 = (S + 2) % 3;
  constexpr int NB = NW * SH / kMaxGroupPlanes;
  const RowCtx c = row_ctx(a);
  const WLBM_CONST uint32_t* sels = row_ptr(a.sels[L - 1]);
  const int i_begin = part * SH;
  float* pl = sP + (2 * (L - 1) + (t & 1)) * NB * 64;
  RowWalls rw{};
  float tg = 0.f, wtg = 0.f, bbt = 0.f;
  uint32_t bbm = 0;
  bool bb = false;
  const WLBM_CONST uint32_t* codes = nullptr;
  if constexpr (WALLS)
    walls_up<NW, SH, K, WF, L, S>(a, g, eR, sP + (2 * (L - 1) + ((t + 1) & 1)) * NB * 64, ec,
                                  y0 - (K - 1) + t - (L - 1), lane, part, rw, tg, wtg, bb, bbm,
                                  bbt, codes);
  float* ql = FLUX ? flux_sums<NB>(fc, L, t) : nullptr;
  const WLBM_CONST float* sx = FLUX ? row_ptr(a.sxtab) : nullptr;
  const WLBM_CONST float* sy = FLUX ? row_ptr(a.sytab) : nullptr;
#pragma unroll
  for (int b0 = 0; b0 < SH; b0 += kMaxGroupPlanes) {
    const int i0 = i_begin + b0;
    float bsum = 0.f, bqx = 0.f, bqy = 0.f;
#pragma unroll
    for (int d = 0; d < kMaxGroupPlanes; ++d) {
      float out = relax_up<SH, K, WF, L, S>(a, g, sel_at(c.tab, sels[i0 + d]), c.wtab[i0 + d],
                                            b0 + d, eR + (L - 1) * 3 * kERow + 1 + lane);
      if constexpr (WALLS)
        out = wall_update(out, c.wtab[i0 + d], rw, codes, i0 + d, tg, wtg, bb, bbm, bbt);
      g.X[L - 1][S][b0 + d] = out;
      bsum += out;
      if constexpr (FLUX) {
        bqx = fmaf(out, sx[i0 + d], bqx);
        bqy = fmaf(out, sy[i0 + d], bqy);
      }
    }
    pl[(i0 / kMaxGroupPlanes) * 64 + lane] = bsum;
    if constexpr (FLUX) {
      ql[(i0 / kMaxGroupPlanes) * 64 + lane] = bqx;
      ql[(NB + i0 / kMaxGroupPlanes) * 64 + lane] = bqy;
    }
  }
  // W of this row (level L-1 holds it in slot S2)
  if constexpr (WF) g.W[L - 1][S] = g.W[L - 2][S2];
  lds_barrier();
  float E = 0.f;
#pragma unroll
  for (int k = 0; k < NB; ++k) E += pl[k * 64 + lane];
  g.E[L - 1][S] = WF ? E * g.W[L - 1][S] : E;
  if constexpr (FLUX) {
    flux_level<NW, NB, K>(a, fc, L, t, y0 - (K - 1) + t - (L - 1), y0, lane, part);
  }
  if constexpr (WALLS) {
    if (rw.outside) {
#pragma unroll
      for (int j = 0; j < SH; ++j) g.X[L - 1][S][j] = 0.f;
      g.E[L - 1][S] = 0.f;
      if constexpr (WF) g.W[L - 1][S] = 0.f;
    }
  }
  eR[(L * 3 + S) * kERow + 1 + lane] = g.E[L - 1][S];
  __builtin_amdgcn_wave_barrier();
}

// The output level K at iteration t: row ro = r - (K-1), stored with the
// ghost copies of periodic edges.
template <int NW, int SH, int K, bool WF, int S, bool WALLS, bool FLUX>
__device__ __forceinline__ void level_out(const FusedArgs& a, Ring<SH, K>& g, float* sP,
                                          const float* eR, const EdgeCtx& ec, int t, int x0,
                                          int y0, int lane, int part, bool out_lane,
                                          FluxCtx& fc) {
  constexpr int NB = NW * SH / kMaxGroupPlanes;
  const RowCtx c = row_ctx(a);
  const WLBM_CONST uint32_t* sels = row_ptr(a.sels[K - 1]);
  const int ny = a.ny, pitch = a.pitch, nx = a.nx;
  const long long plane = a.plane;
  const int i_begin = part * SH;
  const int ro = y0 - (K - 1) + t - (K - 1);
  const bool store = out_lane && ro < ny;
  const int xo = x0 - kLane0<K, WALLS> + lane;
  const bool px = !WALLS || a.x_edge == kPeriodic;
  const bool py = !WALLS || a.y_edge == kPeriodic;
  // byte offsets of the cell and its ghosts (used only where stored)
  const int row_o = (ro + 1) * pitch + kXOff;
  const uint32_t ob = uint32_t((row_o + xo) * 4);
  // Ghost copies of this cell in the frame of periodic edges (nx >= 2 kGhost
  // and ny >= 2, so a cell has at most one ghost column and one ghost row):
  // columns 0 .. kGhost-1 are copied to nx .. nx+kGhost-1 and columns
  // nx-kGhost .. nx-1 to -kGhost .. -1; rows 0 and ny - 1 to ny and -1.  Only
  // blocks on the lattice's edge have any, which the whole block knows.
  const bool edge = x0 == 0 || x0 + kStrip<K> + kGhost - 1 >= nx || ro == 0 || ro == ny - 1;
  const bool gx = store && px && (xo < kGhost || xo >= nx - kGhost);
  const bool gy = store && py && (ro == 0 || ro == ny - 1);
  const int xg = xo < kGhost ? xo + nx : xo - nx;
  const int yg = ro == 0 ? ny : -1;
  const int row_g = (yg + 1) * pitch + kXOff;
  const uint32_t obx = uint32_t((row_o + xg) * 4);
  const uint32_t oby = uint32_t((row_g + xo) * 4);
  const uint32_t obxy = uint32_t((row_g + xg) * 4);
  float* po = sP + (2 * (K - 1) + (t & 1)) * NB * 64;
  RowWalls rw{};
  float tg = 0.f, wtg = 0.f, bbt = 0.f;
  uint32_t bbm = 0;
  bool bb = false;
  const WLBM_CONST uint32_t* codes = nullptr;
  if constexpr (WALLS)
    walls_up<NW, SH, K, WF, K, S>(a, g, eR, sP + (2 * (K - 1) + ((t + 1) & 1)) * NB * 64, ec, ro,
                                  lane, part, rw, tg, wtg, bb, bbm, bbt, codes);
  float* qo = FLUX ? flux_sums<NB>(fc, K, t) : nullptr;
  const WLBM_CONST float* sx = FLUX ? row_ptr(a.sxtab) : nullptr;
  const WLBM_CONST float* sy = FLUX ? row_ptr(a.sytab) : nullptr;
#pragma unroll
  for (int b0 = 0; b0 < SH; b0 += kMaxGroupPlanes) {
    const int i0 = i_begin + b0;
    float bsum = 0.f, bqx = 0.f, bqy = 0.f;
    const rsrc_t ro_rs = make_rsrc(a.e_out + (long long)i0 * plane,
                                   uint32_t(kMaxGroupPlanes * plane * 4));
    float o[kMaxGroupPlanes];
#pragma unroll
    for (int d = 0; d < kMaxGroupPlanes; ++d) {
      float out = relax_up<SH, K, WF, K, S>(a, g, sel_at(c.tab, sels[i0 + d]), c.wtab[i0 + d],
                                            b0 + d, eR + (K - 1) * 3 * kERow + 1 + lane);
      if constexpr (WALLS)
        out = wall_update(out, c.wtab[i0 + d], rw, codes, i0 + d, tg, wtg, bb, bbm, bbt);
      bsum += out;
      o[d] = out;
      if constexpr (FLUX) {
        bqx = fmaf(out, sx[i0 + d], bqx);
        bqy = fmaf(out, sy[i0 + d], bqy);
      }
    }
    po[(i0 / kMaxGroupPlanes) * 64 + lane] = bsum;
    if constexpr (FLUX) {
      qo[(i0 / kMaxGroupPlanes) * 64 + lane] = bqx;
      qo[(NB + i0 / kMaxGroupPlanes) * 64 + lane] = bqy;
    }
    // the batch's stores, under one lane mask each
    auto put = [&](uint32_t off) {
#pragma unroll
      for (int d = 0; d < kMaxGroupPlanes; ++d)
        buf_store_stream(o[d], ro_rs, off, uint32_t(d) * c.plane_bytes);
    };
    if (store) put(ob);
    if (edge) {
      if (gx) put(obx);
      if (gy) put(oby);
      if (gx && gy) put(obxy);
    }
  }
  lds_barrier();
  if (part == 0 && store) {
    float E = 0.f;
#pragma unroll
    for (int k = 0; k < NB; ++k) E += po[k * 64 + lane];
    const rsrc_t Ers = make_rsrc(a.E_out, c.plane_bytes);
    buf_store(E, Ers, ob);
    if (edge) {
      if (gx) buf_store(E, Ers, obx);
      if (gy) buf_store(E, Ers, oby);
      if (gx && gy) buf_store(E, Ers, obxy);
    }
  }
  if constexpr (FLUX) {
    flux_out<NW, NB, K>(a, fc, t, ro, y0, lane, part);
  }
}

// Iteration t (ring slot S = t mod 3): level 1, then each higher level once
// the three rows it reads exist.
template <int NW, int SH, int K, bool WF, int S, bool WALLS, bool FLUX>
__device__ __forceinline__ void iteration(const FusedArgs& a, Ring<SH, K>& g, float* sP,
                                          float* eR, const EdgeCtx& ec, int t, int x0, int y0,
                                          int lane, int part, uint32_t lcol, bool out_lane,
                                          FluxCtx& fc) {
  level1<NW, SH, K, WF, S, WALLS, FLUX>(a, g, sP, eR, ec, t, y0, lane, part, lcol, fc);
  if constexpr (K >= 3) {
    if (t < 2) return;
    level_mid<NW, SH, K, WF, 2, S, WALLS, FLUX>(a, g, sP, eR, ec, t, y0, lane, part, fc);
  }
  if constexpr (K >= 4) {
    if (t < 4) return;
    level_mid<NW, SH, K, WF, 3, S, WALLS, FLUX>(a, g, sP, eR, ec, t, y0, lane, part, fc);
  }
  if (t < 2 * (K - 1)) return;
  level_out<NW, SH, K, WF, S, WALLS, FLUX>(a, g, sP, eR, ec, t, x0, y0, lane, part, out_lane,
                                           fc);
}

// One block's strip (x0, y0): the rows and lanes of the iteration loop.
template <int NW, int SH, bool WF, int K, bool WALLS, bool FLUX>
__device__ __forceinline__ void run_block(const FusedArgs& a, float* sP, float* sEr, float* sQ,
                                          int x0, int y0) {
  const int lane = threadIdx.x & 63;
  const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // this lane's column; lanes past the ghost frame read its last column
  // (their values are never used), so that every read stays inside the row
  // and its padding
  constexpr int L0 = kLane0<K, WALLS>;
  const int x = x0 - L0 + lane;
  const int xl = x < a.nx + kGhost - 1 ? x : a.nx + kGhost - 1;
  const uint32_t lcol = uint32_t((kXOff + xl) * 4);
  const bool out_lane = lane >= L0 && lane < L0 + kStrip<K> && x < a.nx;
  FluxCtx fc{};
  if constexpr (FLUX) {
    constexpr int NB = NW * SH / kMaxGroupPlanes;
    fc.sQ = sQ;
    fc.sF = sQ + 2 * K * 2 * NB * 64;
    fc.x = x;
    fc.out_lane = out_lane;
    // the window sums of the first output row, unless a step of this launch
    // starts the window
    if (a.flux_levels != 0 && a.flux_first == 0 && out_lane && y0 < a.ny) {
      const long long o = (long long)y0 * a.nx + x;
      if (part == 0) fc.p[0] = a.qsx[o];
      if (part == (NW == 1 ? 0 : 1)) fc.p[NW == 1 ? 1 : 0] = a.qsy[o];
    }
  }
  EdgeCtx ec{};
  if constexpr (WALLS) {
    ec.x = x;
    ec.x_in = x >= 0 && x < a.nx;
    const bool xbb = a.x_edge == kBlackbody;
    ec.xbb = (xbb && (x == 0 || x == a.nx - 1)) ? 0xffffffffu : 0u;
    ec.xbb_t = x == 0 ? a.t_x_lo : a.t_x_hi;
    ec.blk_xbb = xbb && (x0 - L0 <= 0 || (x0 - L0 <= a.nx - 1 && a.nx - 1 <= x0 - L0 + 63));
  }

  Ring<SH, K> g;
  // step-n E of rows r0 - 1 and r0 (r0 = y0 - (K-1), the first level-1 row)
  // into slots 0 and 1; the loads of row r0 bring row r0 + 1 into slot 2
  const uint32_t plane_bytes = uint32_t(a.plane * 4);
  const int r0 = y0 - (K - 1);
  const bool wrap_y = !WALLS || a.y_edge == kPeriodic;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int ra = r0 - 1 + k;
    const int row = wrap_y ? wrap_index(ra, a.ny) : min(max(ra, 0), a.ny - 1);
    const bool valid = wrap_y || (ra >= 0 && ra < a.ny);
    const uint32_t rb = uint32_t((row + 1) * a.pitch * 4);
    g.rb[k] = rb;
    const float Ev = buf_load(make_rsrc(a.E_in, plane_bytes), lcol, rb);
    if constexpr (WF) {
      const float Wv = buf_load(make_rsrc(a.Wf, plane_bytes), lcol, rb);
      g.Wn[k] = valid ? Wv : 0.f;
      g.En[k] = valid ? Ev * Wv : 0.f;
    } else {
      g.En[k] = valid ? Ev : 0.f;
    }
  }
  float* eR = sEr;
  // the pads either side of each row (read only by lanes whose results are
  // never used) hold zero
  if (lane < 3 * K) eR[lane * kERow] = eR[lane * kERow + kERow - 1] = 0.f;
  eR[1 + lane] = g.En[0];
  eR[kERow + 1 + lane] = g.En[1];
  g.wn = wrap_y ? wrap_index(r0, a.ny) : r0;
  issue_row<SH, K, WF, 2, WALLS>(a, g, part * SH, lcol);
  // a.rows + 2 (K - 1) is a multiple of 3 (the loop is unrolled by three)
  const int T = a.rows + 2 * (K - 1);
  for (int t = 0; t < T; t += 3) {
    iteration<NW, SH, K, WF, 0, WALLS, FLUX>(a, g, sP, eR, ec, t, x0, y0, lane, part, lcol,
                                             out_lane, fc);
    iteration<NW, SH, K, WF, 1, WALLS, FLUX>(a, g, sP, eR, ec, t + 1, x0, y0, lane, part, lcol,
                                             out_lane, fc);
    iteration<NW, SH, K, WF, 2, WALLS, FLUX>(a, g, sP, eR, ec, t + 2, x0, y0, lane, part, lcol,
                                             out_lane, fc);
  }
}

template <int NW, int SH, bool WF, int K, bool WALLS, bool FLUX>
__device__ __forceinline__ void stepk_block(const FusedArgs& a, float* sP, float* sEr, float* sQ) {
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (b % a.strips_x) * kStrip<K>;
  const int y0 = (b / a.strips_x) * a.rows;
  if constexpr (WALLS) {
    // A block none of whose levels reaches a wall row, a row beyond a
    // non-periodic y edge or a blackbody column runs the code of periodic
    // lattices (its ghost reads and writes are those of periodic edges, or
    // none).  Its level-1 rows are y0 - (K-1) .. y0 + rows - 1 + (K-1) and
    // its lanes x0 - K .. x0 - K + 63.
    const bool rows_free = a.y_edge == kPeriodic ||
                           (y0 - (K - 1) >= 1 && y0 + a.rows - 1 + (K - 1) <= a.ny - 2);
    const bool cols_free =
        a.x_edge == kPeriodic || (x0 - K >= 1 && x0 - K + 63 <= a.nx - 2);
    if (rows_free && cols_free) {
      run_block<NW, SH, WF, K, false, FLUX>(a, sP, sEr, sQ, x0, y0);
      return;
    }
  }
  run_block<NW, SH, WF, K, WALLS, FLUX>(a, sP, sEr, sQ, x0, y0);
}

// E batch sums: [level 1 .. K][row parity][batch of 8 directions][lane]
template <int NW, int SH, int K>
constexpr int kSumFloats = 2 * K * (NW * SH / kMaxGroupPlanes) * 64;
// heat-flux batch sums: as the E sums, x and y; then the ring of step sums
template <int NW, int SH, int K>
constexpr int kFluxFloats = 2 * kSumFloats<NW, SH, K> + K * K * 2 * 64;

template <int NW, int SH, bool WF, int K, bool WALLS>
__global__ __launch_bounds__(64 * NW) void k_stepk(const FusedArgs a) {
  __shared__ float sP[kSumFloats<NW, SH, K>];
  // the E rings of the block: step n, then levels 1 .. K-1
  __shared__ float sEr[K * 3 * kERow];
  stepk_block<NW, SH, WF, K, WALLS, false>(a, sP, sEr, nullptr);
}

// With the heat flux of flux-window steps: held to 128 registers a lane
// (four waves a SIMD; the flux sums would otherwise take the count past it
// and halve the resident blocks).
template <int NW, int SH, bool WF, int K, bool WALLS>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void k_stepk_flux(
    const FusedArgs a) {
  __shared__ float sP[kSumFloats<NW, SH, K>];
  __shared__ float sEr[K * 3 * kERow];
  __shared__ float sQ[kFluxFloats<NW, SH, K>];
  stepk_block<NW, SH, WF, K, WALLS, true>(a, sP, sEr, sQ);
}

// A lattice's arguments from the batch's device table, field by field
// through the scalar cache (so that they land in scalar registers, as kernel
// arguments do).
__device__ __forceinline__ FusedArgs load_args(const WLBM_CONST FusedArgs* p) {
  FusedArgs a;
  a.e_in = p->e_in;
  a.e_out = p->e_out;
  a.E_in = p->E_in;
  a.E_out = p->E_out;
  a.Wf = p->Wf;
  a.pulls = p->pulls;
#pragma unroll
  for (int m = 0; m < 4; ++m) a.sels[m] = p->sels[m];
  a.wtab = p->wtab;
  a.W = p->W;
  a.nx = p->nx;
  a.ny = p->ny;
  a.q = p->q;
  a.pitch = p->pitch;
  a.plane = p->plane;
  a.strips_x = p->strips_x;
  a.strips_y = p->strips_y;
  a.rows = p->rows;
  a.x_edge = p->x_edge;
  a.y_edge = p->y_edge;
  a.t_x_lo = p->t_x_lo;
  a.t_x_hi = p->t_x_hi;
  a.t_y_lo = p->t_y_lo;
  a.t_y_hi = p->t_y_hi;
  a.codes = p->codes;
  a.ins = p->ins;
  return a;
}
__device__ __forceinline__ void load_flux_args(FusedArgs& a, const WLBM_CONST FusedArgs* p) {
  a.qsx = p->qsx;
  a.qsy = p->qsy;
  a.sxtab = p->sxtab;
  a.sytab = p->sytab;
}

// K steps of n lattices in one launch (the in-plane film sweeps of Sec. 3.5
// run many lattices of different thickness and Knudsen number): each block
// finds its lattice in the prefix table of block counts, takes that
// lattice's arguments for the current buffer parity from the device table
// and its per-step tables from its rings (scalar loads), and runs the block
// as k_stepk does.
template <int NW, int SH, bool WF, int K, bool FLUX>
__device__ __forceinline__ void stepk_batch_block(const FusedBatchArgs& b, float* sP, float* sEr,
                                                  float* sQ) {
  const int gb = xcd_tile(blockIdx.x, gridDim.x);
  const WLBM_CONST int* first = scalar_ptr(b.first);
  int j = 0;
  while (j + 1 < b.n && gb >= first[j + 1]) ++j;
  j = __builtin_amdgcn_readfirstlane(j);
  FusedArgs a = load_args(scalar_ptr(b.lats) + 2 * j + b.parity);
  if constexpr (FLUX) {
    load_flux_args(a, scalar_ptr(b.lats) + 2 * j + b.parity);
    a.flux_levels = b.flux_levels;
    a.flux_first = b.flux_first;
  }
  const size_t q = size_t(a.q);
  const uint32_t* sel0 = scalar_ptr(b.sels)[j] + size_t(b.row) * q;
#pragma unroll
  for (int m = 0; m < K; ++m) a.sels[m] = sel0 + size_t(m) * q;
  a.pulls = scalar_ptr(b.pulls)[j] + size_t(b.row) * q;
  a.codes = reinterpret_cast<const uint32_t*>(scalar_ptr(b.codes)[j] + size_t(b.row) * q);
  a.ins = scalar_ptr(b.ins)[j] + 4 * b.row;
  const int lb = gb - first[j];
  const int x0 = (lb % a.strips_x) * kStrip<K>;
  const int y0 = (lb / a.strips_x) * a.rows;
  const bool rows_free = a.y_edge == kPeriodic ||
                         (y0 - (K - 1) >= 1 && y0 + a.rows - 1 + (K - 1) <= a.ny - 2);
  const bool cols_free = a.x_edge == kPeriodic || (x0 - K >= 1 && x0 - K + 63 <= a.nx - 2);
  if (rows_free && cols_free)
    run_block<NW, SH, WF, K, false, FLUX>(a, sP, sEr, sQ, x0, y0);
  else
    run_block<NW, SH, WF, K, true, FLUX>(a, sP, sEr, sQ, x0, y0);
}

template <int NW, int SH, bool WF, int K>
__global__ __launch_bounds__(64 * NW) void k_stepk_batch(const FusedBatchArgs b) {
  __shared__ float sP[kSumFloats<NW, SH, K>];
  __shared__ float sEr[K * 3 * kERow];
  stepk_batch_block<NW, SH, WF, K, false>(b, sP, sEr, nullptr);
}

template <int NW, int SH, bool WF, int K>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void
k_stepk_batch_flux(const FusedBatchArgs b) {
  __shared__ float sP[kSumFloats<NW, SH, K>];
  __shared__ float sEr[K * 3 * kERow];
  __shared__ float sQ[kFluxFloats<NW, SH, K>];
  stepk_batch_block<NW, SH, WF, K, true>(b, sP, sEr, sQ);
}

template <int NW, int SH, int K, bool FLUX>
hipError_t launchk_batch(const FusedBatchArgs& b, bool wf, hipStream_t s) {
  const dim3 grid(b.nblocks), block(64 * NW);
  if constexpr (FLUX) {
    if (wf)
      hipLaunchKernelGGL((k_stepk_batch_flux<NW, SH, true, K>), grid, block, 0, s, b);
    else
      hipLaunchKernelGGL((k_stepk_batch_flux<NW, SH, false, K>), grid, block, 0, s, b);
  } else {
    if (wf)
      hipLaunchKernelGGL((k_stepk_batch<NW, SH, true, K>), grid, block, 0, s, b);
    else
      hipLaunchKernelGGL((k_stepk_batch<NW, SH, false, K>), grid, block, 0, s, b);
  }
  return hipGetLastError();
}

template <int K, bool FLUX>
hipError_t launch_fused_batch_qk(const FusedBatchArgs& b, int q, bool per_cell, hipStream_t s) {
  if constexpr (K == 2) {
    switch (q) {
      case 80: return launchk_batch<5, 16, K, FLUX>(b, per_cell, s);
      case 96: return launchk_batch<6, 16, K, FLUX>(b, per_cell, s);
      case 112: return launchk_batch<7, 16, K, FLUX>(b, per_cell, s);
      case 128: return launchk_batch<8, 16, K, FLUX>(b, per_cell, s);
      default: break;
    }
  }
  switch (q) {
    case 8: return launchk_batch<1, 8, K, FLUX>(b, per_cell, s);
    case 16: return launchk_batch<2, 8, K, FLUX>(b, per_cell, s);
    case 24: return launchk_batch<3, 8, K, FLUX>(b, per_cell, s);
    case 32: return launchk_batch<4, 8, K, FLUX>(b, per_cell, s);
    case 40: return launchk_batch<5, 8, K, FLUX>(b, per_cell, s);
    case 48: return launchk_batch<6, 8, K, FLUX>(b, per_cell, s);
    case 56: return launchk_batch<7, 8, K, FLUX>(b, per_cell, s);
    case 64: return launchk_batch<8, 8, K, FLUX>(b, per_cell, s);
    case 72: return launchk_batch<9, 8, K, FLUX>(b, per_cell, s);
    case 80: 
      if constexpr (K != 2) return launchk_batch<10, 8, K, FLUX>(b, per_cell, s);
      break;
    case 88: return launchk_batch<11, 8, K, FLUX>(b, per_cell, s);
    case 96: 
      if constexpr (K != 2) return launchk_batch<12, 8, K, FLUX>(b, per_cell, s);
      break;
    case 104: return launchk_batch<13, 8, K, FLUX>(b, per_cell, s);
    case 112: 
      if constexpr (K != 2) return launchk_batch<14, 8, K, FLUX>(b, per_cell, s);
      break;
    case 120: return launchk_batch<15, 8, K, FLUX>(b, per_cell, s);
    case 128: 
      if constexpr (K != 2) return launchk_batch<16, 8, K, FLUX>(b, per_cell, s);
      break;
    default: break;
  }
  if constexpr (K == 2) {
    if (q == 192) return launchk_batch<12, 16, K, FLUX>(b, per_cell, s);
    if (q == 256) return launchk_batch<16, 16, K, FLUX>(b, per_cell, s);
  }
  return hipErrorInvalidValue;
}

template <int NW, int SH, bool WALLS, int K, bool FLUX>
hipError_t launchk(const FusedArgs& a, bool wf, hipStream_t s) {
  const dim3 grid(a.strips_x * a.strips_y), block(64 * NW);
  if constexpr (FLUX) {
    if (wf)
      hipLaunchKernelGGL((k_stepk_flux<NW, SH, true, K, WALLS>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_stepk_flux<NW, SH, false, K, WALLS>), grid, block, 0, s, a);
  } else {
    if (wf)
      hipLaunchKernelGGL((k_stepk<NW, SH, true, K, WALLS>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_stepk<NW, SH, false, K, WALLS>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

template <int NW, int SH, bool WALLS, int K>
int blocks_per_cu_tmpl(bool wf) {
  int n = 0;
  const int bs = 64 * NW;
  const hipError_t e =
      wf ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stepk<NW, SH, true, K, WALLS>, bs, 0)
         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stepk<NW, SH, false, K, WALLS>, bs,
                                                        0);
  return e == hipSuccess ? n : 0;
}

// Dispatch on q: one wave per 8 directions up to q = 128 (blocks of up to 16
// waves), except at two steps per launch for q = 80, 96, 112 and 128, which
// run half as many waves of 16 directions (each wave then adds its E batch
// sums for twice the directions; three or four steps need the registers of
// 8 directions a wave), and 12 or 16 waves of 16 directions for q = 192 and
// 256 (two steps per launch: a block of 16 waves must keep to 128 registers
// a lane so that four waves share each SIMD).  Measured on MI355X, 1024 x
// 1024 periodic, q = 128: two steps 997 G updates/s with 16 directions a
// wave, 963 with 8; four steps 1352 with 8 (1022 with 16).
template <bool WALLS, int K, bool FLUX>
hipError_t launch_fused_qk(const FusedArgs& a, bool per_cell, hipStream_t s) {
  if constexpr (K == 2) {
    switch (a.q) {
      case 80: return launchk<5, 16, WALLS, K, FLUX>(a, per_cell, s);
      case 96: return launchk<6, 16, WALLS, K, FLUX>(a, per_cell, s);
      case 112: return launchk<7, 16, WALLS, K, FLUX>(a, per_cell, s);
      case 128: return launchk<8, 16, WALLS, K, FLUX>(a, per_cell, s);
      default: break;
    }
  }
  switch (a.q) {
    case 8: return launchk<1, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 16: return launchk<2, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 24: return launchk<3, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 32: return launchk<4, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 40: return launchk<5, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 48: return launchk<6, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 56: return launchk<7, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 64: return launchk<8, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 72: return launchk<9, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 80: 
      if constexpr (K != 2) return launchk<10, 8, WALLS, K, FLUX>(a, per_cell, s);
      break;
    case 88: return launchk<11, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 96: 
      if constexpr (K != 2) return launchk<12, 8, WALLS, K, FLUX>(a, per_cell, s);
      break;
    case 104: return launchk<13, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 112: 
      if constexpr (K != 2) return launchk<14, 8, WALLS, K, FLUX>(a, per_cell, s);
      break;
    case 120: return launchk<15, 8, WALLS, K, FLUX>(a, per_cell, s);
    case 128: 
      if constexpr (K != 2) return launchk<16, 8, WALLS, K, FLUX>(a, per_cell, s);
      break;
    default: break;
  }
  if constexpr (K == 2) {
    if (a.q == 192) return launchk<12, 16, WALLS, K, FLUX>(a, per_cell, s);
    if (a.q == 256) return launchk<16, 16, WALLS, K, FLUX>(a, per_cell, s);
  }
  return hipErrorInvalidValue;
}

template <bool WALLS, int K>
int blocks_per_cu_qk(int q, bool per_cell) {
  if constexpr (K == 2) {
    switch (q) {
      case 80: return blocks_per_cu_tmpl<5, 16, WALLS, K>(per_cell);
      case 96: return blocks_per_cu_tmpl<6, 16, WALLS, K>(per_cell);
      case 112: return blocks_per_cu_tmpl<7, 16, WALLS, K>(per_cell);
      case 128: return blocks_per_cu_tmpl<8, 16, WALLS, K>(per_cell);
      default: break;
    }
  }
  switch (q) {
    case 8: return blocks_per_cu_tmpl<1, 8, WALLS, K>(per_cell);
    case 16: return blocks_per_cu_tmpl<2, 8, WALLS, K>(per_cell);
    case 24: return blocks_per_cu_tmpl<3, 8, WALLS, K>(per_cell);
    case 32: return blocks_per_cu_tmpl<4, 8, WALLS, K>(per_cell);
    case 40: return blocks_per_cu_tmpl<5, 8, WALLS, K>(per_cell);
    case 48: return blocks_per_cu_tmpl<6, 8, WALLS, K>(per_cell);
    case 56: return blocks_per_cu_tmpl<7, 8, WALLS, K>(per_cell);
    case 64: return blocks_per_cu_tmpl<8, 8, WALLS, K>(per_cell);
    case 72: return blocks_per_cu_tmpl<9, 8, WALLS, K>(per_cell);
    case 80: 
      if constexpr (K != 2) return blocks_per_cu_tmpl<10, 8, WALLS, K>(per_cell);
      break;
    case 88: return blocks_per_cu_tmpl<11, 8, WALLS, K>(per_cell);
    case 96: 
      if constexpr (K != 2) return blocks_per_cu_tmpl<12, 8, WALLS, K>(per_cell);
      break;
    case 104: return blocks_per_cu_tmpl<13, 8, WALLS, K>(per_cell);
    case 112: 
      if constexpr (K != 2) return blocks_per_cu_tmpl<14, 8, WALLS, K>(per_cell);
      break;
    case 120: return blocks_per_cu_tmpl<15, 8, WALLS, K>(per_cell);
    case 128: 
      if constexpr (K != 2) return blocks_per_cu_tmpl<16, 8, WALLS, K>(per_cell);
      break;
    default: break;
  }
  if constexpr (K == 2) {
    if (q == 192) return blocks_per_cu_tmpl<12, 16, WALLS, K>(per_cell);
    if (q == 256) return blocks_per_cu_tmpl<16, 16, WALLS, K>(per_cell);
  }
  return 0;
}

}  // namespace
}  // namespace wlbm
