// Several time steps of the worm-LBM per launch (temporal blocking) for
// gfx950.
//
// One launch of k_stepk<..., K> advances a periodic lattice by steps n+1 ..
// n+K, K = 2, 3 or 4 (Sec. 2.3 Eq. algorithm, pull form as in k_step): each
// population is read from HBM once and written once per K steps, instead of
// once per step.
//
// A block owns a strip of kStrip columns and a.rows rows of the output.  Its NW
// waves cover the same 64 columns x0-K .. x0+63-K, one per lane, and take SH
// directions each (8, or 16 above Q = 64).  Rows are pipelined: at iteration
// t the waves compute level 1 (step n+1) of row r = y0-(K-1)+t from the
// step-n populations in HBM, then level l of row r-(l-1) for l = 2 .. K from
// level l-1, whose rows r-l .. r-l+2 are held in registers, a ring of three
// rows per level; level K is the output.  The one-cell shifts in x of the
// pulled populations are lane shifts of a whole wave (DPP wave_shr /
// wave_shl), so level l is valid on lanes l .. 63-l; E, which every
// direction reads at its own move, is read from the wave's own LDS copy of
// the three E rows at a shifted address.  Step-n rows wrap by comparison as
// they advance (the pulls of a wrapped row reach the ghost rows); columns
// read the ghost frame of periodic x edges (kGhost columns deep), which must
// be valid on entry (the caller refreshes it with k_fill_ghosts after other
// producers) and which the kernel writes for its output.  E of each row of
// each level is summed over the waves in LDS in k_step's order (8-direction
// batch sums in batch order), and every update uses k_step's arithmetic, so
// one launch gives the same bits as K k_step launches.
//
// Scalar work per direction is kept to loads: the host writes, per step and
// direction, the byte offset of the direction's entry in the selection table
// and, for the first step, the offset of its pulled population, so the kernel
// decodes no schedule codes (scalar instruction issue limits this kernel as
// much as vector issue does).
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
// Ghost columns written on each side by every multi-step launch (the most
// any K reads), so that launches of different K can follow each other.
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
// Selections by a direction's move are wave-uniform.  Rather than comparing
// and selecting on the decoded move in scalar code for every direction and
// row, the kernel loads the entry of the move's code from this table (one
// scalar load per direction, at a byte offset the host writes per step and
// direction) and selects with bitwise operations.  Entry c, for code
// c = dx + 1 | (dy + 1) << 2 | hop << 4 with (hx, hy) the move on a hop and
// (0, 0) on a pause: the lane masks of hy = -1, hy = 0, hx > 0 and hx < 0,
// then, for each iteration slot S, the byte offset of E at (x - dx, rho - dy)
// in a wave's LDS copy of an E ring, from the lane's own entry in slot 0
// (rows rho - 1, rho, rho + 1 are in slots S, S + 2, S + 1 mod 3).
enum SelWord : int { kHyLo, kHyMid, kHxPos, kHxNeg, kEOff0, kEOff1, kEOff2, kSelWords = 8 };
// Row length (floats) of a wave's private LDS copy of one E row: 64 lanes
// and one pad either side for the lane shifts.
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
  int wn;                  // wrapped index of the newest step-n row loaded
};

// Issue the loads of level-1 row r: the step-n populations each of this
// wave's directions pulls (row r - hy, column x - hx) into g.V, and step-n E
// (and W) of row r + 1 into ring slot SN.  Nothing waits for them here.
// With three or four steps per launch the wave issues them at raised priority
// so that they leave early (four steps at 1024 x 1024, Q = 64: +2 %; with
// two steps raising it cost 2 %).
template <int SH, int K, bool WF, int SN>
__device__ __forceinline__ void issue_row(const FusedArgs& a, Ring<SH, K>& g, int i_begin,
                                          uint32_t lcol) {
  if constexpr (K >= 3) __builtin_amdgcn_s_setprio(3);
  const WLBM_CONST uint32_t* pulls = row_ptr(a.pulls);
  const long long plane = a.plane;
  const uint32_t plane_bytes = uint32_t(plane * 4);
  // the rows advance by one per call: wrap the newest index by comparison
  g.wn = g.wn + 1 == a.ny ? 0 : g.wn + 1;
  g.rb[SN] = uint32_t((g.wn + 1) * a.pitch * 4);
  const uint32_t rb_m = g.rb[SN], rb_0 = g.rb[(SN + 2) % 3];
  {
    const float Ev = buf_load(make_rsrc(a.E_in, plane_bytes), lcol, rb_m);
    if constexpr (WF) {
      const float Wv = buf_load(make_rsrc(a.Wf, plane_bytes), lcol, rb_m);
      g.Wn[SN] = Wv;
      g.En[SN] = Ev * Wv;
    } else {
      g.En[SN] = Ev;
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

// Level 1 at iteration t (row r = y0 - (K-1) + t, ring slot S = t mod 3)
// from the step-n loads; then the loads of the next row are issued, and E of
// row r is summed.  Step-n slots: rows r-1, r, r+1 are S, S+1, S+2 (mod 3).
template <int NW, int SH, int K, bool WF, int S>
__device__ __forceinline__ void level1(const FusedArgs& a, Ring<SH, K>& g, float* sP, float* eR,
                                       int t, int y0, int lane, int part, uint32_t lcol) {
  constexpr int S1 = (S + 1) % 3, S2 = (S + 2) % 3;
  constexpr int NB = NW * SH / kMaxGroupPlanes;   // batches of 8 directions
  const RowCtx c = row_ctx(a);
  const WLBM_CONST uint32_t* sels = row_ptr(a.sels[0]);
  const int i_begin = part * SH;
  float* p1 = sP + (t & 1) * NB * 64;
  // step-n E of row r + 1 (loaded during the previous iteration) into this
  // wave's LDS copy; rows r - 1 and r are there already
  eR[S2 * kERow + 1 + lane] = g.En[S2];
  __builtin_amdgcn_wave_barrier();
  const float* eLane0 = eR + 1 + lane;
#pragma unroll
  for (int b0 = 0; b0 < SH; b0 += kMaxGroupPlanes) {
    const int i0 = i_begin + b0;
    float bsum = 0.f;
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
      g.X[0][S][b0 + d] = out;
      bsum += out;
    }
    p1[(i0 / kMaxGroupPlanes) * 64 + lane] = bsum;
  }
  // W of this row for the next level, before slot S is refilled
  if constexpr (WF) g.W[0][S] = g.Wn[S1];
  const float Wrow = WF ? g.Wn[S1] : 1.f;
  // loads of the next level-1 row (its step-n row r + 2 goes to slot S)
  if (t + 1 < a.rows + 2 * (K - 1)) issue_row<SH, K, WF, S>(a, g, i_begin, lcol);
  // E of row r: the batch sums in batch order, as k_step adds them
  lds_barrier();
  float E = 0.f;
#pragma unroll
  for (int k = 0; k < NB; ++k) E += p1[k * 64 + lane];
  g.E[0][S] = WF ? E * Wrow : E;
  // this wave's LDS copy of the row, read with lane shifts by the next level
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

// An intermediate level L (2 .. K-1) at iteration t: row r - (L-1) into ring
// slot S of level L, and its E.
template <int NW, int SH, int K, bool WF, int L, int S>
__device__ __forceinline__ void level_mid(const FusedArgs& a, Ring<SH, K>& g, float* sP,
                                          float* eR, int t, int lane, int part) {
  constexpr int S2 = (S + 2) % 3;
  constexpr int NB = NW * SH / kMaxGroupPlanes;
  const RowCtx c = row_ctx(a);
  const WLBM_CONST uint32_t* sels = row_ptr(a.sels[L - 1]);
  const int i_begin = part * SH;
  float* pl = sP + (2 * (L - 1) + (t & 1)) * NB * 64;
#pragma unroll
  for (int b0 = 0; b0 < SH; b0 += kMaxGroupPlanes) {
    const int i0 = i_begin + b0;
    float bsum = 0.f;
#pragma unroll
    for (int d = 0; d < kMaxGroupPlanes; ++d) {
      const float out = relax_up<SH, K, WF, L, S>(a, g, sel_at(c.tab, sels[i0 + d]), c.wtab[i0 + d],
                                                  b0 + d, eR + (L - 1) * 3 * kERow + 1 + lane);
      g.X[L - 1][S][b0 + d] = out;
      bsum += out;
    }
    pl[(i0 / kMaxGroupPlanes) * 64 + lane] = bsum;
  }
  // W of this row (level L-1 holds it in slot S2)
  if constexpr (WF) g.W[L - 1][S] = g.W[L - 2][S2];
  lds_barrier();
  float E = 0.f;
#pragma unroll
  for (int k = 0; k < NB; ++k) E += pl[k * 64 + lane];
  g.E[L - 1][S] = WF ? E * g.W[L - 1][S] : E;
  eR[(L * 3 + S) * kERow + 1 + lane] = g.E[L - 1][S];
  __builtin_amdgcn_wave_barrier();
}

// The output level K at iteration t: row ro = r - (K-1), stored with its
// ghost copies.
template <int NW, int SH, int K, bool WF, int S>
__device__ __forceinline__ void level_out(const FusedArgs& a, Ring<SH, K>& g, float* sP,
                                          const float* eR, int t, int x0, int y0, int lane,
                                          int part, bool out_lane) {
  constexpr int NB = NW * SH / kMaxGroupPlanes;
  const RowCtx c = row_ctx(a);
  const WLBM_CONST uint32_t* sels = row_ptr(a.sels[K - 1]);
  const int ny = a.ny, pitch = a.pitch, nx = a.nx;
  const long long plane = a.plane;
  const int i_begin = part * SH;
  const int ro = y0 - (K - 1) + t - (K - 1);
  const bool store = out_lane && ro < ny;
  const int xo = x0 - K + lane;
  // byte offsets of the cell and its ghosts (used only where stored)
  const int row_o = (ro + 1) * pitch + kXOff;
  const uint32_t ob = uint32_t((row_o + xo) * 4);
  // Ghost copies of this cell in the frame (nx >= 2 kGhost and ny >= 2, so
  // a cell has at most one ghost column and one ghost row): columns 0 ..
  // kGhost-1 are copied to nx .. nx+kGhost-1 and columns nx-kGhost .. nx-1 to
  // -kGhost .. -1; rows 0 and ny - 1 to ny and -1.  Only blocks on the
  // lattice's edge have any, which the whole block knows.
  const bool edge = x0 == 0 || x0 + kStrip<K> + kGhost - 1 >= nx || ro == 0 || ro == ny - 1;
  const bool gx = store && (xo < kGhost || xo >= nx - kGhost);
  const bool gy = store && (ro == 0 || ro == ny - 1);
  const int xg = xo < kGhost ? xo + nx : xo - nx;
  const int yg = ro == 0 ? ny : -1;
  const int row_g = (yg + 1) * pitch + kXOff;
  const uint32_t obx = uint32_t((row_o + xg) * 4);
  const uint32_t oby = uint32_t((row_g + xo) * 4);
  const uint32_t obxy = uint32_t((row_g + xg) * 4);
  float* po = sP + (2 * (K - 1) + (t & 1)) * NB * 64;
#pragma unroll
  for (int b0 = 0; b0 < SH; b0 += kMaxGroupPlanes) {
    const int i0 = i_begin + b0;
    float bsum = 0.f;
    const rsrc_t ro_rs = make_rsrc(a.e_out + (long long)i0 * plane,
                                   uint32_t(kMaxGroupPlanes * plane * 4));
    float o[kMaxGroupPlanes];
#pragma unroll
    for (int d = 0; d < kMaxGroupPlanes; ++d) {
      const float out = relax_up<SH, K, WF, K, S>(a, g, sel_at(c.tab, sels[i0 + d]), c.wtab[i0 + d],
                                                  b0 + d, eR + (K - 1) * 3 * kERow + 1 + lane);
      bsum += out;
      o[d] = out;
    }
    po[(i0 / kMaxGroupPlanes) * 64 + lane] = bsum;
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
}

// Iteration t (ring slot S = t mod 3): level 1, then each higher level once
// the three rows it reads exist.
template <int NW, int SH, int K, bool WF, int S>
__device__ __forceinline__ void iteration(const FusedArgs& a, Ring<SH, K>& g, float* sP,
                                          float* eR, int t, int x0, int y0, int lane, int part,
                                          uint32_t lcol, bool out_lane) {
  level1<NW, SH, K, WF, S>(a, g, sP, eR, t, y0, lane, part, lcol);
  if constexpr (K >= 3) {
    if (t < 2) return;
    level_mid<NW, SH, K, WF, 2, S>(a, g, sP, eR, t, lane, part);
  }
  if constexpr (K >= 4) {
    if (t < 4) return;
    level_mid<NW, SH, K, WF, 3, S>(a, g, sP, eR, t, lane, part);
  }
  if (t < 2 * (K - 1)) return;
  level_out<NW, SH, K, WF, S>(a, g, sP, eR, t, x0, y0, lane, part, out_lane);
}

// Ghost frame of a periodic lattice written by another producer (k_step
// writes the first ghost column and row only): every ghost cell (columns
// -kGhost .. -1 and nx .. nx+kGhost-1 of rows 0 .. ny-1, and rows -1, ny of
// columns -kGhost .. nx+kGhost-1) of planes 0 .. nplanes-1 copies the cell it
// wraps to.
__global__ __launch_bounds__(kBlock) void k_fill_ghosts(float* base, long long plane, int nplanes,
                                                       int nx, int ny, int pitch) {
  const long long ncol = 2LL * kGhost * ny, nrow = 2LL * (nx + 2 * kGhost);
  const long long nper = ncol + nrow;
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= nper * nplanes) return;
  const int p = int(t / nper);
  const long long g = t - (long long)p * nper;
  int gx, gy;
  if (g < ncol) {
    const int k = int(g / ny);
    gy = int(g - (long long)k * ny);
    gx = k < kGhost ? k - kGhost : nx + k - kGhost;
  } else {
    const long long h = g - ncol;
    const int k = int(h / (nx + 2 * kGhost));
    gx = int(h - (long long)k * (nx + 2 * kGhost)) - kGhost;
    gy = k == 0 ? -1 : ny;
  }
  float* pl = base + (long long)p * plane;
  pl[cell(gx, gy, pitch)] = pl[cell(wrap_index(gx, nx), wrap_index(gy, ny), pitch)];
}

template <int NW, int SH, bool WF, int K>
__global__ __launch_bounds__(64 * NW) void k_stepk(const FusedArgs a) {
  // E batch sums: [level 1 .. K][row parity][batch of 8 directions][lane]
  __shared__ float sP[2 * K * (NW * SH / kMaxGroupPlanes) * 64];
  // each wave's own copy of the E rings: step n, then levels 1 .. K-1
  __shared__ float sEr[NW][K * 3 * kERow];
  const int lane = threadIdx.x & 63;
  const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (b % a.strips_x) * kStrip<K>;
  const int y0 = (b / a.strips_x) * a.rows;
  // this lane's column; lanes past the ghost frame read its last column
  // (their values are never used), so that every read stays inside the row
  // and its padding
  const int x = x0 - K + lane;
  const int xl = x < a.nx + kGhost - 1 ? x : a.nx + kGhost - 1;
  const uint32_t lcol = uint32_t((kXOff + xl) * 4);
  const bool out_lane = lane >= K && lane < K + kStrip<K> && x < a.nx;

  Ring<SH, K> g;
  // step-n E of rows r0 - 1 and r0 (r0 = y0 - (K-1), the first level-1 row)
  // into slots 0 and 1; the loads of row r0 bring row r0 + 1 into slot 2
  const uint32_t plane_bytes = uint32_t(a.plane * 4);
  const int r0 = y0 - (K - 1);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const uint32_t rb = uint32_t((wrap_index(r0 - 1 + k, a.ny) + 1) * a.pitch * 4);
    g.rb[k] = rb;
    const float Ev = buf_load(make_rsrc(a.E_in, plane_bytes), lcol, rb);
    if constexpr (WF) {
      const float Wv = buf_load(make_rsrc(a.Wf, plane_bytes), lcol, rb);
      g.Wn[k] = Wv;
      g.En[k] = Ev * Wv;
    } else {
      g.En[k] = Ev;
    }
  }
  float* eR = sEr[part];
  // the pads either side of each row (read only by lanes whose results are
  // never used) hold zero
  if (lane < 3 * K) eR[lane * kERow] = eR[lane * kERow + kERow - 1] = 0.f;
  eR[1 + lane] = g.En[0];
  eR[kERow + 1 + lane] = g.En[1];
  g.wn = wrap_index(r0, a.ny);
  issue_row<SH, K, WF, 2>(a, g, part * SH, lcol);
  // a.rows + 2 (K - 1) is a multiple of 3 (the loop is unrolled by three)
  const int T = a.rows + 2 * (K - 1);
  for (int t = 0; t < T; t += 3) {
    iteration<NW, SH, K, WF, 0>(a, g, sP, eR, t, x0, y0, lane, part, lcol, out_lane);
    iteration<NW, SH, K, WF, 1>(a, g, sP, eR, t + 1, x0, y0, lane, part, lcol, out_lane);
    iteration<NW, SH, K, WF, 2>(a, g, sP, eR, t + 2, x0, y0, lane, part, lcol, out_lane);
  }
}

template <int NW, int SH>
hipError_t launchk(const FusedArgs& a, int k, bool wf, hipStream_t s) {
  const dim3 grid(a.strips_x * a.strips_y), block(64 * NW);
  if (k == 2) {
    if (wf)
      hipLaunchKernelGGL((k_stepk<NW, SH, true, 2>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_stepk<NW, SH, false, 2>), grid, block, 0, s, a);
  } else if (k == 3) {
    if (wf)
      hipLaunchKernelGGL((k_stepk<NW, SH, true, 3>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_stepk<NW, SH, false, 3>), grid, block, 0, s, a);
  } else if (k == 4) {
    if (wf)
      hipLaunchKernelGGL((k_stepk<NW, SH, true, 4>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_stepk<NW, SH, false, 4>), grid, block, 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t fill_ghosts(float* base, long long plane, int nplanes, int nx, int ny, int pitch,
                       hipStream_t s) {
  const long long n = (2LL * kGhost * ny + 2LL * (nx + 2 * kGhost)) * nplanes;
  hipLaunchKernelGGL(k_fill_ghosts, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     base, plane, nplanes, nx, ny, pitch);
  return hipGetLastError();
}

int fused_strips_x(int nx, int k) {
  const int w = k == 4 ? kStrip<4> : (k == 3 ? kStrip<3> : kStrip<2>);
  return (nx + w - 1) / w;
}

// Candidate block heights for k steps per launch: R + 2 (k - 1) a multiple
// of 3, R up to 62, and no taller than needed to cover ny in one block row.
// Taller blocks re-read fewer halo rows but give fewer blocks, and how the
// last round of resident blocks fills the GPU depends on the lattice, so the
// caller times them (at 1024 x 1024, Q = 64, three steps per launch: R = 23
// 1159, 29 963, 35 1058, 47 1064 G updates/s).
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

template <int NW, int SH>
int blocks_per_cu_tmpl(int k, bool wf) {
  int n = 0;
  hipError_t e = hipSuccess;
  const int bs = 64 * NW;
  if (k == 2)
    e = wf ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stepk<NW, SH, true, 2>, bs, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stepk<NW, SH, false, 2>, bs, 0);
  else if (k == 3)
    e = wf ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stepk<NW, SH, true, 3>, bs, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stepk<NW, SH, false, 3>, bs, 0);
  else
    e = wf ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stepk<NW, SH, true, 4>, bs, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stepk<NW, SH, false, 4>, bs, 0);
  return e == hipSuccess ? n : 0;
}

int fused_blocks_per_cu(int q, int k, bool per_cell) {
  if (q <= 64) {
    switch (q / 8) {
      case 1: return blocks_per_cu_tmpl<1, 8>(k, per_cell);
      case 2: return blocks_per_cu_tmpl<2, 8>(k, per_cell);
      case 3: return blocks_per_cu_tmpl<3, 8>(k, per_cell);
      case 4: return blocks_per_cu_tmpl<4, 8>(k, per_cell);
      case 5: return blocks_per_cu_tmpl<5, 8>(k, per_cell);
      case 6: return blocks_per_cu_tmpl<6, 8>(k, per_cell);
      case 7: return blocks_per_cu_tmpl<7, 8>(k, per_cell);
      case 8: return blocks_per_cu_tmpl<8, 8>(k, per_cell);
      default: return 0;
    }
  }
  switch (q / 16) {
    case 5: return blocks_per_cu_tmpl<5, 16>(k, per_cell);
    case 6: return blocks_per_cu_tmpl<6, 16>(k, per_cell);
    case 7: return blocks_per_cu_tmpl<7, 16>(k, per_cell);
    case 8: return blocks_per_cu_tmpl<8, 16>(k, per_cell);
    default: return 0;
  }
}

// Waves per block: one per 8 directions up to q = 64, one per 16 up to 128.
bool fused_supported(int q, int nx, int ny) {
  return nx >= 2 * kGhost && ny >= 2 && q % kMaxGroupPlanes == 0 &&
         (q <= 64 || (q <= 128 && q % 16 == 0));
}

hipError_t launch_fused(const FusedArgs& a, int k, bool per_cell, hipStream_t s) {
  if (a.q <= 64) {
    switch (a.q / 8) {
      case 1: return launchk<1, 8>(a, k, per_cell, s);
      case 2: return launchk<2, 8>(a, k, per_cell, s);
      case 3: return launchk<3, 8>(a, k, per_cell, s);
      case 4: return launchk<4, 8>(a, k, per_cell, s);
      case 5: return launchk<5, 8>(a, k, per_cell, s);
      case 6: return launchk<6, 8>(a, k, per_cell, s);
      case 7: return launchk<7, 8>(a, k, per_cell, s);
      case 8: return launchk<8, 8>(a, k, per_cell, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (a.q / 16) {
    case 5: return launchk<5, 16>(a, k, per_cell, s);
    case 6: return launchk<6, 16>(a, k, per_cell, s);
    case 7: return launchk<7, 16>(a, k, per_cell, s);
    case 8: return launchk<8, 16>(a, k, per_cell, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wlbm
