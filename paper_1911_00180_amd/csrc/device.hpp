// Device-side data layout and kernel launch interface of the worm-LBM
// library.  Shared by the library's .hip sources only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wlbm {

// Padded HBM layout of every per-cell field (populations, E, W field).
// A field plane holds rows y = -1 .. ny and columns x = -4 .. nx + 3, where
// rows -1 and ny and columns -4 .. -1, nx .. nx + 3 are ghosts: for a
// periodic edge they hold copies of the opposite edge, otherwise they stay
// zero.  k_step writes the first ghost column / row (-1, nx, ny) of what it
// produces; the multi-step kernels, which read up to four ghost columns,
// write all four, and fill_ghosts refreshes them after other producers.
// Cell (x, y) sits at (y + 1) * pitch + kXOff + x, so that x = 0 starts a
// 128-byte line and a wave's 64 consecutive cells are two whole lines; each
// row has at least five cells of padding after x = nx - 1.  Populations are
// [q] such planes (structure of arrays).
constexpr int kXOff = 32;
constexpr int kBlock = 256;
constexpr int kMaxQ = 1024;

enum Edge { kPeriodic = 0, kBlackbody = 1, kDiffuse = 2 };

inline int padded_pitch(int nx) { return ((nx + kXOff + 5 + 31) / 32) * 32; }
inline int64_t padded_plane(int nx, int ny) { return int64_t(ny + 2) * padded_pitch(nx); }

// Schedule code of one direction on one step: bits 0-1 dx+1, bits 2-3 dy+1,
// bit 4 hop.  Rows of q bytes, read four directions per 32-bit word.
inline uint8_t pack_code(int dx, int dy, int hop) {
  return uint8_t((dx + 1) | ((dy + 1) << 2) | (hop << 4));
}

struct StepArgs {
  const float* e_in;
  float* e_out;
  const float* E_in;
  float* E_out;
  const float* Wf;        // padded per-cell corrected weight (per-cell mode)
  double* qsx;            // heat-flux window sums, [ny][nx] (flux mode), float64
  double* qsy;
  const uint32_t* codes;  // schedule row of this step
  // k_step only: per direction, the byte offset of its pulled population and
  // of its entry in the multi-step kernels' selection table (move code times
  // kSelEntryBytes) for this step; k_step_batch decodes the codes instead
  const uint32_t* pulls;
  const uint32_t* sels;
  const float* wtab;      // [q] weights
  const float* sxtab;     // [q] unit vectors
  const float* sytab;
  const int* mtab;        // [q] index of each direction's mirror image in a y wall
  float W;                // uniform corrected weight
  float spec;             // diffuse y walls: specular fraction p
  // Diffuse walls: sums of w_i over the directions whose pending move points
  // into the domain through the lo (dy = +1) / hi (dy = -1) wall on this
  // step, over the hopping ones and over all of them.
  float in_lo_hop, in_lo_all, in_hi_hop, in_hi_all;
  float t_x_lo, t_x_hi, t_y_lo, t_y_hi;
  int nx, ny, q, pitch;
  long long plane;
  int x_edge, y_edge;
  int tiles_x, ntiles;
  int q_first;            // flux mode: 1 on the first step of the window
};

struct Geometry {
  int nx, ny, q, pitch;
  long long plane;
  int x_edge, y_edge;
};

struct Walls {
  float x_lo, x_hi, y_lo, y_hi;
};

// Collide-and-stream of one time step.  Tiles are 64 cells wide and
// 4 / split rows tall; the directions of each cell are split over `split`
// waves (1, 2 or 4; q must be a multiple of 8 * split).  per_cell selects the
// per-cell weight field; flux accumulates the heat flux into qsx/qsy.  The
// kernel addresses a batch of kMaxGroupPlanes consecutive direction planes
// through one buffer descriptor, so that many planes (plus one row and
// column) must fit in 4 GiB.
constexpr int kMaxGroupPlanes = 8;
hipError_t launch_step(const StepArgs& a, int split, bool per_cell, bool flux, hipStream_t s);
int tiles_x_for(int nx);
int tiles_y_for(int ny, int split);
// Dynamic LDS of a step block: the 8-direction batch sums of E' when the
// directions of a cell are split over several waves.
size_t step_batch_lds_bytes(int q, int split);

// K = 2, 3 or 4 time steps (n+1 .. n+K) of a lattice with periodic x and y
// edges in one launch; codes[k] is the schedule row of step n+1+k.  Same
// results as K launch_step calls.
// Bytes per schedule code in the multi-step kernels' selection table.
constexpr uint32_t kSelEntryBytes = 32;
struct FusedArgs {
  const float* e_in;
  float* e_out;
  const float* E_in;
  float* E_out;
  const float* Wf;
  // Byte offset of the population that direction i pulls on the launch's
  // first step, from a cell's row and column, one row and one float up:
  // (1 - hy) pitch 4 + 4 (1 - hx) + (i mod 8) plane 4, with (hx, hy) the
  // move on a hop and (0, 0) on a pause.
  const uint32_t* pulls;
  // Per step of the launch: direction i's byte offset into the selection
  // table of the kernel (its schedule code times the table's entry size).
  const uint32_t* sels[4];
  const float* wtab;
  float W;
  int nx, ny, q, pitch;
  long long plane;
  int strips_x, strips_y;
  int rows;   // output rows per block: rows + 2 (k - 1) a multiple of 3
  // Edges (x: periodic or blackbody; y: periodic, blackbody or fully
  // diffuse) and blackbody temperatures.
  int x_edge, y_edge;
  float t_x_lo, t_x_hi, t_y_lo, t_y_hi;
  // The schedule row of the launch's first step (step m of the launch at
  // codes + m q / 4; wall rows decode it) and its four sums of inward weights
  // of the diffuse walls (as StepArgs: lo hopping, lo all, hi hopping, hi all;
  // step m at ins + 4 m), in device memory uploaded with the schedule.
  const uint32_t* codes;
  const float* ins;
  // Heat flux of flux-window steps (the flux kernels only): bit m - 1 of
  // flux_levels set for step m of the launch (1 .. K) in the window; the
  // window's float64 sums qsx, qsy ([ny][nx]) are set by step flux_first
  // (0: by none of the launch's steps) and added to by the others; sxtab,
  // sytab: s_x,i and s_y,i.
  double* qsx;
  double* qsy;
  const float* sxtab;
  const float* sytab;
  uint32_t flux_levels;
  int flux_first;
};
// K = 2 .. 4 steps of n lattices with the same q and per-cell field use in
// one launch.  lats holds each lattice's arguments for buffer parity 0 and 1
// ([2n], on the device; the per-step fields are taken from the rings below);
// first[j] is the first block of lattice j, first[n] = nblocks.  Lattice j's
// per-step tables are rings of two schedule chunks: selection offsets
// (sels[j]), pull offsets of its geometry (pulls[j]), schedule rows
// (codes[j], q bytes a step) and inward-weight sums (ins[j], 4 a step); the
// launch's first step is ring row `row`.
struct FusedBatchArgs {
  const FusedArgs* lats;
  const int* first;
  const uint32_t* const* sels;
  const uint32_t* const* pulls;
  const uint8_t* const* codes;
  const float* const* ins;
  int row;
  int n, nblocks, parity;
  // flux-window steps of the launch, as FusedArgs (the same for every
  // lattice; each lattice's sums and tables are in lats)
  uint32_t flux_levels;
  int flux_first;
};
// flux: the flux kernels (b.flux_levels != 0).
hipError_t launch_fused_batch(const FusedBatchArgs& b, int q, int k, bool per_cell, bool flux,
                              hipStream_t s);
hipError_t launch_fused_batch_walls2(const FusedBatchArgs& b, int q, bool per_cell,
                                     hipStream_t s);
hipError_t launch_fused_batch_walls3(const FusedBatchArgs& b, int q, bool per_cell,
                                     hipStream_t s);
hipError_t launch_fused_batch_walls4(const FusedBatchArgs& b, int q, bool per_cell,
                                     hipStream_t s);
hipError_t launch_fused_batch_flux2(const FusedBatchArgs& b, int q, bool per_cell,
                                    hipStream_t s);
hipError_t launch_fused_batch_flux3(const FusedBatchArgs& b, int q, bool per_cell,
                                    hipStream_t s);
hipError_t launch_fused_batch_flux4(const FusedBatchArgs& b, int q, bool per_cell,
                                    hipStream_t s);

// K = 2 .. 4 steps per launch; lattices with walls run the kernels of
// fused_walls{2,3,4}.hip, launches with flux-window steps (flux: a.flux_levels
// != 0) those of fused_flux{2,3,4}.hip.
hipError_t launch_fused(const FusedArgs& a, int k, bool per_cell, bool flux, hipStream_t s);
hipError_t launch_fused_walls2(const FusedArgs& a, bool per_cell, hipStream_t s);
hipError_t launch_fused_walls3(const FusedArgs& a, bool per_cell, hipStream_t s);
hipError_t launch_fused_walls4(const FusedArgs& a, bool per_cell, hipStream_t s);
hipError_t launch_fused_flux2(const FusedArgs& a, bool per_cell, hipStream_t s);
hipError_t launch_fused_flux3(const FusedArgs& a, bool per_cell, hipStream_t s);
hipError_t launch_fused_flux4(const FusedArgs& a, bool per_cell, hipStream_t s);
int fused_blocks_per_cu_walls2(int q, bool per_cell);
int fused_blocks_per_cu_walls3(int q, bool per_cell);
int fused_blocks_per_cu_walls4(int q, bool per_cell);
// Ghost frame of nplanes planes from the cells they wrap to: the four ghost
// columns each side if px (periodic x), the ghost rows if py.
hipError_t fill_ghosts(float* base, long long plane, int nplanes, int nx, int ny, int pitch,
                       bool px, bool py, hipStream_t s);
int fused_strips_x(int nx, int k);
// Candidate output rows per block for k steps per launch (at most max_cand,
// written to cand); returns their number.
int fused_row_candidates(int ny, int k, int* cand, int max_cand);
// Whether the multi-step kernels take this lattice: q a multiple of 8 up to
// 128, or q = 192 or 256 (two steps per launch), nx >= 8, ny >= 2.
bool fused_supported(int q, int nx, int ny);
// Resident blocks per CU of the k-step kernel for q directions and these
// edges (occupancy query of the runtime; 0 if it fails).
int fused_blocks_per_cu(int q, int k, bool per_cell, bool walls);

// One time step of n lattices in one launch (same split, per-cell field use
// and step; lattices with the same q, direction set and grid speeds share a
// schedule ring).  lats holds, for each lattice j, its arguments for buffer
// parity 0 and 1 ([2n], on the device); first[j] is the first block of
// lattice j, first[n] = nblocks.  The per-step fields of StepArgs (codes,
// wall sums, q_first) come from here.
struct BatchStepArgs {
  const StepArgs* lats;
  const int* first;
  // This step's schedule row and sums of inward weights of diffuse walls
  // (in_lo_hop, in_lo_all, in_hi_hop, in_hi_all), in device memory uploaded
  // with the schedule, so that a captured launch reads the values of its
  // step.  With one direction set in the batch: codes and ins.  With several
  // (grouped launch): lattice j's rings start at ring_codes[j] and
  // ring_ins[j], and the step is their row `row`.
  const uint32_t* codes;
  const float* ins;
  const uint32_t* const* ring_codes;
  const float* const* ring_ins;
  int row;
  int n, nblocks, parity, q_first;
  int q;   // largest q of the batch (sizes the dynamic LDS)
};
hipError_t launch_step_batch(const BatchStepArgs& b, int split, bool per_cell, bool flux,
                             bool grouped, hipStream_t s);

// e_i = w_i T0 (T0 unpadded [ny][nx]), blackbody walls, E, ghosts.
hipError_t launch_init_temperature(const Geometry& g, const float* T0, float* e, float* E,
                                   const float* wtab, Walls walls, hipStream_t s);
// e from an unpadded [q][ny][nx] array, blackbody walls, E, ghosts.
hipError_t launch_init_populations(const Geometry& g, const float* src, float* e, float* E,
                                   const float* wtab, Walls walls, hipStream_t s);
hipError_t launch_read_populations(const Geometry& g, const float* e, float* dst, hipStream_t s);
// Overwrite the n source cells (x, y) = cells[2s], cells[2s+1] with the
// imposed DDEDs vals[s][q], and E with their sum.
hipError_t launch_apply_sources(const Geometry& g, float* e, float* E, const int32_t* cells,
                                const float* vals, int n, hipStream_t s);
hipError_t launch_read_field(const Geometry& g, const float* f, float* dst, hipStream_t s);
// dst[y][x] += a * f(x, y) (f padded, dst unpadded).
hipError_t launch_axpy_field(const Geometry& g, float a, const float* f, float* dst,
                             hipStream_t s);
hipError_t launch_read_flux(const Geometry& g, const float* e, const float* sxtab,
                            const float* sytab, float* qx, float* qy, hipStream_t s);
hipError_t launch_scale_pair(int n, const double* ax, const double* ay, double scale, float* bx,
                             float* by, hipStream_t s);
// Totals in float64: out[0] = sum E, out[1] = sum q_x, out[2] = sum q_y.
hipError_t launch_totals(const Geometry& g, const float* e, const float* E, const float* sxtab,
                         const float* sytab, double* partials, int max_blocks, double* out,
                         hipStream_t s);
// Float64 sums of q_x, q_y over columns x0 <= x < x1, all rows: out[0], out[1]
// (out[2] = 0).  window != 0: from the flux-window sums qsx/qsy; else from e.
hipError_t launch_flux_sum(const Geometry& g, const float* e, const float* sxtab,
                           const float* sytab, const double* qsx, const double* qsy, int window,
                           int x0, int x1, double* partials, int max_blocks, double* out,
                           hipStream_t s);
// Per-cell corrected weight from an MFP field: check pass (sets *flag on a
// non-positive MFP or an unstable/non-finite weight), then write pass.
hipError_t launch_check_mfp(const Geometry& g, const float* mfp, double lam, double f, int corr,
                            int* flag, hipStream_t s);
hipError_t launch_write_wfield(const Geometry& g, const float* mfp, double lam, double f,
                               int corr, float* Wf, float* Wraw, hipStream_t s);

// Reverse step m of the adjoint: reads lam^m (zero at blackbody cells and
// beyond non-periodic edges), its eight move-class partial sums H^m and the
// forward state e^{m-1}, E^{m-1}; writes lam^{m-1} and H^{m-1} (classes by
// the moves of step m-1) and adds to the float64 per-cell accumulators gW
// (dL/dW_corr) and gB (wall cells: dL/de^{m-1} summed with the weights).
struct AdjArgs {
  const float* lam_in;
  float* lam_out;
  const float* H_in;      // 8 padded planes
  float* H_out;
  const float* e_prev;    // q padded planes
  const float* E_prev;    // padded plane
  const float* Wf;        // per-cell corrected weight (per-cell mode)
  double* gW;             // [ny][nx]
  double* gB;             // [ny][nx], wall cells only
  const uint32_t* codes;       // schedule row of step m
  const uint32_t* codes_next;  // schedule row of step m-1 (any row for m = 1)
  const float* wtab;
  float W;
  int nx, ny, q, pitch;
  long long plane;
  int x_edge, y_edge;
  int tiles_x, ntiles;
};

// Adds dL/dT = vals[p] at probe cells (x, y) = cells[2p], cells[2p+1] to
// lam (all directions) and H (class c gets vals[p] * wcls[c]); at wall cells
// to gB instead, times wall_w = sum_i w_i.  Sets *flag for a cell outside
// the lattice.
struct AdjSeedArgs {
  float* lam;
  float* H;
  double* gB;
  const int32_t* cells;
  const float* vals;
  int* flag;
  int n;
  float wcls[8];
  double wall_w;
  int nx, ny, q, pitch;
  long long plane;
  int x_edge, y_edge;
};

hipError_t launch_adjoint(const AdjArgs& a, int split, bool per_cell, hipStream_t s);
hipError_t launch_adj_seed(const AdjSeedArgs& a, hipStream_t s);
// Per-cell dL/dMFP from dL/dW_corr; Wraw is the [ny][nx] field of W = 1/MFP
// or NULL for the uniform W_uniform.
hipError_t launch_adj_grad_mfp(const Geometry& g, const double* gW, const float* Wraw,
                               double W_uniform, double lam, double f, int corr, float* out,
                               hipStream_t s);
hipError_t launch_adj_grad_t0(const Geometry& g, const float* lam, const float* wtab, float* out,
                              hipStream_t s);
// out[0..3] = dL/dT of the x_lo, x_hi, y_lo, y_hi walls.
hipError_t launch_adj_walls(const Geometry& g, const double* gB, double* out, hipStream_t s);
hipError_t launch_read_probes(const Geometry& g, const float* E, const int32_t* cells, int n,
                              float* out, hipStream_t s);

// Move class 0..7 of a D2Q8 move, as the adjoint kernel numbers its partial
// sums (host copy of the device rule).
inline int host_move_class(int dx, int dy) {
  const int c = (dx + 1) * 3 + (dy + 1);
  return c - (c > 4 ? 1 : 0);
}

}  // namespace wlbm
