// Internal declarations shared by the C-ABI sources of libwormlbm.so
// (api.hip: lattice set-up, stepping and readout; api_states.hip: saved
// states, tapes and the adjoint; api_batch.hip: batches; api_tune.hip: launch
// configuration and tuning).  Not part of the interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/wormlbm.h"
#include "device.hpp"
#include "tables.hpp"

namespace wlbm {

// Sets the calling thread's last-error message and returns st.
wlbm_status fail(wlbm_status st, const char* fmt, ...);
// The calling thread's last-error message.
const char* last_error_text();

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::wlbm::fail(WLBM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kReduceBlocks = 1024;
constexpr int kDefaultChunk = 240;   // a multiple of 2, 3 and 4 (steps per launch)
constexpr int64_t kMaxSteps = (int64_t(1) << 31) - 1;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of the lattice workspace regions.
struct Carve {
  size_t e[2], E[2], Wf, Wraw, qsx, qsy, partials, totals, flag, sched, pulls, ins, wtab, sxtab,
      sytab, mtab, total;
};

// Lattices that the multi-step kernels can advance.
bool fusable(const wlbm_params& p);
int chunk_steps(const wlbm_params& p);
Carve carve(const wlbm_params& p);

// Byte offsets of the adjoint workspace regions.
struct AdjCarve {
  size_t lam[2], H[2], gW, gB, sched, walls, flag, total;
};
AdjCarve adj_carve(const wlbm_params& p);

inline size_t state_bytes_of(const wlbm_params& p) {
  return align_up(size_t(padded_plane(p.nx, p.ny)) * sizeof(float) * size_t(p.q + 1));
}

}  // namespace wlbm

struct wlbm_lattice {
  wlbm_params p{};
  wlbm::DirSet dirs;
  wlbm::TasState tas;
  wlbm::Geometry g{};
  hipStream_t stream = nullptr;
  int device = 0;           // GPU holding the workspace
  char* ws = nullptr;
  wlbm::Carve c{};
  int cur = 0;              // population buffer holding the current state
  float W = 0.f;            // uniform corrected weight
  bool per_cell = false;    // per-cell weight field active
  int split = 1;            // waves sharing the directions of one cell
  int chunk = wlbm::kDefaultChunk;
  // Output rows per block of the k-step kernels, per [per_cell][k]: fixed by
  // wlbm_set_block_rows or wlbm_tune_block_rows; 0 = the launch model's pick.
  int rows[2][5] = {};
  mutable int model_rows[2][5] = {};   // the launch model's pick, once computed
  // The current population and E planes hold their whole ghost frame (as
  // the multi-step kernels write it); other producers write the first ghost
  // column and row only.
  bool ghosts_full = false;
  bool wf_ghosts_full = false;   // the same for the per-cell weight field
  uint8_t* pinned[2] = {nullptr, nullptr};
  uint32_t* pinned_pulls[2] = {nullptr, nullptr};   // staging of the pull offsets
  float* pinned_ins[2] = {nullptr, nullptr};        // staging of the inward-weight sums
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_pending[2] = {false, false};
  int64_t chunk_counter = 0;
  int flux_window = 0;
  bool flux_valid = false;
  bool broken = false;
  wlbm::Walls walls{};
  wlbm::ScheduleBook book;  // schedule rows of any step, for restarts and the adjoint
  // internal sources (caller's device arrays, kept valid by the caller)
  int nsrc = 0;
  const int32_t* src_cells = nullptr;
  const float* src_vals = nullptr;
  // adjoint (reverse pass) state
  char* aws = nullptr;      // caller's adjoint workspace
  wlbm::AdjCarve ac{};
  int acur = 0;             // lam / H buffer holding lam^am
  int64_t am = -1;          // adjoint step index; -1 when no reverse pass is active

  float* ptr(size_t off) { return reinterpret_cast<float*>(ws + off); }
  double* dptr(size_t off) { return reinterpret_cast<double*>(ws + off); }
  float* aptr(size_t off) { return reinterpret_cast<float*>(aws + off); }
};

namespace wlbm {

wlbm_status check_lat(const wlbm_lattice* l);
wlbm_status check_steps(const wlbm_lattice* l, int64_t nsteps);
// Default direction split for q (as many waves per cell as q allows, up to
// four).
int auto_split(int q);
// Advance nsteps (validated by the caller); with a tape, step k writes its
// output into tape slot k.
wlbm_status run_steps(wlbm_lattice* l, int64_t nsteps, char* tape, size_t slot_bytes);
// Whether run_steps may advance this lattice several steps per launch (with
// no tape and no flux window), and at most how many.
bool lattice_fuses(const wlbm_lattice* l);
int fused_k_cap(const wlbm_lattice* l);
// Steps per launch the lattice's multi-step launches take: step_fusion 2 .. 4,
// or for 1 (automatic) four, two for lattices with walls and q above 64 or a
// per-cell field (measured fastest), capped by fused_k_cap.
int fused_k_max(const wlbm_lattice* l);
// Output rows per block of the k-step kernel for the lattice's current
// weight mode: the fixed or tuned height, else the launch model's pick.
int block_rows_for(const wlbm_lattice* l, int k);
// Per-device set-up of the allocation-free readout (api_noalloc.hip).
wlbm_status noalloc_setup(int device);

}  // namespace wlbm
