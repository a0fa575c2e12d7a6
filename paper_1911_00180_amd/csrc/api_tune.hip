// C-ABI of libwormlbm.so (declared in include/wormlbm.h): launch
// configuration of the step kernels and its tuning.
//
// Two choices affect only speed, never results: the direction split of the
// single-step kernel (waves sharing one cell's directions) and the block
// height (output rows per block) of the kernels that advance k = 2 .. 4 steps
// per launch.  Neither is timed implicitly: wlbm_step uses the split of the
// parameters (or the default for q) and the height the caller fixed or a
// tuning call chose, else the launch model's pick below; wlbm_autotune and
// wlbm_tune_block_rows time the candidates on a saved state and restore it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "api_internal.hpp"

namespace wlbm {

// Row iterations of a block (R + 2 (k - 1)) that the launch model allows on a
// lattice with walls.
constexpr int kMaxWalledIterations = 18;

// Launch model of the k-step kernel: blocks run in rounds of (resident
// blocks per CU) x (CUs); a block of R output rows iterates over R + 2 (k-1)
// rows (the halo of the k levels).  The height with the fewest row
// iterations over all rounds, (rounds) x (R + 2 (k - 1)), is picked; among
// equals the taller (fewer blocks).  At 1024 x 1024, Q = 64, four steps per
// launch this gives the 45-row blocks (22 x 23 = 506 blocks, one round of
// 512) that timing also picks.  On a lattice with walls the blocks that touch
// one run the slower walled code, and short blocks measured faster: only
// heights of at most 18 row iterations are considered there (four steps per
// launch, 1024 x 1024 x 64 with blackbody x edges: 12 rows 0.060 ms per step
// against 0.075 at the 45 rows the unrestricted model picks; 2048 x 2048 x
// 128 with a per-cell field and blackbody x edges, two steps: 16 rows 0.571
// against 0.618 at 61; 4096 x 4096 x 256, blackbody x and diffuse y: 16 rows
// 4.26 against 4.29 at 58).
int block_rows_for(const wlbm_lattice* l, int k) {
  const int pc = l->per_cell ? 1 : 0;
  if (l->rows[pc][k]) return l->rows[pc][k];
  if (l->model_rows[pc][k]) return l->model_rows[pc][k];
  int cand[32];
  const int nc = fused_row_candidates(l->g.ny, k, cand, 32);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  const bool walls = l->g.x_edge != kPeriodic || l->g.y_edge != kPeriodic;
  const long long cap =
      (long long)std::max(1, fused_blocks_per_cu(l->p.q, k, l->per_cell, walls)) * cus;
  const long long sx = fused_strips_x(l->g.nx, k);
  int best = cand[0];
  long long best_cost = -1;
  for (int c = 0; c < nc; ++c) {
    const int R = cand[c];
    if (walls && c > 0 && R + 2 * (k - 1) > kMaxWalledIterations) break;
    const long long nb = sx * ((l->g.ny + R - 1) / R);
    const long long cost = ((nb + cap - 1) / cap) * (R + 2 * (k - 1));
    if (best_cost < 0 || cost <= best_cost) {
      best_cost = cost;
      best = R;
    }
  }
  l->model_rows[pc][k] = best;
  return best;
}

}  // namespace wlbm

using namespace wlbm;

extern "C" {

wlbm_status wlbm_set_dir_split(wlbm_lattice* l, int32_t split) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (split == 0) {
    l->split = auto_split(l->p.q);
    return WLBM_OK;
  }
  if (split != 1 && split != 2 && split != 4)
    return fail(WLBM_EINVAL, "dir_split must be 0, 1, 2 or 4");
  if (l->p.q % (kMaxGroupPlanes * split) != 0)
    return fail(WLBM_EINVAL, "q = %d cannot be split over %d waves", l->p.q, split);
  if (step_batch_lds_bytes(l->p.q, split) > 48 * 1024)
    return fail(WLBM_EINVAL, "q = %d is too large for a split over %d waves", l->p.q, split);
  l->split = split;
  return WLBM_OK;
}

int32_t wlbm_get_dir_split(const wlbm_lattice* l) { return l ? l->split : -1; }

wlbm_status wlbm_autotune(wlbm_lattice* l, void* d_state, size_t bytes, int32_t steps,
                          float* ms_by_split, int32_t* chosen) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (steps < 1 || steps > 10000) return fail(WLBM_EINVAL, "steps must be in 1 .. 10000");
  if (l->tas.n + steps + 2 > kMaxSteps) return fail(WLBM_EINVAL, "step count would overflow");
  const int64_t step0 = l->tas.n;
  const bool flux_valid = l->flux_valid;
  const int flux_window = l->flux_window;
  const int keep_split = l->split;
  const int keep_fusion = l->p.step_fusion;
  st = wlbm_save_state(l, d_state, bytes);
  if (st) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(WLBM_EHIP, "hipEventCreate failed: %s", hipGetErrorString(he));
  }
  const int cand[3] = {1, 2, 4};
  float best = 0.f;
  int best_split = keep_split;
  bool have = false;
  l->flux_window = 0;  // the tuning steps leave the flux-window sums alone
  l->p.step_fusion = 0;  // the split is the single-step kernel's: time that one
  for (int k = 0; k < 3 && st == WLBM_OK; ++k) {
    float ms = -1.f;
    if (l->p.q % (kMaxGroupPlanes * cand[k]) == 0 &&
        step_batch_lds_bytes(l->p.q, cand[k]) <= 48 * 1024) {
      l->split = cand[k];
      st = run_steps(l, 2, nullptr, 0);  // warm-up
      if (!st && (he = hipEventRecord(e0, l->stream)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventRecord failed: %s", hipGetErrorString(he));
      if (!st) st = run_steps(l, steps, nullptr, 0);
      if (!st && (he = hipEventRecord(e1, l->stream)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventRecord failed: %s", hipGetErrorString(he));
      if (!st && (he = hipEventSynchronize(e1)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventSynchronize failed: %s", hipGetErrorString(he));
      if (!st && (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventElapsedTime failed: %s", hipGetErrorString(he));
      if (!st) {
        ms /= float(steps);
        if (!have || ms < best) {
          best = ms;
          best_split = cand[k];
          have = true;
        }
      }
      if (!st) st = wlbm_load_state(l, d_state, bytes, step0);
    }
    if (ms_by_split) ms_by_split[k] = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  l->flux_window = flux_window;
  l->p.step_fusion = keep_fusion;
  if (st) {
    l->split = keep_split;
    return st;
  }
  l->split = best_split;
  l->flux_valid = flux_valid;
  if (chosen) *chosen = best_split;
  return WLBM_OK;
}


int32_t wlbm_get_steps_per_launch(const wlbm_lattice* l) {
  if (!l) return -1;
  return lattice_fuses(l) ? fused_k_max(l) : 1;
}

int32_t wlbm_get_block_rows(const wlbm_lattice* l, int32_t k) {
  if (!l || k < 2 || k > 4) return -1;
  if (!lattice_fuses(l)) return 0;
  return block_rows_for(l, k);
}

wlbm_status wlbm_set_block_rows(wlbm_lattice* l, int32_t k, int32_t rows) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (k < 2 || k > 4) return fail(WLBM_EINVAL, "k must be 2, 3 or 4 (got %d)", k);
  if (rows < 0 || rows > 62 || (rows > 0 && (rows + 2 * (k - 1)) % 3 != 0))
    return fail(WLBM_EINVAL,
                "rows must be 0 or 1 .. 62 with rows + 2 (k - 1) a multiple of 3 (got %d)", rows);
  l->rows[l->per_cell ? 1 : 0][k] = rows;
  return WLBM_OK;
}

wlbm_status wlbm_tune_block_rows(wlbm_lattice* l, void* d_state, size_t bytes, int32_t k,
                                 int32_t launches, int32_t* rows_out) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (k < 2 || k > 4) return fail(WLBM_EINVAL, "k must be 2, 3 or 4 (got %d)", k);
  if (launches < 1 || launches > 1000) return fail(WLBM_EINVAL, "launches must be in 1 .. 1000");
  if (!lattice_fuses(l))
    return fail(WLBM_EINVAL, "this lattice runs one step per launch (its edges, sources, q or "
                             "size rule out the multi-step kernels, or step_fusion is 0)");
  if (k > fused_k_cap(l))
    return fail(WLBM_EINVAL, "this lattice runs at most %d steps per launch", fused_k_cap(l));
  // a launch never crosses a schedule chunk: time whole launches of k steps
  const int per_call = std::max(1, std::min<int>(launches, l->chunk / k));
  const int64_t warm = 2, need = (warm + launches) * int64_t(k);
  if (l->tas.n + need > kMaxSteps) return fail(WLBM_EINVAL, "step count would overflow");
  const int64_t step0 = l->tas.n;
  const bool flux_valid = l->flux_valid;
  const int flux_window = l->flux_window;
  const int keep_fusion = l->p.step_fusion;
  const int pc = l->per_cell ? 1 : 0;
  const int keep_rows = l->rows[pc][k];
  st = wlbm_save_state(l, d_state, bytes);
  if (st) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(WLBM_EHIP, "hipEventCreate failed: %s", hipGetErrorString(he));
  }
  int cand[32];
  const int nc = fused_row_candidates(l->g.ny, k, cand, 32);
  std::vector<float> best(size_t(nc), -1.f);
  l->flux_window = 0;       // the timed steps leave the flux-window sums alone
  l->p.step_fusion = k;     // k steps per launch (a multiple of k steps each call)
  // two passes over the candidates, each keeping its best time
  for (int pass = 0; pass < 2 && st == WLBM_OK; ++pass) {
    for (int c = 0; c < nc && st == WLBM_OK; ++c) {
      l->rows[pc][k] = cand[c];
      st = run_steps(l, warm * k, nullptr, 0);
      if (!st && (he = hipEventRecord(e0, l->stream)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventRecord failed: %s", hipGetErrorString(he));
      for (int64_t left = launches; !st && left > 0; left -= per_call)
        st = run_steps(l, std::min<int64_t>(left, per_call) * k, nullptr, 0);
      float ms = -1.f;
      if (!st && (he = hipEventRecord(e1, l->stream)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventRecord failed: %s", hipGetErrorString(he));
      if (!st && (he = hipEventSynchronize(e1)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventSynchronize failed: %s", hipGetErrorString(he));
      if (!st && (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventElapsedTime failed: %s", hipGetErrorString(he));
      if (!st && (best[size_t(c)] < 0.f || ms < best[size_t(c)])) best[size_t(c)] = ms;
      if (!st) st = wlbm_load_state(l, d_state, bytes, step0);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  l->flux_window = flux_window;
  l->p.step_fusion = keep_fusion;
  if (st) {
    l->rows[pc][k] = keep_rows;
    return st;
  }
  int b = 0;
  for (int c = 1; c < nc; ++c)
    if (best[size_t(c)] < best[size_t(b)]) b = c;
  l->rows[pc][k] = cand[b];
  l->flux_valid = flux_valid;
  if (rows_out) *rows_out = cand[b];
  return WLBM_OK;
}

}  // extern "C"
