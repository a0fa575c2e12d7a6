// C-ABI of libwormlbm.so (declared in include/wormlbm.h): saved states,
// tapes, probe reads and the adjoint (reverse mode) of the worm-LBM step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <exception>
#include <vector>

#include "api_internal.hpp"

using namespace wlbm;

extern "C" {

wlbm_status wlbm_state_bytes(const wlbm_lattice* l, size_t* bytes) {
  if (!l) return fail(WLBM_EINVAL, "lattice is NULL");
  if (!bytes) return fail(WLBM_EINVAL, "bytes is NULL");
  *bytes = state_bytes_of(l->p);
  return WLBM_OK;
}

wlbm_status wlbm_step_tape(wlbm_lattice* l, int64_t nsteps, void* d_tape, size_t slot_bytes) {
  wlbm_status st = check_lat(l);
  if (!st) st = check_steps(l, nsteps);
  if (st) return st;
  if (nsteps == 0) return WLBM_OK;
  if (!d_tape) return fail(WLBM_EINVAL, "tape is NULL");
  if (reinterpret_cast<uintptr_t>(d_tape) % kAlign || slot_bytes % kAlign)
    return fail(WLBM_EINVAL, "tape and slot size must be 256-byte aligned");
  if (slot_bytes < state_bytes_of(l->p))
    return fail(WLBM_EINVAL, "slot of %zu bytes is smaller than a state (%zu bytes)", slot_bytes,
                state_bytes_of(l->p));
  return run_steps(l, nsteps, static_cast<char*>(d_tape), slot_bytes);
}

wlbm_status wlbm_save_state(wlbm_lattice* l, void* d_buf, size_t bytes) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!d_buf) return fail(WLBM_EINVAL, "state buffer is NULL");
  if (bytes < state_bytes_of(l->p))
    return fail(WLBM_EINVAL, "state buffer of %zu bytes is smaller than a state (%zu bytes)",
                bytes, state_bytes_of(l->p));
  const size_t pbytes = size_t(l->g.plane) * sizeof(float);
  char* b = static_cast<char*>(d_buf);
  HIP_TRY(hipMemcpyAsync(b, l->ptr(l->c.e[l->cur]), pbytes * l->p.q, hipMemcpyDeviceToDevice,
                         l->stream));
  HIP_TRY(hipMemcpyAsync(b + pbytes * l->p.q, l->ptr(l->c.E[l->cur]), pbytes,
                         hipMemcpyDeviceToDevice, l->stream));
  return WLBM_OK;
}

wlbm_status wlbm_load_state(wlbm_lattice* l, const void* d_buf, size_t bytes, int64_t step) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!d_buf) return fail(WLBM_EINVAL, "state buffer is NULL");
  if (bytes < state_bytes_of(l->p))
    return fail(WLBM_EINVAL, "state buffer of %zu bytes is smaller than a state (%zu bytes)",
                bytes, state_bytes_of(l->p));
  if (step < 0 || step > kMaxSteps) return fail(WLBM_EINVAL, "step must be in 0 .. 2^31 - 1");
  const size_t pbytes = size_t(l->g.plane) * sizeof(float);
  const char* b = static_cast<const char*>(d_buf);
  HIP_TRY(hipMemcpyAsync(l->ptr(l->c.e[l->cur]), b, pbytes * l->p.q, hipMemcpyDeviceToDevice,
                         l->stream));
  HIP_TRY(hipMemcpyAsync(l->ptr(l->c.E[l->cur]), b + pbytes * l->p.q, pbytes,
                         hipMemcpyDeviceToDevice, l->stream));
  try {
    l->book.state_at(step, l->tas);
  } catch (const std::exception& e) {
    return fail(WLBM_ENOMEM, "schedule restore failed: %s", e.what());
  }
  l->flux_valid = false;
  l->ghosts_full = false;
  return WLBM_OK;
}

wlbm_status wlbm_read_probes(wlbm_lattice* l, int32_t n, const int32_t* d_cells, float* d_T) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (n < 0) return fail(WLBM_EINVAL, "probe count must be >= 0");
  if (n > 0 && (!d_cells || !d_T)) return fail(WLBM_EINVAL, "probe arrays must not be NULL");
  HIP_TRY(launch_read_probes(l->g, l->ptr(l->c.E[l->cur]), d_cells, n, d_T, l->stream));
  return WLBM_OK;
}

wlbm_status wlbm_adjoint_bytes(const wlbm_lattice* l, size_t* bytes) {
  if (!l) return fail(WLBM_EINVAL, "lattice is NULL");
  if (!bytes) return fail(WLBM_EINVAL, "bytes is NULL");
  *bytes = adj_carve(l->p).total;
  return WLBM_OK;
}

wlbm_status wlbm_adjoint_begin(wlbm_lattice* l, void* d_ws, size_t bytes, int64_t step) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (l->p.y_edge == WLBM_EDGE_DIFFUSE)
    return fail(WLBM_EINVAL, "the adjoint covers periodic and blackbody edges only");
  if (l->nsrc) return fail(WLBM_EINVAL, "the adjoint does not cover internal sources");
  if (step < 0 || step > kMaxSteps) return fail(WLBM_EINVAL, "step must be in 0 .. 2^31 - 1");
  if (!d_ws) return fail(WLBM_EINVAL, "adjoint workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign)
    return fail(WLBM_EINVAL, "adjoint workspace must be 256-byte aligned");
  const AdjCarve ac = adj_carve(l->p);
  if (bytes < ac.total)
    return fail(WLBM_ENOMEM, "adjoint workspace too small: %zu bytes given, %zu needed", bytes,
                ac.total);
  HIP_TRY(hipMemsetAsync(d_ws, 0, ac.total, l->stream));
  l->aws = static_cast<char*>(d_ws);
  l->ac = ac;
  l->acur = 0;
  l->am = step;
  return WLBM_OK;
}

wlbm_status wlbm_adjoint_seed(wlbm_lattice* l, int32_t n, const int32_t* d_cells,
                              const float* d_dT) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (l->am < 0) return fail(WLBM_ESTATE, "no reverse pass: call wlbm_adjoint_begin first");
  if (n < 0) return fail(WLBM_EINVAL, "probe count must be >= 0");
  if (n == 0) return WLBM_OK;
  if (!d_cells || !d_dT) return fail(WLBM_EINVAL, "seed arrays must not be NULL");
  const int q = l->p.q;
  AdjSeedArgs a{};
  a.lam = l->aptr(l->ac.lam[l->acur]);
  a.H = l->aptr(l->ac.H[l->acur]);
  a.gB = reinterpret_cast<double*>(l->aws + l->ac.gB);
  a.cells = d_cells;
  a.vals = d_dT;
  a.flag = reinterpret_cast<int*>(l->aws + l->ac.flag);
  a.n = n;
  double wc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double wall_w = 0.0;
  for (int i = 0; i < q; ++i) wall_w += l->dirs.w[i];
  if (l->am >= 1) {
    // the partial sums of lam^am are classed by the moves of step am
    std::vector<int8_t> dx(q), dy(q);
    std::vector<uint8_t> hop(q);
    try {
      l->book.rows(l->am, 1, dx.data(), dy.data(), hop.data());
    } catch (const std::exception& e) {
      return fail(WLBM_ENOMEM, "schedule restore failed: %s", e.what());
    }
    for (int i = 0; i < q; ++i) wc[host_move_class(dx[i], dy[i])] += l->dirs.w[i];
  }
  for (int c = 0; c < 8; ++c) a.wcls[c] = float(wc[c]);
  a.wall_w = wall_w;
  a.nx = l->g.nx;
  a.ny = l->g.ny;
  a.q = q;
  a.pitch = l->g.pitch;
  a.plane = l->g.plane;
  a.x_edge = l->g.x_edge;
  a.y_edge = l->g.y_edge;
  HIP_TRY(launch_adj_seed(a, l->stream));
  return WLBM_OK;
}

wlbm_status wlbm_adjoint_steps(wlbm_lattice* l, int64_t n, const void* d_states,
                               size_t slot_bytes) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (l->am < 0) return fail(WLBM_ESTATE, "no reverse pass: call wlbm_adjoint_begin first");
  if (n < 0 || n > l->am)
    return fail(WLBM_EINVAL, "n must be in 0 .. %lld (the current adjoint step)",
                (long long)l->am);
  if (n == 0) return WLBM_OK;
  if (!d_states) return fail(WLBM_EINVAL, "states pointer is NULL");
  if (reinterpret_cast<uintptr_t>(d_states) % kAlign || slot_bytes % kAlign)
    return fail(WLBM_EINVAL, "states and slot size must be 256-byte aligned");
  if (slot_bytes < state_bytes_of(l->p))
    return fail(WLBM_EINVAL, "slot of %zu bytes is smaller than a state (%zu bytes)", slot_bytes,
                state_bytes_of(l->p));
  const int q = l->p.q;
  const char* states = static_cast<const char*>(d_states);
  const int64_t m0 = l->am;
  const int64_t base = m0 - n;  // step of the state in slot 0
  AdjArgs a{};
  a.Wf = l->ptr(l->c.Wf);
  a.gW = reinterpret_cast<double*>(l->aws + l->ac.gW);
  a.gB = reinterpret_cast<double*>(l->aws + l->ac.gB);
  a.wtab = l->ptr(l->c.wtab);
  a.W = l->W;
  a.nx = l->g.nx;
  a.ny = l->g.ny;
  a.q = q;
  a.pitch = l->g.pitch;
  a.plane = l->g.plane;
  a.x_edge = l->g.x_edge;
  a.y_edge = l->g.y_edge;
  a.tiles_x = tiles_x_for(l->g.nx);
  a.ntiles = a.tiles_x * tiles_y_for(l->g.ny, l->split);
  std::vector<int8_t> dx, dy;
  std::vector<uint8_t> hop;
  const int64_t per = l->chunk - 1;  // reverse steps per upload: rows m-cnt .. m
  int64_t done = 0;
  while (done < n) {
    const int64_t cnt = std::min<int64_t>(per, n - done);
    const int64_t m_hi = m0 - done;
    const int64_t first = std::max<int64_t>(1, m_hi - cnt);
    const int64_t nrows = m_hi - first + 1;
    const int slot = int(l->chunk_counter & 1);
    if (l->ev_pending[slot]) {
      hipError_t e = hipEventSynchronize(l->ev[slot]);
      if (e != hipSuccess) {
        l->broken = true;
        return fail(WLBM_EHIP, "hipEventSynchronize failed: %s", hipGetErrorString(e));
      }
      l->ev_pending[slot] = false;
    }
    dx.resize(size_t(nrows) * q);
    dy.resize(size_t(nrows) * q);
    hop.resize(size_t(nrows) * q);
    try {
      l->book.rows(first, nrows, dx.data(), dy.data(), hop.data());
    } catch (const std::exception& e) {
      return fail(WLBM_ENOMEM, "schedule restore failed: %s", e.what());
    }
    uint8_t* rows = l->pinned[slot];
    for (size_t k = 0; k < size_t(nrows) * q; ++k) rows[k] = pack_code(dx[k], dy[k], hop[k]);
    uint8_t* dev_rows =
        reinterpret_cast<uint8_t*>(l->aws + l->ac.sched) + size_t(slot) * l->chunk * q;
    hipError_t e = hipMemcpyAsync(dev_rows, rows, size_t(nrows) * q, hipMemcpyHostToDevice,
                                  l->stream);
    if (e == hipSuccess) e = hipEventRecord(l->ev[slot], l->stream);
    if (e != hipSuccess) {
      l->broken = true;
      return fail(WLBM_EHIP, "schedule upload failed: %s", hipGetErrorString(e));
    }
    l->ev_pending[slot] = true;
    ++l->chunk_counter;
    for (int64_t j = 0; j < cnt; ++j) {
      const int64_t m = m_hi - j;
      const uint8_t* row_m = dev_rows + size_t(m - first) * q;
      const uint8_t* row_next = m - 1 >= 1 ? dev_rows + size_t(m - 1 - first) * q : row_m;
      const char* sp = states + size_t(m - 1 - base) * slot_bytes;
      a.codes = reinterpret_cast<const uint32_t*>(row_m);
      a.codes_next = reinterpret_cast<const uint32_t*>(row_next);
      a.e_prev = reinterpret_cast<const float*>(sp);
      a.E_prev = reinterpret_cast<const float*>(sp) + size_t(q) * l->g.plane;
      a.lam_in = l->aptr(l->ac.lam[l->acur]);
      a.lam_out = l->aptr(l->ac.lam[1 - l->acur]);
      a.H_in = l->aptr(l->ac.H[l->acur]);
      a.H_out = l->aptr(l->ac.H[1 - l->acur]);
      e = launch_adjoint(a, l->split, l->per_cell, l->stream);
      if (e != hipSuccess) {
        l->broken = true;
        return fail(WLBM_EHIP, "adjoint kernel launch failed: %s", hipGetErrorString(e));
      }
      l->acur = 1 - l->acur;
    }
    done += cnt;
  }
  l->am = m0 - n;
  return WLBM_OK;
}

wlbm_status wlbm_adjoint_read(wlbm_lattice* l, float* d_g_mfp, float* d_g_T0, double* g_walls) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (l->am < 0) return fail(WLBM_ESTATE, "no reverse pass: call wlbm_adjoint_begin first");
  const double f = l->p.emulate_3d ? 1.5 : 1.0;
  const double W = std::isinf(l->p.mfp_cells) ? 0.0 : 1.0 / l->p.mfp_cells;
  if (d_g_mfp)
    HIP_TRY(launch_adj_grad_mfp(l->g, reinterpret_cast<const double*>(l->aws + l->ac.gW),
                                l->per_cell ? l->ptr(l->c.Wraw) : nullptr, W,
                                l->dirs.lambda_corr, f, l->p.mfp_correction, d_g_mfp,
                                l->stream));
  if (d_g_T0)
    HIP_TRY(launch_adj_grad_t0(l->g, l->aptr(l->ac.lam[l->acur]), l->ptr(l->c.wtab), d_g_T0,
                               l->stream));
  double* dev_walls = reinterpret_cast<double*>(l->aws + l->ac.walls);
  HIP_TRY(launch_adj_walls(l->g, reinterpret_cast<const double*>(l->aws + l->ac.gB), dev_walls,
                           l->stream));
  double hw[4];
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(hw, dev_walls, sizeof(hw), hipMemcpyDeviceToHost, l->stream));
  HIP_TRY(hipMemcpyAsync(&flag, l->aws + l->ac.flag, sizeof(int), hipMemcpyDeviceToHost,
                         l->stream));
  HIP_TRY(hipStreamSynchronize(l->stream));
  if (flag) return fail(WLBM_EINVAL, "a seed cell was outside the lattice (it was skipped)");
  if (g_walls)
    for (int k = 0; k < 4; ++k) g_walls[k] = hw[k];
  return WLBM_OK;
}

int64_t wlbm_adjoint_step_index(const wlbm_lattice* l) { return l ? l->am : -1; }

}  // extern "C"
