// C-ABI of libwormlbm.so (declared in include/wormlbm.h): batches of
// lattices advanced together, one kernel launch per time step for all of
// them (the in-plane film sweeps of Sec. 3.5 run many lattices of different
// thickness and Knudsen number at once).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "api_internal.hpp"

using namespace wlbm;

// A set of lattices advanced together, one launch per step.
// Lattices of a batch with one direction set (q, set, grid speeds) share a
// schedule: one ring of 2 chunks of rows in the batch workspace, and its
// rows of inward-weight sums.
struct BatchGroup {
  wlbm_lattice* lead = nullptr;   // the first member; its directions define the group
  size_t sched = 0, ins = 0;      // workspace offsets of the group's rings
  size_t stage = 0;               // offset of its rows in a pinned staging buffer
};

struct wlbm_batch {
  std::vector<wlbm_lattice*> lats;
  std::vector<int> group;         // group of each lattice
  std::vector<BatchGroup> groups;
  int qmax = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t off_args = 0, off_first = 0, off_rc = 0, off_ri = 0;
  int chunk = 0;
  uint8_t* pinned[2] = {nullptr, nullptr};     // staging of the schedule rows of every group
  float* pinned_ins[2] = {nullptr, nullptr};   // staging of the per-step wall sums
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_pending[2] = {false, false};
  int64_t chunk_counter = 0;
  char* table = nullptr;        // pinned staging of the argument table
  hipEvent_t table_ev = nullptr;
  bool table_pending = false;
  // With graphs on (wlbm_batch_set_graphs), full schedule chunks run as one
  // launch of a captured HIP graph per schedule-ring slot; key: what the
  // graph was captured for.  Off by default: the host enqueues per-step
  // launches faster than the GPU runs them, so graphs measured no gain.
  bool use_graphs = false;
  hipStream_t cap = nullptr;    // private stream the graphs are captured on
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int64_t gkey[2] = {-1, -1};
};

namespace {

struct BatchCarve {
  size_t args, first, rc, ri, total;
  std::vector<size_t> sched, ins;   // per group
};

bool same_directions(const wlbm_lattice* a, const wlbm_lattice* b) {
  return a->p.q == b->p.q && a->p.dirs == b->p.dirs && a->dirs.vgrid == b->dirs.vgrid;
}

// Group index of each lattice (first-seen order) and the lead of each group.
void form_groups(wlbm_lattice* const* lats, int n, std::vector<int>& group,
                 std::vector<wlbm_lattice*>& leads) {
  group.assign(size_t(n), -1);
  leads.clear();
  for (int j = 0; j < n; ++j) {
    for (size_t g = 0; g < leads.size() && group[j] < 0; ++g)
      if (same_directions(leads[g], lats[j])) group[j] = int(g);
    if (group[j] < 0) {
      group[j] = int(leads.size());
      leads.push_back(lats[j]);
    }
  }
}

BatchCarve batch_carve(int n, const std::vector<wlbm_lattice*>& leads, int chunk) {
  BatchCarve c{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  c.args = take(size_t(2) * n * sizeof(StepArgs));
  c.first = take(size_t(n + 1) * sizeof(int));
  c.rc = take(size_t(n) * sizeof(void*));   // per lattice: its group's schedule ring
  c.ri = take(size_t(n) * sizeof(void*));   // and ring of inward-weight sums
  for (const wlbm_lattice* l : leads) {
    c.sched.push_back(take(size_t(2) * chunk * l->p.q));
    c.ins.push_back(take(size_t(2) * chunk * 4 * sizeof(float)));
  }
  c.total = off;
  return c;
}

wlbm_status check_members(wlbm_lattice* const* lats, int32_t n) {
  if (!lats) return fail(WLBM_EINVAL, "lattice list is NULL");
  if (n < 1 || n > 4096) return fail(WLBM_EINVAL, "a batch holds 1 .. 4096 lattices");
  for (int j = 0; j < n; ++j) {
    wlbm_status st = check_lat(lats[j]);
    if (st) return st;
    const wlbm_lattice* a = lats[0];
    const wlbm_lattice* b = lats[j];
    if (b->tas.n != a->tas.n)
      return fail(WLBM_EINVAL, "lattice %d: all lattices of a batch must be at the same step", j);
    if (b->split != a->split || b->per_cell != a->per_cell || b->chunk != a->chunk)
      return fail(WLBM_EINVAL,
                  "lattice %d: direction split, per-cell field use and schedule chunk must agree", j);
    if (b->flux_window != a->flux_window)
      return fail(WLBM_EINVAL, "lattice %d: flux windows must agree", j);
    for (int k = 0; k < j; ++k)
      if (lats[k] == b) return fail(WLBM_EINVAL, "lattice %d appears twice in the batch", j);
  }
  return WLBM_OK;
}

}  // namespace

extern "C" {

wlbm_status wlbm_batch_bytes(wlbm_lattice* const* lats, int32_t n, size_t* bytes) {
  wlbm_status st = check_members(lats, n);
  if (st) return st;
  if (!bytes) return fail(WLBM_EINVAL, "bytes is NULL");
  std::vector<int> group;
  std::vector<wlbm_lattice*> leads;
  form_groups(lats, n, group, leads);
  *bytes = batch_carve(n, leads, lats[0]->chunk).total;
  return WLBM_OK;
}

wlbm_status wlbm_batch_create(wlbm_lattice* const* lats, int32_t n, void* d_ws, size_t bytes,
                              void* stream, wlbm_batch** out) {
  if (!out) return fail(WLBM_EINVAL, "out is NULL");
  *out = nullptr;
  wlbm_status st = check_members(lats, n);
  if (st) return st;
  std::vector<int> group;
  std::vector<wlbm_lattice*> leads;
  form_groups(lats, n, group, leads);
  const BatchCarve bc = batch_carve(n, leads, lats[0]->chunk);
  if (!d_ws) return fail(WLBM_EINVAL, "batch workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign)
    return fail(WLBM_EINVAL, "batch workspace must be 256-byte aligned");
  if (bytes < bc.total)
    return fail(WLBM_ENOMEM, "batch workspace too small: %zu bytes given, %zu needed", bytes,
                bc.total);
  wlbm_batch* b = new (std::nothrow) wlbm_batch();
  if (!b) return fail(WLBM_ENOMEM, "host allocation failed");
  b->lats.assign(lats, lats + n);
  b->group = group;
  b->stream = static_cast<hipStream_t>(stream);
  b->ws = static_cast<char*>(d_ws);
  b->off_args = bc.args;
  b->off_first = bc.first;
  b->off_rc = bc.rc;
  b->off_ri = bc.ri;
  b->chunk = lats[0]->chunk;
  size_t stage = 0;
  for (size_t g = 0; g < leads.size(); ++g) {
    BatchGroup bg;
    bg.lead = leads[g];
    bg.sched = bc.sched[g];
    bg.ins = bc.ins[g];
    bg.stage = stage;
    stage += size_t(b->chunk) * leads[g]->p.q;
    b->groups.push_back(bg);
    b->qmax = std::max(b->qmax, leads[g]->p.q);
  }
  const size_t ngroups = leads.size();
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipHostMalloc(reinterpret_cast<void**>(&b->pinned[k]), stage, hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&b->pinned_ins[k]),
                        ngroups * b->chunk * 4 * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&b->table), bc.ri + size_t(n) * sizeof(void*),
                      hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->table_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)wlbm_batch_destroy(b);
    return fail(WLBM_ENOMEM, "batch set-up failed: %s", hipGetErrorString(e));
  }
  *out = b;
  return WLBM_OK;
}

wlbm_status wlbm_batch_step(wlbm_batch* b, int64_t nsteps) {
  if (!b) return fail(WLBM_EINVAL, "batch is NULL");
  const int n = int(b->lats.size());
  wlbm_status st = check_members(b->lats.data(), n);
  if (st) return st;
  for (int j = 0; j < n; ++j)
    if (!same_directions(b->groups[size_t(b->group[j])].lead, b->lats[j]))
      return fail(WLBM_EINVAL,
                  "lattice %d: its directions or grid speeds changed since the batch was "
                  "created; create the batch again", j);
  wlbm_lattice* l0 = b->lats[0];
  st = check_steps(l0, nsteps);
  if (st) return st;
  if (nsteps == 0) return WLBM_OK;
  const int ngroups = int(b->groups.size());
  // argument table: lattice j, buffer parity p (p = 1 after an odd number of
  // steps of this call); wall temperatures and fields as they are now.  The
  // pinned staging copy of the previous call must have been consumed.
  if (b->table_pending) {
    hipError_t e = hipEventSynchronize(b->table_ev);
    if (e != hipSuccess) return fail(WLBM_EHIP, "hipEventSynchronize failed: %s",
                                     hipGetErrorString(e));
    b->table_pending = false;
  }
  StepArgs* table = reinterpret_cast<StepArgs*>(b->table);
  int* first = reinterpret_cast<int*>(b->table + b->off_first);
  const void** ring_codes = reinterpret_cast<const void**>(b->table + b->off_rc);
  const void** ring_ins = reinterpret_cast<const void**>(b->table + b->off_ri);
  first[0] = 0;
  for (int j = 0; j < n; ++j) {
    wlbm_lattice* l = b->lats[j];
    const BatchGroup& bg = b->groups[size_t(b->group[j])];
    ring_codes[j] = b->ws + bg.sched;
    ring_ins[j] = b->ws + bg.ins;
    for (int par = 0; par < 2; ++par) {
      StepArgs& a = table[size_t(2) * j + par];
      const int in = l->cur ^ par;
      a.e_in = l->ptr(l->c.e[in]);
      a.e_out = l->ptr(l->c.e[1 - in]);
      a.E_in = l->ptr(l->c.E[in]);
      a.E_out = l->ptr(l->c.E[1 - in]);
      a.Wf = l->ptr(l->c.Wf);
      a.qsx = l->ptr(l->c.qsx);
      a.qsy = l->ptr(l->c.qsy);
      a.wtab = l->ptr(l->c.wtab);
      a.sxtab = l->ptr(l->c.sxtab);
      a.sytab = l->ptr(l->c.sytab);
      a.mtab = reinterpret_cast<const int*>(l->ws + l->c.mtab);
      a.W = l->W;
      a.spec = float(l->p.y_specularity);
      a.t_x_lo = l->walls.x_lo;
      a.t_x_hi = l->walls.x_hi;
      a.t_y_lo = l->walls.y_lo;
      a.t_y_hi = l->walls.y_hi;
      a.nx = l->g.nx;
      a.ny = l->g.ny;
      a.q = l->p.q;
      a.pitch = l->g.pitch;
      a.plane = l->g.plane;
      a.x_edge = l->g.x_edge;
      a.y_edge = l->g.y_edge;
      a.tiles_x = tiles_x_for(l->g.nx);
      a.ntiles = a.tiles_x * tiles_y_for(l->g.ny, l->split);
    }
    first[size_t(j) + 1] = first[size_t(j)] + table[size_t(2) * j].ntiles;
  }
  // the table, first[] and the ring pointers sit at the same offsets in the
  // staging buffer and in the workspace, so one copy moves them all
  HIP_TRY(hipMemcpyAsync(b->ws, b->table, b->off_ri + size_t(n) * sizeof(void*),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipEventRecord(b->table_ev, b->stream));
  b->table_pending = true;
  BatchStepArgs ba{};
  ba.lats = reinterpret_cast<const StepArgs*>(b->ws + b->off_args);
  ba.first = reinterpret_cast<const int*>(b->ws + b->off_first);
  ba.n = n;
  ba.nblocks = first[size_t(n)];
  ba.q = b->qmax;
  ba.ring_codes = reinterpret_cast<const uint32_t* const*>(b->ws + b->off_rc);
  ba.ring_ins = reinterpret_cast<const float* const*>(b->ws + b->off_ri);
  const bool grouped = ngroups > 1;
  // group 0's row and sums of step j in ring slot `slot`
  const BatchGroup& g0 = b->groups[0];
  auto rows0 = [&](int slot_, int j) {
    return reinterpret_cast<const uint32_t*>(b->ws + g0.sched +
                                             (size_t(slot_) * b->chunk + j) * g0.lead->p.q);
  };
  auto ins0 = [&](int slot_, int j) {
    return reinterpret_cast<const float*>(b->ws + g0.ins) + (size_t(slot_) * b->chunk + j) * 4;
  };
  const int64_t flux_from = l0->flux_window > 0 ? nsteps - l0->flux_window : nsteps;
  bool has_sources = false;
  for (wlbm_lattice* l : b->lats) has_sources = has_sources || l->nsrc > 0;
  // each group advances its own schedule state
  std::vector<TasState> tas;
  for (const BatchGroup& bg : b->groups) tas.push_back(bg.lead->tas);
  std::vector<int8_t> dx(size_t(b->qmax)), dy(size_t(b->qmax));
  std::vector<uint8_t> hop(size_t(b->qmax));
  int64_t done = 0;
  while (done < nsteps) {
    const int cnt = int(std::min<int64_t>(b->chunk, nsteps - done));
    const int slot = int(b->chunk_counter & 1);
    if (b->ev_pending[slot]) {
      hipError_t e = hipEventSynchronize(b->ev[slot]);
      if (e != hipSuccess) return fail(WLBM_EHIP, "hipEventSynchronize failed: %s",
                                       hipGetErrorString(e));
      b->ev_pending[slot] = false;
    }
    // Build the schedule rows of this chunk (Sec. 2.3, Sec. 2.5) and the
    // per-step sums of inward weights used by diffuse walls, for each group,
    // and upload them into the group's ring slot.
    hipError_t e = hipSuccess;
    for (int g = 0; g < ngroups && e == hipSuccess; ++g) {
      const BatchGroup& bg = b->groups[size_t(g)];
      const wlbm_lattice* lead = bg.lead;
      const int q = lead->p.q;
      uint8_t* rows = b->pinned[slot] + bg.stage;
      float* insums = b->pinned_ins[slot] + size_t(g) * b->chunk * 4;
      for (int j = 0; j < cnt; ++j) {
        tas_advance(lead->dirs, tas[size_t(g)], dx.data(), dy.data(), hop.data());
        for (int m = 0; m < n; ++m)
          if (b->group[m] == g) b->lats[m]->book.note(tas[size_t(g)]);
        double lo_h = 0, lo_a = 0, hi_h = 0, hi_a = 0;
        for (int i = 0; i < q; ++i) {
          rows[size_t(j) * q + i] = pack_code(dx[i], dy[i], hop[i]);
          if (dy[i] == 1) {
            lo_a += lead->dirs.w[i];
            if (hop[i]) lo_h += lead->dirs.w[i];
          } else if (dy[i] == -1) {
            hi_a += lead->dirs.w[i];
            if (hop[i]) hi_h += lead->dirs.w[i];
          }
        }
        insums[4 * j] = float(lo_h);
        insums[4 * j + 1] = float(lo_a);
        insums[4 * j + 2] = float(hi_h);
        insums[4 * j + 3] = float(hi_a);
      }
      uint8_t* dev_rows =
          reinterpret_cast<uint8_t*>(b->ws + bg.sched) + size_t(slot) * b->chunk * q;
      float* dev_ins = reinterpret_cast<float*>(b->ws + bg.ins) + size_t(slot) * b->chunk * 4;
      e = hipMemcpyAsync(dev_rows, rows, size_t(cnt) * q, hipMemcpyHostToDevice, b->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(dev_ins, insums, size_t(cnt) * 4 * sizeof(float),
                           hipMemcpyHostToDevice, b->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(b->ev[slot], b->stream);
    if (e != hipSuccess) return fail(WLBM_EHIP, "schedule upload failed: %s", hipGetErrorString(e));
    b->ev_pending[slot] = true;
    ++b->chunk_counter;
    // A whole chunk with no flux-window step and no sources, starting on an
    // even step of this call, is one launch of the slot's captured graph:
    // its kernels read the schedule rows and sums just uploaded, and the
    // argument table of this call.
    const bool graph = b->use_graphs && cnt == b->chunk && b->chunk % 2 == 0 &&
                       done % 2 == 0 && done + cnt <= flux_from && !has_sources;
    if (graph) {
      const int64_t key = (int64_t(ba.nblocks) << 8) | (int64_t(l0->split) << 1) |
                          int64_t(l0->per_cell ? 1 : 0);
      if (!b->gexec[slot] || b->gkey[slot] != key) {
        if (b->gexec[slot]) {
          // the old graph may still be running: let it finish first
          e = hipStreamSynchronize(b->stream);
          if (e == hipSuccess) e = hipGraphExecDestroy(b->gexec[slot]);
          b->gexec[slot] = nullptr;
          b->gkey[slot] = -1;
        }
        hipGraph_t gr = nullptr;
        if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
          hipError_t el = hipSuccess;
          for (int j = 0; j < cnt && el == hipSuccess; ++j) {
            BatchStepArgs bj = ba;
            bj.row = slot * b->chunk + j;
            bj.codes = rows0(slot, j);
            bj.ins = ins0(slot, j);
            bj.parity = j & 1;
            bj.q_first = 0;
            el = launch_step_batch(bj, l0->split, l0->per_cell, false, grouped, b->cap);
          }
          e = hipStreamEndCapture(b->cap, &gr);
          if (el != hipSuccess) e = el;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec[slot], gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
        if (e != hipSuccess) {
          for (wlbm_lattice* l : b->lats) l->broken = true;
          return fail(WLBM_EHIP, "batch graph capture failed: %s", hipGetErrorString(e));
        }
        b->gkey[slot] = key;
      }
      e = hipGraphLaunch(b->gexec[slot], b->stream);
      if (e != hipSuccess) {
        for (wlbm_lattice* l : b->lats) l->broken = true;
        return fail(WLBM_EHIP, "batch graph launch failed: %s", hipGetErrorString(e));
      }
      done += cnt;
      continue;
    }
    for (int j = 0; j < cnt; ++j) {
      const int64_t k = done + j;
      const bool flux = k >= flux_from;
      ba.row = slot * b->chunk + j;
      ba.codes = rows0(slot, j);
      ba.ins = ins0(slot, j);
      ba.parity = int(k & 1);
      ba.q_first = (flux && k == flux_from) ? 1 : 0;
      e = launch_step_batch(ba, l0->split, l0->per_cell, flux, grouped, b->stream);
      for (int jl = 0; jl < n && e == hipSuccess; ++jl) {
        wlbm_lattice* l = b->lats[jl];
        if (!l->nsrc) continue;
        const int out = 1 - (l->cur ^ int(k & 1));
        e = launch_apply_sources(l->g, l->ptr(l->c.e[out]), l->ptr(l->c.E[out]), l->src_cells,
                                 l->src_vals, l->nsrc, b->stream);
      }
      if (e != hipSuccess) {
        for (wlbm_lattice* l : b->lats) l->broken = true;
        return fail(WLBM_EHIP, "batch step launch failed: %s", hipGetErrorString(e));
      }
    }
    done += cnt;
  }
  for (int j = 0; j < n; ++j) {
    wlbm_lattice* l = b->lats[j];
    l->tas = tas[size_t(b->group[j])];
    l->cur ^= int(nsteps & 1);
    l->flux_valid = l->flux_window > 0 && nsteps >= l->flux_window;
    l->ghosts_full = false;
  }
  return WLBM_OK;
}

wlbm_status wlbm_batch_set_graphs(wlbm_batch* b, int32_t on) {
  if (!b) return fail(WLBM_EINVAL, "batch is NULL");
  if (on != 0 && on != 1) return fail(WLBM_EINVAL, "on must be 0 or 1");
  b->use_graphs = on != 0;
  return WLBM_OK;
}

wlbm_status wlbm_batch_destroy(wlbm_batch* b) {
  if (!b) return WLBM_OK;
  hipError_t e = hipStreamSynchronize(b->stream);
  for (int k = 0; k < 2; ++k) {
    if (b->gexec[k]) (void)hipGraphExecDestroy(b->gexec[k]);
    if (b->pinned[k]) (void)hipHostFree(b->pinned[k]);
    if (b->pinned_ins[k]) (void)hipHostFree(b->pinned_ins[k]);
    if (b->ev[k]) (void)hipEventDestroy(b->ev[k]);
  }
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->table) (void)hipHostFree(b->table);
  if (b->table_ev) (void)hipEventDestroy(b->table_ev);
  delete b;
  if (e != hipSuccess) return fail(WLBM_EHIP, "stream sync at destroy: %s", hipGetErrorString(e));
  return WLBM_OK;
}


}  // extern "C"
