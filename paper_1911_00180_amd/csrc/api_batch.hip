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

// Lattices of one group with the same padded geometry (row pitch and plane
// size) share the pull offsets of the multi-step kernel.
struct BatchGeo {
  int group = 0;
  int pitch = 0;
  long long plane = 0;
  size_t pulls = 0;               // workspace offset of its ring of pull offsets
  size_t stage = 0;               // offset of its rows in a pinned staging buffer (words)
};

struct wlbm_batch {
  std::vector<wlbm_lattice*> lats;
  std::vector<int> group;         // group of each lattice
  std::vector<BatchGroup> groups;
  std::vector<int> geo;           // geometry of each lattice
  std::vector<BatchGeo> geos;
  std::vector<size_t> sels;       // per group: workspace offset of its selection-offset ring
  std::vector<size_t> sels_stage; // per group: its rows in the pinned staging (words)
  int qmax = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t off_args = 0, off_first = 0, off_rc = 0, off_ri = 0;
  // multi-step launches: argument table, prefix of block counts and, per
  // lattice, its rings (selection offsets, pull offsets, codes, wall sums)
  size_t off_fargs = 0, off_ffirst = 0, off_fsel = 0, off_fpull = 0, off_fcode = 0,
         off_fins = 0, table_bytes = 0;
  int chunk = 0;
  uint8_t* pinned[2] = {nullptr, nullptr};     // staging of the schedule rows of every group
  float* pinned_ins[2] = {nullptr, nullptr};   // staging of the per-step wall sums
  uint32_t* pinned_sels[2] = {nullptr, nullptr};    // staging of the selection offsets
  uint32_t* pinned_pulls[2] = {nullptr, nullptr};   // staging of the pull offsets
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
  size_t args, first, rc, ri, fargs, ffirst, fsel, fpull, fcode, fins, total;
  std::vector<size_t> sched, ins, sels;   // per group
  std::vector<size_t> pulls;              // per geometry
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

// Geometry index of each lattice: lattices of one group with the same row
// pitch and plane size (first-seen order).
void form_geos(wlbm_lattice* const* lats, int n, const std::vector<int>& group,
               std::vector<int>& geo, std::vector<BatchGeo>& geos) {
  geo.assign(size_t(n), -1);
  geos.clear();
  for (int j = 0; j < n; ++j) {
    for (size_t k = 0; k < geos.size() && geo[j] < 0; ++k)
      if (geos[k].group == group[j] && geos[k].pitch == lats[j]->g.pitch &&
          geos[k].plane == lats[j]->g.plane)
        geo[j] = int(k);
    if (geo[j] < 0) {
      geo[j] = int(geos.size());
      BatchGeo g;
      g.group = group[j];
      g.pitch = lats[j]->g.pitch;
      g.plane = lats[j]->g.plane;
      geos.push_back(g);
    }
  }
}

// The argument tables come first and in one block (one upload per call);
// the rings follow.
BatchCarve batch_carve(int n, const std::vector<wlbm_lattice*>& leads,
                       const std::vector<BatchGeo>& geos, int chunk) {
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
  c.fargs = take(size_t(2) * n * sizeof(FusedArgs));
  c.ffirst = take(size_t(n + 1) * sizeof(int));
  c.fsel = take(size_t(n) * sizeof(void*));
  c.fpull = take(size_t(n) * sizeof(void*));
  c.fcode = take(size_t(n) * sizeof(void*));
  c.fins = take(size_t(n) * sizeof(void*));
  for (const wlbm_lattice* l : leads) {
    c.sched.push_back(take(size_t(2) * chunk * l->p.q));
    c.ins.push_back(take(size_t(2) * chunk * 4 * sizeof(float)));
    c.sels.push_back(take(size_t(2) * chunk * l->p.q * sizeof(uint32_t)));
  }
  for (const BatchGeo& g : geos)
    c.pulls.push_back(take(size_t(2) * chunk * leads[size_t(g.group)]->p.q * sizeof(uint32_t)));
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

// Steps per launch of the batch's multi-step launches: the fewest any member
// allows, when every member takes the multi-step kernels and all have one q
// (the kernel's shape); 0 if the batch runs one step per launch.
int batch_fused_k(const wlbm_batch* b) {
  int k = 4;
  for (const wlbm_lattice* l : b->lats) {
    if (!lattice_fuses(l) || l->p.q != b->qmax) return 0;
    k = std::min(k, fused_k_max(l));
  }
  return k >= 2 ? k : 0;
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
  std::vector<int> geo;
  std::vector<BatchGeo> geos;
  form_geos(lats, n, group, geo, geos);
  *bytes = batch_carve(n, leads, geos, lats[0]->chunk).total;
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
  std::vector<int> geo;
  std::vector<BatchGeo> geos;
  form_geos(lats, n, group, geo, geos);
  const BatchCarve bc = batch_carve(n, leads, geos, lats[0]->chunk);
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
  b->off_fargs = bc.fargs;
  b->off_ffirst = bc.ffirst;
  b->off_fsel = bc.fsel;
  b->off_fpull = bc.fpull;
  b->off_fcode = bc.fcode;
  b->off_fins = bc.fins;
  b->table_bytes = bc.fins + size_t(n) * sizeof(void*);
  b->chunk = lats[0]->chunk;
  size_t stage = 0, stage_sels = 0;
  for (size_t g = 0; g < leads.size(); ++g) {
    BatchGroup bg;
    bg.lead = leads[g];
    bg.sched = bc.sched[g];
    bg.ins = bc.ins[g];
    bg.stage = stage;
    stage += size_t(b->chunk) * leads[g]->p.q;
    b->groups.push_back(bg);
    b->sels.push_back(bc.sels[g]);
    b->sels_stage.push_back(stage_sels);
    stage_sels += size_t(b->chunk) * leads[g]->p.q;
    b->qmax = std::max(b->qmax, leads[g]->p.q);
  }
  b->geo = geo;
  b->geos = geos;
  size_t stage_pulls = 0;
  for (size_t k = 0; k < geos.size(); ++k) {
    b->geos[k].pulls = bc.pulls[k];
    b->geos[k].stage = stage_pulls;
    stage_pulls += size_t(b->chunk) * leads[size_t(geos[k].group)]->p.q;
  }
  const size_t ngroups = leads.size();
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipHostMalloc(reinterpret_cast<void**>(&b->pinned[k]), stage, hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&b->pinned_ins[k]),
                        ngroups * b->chunk * 4 * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&b->pinned_sels[k]),
                        stage_sels * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&b->pinned_pulls[k]),
                        stage_pulls * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&b->table), b->table_bytes, hipHostMallocDefault);
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
  // Several steps per launch when every lattice takes the multi-step kernels
  // and all have one q (the kernel's shape): k_max steps per launch, the
  // fewest any lattice allows; the steps left over at chunk ends run one per
  // launch.
  const int k_max = batch_fused_k(b);
  const bool fuse = k_max >= 2;
  // argument tables: lattice j, buffer parity p (p = 1 after an odd number of
  // launches of this call); wall temperatures and fields as they are now.
  // The pinned staging copy of the previous call must have been consumed.
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
  FusedArgs* ftable = reinterpret_cast<FusedArgs*>(b->table + b->off_fargs);
  int* ffirst = reinterpret_cast<int*>(b->table + b->off_ffirst);
  const void** fsel = reinterpret_cast<const void**>(b->table + b->off_fsel);
  const void** fpull = reinterpret_cast<const void**>(b->table + b->off_fpull);
  const void** fcode = reinterpret_cast<const void**>(b->table + b->off_fcode);
  const void** fins = reinterpret_cast<const void**>(b->table + b->off_fins);
  first[0] = 0;
  ffirst[0] = 0;
  for (int j = 0; j < n; ++j) {
    wlbm_lattice* l = b->lats[j];
    const BatchGroup& bg = b->groups[size_t(b->group[j])];
    ring_codes[j] = b->ws + bg.sched;
    ring_ins[j] = b->ws + bg.ins;
    fsel[j] = b->ws + b->sels[size_t(b->group[j])];
    fpull[j] = b->ws + b->geos[size_t(b->geo[j])].pulls;
    fcode[j] = b->ws + bg.sched;
    fins[j] = b->ws + bg.ins;
    const int rows = fuse ? block_rows_for(l, k_max) : 1;
    for (int par = 0; par < 2; ++par) {
      StepArgs& a = table[size_t(2) * j + par];
      const int in = l->cur ^ par;
      a.e_in = l->ptr(l->c.e[in]);
      a.e_out = l->ptr(l->c.e[1 - in]);
      a.E_in = l->ptr(l->c.E[in]);
      a.E_out = l->ptr(l->c.E[1 - in]);
      a.Wf = l->ptr(l->c.Wf);
      a.qsx = l->dptr(l->c.qsx);
      a.qsy = l->dptr(l->c.qsy);
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
      FusedArgs& f = ftable[size_t(2) * j + par];
      f = FusedArgs{};
      f.e_in = a.e_in;
      f.e_out = a.e_out;
      f.E_in = a.E_in;
      f.E_out = a.E_out;
      f.Wf = a.Wf;
      f.wtab = a.wtab;
      f.W = a.W;
      f.nx = a.nx;
      f.ny = a.ny;
      f.q = a.q;
      f.pitch = a.pitch;
      f.plane = a.plane;
      f.rows = rows;
      f.strips_x = fused_strips_x(a.nx, std::max(k_max, 2));
      f.strips_y = (a.ny + rows - 1) / rows;
      f.x_edge = a.x_edge;
      f.y_edge = a.y_edge;
      f.t_x_lo = a.t_x_lo;
      f.t_x_hi = a.t_x_hi;
      f.t_y_lo = a.t_y_lo;
      f.t_y_hi = a.t_y_hi;
      f.qsx = a.qsx;
      f.qsy = a.qsy;
      f.sxtab = a.sxtab;
      f.sytab = a.sytab;
    }
    first[size_t(j) + 1] = first[size_t(j)] + table[size_t(2) * j].ntiles;
    ffirst[size_t(j) + 1] =
        ffirst[size_t(j)] + ftable[size_t(2) * j].strips_x * ftable[size_t(2) * j].strips_y;
  }
  // the tables sit at the same offsets in the staging buffer and in the
  // workspace, so one copy moves them all
  HIP_TRY(hipMemcpyAsync(b->ws, b->table, b->table_bytes, hipMemcpyHostToDevice, b->stream));
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
  FusedBatchArgs fb{};
  fb.lats = reinterpret_cast<const FusedArgs*>(b->ws + b->off_fargs);
  fb.first = reinterpret_cast<const int*>(b->ws + b->off_ffirst);
  fb.sels = reinterpret_cast<const uint32_t* const*>(b->ws + b->off_fsel);
  fb.pulls = reinterpret_cast<const uint32_t* const*>(b->ws + b->off_fpull);
  fb.codes = reinterpret_cast<const uint8_t* const*>(b->ws + b->off_fcode);
  fb.ins = reinterpret_cast<const float* const*>(b->ws + b->off_fins);
  fb.n = n;
  fb.nblocks = ffirst[size_t(n)];
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
  // The multi-step kernels read the ghost frame of periodic edges, which
  // other producers write only in part: refresh it before a multi-step
  // launch that follows them (the current buffer of a lattice after `fl`
  // launches of this call is cur ^ (fl & 1)).
  std::vector<bool> frame_ok(static_cast<size_t>(n), false);
  for (int j = 0; j < n; ++j) frame_ok[size_t(j)] = b->lats[j]->ghosts_full;
  auto refresh = [&](int64_t fl) -> hipError_t {
    for (int j = 0; j < n; ++j) {
      wlbm_lattice* l = b->lats[j];
      const bool px = l->g.x_edge == kPeriodic, py = l->g.y_edge == kPeriodic;
      const int buf = l->cur ^ int(fl & 1);
      hipError_t e = hipSuccess;
      if (!frame_ok[size_t(j)]) {
        e = fill_ghosts(l->ptr(l->c.e[buf]), l->g.plane, l->p.q, l->g.nx, l->g.ny, l->g.pitch,
                        px, py, b->stream);
        if (e == hipSuccess)
          e = fill_ghosts(l->ptr(l->c.E[buf]), l->g.plane, 1, l->g.nx, l->g.ny, l->g.pitch, px,
                          py, b->stream);
        frame_ok[size_t(j)] = true;
      }
      if (e == hipSuccess && l->per_cell && !l->wf_ghosts_full) {
        e = fill_ghosts(l->ptr(l->c.Wf), l->g.plane, 1, l->g.nx, l->g.ny, l->g.pitch, px, py,
                        b->stream);
        if (e == hipSuccess) l->wf_ghosts_full = true;
      }
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  // each group advances its own schedule state
  std::vector<TasState> tas;
  for (const BatchGroup& bg : b->groups) tas.push_back(bg.lead->tas);
  std::vector<int8_t> dx(size_t(b->chunk) * b->qmax), dy(size_t(b->chunk) * b->qmax);
  std::vector<uint8_t> hop(size_t(b->chunk) * b->qmax);
  int64_t done = 0;
  int64_t flips = 0;          // launches so far: the buffer parity
  bool last_fused = false;
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
    // with (for multi-step launches) the selection offsets of the group and
    // the pull offsets of each geometry, and upload them into the rings.
    hipError_t e = hipSuccess;
    for (int g = 0; g < ngroups && e == hipSuccess; ++g) {
      const BatchGroup& bg = b->groups[size_t(g)];
      const wlbm_lattice* lead = bg.lead;
      const int q = lead->p.q;
      uint8_t* rows = b->pinned[slot] + bg.stage;
      float* insums = b->pinned_ins[slot] + size_t(g) * b->chunk * 4;
      for (int j = 0; j < cnt; ++j) {
        int8_t* dxj = dx.data() + size_t(j) * q;
        int8_t* dyj = dy.data() + size_t(j) * q;
        uint8_t* hopj = hop.data() + size_t(j) * q;
        tas_advance(lead->dirs, tas[size_t(g)], dxj, dyj, hopj);
        for (int m = 0; m < n; ++m)
          if (b->group[m] == g) b->lats[m]->book.note(tas[size_t(g)]);
        double lo_h = 0, lo_a = 0, hi_h = 0, hi_a = 0;
        for (int i = 0; i < q; ++i) {
          rows[size_t(j) * q + i] = pack_code(dxj[i], dyj[i], hopj[i]);
          if (dyj[i] == 1) {
            lo_a += lead->dirs.w[i];
            if (hopj[i]) lo_h += lead->dirs.w[i];
          } else if (dyj[i] == -1) {
            hi_a += lead->dirs.w[i];
            if (hopj[i]) hi_h += lead->dirs.w[i];
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
      if (fuse && e == hipSuccess) {
        uint32_t* sels = b->pinned_sels[slot] + b->sels_stage[size_t(g)];
        for (size_t k = 0; k < size_t(cnt) * q; ++k) sels[k] = uint32_t(rows[k]) * kSelEntryBytes;
        e = hipMemcpyAsync(reinterpret_cast<uint32_t*>(b->ws + b->sels[size_t(g)]) +
                               size_t(slot) * b->chunk * q,
                           sels, size_t(cnt) * q * sizeof(uint32_t), hipMemcpyHostToDevice,
                           b->stream);
        for (size_t k = 0; k < b->geos.size() && e == hipSuccess; ++k) {
          const BatchGeo& geo = b->geos[k];
          if (geo.group != g) continue;
          const uint32_t pitch4 = uint32_t(geo.pitch) * 4u, plane4 = uint32_t(geo.plane) * 4u;
          uint32_t* pw = b->pinned_pulls[slot] + geo.stage;
          for (int j = 0; j < cnt; ++j)
            for (int i = 0; i < q; ++i) {
              const size_t ji = size_t(j) * q + i;
              const int hx = hop[ji] ? dx[ji] : 0, hy = hop[ji] ? dy[ji] : 0;
              pw[ji] = uint32_t(1 - hy) * pitch4 + uint32_t(4 * (1 - hx)) +
                       uint32_t(i % kMaxGroupPlanes) * plane4;
            }
          e = hipMemcpyAsync(reinterpret_cast<uint32_t*>(b->ws + geo.pulls) +
                                 size_t(slot) * b->chunk * q,
                             pw, size_t(cnt) * q * sizeof(uint32_t), hipMemcpyHostToDevice,
                             b->stream);
        }
      }
    }
    if (e == hipSuccess) e = hipEventRecord(b->ev[slot], b->stream);
    if (e != hipSuccess) return fail(WLBM_EHIP, "schedule upload failed: %s", hipGetErrorString(e));
    b->ev_pending[slot] = true;
    ++b->chunk_counter;
    // A whole chunk of single steps with no flux-window step and no sources,
    // starting on an even launch of this call, is one launch of the slot's
    // captured graph: its kernels read the schedule rows and sums just
    // uploaded, and the argument table of this call.
    const bool graph = !fuse && b->use_graphs && cnt == b->chunk && b->chunk % 2 == 0 &&
                       flips % 2 == 0 && done + cnt <= flux_from && !has_sources;
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
      flips += cnt;
      last_fused = false;
      std::fill(frame_ok.begin(), frame_ok.end(), false);
      continue;
    }
    for (int j = 0; j < cnt; ++j) {
      const int64_t k = done + j;
      const bool flux = k >= flux_from;
      if (fuse && j + k_max <= cnt) {
        // steps k .. k + k_max - 1 in one launch; those in the flux window
        // add their heat flux to the window's sums in the launch
        fb.row = slot * b->chunk + j;
        fb.parity = int(flips & 1);
        fb.flux_levels = 0;
        for (int m = 0; m < k_max; ++m)
          if (k + m >= flux_from) fb.flux_levels |= 1u << m;
        fb.flux_first =
            (flux_from >= k && flux_from < k + k_max) ? int(flux_from - k) + 1 : 0;
        e = refresh(flips);
        if (e == hipSuccess)
          e = launch_fused_batch(fb, b->qmax, k_max, l0->per_cell, fb.flux_levels != 0,
                                 b->stream);
        if (e != hipSuccess) {
          for (wlbm_lattice* l : b->lats) l->broken = true;
          return fail(WLBM_EHIP, "batch multi-step launch failed: %s", hipGetErrorString(e));
        }
        ++flips;
        last_fused = true;
        j += k_max - 1;
        continue;
      }
      ba.row = slot * b->chunk + j;
      ba.codes = rows0(slot, j);
      ba.ins = ins0(slot, j);
      ba.parity = int(flips & 1);
      ba.q_first = (flux && k == flux_from) ? 1 : 0;
      e = launch_step_batch(ba, l0->split, l0->per_cell, flux, grouped, b->stream);
      for (int jl = 0; jl < n && e == hipSuccess; ++jl) {
        wlbm_lattice* l = b->lats[jl];
        if (!l->nsrc) continue;
        const int out = 1 - (l->cur ^ int(flips & 1));
        e = launch_apply_sources(l->g, l->ptr(l->c.e[out]), l->ptr(l->c.E[out]), l->src_cells,
                                 l->src_vals, l->nsrc, b->stream);
      }
      if (e != hipSuccess) {
        for (wlbm_lattice* l : b->lats) l->broken = true;
        return fail(WLBM_EHIP, "batch step launch failed: %s", hipGetErrorString(e));
      }
      ++flips;
      last_fused = false;
      std::fill(frame_ok.begin(), frame_ok.end(), false);
    }
    done += cnt;
  }
  for (int j = 0; j < n; ++j) {
    wlbm_lattice* l = b->lats[j];
    l->tas = tas[size_t(b->group[j])];
    l->cur ^= int(flips & 1);
    l->flux_valid = l->flux_window > 0 && nsteps >= l->flux_window;
    l->ghosts_full = last_fused;
  }
  return WLBM_OK;
}

int32_t wlbm_batch_get_steps_per_launch(const wlbm_batch* b) {
  if (!b) return -1;
  const int k = batch_fused_k(b);
  return k >= 2 ? k : 1;
}

wlbm_status wlbm_batch_tune_block_rows(wlbm_batch* b, void* d_states, size_t bytes,
                                       int32_t launches, int32_t* rows_out) {
  if (!b) return fail(WLBM_EINVAL, "batch is NULL");
  wlbm_status st = check_members(b->lats.data(), int32_t(b->lats.size()));
  if (st) return st;
  if (launches < 1 || launches > 1000) return fail(WLBM_EINVAL, "launches must be in 1 .. 1000");
  const int k = batch_fused_k(b);
  if (k < 2)
    return fail(WLBM_EINVAL, "this batch runs one step per launch (a member's edges, sources, q "
                             "or size rule out the multi-step kernels, or the members' q differ)");
  if (!d_states) return fail(WLBM_EINVAL, "state buffer is NULL");
  // one slot per member, each 256-byte aligned
  std::vector<size_t> off(b->lats.size()), len(b->lats.size());
  size_t need = 0;
  for (size_t j = 0; j < b->lats.size(); ++j) {
    st = wlbm_state_bytes(b->lats[j], &len[j]);
    if (st) return st;
    off[j] = need;
    need = align_up(need + len[j]);
  }
  if (bytes < need)
    return fail(WLBM_EINVAL, "state buffer holds %zu bytes, the members' states need %zu", bytes,
                need);
  if (reinterpret_cast<uintptr_t>(d_states) % kAlign)
    return fail(WLBM_EINVAL, "state buffer must be 256-byte aligned");
  wlbm_lattice* l0 = b->lats[0];
  const int pc = l0->per_cell ? 1 : 0;
  const int64_t warm = 2, need_steps = (warm + launches) * int64_t(k);
  if (l0->tas.n + need_steps > kMaxSteps) return fail(WLBM_EINVAL, "step count would overflow");
  const int64_t step0 = l0->tas.n;
  // whole launches of k steps: a launch never crosses a schedule chunk
  const int per_call = std::max(1, std::min<int>(launches, b->chunk / k));
  char* buf = static_cast<char*>(d_states);
  // the members' state moves run on the batch's stream while tuning, and
  // their flux-window sums are left alone
  std::vector<hipStream_t> keep_stream(b->lats.size());
  std::vector<int> keep_window(b->lats.size()), keep_rows(b->lats.size());
  std::vector<uint8_t> keep_valid(b->lats.size());
  for (size_t j = 0; j < b->lats.size(); ++j) {
    wlbm_lattice* l = b->lats[j];
    keep_stream[j] = l->stream;
    keep_window[j] = l->flux_window;
    keep_valid[j] = l->flux_valid ? 1 : 0;
    keep_rows[j] = l->rows[pc][k];
    l->stream = b->stream;
    l->flux_window = 0;
  }
  auto restore_members = [&]() {
    for (size_t j = 0; j < b->lats.size(); ++j) {
      wlbm_lattice* l = b->lats[j];
      l->stream = keep_stream[j];
      l->flux_window = keep_window[j];
      l->flux_valid = keep_valid[j] != 0;
    }
  };
  for (size_t j = 0; j < b->lats.size() && !st; ++j)
    st = wlbm_save_state(b->lats[j], buf + off[j], len[j]);
  int ny_max = 1;
  for (const wlbm_lattice* l : b->lats) ny_max = std::max(ny_max, l->g.ny);
  int cand[32];
  const int nc = fused_row_candidates(ny_max, k, cand, 32);
  std::vector<float> best(size_t(nc), -1.f);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipSuccess;
  if (!st && (he = hipEventCreate(&e0)) != hipSuccess)
    st = fail(WLBM_EHIP, "hipEventCreate failed: %s", hipGetErrorString(he));
  if (!st && (he = hipEventCreate(&e1)) != hipSuccess)
    st = fail(WLBM_EHIP, "hipEventCreate failed: %s", hipGetErrorString(he));
  // two passes over the candidates (one height for every member), each
  // keeping its best time; the states are restored after every trial
  for (int pass = 0; pass < 2 && !st; ++pass) {
    for (int c = 0; c < nc && !st; ++c) {
      for (wlbm_lattice* l : b->lats) l->rows[pc][k] = cand[c];
      st = wlbm_batch_step(b, warm * k);
      if (!st && (he = hipEventRecord(e0, b->stream)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventRecord failed: %s", hipGetErrorString(he));
      for (int64_t left = launches; !st && left > 0; left -= per_call)
        st = wlbm_batch_step(b, std::min<int64_t>(left, per_call) * k);
      float ms = -1.f;
      if (!st && (he = hipEventRecord(e1, b->stream)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventRecord failed: %s", hipGetErrorString(he));
      if (!st && (he = hipEventSynchronize(e1)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventSynchronize failed: %s", hipGetErrorString(he));
      if (!st && (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
        st = fail(WLBM_EHIP, "hipEventElapsedTime failed: %s", hipGetErrorString(he));
      if (!st && (best[size_t(c)] < 0.f || ms < best[size_t(c)])) best[size_t(c)] = ms;
      for (size_t j = 0; j < b->lats.size() && !st; ++j)
        st = wlbm_load_state(b->lats[j], buf + off[j], len[j], step0);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) {
    for (size_t j = 0; j < b->lats.size(); ++j) b->lats[j]->rows[pc][k] = keep_rows[j];
    restore_members();
    return st;
  }
  int bi = 0;
  for (int c = 1; c < nc; ++c)
    if (best[size_t(c)] < best[size_t(bi)]) bi = c;
  for (wlbm_lattice* l : b->lats) l->rows[pc][k] = cand[bi];
  restore_members();
  if (rows_out) *rows_out = cand[bi];
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
    if (b->pinned_sels[k]) (void)hipHostFree(b->pinned_sels[k]);
    if (b->pinned_pulls[k]) (void)hipHostFree(b->pinned_pulls[k]);
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
