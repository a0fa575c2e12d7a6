// C-ABI of libwormlbm.so (declared in include/wormlbm.h).
//
// A lattice handle owns the host tables (direction set, weights, corrected
// relaxation weight), the host TAS state and two pinned staging buffers for
// schedule uploads; all device memory is the caller's workspace, carved into
// the regions below.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "../../include/wormlbm.h"
#include "device.hpp"
#include "tables.hpp"

using namespace wlbm;

namespace {

thread_local std::string g_last_error;

wlbm_status fail(wlbm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(WLBM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));            \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kReduceBlocks = 1024;
constexpr int kDefaultChunk = 240;   // a multiple of 2, 3 and 4 (steps per launch)
constexpr int64_t kMaxSteps = (int64_t(1) << 31) - 1;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of the workspace regions.
struct Carve {
  size_t e[2], E[2], Wf, Wraw, qsx, qsy, partials, totals, flag, sched, pulls, wtab, sxtab, sytab,
      mtab, total;
};

// Lattices that the multi-step kernels can advance (both edges periodic).
bool fusable(const wlbm_params& p) {
  return p.x_edge == WLBM_EDGE_PERIODIC && p.y_edge == WLBM_EDGE_PERIODIC &&
         fused_supported(p.q, p.nx, p.ny);
}

int chunk_steps(const wlbm_params& p) { return p.sched_chunk ? p.sched_chunk : kDefaultChunk; }

Carve carve(const wlbm_params& p) {
  Carve c{};
  const size_t plane = size_t(padded_plane(p.nx, p.ny)) * sizeof(float);
  const size_t cells = size_t(p.nx) * size_t(p.ny) * sizeof(float);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  c.e[0] = take(plane * size_t(p.q));
  c.e[1] = take(plane * size_t(p.q));
  c.E[0] = take(plane);
  c.E[1] = take(plane);
  c.Wf = take(plane);
  c.Wraw = take(cells);
  c.qsx = take(cells);
  c.qsy = take(cells);
  c.partials = take(size_t(kReduceBlocks) * 3 * sizeof(double));
  c.totals = take(4 * sizeof(double));
  c.flag = take(sizeof(int));
  c.sched = take(size_t(2) * chunk_steps(p) * size_t(p.q));
  // per step, the multi-step kernels' pull offsets and selection-table
  // offsets of every direction (FusedArgs::pulls, FusedArgs::sels)
  c.pulls = take(fusable(p) ? size_t(4) * chunk_steps(p) * size_t(p.q) * sizeof(uint32_t) : 0);
  c.wtab = take(size_t(p.q) * sizeof(float));
  c.sxtab = take(size_t(p.q) * sizeof(float));
  c.sytab = take(size_t(p.q) * sizeof(float));
  c.mtab = take(size_t(p.q) * sizeof(int));
  c.total = off;
  return c;
}

wlbm_status validate(const wlbm_params* p) {
  if (!p) return fail(WLBM_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nx > (1 << 20) || p->ny > (1 << 20))
    return fail(WLBM_EINVAL, "nx, ny must be in 1..2^20 (got %d, %d)", p->nx, p->ny);
  if (p->q < 8 || p->q > kMaxQ || p->q % 8 != 0)
    return fail(WLBM_EINVAL, "q must be a multiple of 8 in 8..%d (got %d)", kMaxQ, p->q);
  if (p->dirs != WLBM_DIRS_UNIFORM && p->dirs != WLBM_DIRS_RING)
    return fail(WLBM_EINVAL, "unknown direction set %d", p->dirs);
  if (p->x_edge != WLBM_EDGE_PERIODIC && p->x_edge != WLBM_EDGE_BLACKBODY)
    return fail(WLBM_EINVAL, "x edges must be periodic or blackbody (got %d)", p->x_edge);
  if (p->y_edge != WLBM_EDGE_PERIODIC && p->y_edge != WLBM_EDGE_BLACKBODY &&
      p->y_edge != WLBM_EDGE_DIFFUSE)
    return fail(WLBM_EINVAL, "y edges must be periodic, blackbody or diffuse (got %d)",
                p->y_edge);
  if (!(p->mfp_cells > 0.0)) return fail(WLBM_EINVAL, "mfp_cells must be > 0");
  if (p->emulate_3d != 0 && p->emulate_3d != 1) return fail(WLBM_EINVAL, "emulate_3d is 0 or 1");
  if (p->mfp_correction != 0 && p->mfp_correction != 1)
    return fail(WLBM_EINVAL, "mfp_correction is 0 or 1");
  if (p->dir_split != 0 && p->dir_split != 1 && p->dir_split != 2 && p->dir_split != 4)
    return fail(WLBM_EINVAL, "dir_split must be 0, 1, 2 or 4");
  if (p->dir_split && p->q % (kMaxGroupPlanes * p->dir_split) != 0)
    return fail(WLBM_EINVAL, "q = %d cannot be split over %d waves (needs a multiple of %d)",
                p->q, p->dir_split, kMaxGroupPlanes * p->dir_split);
  if (p->dir_split && step_batch_lds_bytes(p->q, p->dir_split) > 48 * 1024)
    return fail(WLBM_EINVAL, "q = %d is too large for a split over %d waves", p->q,
                p->dir_split);
  if (p->sched_chunk != 0 && (p->sched_chunk < 16 || p->sched_chunk > 65536))
    return fail(WLBM_EINVAL, "sched_chunk must be 0 or 16..65536");
  for (int k = 0; k < 3; ++k)
    if (p->reserved[k] != 0) return fail(WLBM_EINVAL, "reserved fields must be zero");
  if (p->step_fusion < 0 || p->step_fusion > 4)
    return fail(WLBM_EINVAL, "step_fusion is 0 (one step per launch), 1 (default), 2, 3 or 4");
  if (!(p->y_specularity >= 0.0 && p->y_specularity <= 1.0))
    return fail(WLBM_EINVAL, "y_specularity must lie in [0, 1]");
  if (!std::isfinite(p->t_x_lo) || !std::isfinite(p->t_x_hi) || !std::isfinite(p->t_y_lo) ||
      !std::isfinite(p->t_y_hi))
    return fail(WLBM_EINVAL, "wall temperatures must be finite");
  // 32-bit byte offsets inside one group of direction planes
  if ((kMaxGroupPlanes * padded_plane(p->nx, p->ny) + 2 * (padded_pitch(p->nx) + 1)) *
          int64_t(sizeof(float)) >=
      (int64_t(1) << 32))
    return fail(WLBM_EINVAL,
                "lattice too large: %d padded planes must stay below 4 GiB (nx*ny up to about "
                "1.3e8 cells)", kMaxGroupPlanes);
  return WLBM_OK;
}

double uniform_wcorr(const wlbm_params& p, double lam, double* W_out) {
  const double W = std::isinf(p.mfp_cells) ? 0.0 : 1.0 / p.mfp_cells;
  if (W_out) *W_out = W;
  return corrected_weight(W, lam, p.emulate_3d != 0, p.mfp_correction != 0);
}

// Byte offsets of the adjoint workspace regions.
struct AdjCarve {
  size_t lam[2], H[2], gW, gB, sched, walls, flag, total;
};

AdjCarve adj_carve(const wlbm_params& p) {
  AdjCarve c{};
  const size_t plane = size_t(padded_plane(p.nx, p.ny)) * sizeof(float);
  const size_t cells = size_t(p.nx) * size_t(p.ny);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  c.lam[0] = take(plane * size_t(p.q));
  c.lam[1] = take(plane * size_t(p.q));
  c.H[0] = take(plane * 8);
  c.H[1] = take(plane * 8);
  c.gW = take(cells * sizeof(double));
  c.gB = take(cells * sizeof(double));
  c.sched = take(size_t(2) * chunk_steps(p) * size_t(p.q));
  c.walls = take(4 * sizeof(double));
  c.flag = take(sizeof(int));
  c.total = off;
  return c;
}

size_t state_bytes_of(const wlbm_params& p) {
  return align_up(size_t(padded_plane(p.nx, p.ny)) * sizeof(float) * size_t(p.q + 1));
}

}  // namespace

// Block height (output rows per block) of a multi-step kernel, chosen by
// timing real launches: in each of kPasses passes over the candidates, a
// candidate height runs kSample back-to-back launches, timed from the end of
// the first to the end of the last (so that the warm-up of the first and the
// overlap of consecutive launches are as in a long run); the candidate with
// the best time over the passes is kept.  The populations do not depend on
// the height, so nothing is repeated or undone.
struct RowTuner {
  static constexpr int kMaxCand = 24;
  static constexpr int kSample = 6;
  static constexpr int kPasses = 2;
  int cand[kMaxCand] = {};
  float ms[kMaxCand] = {};
  int ncand = 0;
  int next = 0;     // launches run while tuning
  int chosen = 0;   // 0 while tuning
};

struct wlbm_lattice {
  wlbm_params p{};
  DirSet dirs;
  TasState tas;
  Geometry g{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Carve c{};
  int cur = 0;              // population buffer holding the current state
  float W = 0.f;            // uniform corrected weight
  bool per_cell = false;    // per-cell weight field active
  int split = 1;            // waves sharing the directions of one cell
  int chunk = kDefaultChunk;
  // Rows per block of the multi-step kernels, per [per_cell][k]: chosen by
  // timing the first launches (the results do not depend on it).
  RowTuner tuner[2][5];
  hipEvent_t tev[2] = {nullptr, nullptr};   // timing events of those launches
  uint8_t* pinned[2] = {nullptr, nullptr};
  uint32_t* pinned_pulls[2] = {nullptr, nullptr};   // staging of the pull offsets
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_pending[2] = {false, false};
  int64_t chunk_counter = 0;
  int flux_window = 0;
  bool flux_valid = false;
  bool broken = false;
  Walls walls{};
  ScheduleBook book;        // schedule rows of any step, for restarts and the adjoint
  // adjoint (reverse pass) state
  // internal sources (caller's device arrays, kept valid by the caller)
  int nsrc = 0;
  const int32_t* src_cells = nullptr;
  const float* src_vals = nullptr;
  char* aws = nullptr;      // caller's adjoint workspace
  AdjCarve ac{};
  int acur = 0;             // lam / H buffer holding lam^am
  int64_t am = -1;          // adjoint step index; -1 when no reverse pass is active

  float* ptr(size_t off) { return reinterpret_cast<float*>(ws + off); }
  float* aptr(size_t off) { return reinterpret_cast<float*>(aws + off); }
};

namespace {

wlbm_status check_lat(const wlbm_lattice* l) {
  if (!l) return fail(WLBM_EINVAL, "lattice is NULL");
  if (l->broken) return fail(WLBM_ESTATE, "lattice is unusable after an earlier HIP error");
  return WLBM_OK;
}

// Default direction split: as many waves per cell as q allows (up to four),
// which keeps waves short-lived; measured best on 1024^2 x 64 and
// 4096^2 x 256 lattices.
int auto_split(int q) {
  constexpr size_t kMaxBatchLds = 48 * 1024;
  if (q % (4 * kMaxGroupPlanes) == 0 && step_batch_lds_bytes(q, 4) <= kMaxBatchLds) return 4;
  if (q % (2 * kMaxGroupPlanes) == 0 && step_batch_lds_bytes(q, 2) <= kMaxBatchLds) return 2;
  return 1;
}

void auto_tiling(wlbm_lattice* l) { l->split = l->p.dir_split ? l->p.dir_split : auto_split(l->p.q); }

}  // namespace

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
  // Full schedule chunks run as one launch of a captured HIP graph per
  // schedule-ring slot; key: what the graph was captured for.
  bool use_graphs = true;
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

void wlbm_default_params(wlbm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = 64;
  p->ny = 64;
  p->q = 16;
  p->dirs = WLBM_DIRS_UNIFORM;
  p->mfp_cells = 16.0;
  p->emulate_3d = 0;
  p->mfp_correction = 1;
  p->x_edge = WLBM_EDGE_PERIODIC;
  p->y_edge = WLBM_EDGE_PERIODIC;
  p->step_fusion = 1;
}

wlbm_status wlbm_workspace_bytes(const wlbm_params* p, size_t* bytes) {
  wlbm_status st = validate(p);
  if (st) return st;
  if (!bytes) return fail(WLBM_EINVAL, "bytes is NULL");
  try {
    DirSet d = build_dirs(p->q, p->dirs);
    if (uniform_wcorr(*p, d.lambda_corr, nullptr) > 1.0)
      return fail(WLBM_EUNSTABLE, "corrected relaxation weight %.17g exceeds 1 (App. A)",
                  uniform_wcorr(*p, d.lambda_corr, nullptr));
  } catch (const std::exception& e) {
    return fail(WLBM_EINVAL, "%s", e.what());
  }
  *bytes = carve(*p).total;
  return WLBM_OK;
}

wlbm_status wlbm_get_directions(const wlbm_params* p, double* sx, double* sy, double* w) {
  wlbm_status st = validate(p);
  if (st) return st;
  try {
    DirSet d = build_dirs(p->q, p->dirs);
    for (int i = 0; i < p->q; ++i) {
      if (sx) sx[i] = d.sx[i];
      if (sy) sy[i] = d.sy[i];
      if (w) w[i] = d.w[i];
    }
  } catch (const std::exception& e) {
    return fail(WLBM_EINVAL, "%s", e.what());
  }
  return WLBM_OK;
}

wlbm_status wlbm_get_constants(const wlbm_params* p, double* lambda_corr, double* w,
                               double* w_corr) {
  wlbm_status st = validate(p);
  if (st) return st;
  try {
    DirSet d = build_dirs(p->q, p->dirs);
    double W;
    const double wc = uniform_wcorr(*p, d.lambda_corr, &W);
    if (lambda_corr) *lambda_corr = d.lambda_corr;
    if (w) *w = W;
    if (w_corr) *w_corr = wc;
  } catch (const std::exception& e) {
    return fail(WLBM_EINVAL, "%s", e.what());
  }
  return WLBM_OK;
}

static wlbm_status check_speeds(int q, const double* v) {
  if (!v) return WLBM_OK;
  for (int i = 0; i < q; ++i)
    if (!(v[i] > 0.0 && v[i] <= 1.0))
      return fail(WLBM_EINVAL, "speed of direction %d is %g; speeds lie in (0, 1]", i, v[i]);
  return WLBM_OK;
}

wlbm_status wlbm_get_schedule(const wlbm_params* p, const double* speeds, int64_t step0,
                              int64_t n, int8_t* moves, int64_t* pos) {
  wlbm_status st = validate(p);
  if (!st) st = check_speeds(p->q, speeds);
  if (st) return st;
  if (step0 < 0 || n < 0 || step0 + n > kMaxSteps)
    return fail(WLBM_EINVAL, "steps must satisfy 0 <= step0, 0 <= n, step0 + n < 2^31");
  if (n > 0 && !moves) return fail(WLBM_EINVAL, "moves is NULL");
  try {
    DirSet d = build_dirs(p->q, p->dirs);
    if (speeds) d.vgrid.assign(speeds, speeds + p->q);
    TasState s;
    s.reset(p->q);
    std::vector<int8_t> dx(p->q), dy(p->q);
    std::vector<uint8_t> hop(p->q);
    for (int64_t k = 0; k < step0 + n; ++k) {
      tas_advance(d, s, dx.data(), dy.data(), hop.data());
      if (k < step0) continue;
      const int64_t row = k - step0;
      for (int i = 0; i < p->q; ++i) {
        const int idx = d2q8_index(dx[i], dy[i]);
        moves[row * p->q + i] = int8_t(hop[i] ? idx : -idx);
        if (pos) {
          pos[(row * p->q + i) * 2] = s.px[i];
          pos[(row * p->q + i) * 2 + 1] = s.py[i];
        }
      }
    }
  } catch (const std::exception& e) {
    return fail(WLBM_EINVAL, "%s", e.what());
  }
  return WLBM_OK;
}

wlbm_status wlbm_create(const wlbm_params* p, void* d_workspace, size_t ws_bytes, void* stream,
                        wlbm_lattice** out) {
  if (!out) return fail(WLBM_EINVAL, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  wlbm_status st = wlbm_workspace_bytes(p, &need);
  if (st) return st;
  if (!d_workspace) return fail(WLBM_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
    return fail(WLBM_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(WLBM_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);

  wlbm_lattice* l = new (std::nothrow) wlbm_lattice();
  if (!l) return fail(WLBM_ENOMEM, "host allocation failed");
  try {
    l->p = *p;
    l->dirs = build_dirs(p->q, p->dirs);
  } catch (const std::exception& e) {
    delete l;
    return fail(WLBM_EINVAL, "%s", e.what());
  }
  l->tas.reset(p->q);
  l->book.reset(&l->dirs);
  l->stream = static_cast<hipStream_t>(stream);
  l->ws = static_cast<char*>(d_workspace);
  l->c = carve(*p);
  l->chunk = chunk_steps(*p);
  l->W = float(uniform_wcorr(*p, l->dirs.lambda_corr, nullptr));
  l->walls = {float(p->t_x_lo), float(p->t_x_hi), float(p->t_y_lo), float(p->t_y_hi)};
  l->g = {p->nx, p->ny, p->q, padded_pitch(p->nx), padded_plane(p->nx, p->ny), p->x_edge,
          p->y_edge};
  auto_tiling(l);

  auto cleanup = [&](wlbm_status s) {
    for (int k = 0; k < 2; ++k) {
      if (l->pinned[k]) (void)hipHostFree(l->pinned[k]);
      if (l->pinned_pulls[k]) (void)hipHostFree(l->pinned_pulls[k]);
      if (l->ev[k]) (void)hipEventDestroy(l->ev[k]);
      if (l->tev[k]) (void)hipEventDestroy(l->tev[k]);
    }
    delete l;
    return s;
  };
  const size_t stage = std::max<size_t>(size_t(l->chunk) * p->q, 4 * size_t(p->q) * sizeof(float));
  for (int k = 0; k < 2; ++k) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&l->pinned[k]), stage, hipHostMallocDefault);
    if (e == hipSuccess && fusable(*p))
      e = hipHostMalloc(reinterpret_cast<void**>(&l->pinned_pulls[k]),
                        size_t(2) * l->chunk * p->q * sizeof(uint32_t), hipHostMallocDefault);
    if (e != hipSuccess) {
      wlbm_status s = fail(WLBM_ENOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
      return cleanup(s);
    }
    e = hipEventCreateWithFlags(&l->ev[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&l->tev[k]);
    if (e != hipSuccess) {
      wlbm_status s = fail(WLBM_EHIP, "hipEventCreate failed: %s", hipGetErrorString(e));
      return cleanup(s);
    }
  }
  // Clear the workspace (ghosts of non-periodic edges must read zero) and
  // upload the direction tables as float32.
  hipError_t e = hipMemsetAsync(l->ws, 0, l->c.total, l->stream);
  float* tabs = reinterpret_cast<float*>(l->pinned[0]);
  for (int i = 0; i < p->q; ++i) {
    tabs[i] = float(l->dirs.w[i]);
    tabs[p->q + i] = float(l->dirs.sx[i]);
    tabs[2 * p->q + i] = float(l->dirs.sy[i]);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(l->ws + l->c.wtab, tabs, p->q * sizeof(float), hipMemcpyHostToDevice,
                       l->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(l->ws + l->c.sxtab, tabs + p->q, p->q * sizeof(float),
                       hipMemcpyHostToDevice, l->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(l->ws + l->c.sytab, tabs + 2 * p->q, p->q * sizeof(float),
                       hipMemcpyHostToDevice, l->stream);
  int* mir = reinterpret_cast<int*>(tabs + 3 * p->q);
  for (int i = 0; i < p->q; ++i) mir[i] = l->dirs.mirror_y[i];
  if (e == hipSuccess)
    e = hipMemcpyAsync(l->ws + l->c.mtab, mir, p->q * sizeof(int), hipMemcpyHostToDevice,
                       l->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(l->stream);
  if (e != hipSuccess) {
    wlbm_status s = fail(WLBM_EHIP, "workspace set-up failed: %s", hipGetErrorString(e));
    return cleanup(s);
  }
  *out = l;
  return WLBM_OK;
}

wlbm_status wlbm_set_stream(wlbm_lattice* l, void* stream) {
  if (!l) return fail(WLBM_EINVAL, "lattice is NULL");
  l->stream = static_cast<hipStream_t>(stream);
  return WLBM_OK;
}

wlbm_status wlbm_set_temperature(wlbm_lattice* l, const float* d_T0) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!d_T0) return fail(WLBM_EINVAL, "T0 is NULL");
  HIP_TRY(launch_init_temperature(l->g, d_T0, l->ptr(l->c.e[l->cur]), l->ptr(l->c.E[l->cur]),
                                  l->ptr(l->c.wtab), l->walls, l->stream));
  HIP_TRY(launch_apply_sources(l->g, l->ptr(l->c.e[l->cur]), l->ptr(l->c.E[l->cur]), l->src_cells,
                               l->src_vals, l->nsrc, l->stream));
  l->flux_valid = false;
  return WLBM_OK;
}

wlbm_status wlbm_set_populations(wlbm_lattice* l, const float* d_e) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!d_e) return fail(WLBM_EINVAL, "populations pointer is NULL");
  HIP_TRY(launch_init_populations(l->g, d_e, l->ptr(l->c.e[l->cur]), l->ptr(l->c.E[l->cur]),
                                  l->ptr(l->c.wtab), l->walls, l->stream));
  HIP_TRY(launch_apply_sources(l->g, l->ptr(l->c.e[l->cur]), l->ptr(l->c.E[l->cur]), l->src_cells,
                               l->src_vals, l->nsrc, l->stream));
  l->flux_valid = false;
  return WLBM_OK;
}

wlbm_status wlbm_set_mfp_field(wlbm_lattice* l, const float* d_mfp) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!d_mfp) {
    l->per_cell = false;
    return WLBM_OK;
  }
  const double f = l->p.emulate_3d ? 1.5 : 1.0;
  int* flag = reinterpret_cast<int*>(l->ws + l->c.flag);
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), l->stream));
  HIP_TRY(launch_check_mfp(l->g, d_mfp, l->dirs.lambda_corr, f, l->p.mfp_correction, flag,
                           l->stream));
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, l->stream));
  HIP_TRY(hipStreamSynchronize(l->stream));
  if (hflag)
    return fail(WLBM_EUNSTABLE,
                "MFP field rejected: a value is not positive, or a corrected weight is above 1 "
                "or not finite (App. A)");
  HIP_TRY(launch_write_wfield(l->g, d_mfp, l->dirs.lambda_corr, f, l->p.mfp_correction,
                              l->ptr(l->c.Wf), l->ptr(l->c.Wraw), l->stream));
  l->per_cell = true;
  return WLBM_OK;
}

wlbm_status wlbm_set_sources(wlbm_lattice* l, int32_t n, const int32_t* d_cells,
                             const float* d_values) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (n < 0) return fail(WLBM_EINVAL, "source count must be >= 0");
  if (n == 0) {
    l->nsrc = 0;
    l->src_cells = nullptr;
    l->src_vals = nullptr;
    return WLBM_OK;
  }
  if (!d_cells || !d_values) return fail(WLBM_EINVAL, "source arrays must not be NULL");
  std::vector<int32_t> cells(size_t(n) * 2);
  HIP_TRY(hipMemcpyAsync(cells.data(), d_cells, cells.size() * sizeof(int32_t),
                         hipMemcpyDeviceToHost, l->stream));
  HIP_TRY(hipStreamSynchronize(l->stream));
  std::vector<uint8_t> seen(size_t(l->g.nx) * l->g.ny, 0);
  for (int s = 0; s < n; ++s) {
    const int x = cells[2 * size_t(s)], y = cells[2 * size_t(s) + 1];
    if (x < 0 || x >= l->g.nx || y < 0 || y >= l->g.ny)
      return fail(WLBM_EINVAL, "source %d at (%d, %d) lies outside the lattice", s, x, y);
    uint8_t& f = seen[size_t(y) * l->g.nx + x];
    if (f) return fail(WLBM_EINVAL, "source %d repeats cell (%d, %d)", s, x, y);
    f = 1;
  }
  l->nsrc = n;
  l->src_cells = d_cells;
  l->src_vals = d_values;
  HIP_TRY(launch_apply_sources(l->g, l->ptr(l->c.e[l->cur]), l->ptr(l->c.E[l->cur]), d_cells,
                               d_values, n, l->stream));
  return WLBM_OK;
}

wlbm_status wlbm_flux_distribution(const wlbm_params* p, double T, double qx, double qy,
                                   double* e) {
  wlbm_status st = validate(p);
  if (st) return st;
  if (!e) return fail(WLBM_EINVAL, "output is NULL");
  try {
    DirSet d = build_dirs(p->q, p->dirs);
    // M = sum_i w_i s_i s_i^T; e_i = w_i (T + s_i . M^-1 q)
    double mxx = 0, mxy = 0, myy = 0;
    for (int i = 0; i < p->q; ++i) {
      mxx += d.w[i] * d.sx[i] * d.sx[i];
      mxy += d.w[i] * d.sx[i] * d.sy[i];
      myy += d.w[i] * d.sy[i] * d.sy[i];
    }
    const double det = mxx * myy - mxy * mxy;
    const double ax = (myy * qx - mxy * qy) / det;
    const double ay = (mxx * qy - mxy * qx) / det;
    for (int i = 0; i < p->q; ++i) e[i] = d.w[i] * (T + d.sx[i] * ax + d.sy[i] * ay);
  } catch (const std::exception& ex) {
    return fail(WLBM_EINVAL, "%s", ex.what());
  }
  return WLBM_OK;
}

wlbm_status wlbm_set_speeds(wlbm_lattice* l, const double* speeds) {
  wlbm_status st = check_lat(l);
  if (!st) st = check_speeds(l->p.q, speeds);
  if (st) return st;
  if (l->tas.n != 0) return fail(WLBM_ESTATE, "grid speeds can only be set at step 0");
  if (speeds)
    l->dirs.vgrid.assign(speeds, speeds + l->p.q);
  else
    l->dirs.vgrid.assign(l->p.q, 1.0);
  l->book.reset(&l->dirs);
  return WLBM_OK;
}

wlbm_status wlbm_set_wall_temperatures(wlbm_lattice* l, double txl, double txh, double tyl,
                                       double tyh) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!std::isfinite(txl) || !std::isfinite(txh) || !std::isfinite(tyl) || !std::isfinite(tyh))
    return fail(WLBM_EINVAL, "wall temperatures must be finite");
  l->walls = {float(txl), float(txh), float(tyl), float(tyh)};
  return WLBM_OK;
}

wlbm_status wlbm_set_flux_window(wlbm_lattice* l, int32_t window) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (window < 0) return fail(WLBM_EINVAL, "flux window must be >= 0");
  l->flux_window = window;
  l->flux_valid = false;
  return WLBM_OK;
}

}  // extern "C"

namespace {

// Advance nsteps (validated by the caller).  Without a tape the state
// alternates between the two population buffers of the workspace.  With a
// tape, step k (0-based) writes its output straight into tape slot k and
// reads slot k-1 (the lattice's current state for k = 0); the last slot is
// then copied into the current buffer.
wlbm_status run_steps(wlbm_lattice* l, int64_t nsteps, char* tape, size_t slot_bytes) {
  const int q = l->p.q;
  const int64_t flux_from = l->flux_window > 0 ? nsteps - l->flux_window : nsteps;
  std::vector<int8_t> dx(q), dy(q);
  std::vector<uint8_t> hop(q);
  std::vector<float> insums;
  StepArgs a{};
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
  a.q = q;
  a.pitch = l->g.pitch;
  a.plane = l->g.plane;
  a.x_edge = l->g.x_edge;
  a.y_edge = l->g.y_edge;
  a.tiles_x = tiles_x_for(l->g.nx);
  a.ntiles = a.tiles_x * tiles_y_for(l->g.ny, l->split);
  // several steps per launch: periodic edges only, no sources, not into a
  // tape, and a lattice the multi-step kernels are built for
  const bool fuse = l->p.step_fusion != 0 && !tape && l->nsrc == 0 &&
                    l->g.x_edge == kPeriodic && l->g.y_edge == kPeriodic &&
                    fused_supported(q, l->g.nx, l->g.ny);
  const int k_max = l->p.step_fusion == 1 ? 4 : l->p.step_fusion;

  // the multi-step kernels read three ghost columns; other producers write
  // the first one only, so the frame is refreshed before the first
  // multi-step launch and after any single step in between
  bool refresh_ghosts = true;

  int64_t done = 0;
  while (done < nsteps) {
    const int cnt = int(std::min<int64_t>(l->chunk, nsteps - done));
    const int slot = int(l->chunk_counter & 1);
    if (l->ev_pending[slot]) {
      hipError_t e = hipEventSynchronize(l->ev[slot]);
      if (e != hipSuccess) {
        l->broken = true;
        return fail(WLBM_EHIP, "hipEventSynchronize failed: %s", hipGetErrorString(e));
      }
      l->ev_pending[slot] = false;
    }
    // Build the schedule rows of this chunk (Sec. 2.3, Sec. 2.5) and the
    // per-step sums of inward weights used by diffuse walls.
    uint8_t* rows = l->pinned[slot];
    // with it, the multi-step kernels' first-step pull offsets (FusedArgs::pulls)
    uint32_t* pw = fuse ? l->pinned_pulls[slot] : nullptr;
    const uint32_t pitch4 = uint32_t(l->g.pitch) * 4u, plane4 = uint32_t(l->g.plane) * 4u;
    insums.assign(size_t(cnt) * 4, 0.f);
    for (int j = 0; j < cnt; ++j) {
      tas_advance(l->dirs, l->tas, dx.data(), dy.data(), hop.data());
      l->book.note(l->tas);
      double lo_h = 0, lo_a = 0, hi_h = 0, hi_a = 0;
      for (int i = 0; i < q; ++i) {
        rows[size_t(j) * q + i] = pack_code(dx[i], dy[i], hop[i]);
        if (pw) {
          const int hx = hop[i] ? dx[i] : 0, hy = hop[i] ? dy[i] : 0;
          pw[size_t(2 * j) * q + i] =
              uint32_t(1 - hy) * pitch4 + uint32_t(4 * (1 - hx)) + uint32_t(i % 8) * plane4;
          pw[size_t(2 * j + 1) * q + i] = uint32_t(rows[size_t(j) * q + i]) * kSelEntryBytes;
        }
        if (dy[i] == 1) {
          lo_a += l->dirs.w[i];
          if (hop[i]) lo_h += l->dirs.w[i];
        } else if (dy[i] == -1) {
          hi_a += l->dirs.w[i];
          if (hop[i]) hi_h += l->dirs.w[i];
        }
      }
      insums[4 * j] = float(lo_h);
      insums[4 * j + 1] = float(lo_a);
      insums[4 * j + 2] = float(hi_h);
      insums[4 * j + 3] = float(hi_a);
    }
    uint8_t* dev_rows = reinterpret_cast<uint8_t*>(l->ws + l->c.sched) + size_t(slot) * l->chunk * q;
    uint32_t* dev_pulls =
        reinterpret_cast<uint32_t*>(l->ws + l->c.pulls) + size_t(2 * slot) * l->chunk * q;
    hipError_t e = hipMemcpyAsync(dev_rows, rows, size_t(cnt) * q, hipMemcpyHostToDevice, l->stream);
    if (e == hipSuccess && pw)
      e = hipMemcpyAsync(dev_pulls, pw, size_t(2 * cnt) * q * sizeof(uint32_t),
                         hipMemcpyHostToDevice, l->stream);
    if (e == hipSuccess) e = hipEventRecord(l->ev[slot], l->stream);
    if (e != hipSuccess) {
      l->broken = true;
      return fail(WLBM_EHIP, "schedule upload failed: %s", hipGetErrorString(e));
    }
    l->ev_pending[slot] = true;
    ++l->chunk_counter;
    for (int j = 0; j < cnt; ++j) {
      const int64_t k = done + j;
      const bool flux = k >= flux_from;
      // steps k .. k+K-1 in one launch (all in this chunk, none in a flux
      // window)
      const int K = int(std::min<int64_t>({int64_t(k_max), int64_t(cnt - j), flux_from - k}));
      if (fuse && K >= 2) {
        FusedArgs a2{};
        a2.e_in = l->ptr(l->c.e[l->cur]);
        a2.e_out = l->ptr(l->c.e[1 - l->cur]);
        a2.E_in = l->ptr(l->c.E[l->cur]);
        a2.E_out = l->ptr(l->c.E[1 - l->cur]);
        a2.Wf = a.Wf;
        a2.pulls = dev_pulls + size_t(2 * j) * q;
        for (int m = 0; m < K; ++m) a2.sels[m] = dev_pulls + size_t(2 * (j + m) + 1) * q;
        a2.wtab = a.wtab;
        a2.W = a.W;
        a2.nx = a.nx;
        a2.ny = a.ny;
        a2.q = q;
        a2.pitch = a.pitch;
        a2.plane = a.plane;
        e = hipSuccess;
        RowTuner& tu = l->tuner[l->per_cell ? 1 : 0][K];
        if (tu.ncand == 0) tu.ncand = fused_row_candidates(a.ny, K, tu.cand, RowTuner::kMaxCand);
        const bool timing = tu.chosen == 0;
        const int ci = (tu.next / RowTuner::kSample) % tu.ncand;
        const int phase = tu.next % RowTuner::kSample;
        const bool first_pass = tu.next < RowTuner::kSample * tu.ncand;
        a2.rows = timing ? tu.cand[ci] : tu.chosen;
        a2.strips_x = fused_strips_x(a.nx, K);
        a2.strips_y = (a.ny + a2.rows - 1) / a2.rows;
        if (refresh_ghosts) {
          e = fill_ghosts(l->ptr(l->c.e[l->cur]), a.plane, q, a.nx, a.ny, a.pitch, l->stream);
          if (e == hipSuccess)
            e = fill_ghosts(l->ptr(l->c.E[l->cur]), a.plane, 1, a.nx, a.ny, a.pitch, l->stream);
          if (e == hipSuccess && l->per_cell)
            e = fill_ghosts(l->ptr(l->c.Wf), a.plane, 1, a.nx, a.ny, a.pitch, l->stream);
          refresh_ghosts = false;
        }
        if (e == hipSuccess) e = launch_fused(a2, K, l->per_cell, l->stream);
        if (e == hipSuccess && timing) {
          if (phase == 0) {
            e = hipEventRecord(l->tev[0], l->stream);
          } else if (phase == RowTuner::kSample - 1) {
            float ms = 0.f;
            e = hipEventRecord(l->tev[1], l->stream);
            if (e == hipSuccess) e = hipEventSynchronize(l->tev[1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, l->tev[0], l->tev[1]);
            if (first_pass || ms < tu.ms[ci]) tu.ms[ci] = ms;
          }
          if (e == hipSuccess && ++tu.next == RowTuner::kPasses * RowTuner::kSample * tu.ncand) {
            int b = 0;
            for (int c = 1; c < tu.ncand; ++c)
              if (tu.ms[c] < tu.ms[b]) b = c;
            tu.chosen = tu.cand[b];
          }
        }
        if (e != hipSuccess) {
          l->broken = true;
          return fail(WLBM_EHIP, "fused step kernel launch failed: %s", hipGetErrorString(e));
        }
        l->cur = 1 - l->cur;
        j += K - 1;
        continue;
      }
      a.codes = reinterpret_cast<const uint32_t*>(dev_rows + size_t(j) * q);
      a.in_lo_hop = insums[4 * j];
      a.in_lo_all = insums[4 * j + 1];
      a.in_hi_hop = insums[4 * j + 2];
      a.in_hi_all = insums[4 * j + 3];
      if (tape) {
        float* in = k == 0 ? nullptr : reinterpret_cast<float*>(tape + size_t(k - 1) * slot_bytes);
        float* out = reinterpret_cast<float*>(tape + size_t(k) * slot_bytes);
        a.e_in = in ? in : l->ptr(l->c.e[l->cur]);
        a.E_in = in ? in + size_t(q) * l->g.plane : l->ptr(l->c.E[l->cur]);
        a.e_out = out;
        a.E_out = out + size_t(q) * l->g.plane;
      } else {
        a.e_in = l->ptr(l->c.e[l->cur]);
        a.e_out = l->ptr(l->c.e[1 - l->cur]);
        a.E_in = l->ptr(l->c.E[l->cur]);
        a.E_out = l->ptr(l->c.E[1 - l->cur]);
      }
      a.q_first = (flux && k == flux_from) ? 1 : 0;
      e = launch_step(a, l->split, l->per_cell, flux, l->stream);
      if (e == hipSuccess)
        e = launch_apply_sources(l->g, a.e_out, a.E_out, l->src_cells, l->src_vals, l->nsrc,
                                 l->stream);
      if (e != hipSuccess) {
        l->broken = true;
        return fail(WLBM_EHIP, "step kernel launch failed: %s", hipGetErrorString(e));
      }
      if (!tape) l->cur = 1 - l->cur;
      refresh_ghosts = true;
    }
    done += cnt;
  }
  if (tape) {
    const char* last = tape + size_t(nsteps - 1) * slot_bytes;
    const size_t pbytes = size_t(l->g.plane) * sizeof(float);
    hipError_t e = hipMemcpyAsync(l->ptr(l->c.e[l->cur]), last, pbytes * q,
                                  hipMemcpyDeviceToDevice, l->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(l->ptr(l->c.E[l->cur]), last + pbytes * q, pbytes,
                         hipMemcpyDeviceToDevice, l->stream);
    if (e != hipSuccess) {
      l->broken = true;
      return fail(WLBM_EHIP, "tape copy failed: %s", hipGetErrorString(e));
    }
  }
  l->flux_valid = l->flux_window > 0 && nsteps >= l->flux_window;
  return WLBM_OK;
}

wlbm_status check_steps(const wlbm_lattice* l, int64_t nsteps) {
  if (nsteps < 0) return fail(WLBM_EINVAL, "nsteps must be >= 0");
  if (l->tas.n + nsteps > kMaxSteps) return fail(WLBM_EINVAL, "step count would exceed 2^31 - 1");
  return WLBM_OK;
}

}  // namespace

extern "C" {

wlbm_status wlbm_step(wlbm_lattice* l, int64_t nsteps) {
  wlbm_status st = check_lat(l);
  if (!st) st = check_steps(l, nsteps);
  if (st) return st;
  if (nsteps == 0) return WLBM_OK;
  return run_steps(l, nsteps, nullptr, 0);
}

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

wlbm_status wlbm_read_temperature(wlbm_lattice* l, float* d_T) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!d_T) return fail(WLBM_EINVAL, "T is NULL");
  HIP_TRY(launch_read_field(l->g, l->ptr(l->c.E[l->cur]), d_T, l->stream));
  return WLBM_OK;
}

wlbm_status wlbm_accumulate_temperature(wlbm_lattice* l, double scale, float* d_T) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!d_T) return fail(WLBM_EINVAL, "T is NULL");
  if (!std::isfinite(scale)) return fail(WLBM_EINVAL, "scale must be finite");
  HIP_TRY(launch_axpy_field(l->g, float(scale), l->ptr(l->c.E[l->cur]), d_T, l->stream));
  return WLBM_OK;
}

wlbm_status wlbm_read_heat_flux(wlbm_lattice* l, float* d_qx, float* d_qy, int32_t averaged) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!d_qx || !d_qy) return fail(WLBM_EINVAL, "flux outputs must not be NULL");
  if (averaged) {
    if (!l->flux_valid)
      return fail(WLBM_ESTATE, "no complete flux window: set one and step at least that far");
    HIP_TRY(launch_scale_pair(l->g.nx * l->g.ny, l->ptr(l->c.qsx), l->ptr(l->c.qsy),
                              1.0f / float(l->flux_window), d_qx, d_qy, l->stream));
  } else {
    HIP_TRY(launch_read_flux(l->g, l->ptr(l->c.e[l->cur]), l->ptr(l->c.sxtab),
                             l->ptr(l->c.sytab), d_qx, d_qy, l->stream));
  }
  return WLBM_OK;
}

wlbm_status wlbm_read_populations(wlbm_lattice* l, float* d_e) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (!d_e) return fail(WLBM_EINVAL, "populations pointer is NULL");
  HIP_TRY(launch_read_populations(l->g, l->ptr(l->c.e[l->cur]), d_e, l->stream));
  return WLBM_OK;
}

wlbm_status wlbm_read_totals(wlbm_lattice* l, double* energy, double* qx_sum, double* qy_sum) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  double* dev = reinterpret_cast<double*>(l->ws + l->c.totals);
  HIP_TRY(launch_totals(l->g, l->ptr(l->c.e[l->cur]), l->ptr(l->c.E[l->cur]),
                        l->ptr(l->c.sxtab), l->ptr(l->c.sytab),
                        reinterpret_cast<double*>(l->ws + l->c.partials), kReduceBlocks, dev,
                        l->stream));
  double h[3];
  HIP_TRY(hipMemcpyAsync(h, dev, sizeof(h), hipMemcpyDeviceToHost, l->stream));
  HIP_TRY(hipStreamSynchronize(l->stream));
  if (energy) *energy = h[0];
  if (qx_sum) *qx_sum = h[1];
  if (qy_sum) *qy_sum = h[2];
  if (!std::isfinite(h[0]) || !std::isfinite(h[1]) || !std::isfinite(h[2]))
    return fail(WLBM_ENONFINITE, "non-finite totals: energy %g, qx %g, qy %g", h[0], h[1], h[2]);
  return WLBM_OK;
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

int32_t wlbm_get_block_rows(const wlbm_lattice* l, int32_t k) {
  if (!l || k < 2 || k > 4) return -1;
  return l->tuner[l->per_cell ? 1 : 0][k].chosen;
}

wlbm_status wlbm_set_block_rows(wlbm_lattice* l, int32_t k, int32_t rows) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (k < 2 || k > 4) return fail(WLBM_EINVAL, "k must be 2, 3 or 4 (got %d)", k);
  if (rows < 0 || rows > 62 || (rows > 0 && (rows + 2 * (k - 1)) % 3 != 0))
    return fail(WLBM_EINVAL,
                "rows must be 0 or 1 .. 62 with rows + 2 (k - 1) a multiple of 3 (got %d)", rows);
  RowTuner& tu = l->tuner[l->per_cell ? 1 : 0][k];
  tu.next = 0;
  tu.chosen = rows;
  return WLBM_OK;
}

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


wlbm_status wlbm_read_flux_mean(wlbm_lattice* l, int32_t x0, int32_t x1, int32_t averaged,
                                double* qx_mean, double* qy_mean) {
  wlbm_status st = check_lat(l);
  if (st) return st;
  if (x0 < 0 || x1 > l->g.nx || x0 >= x1)
    return fail(WLBM_EINVAL, "columns must satisfy 0 <= x0 < x1 <= nx");
  if (averaged && !l->flux_valid)
    return fail(WLBM_ESTATE, "no complete flux window: set one and step at least that far");
  double* dev = reinterpret_cast<double*>(l->ws + l->c.totals);
  HIP_TRY(launch_flux_sum(l->g, l->ptr(l->c.e[l->cur]), l->ptr(l->c.sxtab), l->ptr(l->c.sytab),
                          l->ptr(l->c.qsx), l->ptr(l->c.qsy), averaged ? 1 : 0, x0, x1,
                          reinterpret_cast<double*>(l->ws + l->c.partials), kReduceBlocks, dev,
                          l->stream));
  double h[3];
  HIP_TRY(hipMemcpyAsync(h, dev, sizeof(h), hipMemcpyDeviceToHost, l->stream));
  HIP_TRY(hipStreamSynchronize(l->stream));
  const double scale = 1.0 / (double(x1 - x0) * l->g.ny * (averaged ? l->flux_window : 1));
  if (qx_mean) *qx_mean = h[0] * scale;
  if (qy_mean) *qy_mean = h[1] * scale;
  if (!std::isfinite(h[0]) || !std::isfinite(h[1]))
    return fail(WLBM_ENONFINITE, "non-finite flux sums");
  return WLBM_OK;
}

int64_t wlbm_step_count(const wlbm_lattice* l) { return l ? l->tas.n : -1; }

const char* wlbm_last_error(void) { return g_last_error.c_str(); }

wlbm_status wlbm_destroy(wlbm_lattice* l) {
  if (!l) return WLBM_OK;
  hipError_t e = hipStreamSynchronize(l->stream);
  for (int k = 0; k < 2; ++k) {
    if (l->pinned[k]) (void)hipHostFree(l->pinned[k]);
    if (l->pinned_pulls[k]) (void)hipHostFree(l->pinned_pulls[k]);
    if (l->ev[k]) (void)hipEventDestroy(l->ev[k]);
    if (l->tev[k]) (void)hipEventDestroy(l->tev[k]);
  }
  delete l;
  if (e != hipSuccess) return fail(WLBM_EHIP, "stream sync at destroy: %s", hipGetErrorString(e));
  return WLBM_OK;
}

}  // extern "C"
