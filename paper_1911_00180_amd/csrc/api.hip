// C-ABI of libwormlbm.so (declared in include/wormlbm.h): parameters, lattice
// set-up, stepping and readout.  Saved states and the adjoint are in
// api_states.hip, batches in api_batch.hip, launch configuration and tuning
// in api_tune.hip.
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

#include "api_internal.hpp"

namespace wlbm {

namespace {
thread_local std::string g_last_error;
}  // namespace

wlbm_status fail(wlbm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

const char* last_error_text() { return g_last_error.c_str(); }

bool fusable(const wlbm_params& p) {
  // every edge type except partly specular y walls
  const bool walls_ok = p.y_edge != WLBM_EDGE_DIFFUSE || p.y_specularity == 0.0;
  return walls_ok && fused_supported(p.q, p.nx, p.ny);
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
  // flux-window sums in float64: windows run to millions of steps
  c.qsx = take(2 * cells);
  c.qsy = take(2 * cells);
  c.partials = take(size_t(kReduceBlocks) * 3 * sizeof(double));
  c.totals = take(4 * sizeof(double));
  c.flag = take(sizeof(int));
  c.sched = take(size_t(2) * chunk_steps(p) * size_t(p.q));
  // per step, the multi-step kernels' pull offsets and selection-table
  // offsets of every direction (FusedArgs::pulls, FusedArgs::sels)
  c.pulls = take(size_t(4) * chunk_steps(p) * size_t(p.q) * sizeof(uint32_t));
  // per step, the inward-weight sums of diffuse walls (FusedArgs::ins)
  c.ins = take(fusable(p) ? size_t(2) * chunk_steps(p) * 4 * sizeof(float) : 0);
  c.wtab = take(size_t(p.q) * sizeof(float));
  c.sxtab = take(size_t(p.q) * sizeof(float));
  c.sytab = take(size_t(p.q) * sizeof(float));
  c.mtab = take(size_t(p.q) * sizeof(int));
  c.total = off;
  return c;
}

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


wlbm_status check_lat(const wlbm_lattice* l) {
  if (!l) return fail(WLBM_EINVAL, "lattice is NULL");
  if (l->broken) return fail(WLBM_ESTATE, "lattice is unusable after an earlier HIP error");
  return WLBM_OK;
}

wlbm_status check_steps(const wlbm_lattice* l, int64_t nsteps) {
  if (nsteps < 0) return fail(WLBM_EINVAL, "nsteps must be >= 0");
  if (l->tas.n + nsteps > kMaxSteps) return fail(WLBM_EINVAL, "step count would exceed 2^31 - 1");
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

bool lattice_fuses(const wlbm_lattice* l) {
  return l->p.step_fusion != 0 && l->nsrc == 0 && fusable(l->p);
}

// Along a diffuse wall the dependence reaches two columns per step, which
// the ghost frame of a periodic x edge covers for two steps per launch; q
// above 128 runs at most two steps per launch.
int fused_k_cap(const wlbm_lattice* l) {
  if (l->p.q > 128) return 2;   // 16 waves of 16 directions: registers for two levels
  return (l->g.x_edge == kPeriodic && l->g.y_edge == kDiffuse) ? 2 : 4;
}

// Automatic steps per launch, from measurements on MI355X: periodic
// lattices gain up to four steps (1024^2 x 64: 1, 2, 3, 4 steps 552, 1001,
// 1338, 1648 G updates/s); lattices with walls run a kernel with more
// registers, and with q above 64 (16 directions a wave) or a per-cell field
// two steps were fastest (512 x 256 x 128 diffuse film: 1, 2, 3, 4 steps 291,
// 551, 426, 425 G updates/s).
int fused_k_max(const wlbm_lattice* l) {
  const bool walls = l->g.x_edge != kPeriodic || l->g.y_edge != kPeriodic;
  const int k_auto = walls && (l->p.q > 64 || l->per_cell) ? 2 : 4;
  return std::min(fused_k_cap(l), l->p.step_fusion == 1 ? k_auto : l->p.step_fusion);
}

}  // namespace wlbm

using namespace wlbm;

namespace {

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
  {
    // the device that holds the workspace (the caller's current device if
    // the runtime cannot tell)
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, d_workspace) != hipSuccess ||
        attr.type != hipMemoryTypeDevice || attr.device < 0) {
      (void)hipGetLastError();
      if (hipGetDevice(&attr.device) != hipSuccess) attr.device = 0;
    }
    l->device = attr.device;
  }
  l->c = carve(*p);
  l->chunk = chunk_steps(*p);
  l->W = float(uniform_wcorr(*p, l->dirs.lambda_corr, nullptr));
  l->walls = {float(p->t_x_lo), float(p->t_x_hi), float(p->t_y_lo), float(p->t_y_hi)};
  l->g = {p->nx, p->ny, p->q, padded_pitch(p->nx), padded_plane(p->nx, p->ny), p->x_edge,
          p->y_edge};
  l->split = p->dir_split ? p->dir_split : auto_split(p->q);

  auto cleanup = [&](wlbm_status s) {
    for (int k = 0; k < 2; ++k) {
      if (l->pinned[k]) (void)hipHostFree(l->pinned[k]);
      if (l->pinned_pulls[k]) (void)hipHostFree(l->pinned_pulls[k]);
      if (l->pinned_ins[k]) (void)hipHostFree(l->pinned_ins[k]);
      if (l->ev[k]) (void)hipEventDestroy(l->ev[k]);
    }
    delete l;
    return s;
  };
  const size_t stage = std::max<size_t>(size_t(l->chunk) * p->q, 4 * size_t(p->q) * sizeof(float));
  for (int k = 0; k < 2; ++k) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&l->pinned[k]), stage, hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&l->pinned_pulls[k]),
                        size_t(2) * l->chunk * p->q * sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess && fusable(*p))
      e = hipHostMalloc(reinterpret_cast<void**>(&l->pinned_ins[k]),
                        size_t(l->chunk) * 4 * sizeof(float), hipHostMallocDefault);
    if (e != hipSuccess) {
      wlbm_status s = fail(WLBM_ENOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
      return cleanup(s);
    }
    e = hipEventCreateWithFlags(&l->ev[k], hipEventDisableTiming);
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
  const wlbm_status ns = noalloc_setup(l->device);
  if (ns) return cleanup(ns);
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
  l->ghosts_full = false;
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
  l->ghosts_full = false;
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
  l->wf_ghosts_full = false;
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
  l->ghosts_full = false;
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

namespace wlbm {

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
  a.q = q;
  a.pitch = l->g.pitch;
  a.plane = l->g.plane;
  a.x_edge = l->g.x_edge;
  a.y_edge = l->g.y_edge;
  a.tiles_x = tiles_x_for(l->g.nx);
  a.ntiles = a.tiles_x * tiles_y_for(l->g.ny, l->split);
  // several steps per launch: not into a tape, and a lattice the multi-step
  // kernels are built for
  const bool fuse = !tape && lattice_fuses(l);
  const int k_max = fused_k_max(l);

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
    // with it, per step and direction, the pull offset and the selection-table
    // offset (FusedArgs::pulls / sels, StepArgs::pulls / sels)
    uint32_t* pw = l->pinned_pulls[slot];
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
    float* dev_ins = reinterpret_cast<float*>(l->ws + l->c.ins) + size_t(slot) * l->chunk * 4;
    hipError_t e = hipMemcpyAsync(dev_rows, rows, size_t(cnt) * q, hipMemcpyHostToDevice, l->stream);
    if (e == hipSuccess && pw)
      e = hipMemcpyAsync(dev_pulls, pw, size_t(2 * cnt) * q * sizeof(uint32_t),
                         hipMemcpyHostToDevice, l->stream);
    if (e == hipSuccess && fuse) {
      std::memcpy(l->pinned_ins[slot], insums.data(), size_t(cnt) * 4 * sizeof(float));
      e = hipMemcpyAsync(dev_ins, l->pinned_ins[slot], size_t(cnt) * 4 * sizeof(float),
                         hipMemcpyHostToDevice, l->stream);
    }
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
      // steps k .. k+K-1 in one launch (all in this chunk); those in the
      // flux window add their heat flux to the window's sums in the launch
      const int K = int(std::min<int64_t>(k_max, cnt - j));
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
        a2.rows = block_rows_for(l, K);
        a2.strips_x = fused_strips_x(a.nx, K);
        a2.strips_y = (a.ny + a2.rows - 1) / a2.rows;
        a2.x_edge = a.x_edge;
        a2.y_edge = a.y_edge;
        a2.t_x_lo = a.t_x_lo;
        a2.t_x_hi = a.t_x_hi;
        a2.t_y_lo = a.t_y_lo;
        a2.t_y_hi = a.t_y_hi;
        a2.codes = reinterpret_cast<const uint32_t*>(dev_rows + size_t(j) * q);
        a2.ins = dev_ins + size_t(4) * j;
        for (int m = 0; m < K; ++m)
          if (k + m >= flux_from) a2.flux_levels |= 1u << m;
        a2.flux_first = (flux_from >= k && flux_from < k + K) ? int(flux_from - k) + 1 : 0;
        a2.qsx = a.qsx;
        a2.qsy = a.qsy;
        a2.sxtab = a.sxtab;
        a2.sytab = a.sytab;
        e = hipSuccess;
        // the multi-step kernels read kGhost ghost columns of periodic x
        // edges, which other producers do not write: refresh the frame once
        // before the first multi-step launch that follows them
        const bool px = a.x_edge == kPeriodic, py = a.y_edge == kPeriodic;
        if (!l->ghosts_full) {
          e = fill_ghosts(l->ptr(l->c.e[l->cur]), a.plane, q, a.nx, a.ny, a.pitch, px, py,
                          l->stream);
          if (e == hipSuccess)
            e = fill_ghosts(l->ptr(l->c.E[l->cur]), a.plane, 1, a.nx, a.ny, a.pitch, px, py,
                            l->stream);
        }
        if (e == hipSuccess && l->per_cell && !l->wf_ghosts_full) {
          e = fill_ghosts(l->ptr(l->c.Wf), a.plane, 1, a.nx, a.ny, a.pitch, px, py, l->stream);
          if (e == hipSuccess) l->wf_ghosts_full = true;
        }
        if (e == hipSuccess)
          e = launch_fused(a2, K, l->per_cell, a2.flux_levels != 0, l->stream);
        if (e != hipSuccess) {
          l->broken = true;
          return fail(WLBM_EHIP, "fused step kernel launch failed: %s", hipGetErrorString(e));
        }
        l->cur = 1 - l->cur;
        l->ghosts_full = true;   // the kernel writes the whole frame of its output
        j += K - 1;
        continue;
      }
      a.codes = reinterpret_cast<const uint32_t*>(dev_rows + size_t(j) * q);
      a.pulls = dev_pulls + size_t(2 * j) * q;
      a.sels = dev_pulls + size_t(2 * j + 1) * q;
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
      l->ghosts_full = false;
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

}  // namespace wlbm

extern "C" {

wlbm_status wlbm_step(wlbm_lattice* l, int64_t nsteps) {
  wlbm_status st = check_lat(l);
  if (!st) st = check_steps(l, nsteps);
  if (st) return st;
  if (nsteps == 0) return WLBM_OK;
  return run_steps(l, nsteps, nullptr, 0);
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
    HIP_TRY(launch_scale_pair(l->g.nx * l->g.ny, l->dptr(l->c.qsx), l->dptr(l->c.qsy),
                              1.0 / double(l->flux_window), d_qx, d_qy, l->stream));
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
                          l->dptr(l->c.qsx), l->dptr(l->c.qsy), averaged ? 1 : 0, x0, x1,
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

const char* wlbm_last_error(void) { return wlbm::last_error_text(); }

wlbm_status wlbm_destroy(wlbm_lattice* l) {
  if (!l) return WLBM_OK;
  hipError_t e = hipStreamSynchronize(l->stream);
  for (int k = 0; k < 2; ++k) {
    if (l->pinned[k]) (void)hipHostFree(l->pinned[k]);
    if (l->pinned_pulls[k]) (void)hipHostFree(l->pinned_pulls[k]);
    if (l->pinned_ins[k]) (void)hipHostFree(l->pinned_ins[k]);
    if (l->ev[k]) (void)hipEventDestroy(l->ev[k]);
  }
  delete l;
  if (e != hipSuccess) return fail(WLBM_EHIP, "stream sync at destroy: %s", hipGetErrorString(e));
  return WLBM_OK;
}

}  // extern "C"
