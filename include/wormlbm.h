/*
 * wormlbm.h -- C-ABI of the MI355X worm-LBM library (libwormlbm.so).
 *
 * The library advances the worm lattice Boltzmann method for the gray phonon
 * Boltzmann transport equation on one AMD Instinct MI355X (gfx950):
 * Hammer, Fritz, Bedoya-Martinez, "The worm-LBM, an algorithm for a high
 * number of propagation directions on a lattice Boltzmann grid: the case of
 * phonon transport", arXiv:1911.00180.  Section and equation names below are
 * those of that paper.
 *
 * Units are lattice units: one cell per axial hop, one time step per hop,
 * group velocity 1.  The mean free path (MFP) is given in cells, so the
 * relaxation weight of Eq. W-Kn is W = 1 / MFP.  Temperatures are in the
 * linearised gray model e_eq = T (unit heat capacity), so T = sum_i e_i.
 *
 * Memory.  The caller owns every device buffer: the workspace (size from
 * wlbm_workspace_bytes) and all input/output arrays.  Pointers named d_* are
 * device pointers, the others host pointers.  The library never allocates or
 * frees device memory; it allocates a small amount of pinned host memory per
 * lattice for schedule uploads, freed by wlbm_destroy.  The workspace must
 * stay valid until wlbm_destroy.  Device arrays are row-major float32:
 * fields are [ny][nx] (x fastest), populations are [q][ny][nx].
 *
 * Streams.  All device work of a lattice is enqueued on the HIP stream given
 * at creation (or by wlbm_set_stream), as a hipStream_t passed as void*;
 * NULL means the default stream.  Reads complete in stream order; only
 * wlbm_read_totals, wlbm_set_mfp_field and wlbm_step (once per schedule chunk,
 * to recycle its pinned staging buffer) wait on the host.
 *
 * Errors.  Every call returns a wlbm_status.  Invalid arguments are reported
 * synchronously; a HIP runtime error is reported as WLBM_EHIP by the call that
 * sees it.  wlbm_last_error() returns a thread-local message for the last
 * failing call of the calling thread.  A lattice handle must not be used from
 * two threads at once.
 */
#ifndef WORMLBM_H
#define WORMLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden visibility; these declarations are its
 * exported interface. */
#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility push(default)
#endif

typedef struct wlbm_lattice wlbm_lattice;
typedef struct wlbm_batch wlbm_batch;

typedef enum wlbm_status {
  WLBM_OK = 0,
  WLBM_EINVAL = -1,      /* bad argument or parameter                           */
  WLBM_EUNSTABLE = -2,   /* corrected relaxation weight above 1 (App. A)        */
  WLBM_ENOMEM = -3,      /* workspace too small, or pinned host memory failed   */
  WLBM_EHIP = -4,        /* HIP runtime error                                   */
  WLBM_ENONFINITE = -5,  /* non-finite values found by a readout                */
  WLBM_ESTATE = -6       /* call not valid in the current state                 */
} wlbm_status;

/* Edge types (Sec. 2.6).  x edges: periodic or blackbody.  y edges: periodic,
 * blackbody or adiabatic diffuse.  Both edges of an axis have the same type. */
enum {
  WLBM_EDGE_PERIODIC = 0,
  WLBM_EDGE_BLACKBODY = 1,
  WLBM_EDGE_DIFFUSE = 2
};

/* Direction sets (Sec. 2.4).  UNIFORM: Q directions evenly spaced in angle,
 * theta_i = 2 pi i / Q, weights 1/Q.  RING: the D2Q[M x 8] lattice vectors of
 * the square ring max(|Vx|,|Vy|) = M, M = Q/8, counter-clockwise from (M, 0),
 * weights from the angular gaps (Eq. weight).  Direction i of either set has
 * the index i in every [q] array of this interface. */
enum {
  WLBM_DIRS_UNIFORM = 0,
  WLBM_DIRS_RING = 1
};

typedef struct wlbm_params {
  int32_t nx, ny;            /* lattice size, 1 .. 2^20 each; 8 padded planes    */
                             /* of (nx+64)*(ny+2) floats must fit in 4 GiB       */
  int32_t q;                 /* number of directions, multiple of 8, 8 .. 1024   */
  int32_t dirs;              /* WLBM_DIRS_*                                      */
  double mfp_cells;          /* uniform MFP in cells (> 0; +inf gives W = 0)     */
  int32_t emulate_3d;        /* 1: factor 3/2 of Eq. W-correction                */
  int32_t mfp_correction;    /* 1: Eq. W-correction applied; 0: plain W          */
  int32_t x_edge, y_edge;    /* WLBM_EDGE_*                                      */
  double t_x_lo, t_x_hi;     /* blackbody temperatures at x = 0 and x = nx-1     */
  double t_y_lo, t_y_hi;     /* blackbody temperatures at y = 0 and y = ny-1     */
  int32_t dir_split;         /* waves sharing one cell's directions: 0 (auto),   */
                             /* 1, 2 or 4; q must be a multiple of 8*dir_split   */
  int32_t sched_chunk;       /* steps per schedule upload: 0 (auto) or 16..65536; */
                             /* the workspace holds two chunks of q bytes per    */
                             /* step, and of 2 q 32-bit words per step when the  */
                             /* multi-step kernels apply (both edges periodic)   */
  double y_specularity;      /* diffuse y walls: fraction p in [0, 1] of what    */
                             /* crosses them that is reflected specularly        */
                             /* (Eq. adiabatic-specular); 1 - p is scattered     */
                             /* diffusely (Eq. adiabatic-diffuse)                */
  int32_t step_fusion;       /* time steps per kernel launch where possible      */
                             /* (any edges but partly specular walls, no         */
                             /* sources, q a multiple of 8 up to 128, or 192 or  */
                             /* 256, nx >= 8, ny >= 2, outside tapes; q above    */
                             /* 128, and periodic x with diffuse y: at most      */
                             /* two): 1 =                                        */
                             /* automatic (up to four), 2 .. 4 = at most that    */
                             /* many, 0 = one step per launch.  Results are      */
                             /* identical to single steps in every case.         */
  int32_t reserved[3];       /* must be zero                                     */
} wlbm_params;

/* Fill *p with defaults: 64 x 64, q = 16, uniform directions, MFP 16, f = 1,
 * correction on, all edges periodic, wall temperatures 0, automatic tiling,
 * fully diffuse walls (y_specularity 0), step fusion on. */
void wlbm_default_params(wlbm_params* p);

/* Bytes of device workspace needed for the lattice described by *p.  Host
 * only; valid without a GPU.  Returns WLBM_EINVAL for invalid parameters and
 * WLBM_EUNSTABLE if the uniform corrected weight exceeds 1. */
wlbm_status wlbm_workspace_bytes(const wlbm_params* p, size_t* bytes);

/* Create a lattice in the caller's workspace d_workspace (at least
 * wlbm_workspace_bytes bytes, 256-byte aligned).  Builds the direction tables
 * and relaxation constants (Sec. 2.2-2.5), clears the workspace on `stream`,
 * and leaves all populations zero.  No step is taken.  *out receives the
 * handle, owned by the caller until wlbm_destroy. */
wlbm_status wlbm_create(const wlbm_params* p, void* d_workspace, size_t ws_bytes,
                        void* stream, wlbm_lattice** out);

/* Change the stream used by later calls. */
wlbm_status wlbm_set_stream(wlbm_lattice* lat, void* stream);

/* Initial condition e_i = w_i T0 (Sec. 2.4: the weights set initial and
 * boundary conditions), then the blackbody walls are imposed.  d_T0 is a
 * device [ny][nx] float array, read in stream order. */
wlbm_status wlbm_set_temperature(wlbm_lattice* lat, const float* d_T0);

/* Set all populations from a device [q][ny][nx] array, then impose the
 * blackbody walls.  The populations are the directional energy densities
 * (DDEDs) e_i of Sec. 2.2 Eq. discrete-BTE, one per cell and direction; their
 * sum over i is the cell energy E of Eq. lbm-energy-density.  The array is
 * read in stream order and stays the caller's. */
wlbm_status wlbm_set_populations(wlbm_lattice* lat, const float* d_e);

/* Per-cell mean free path in cells (device [ny][nx]); each cell then relaxes
 * with its own corrected weight: W = 1/MFP (Sec. 2.2 Eq. W-Kn, with the group
 * velocity and time step 1), corrected by Eq. W-correction with the
 * Lambda_corr of Eq. W-correction-factor-gereralized (Sec. 2.4).  The DDED
 * that stays or hops relaxes with the weight of its source cell, and a cell
 * emits its EED with its own weight (the paper has a uniform W; this is the
 * reading taken for a field).  NULL returns to the uniform MFP of the
 * parameters.  Waits for the stream; returns WLBM_EUNSTABLE (and keeps the
 * previous field) if any corrected weight exceeds 1 or is not finite, or if
 * an MFP is not positive. */
wlbm_status wlbm_set_mfp_field(wlbm_lattice* lat, const float* d_mfp);

/* Internal sources (Sec. 2.6, Eq. isotropic and Eq. anisotropic): the DDEDs
 * of n distinct cells d_cells (device [n][2] int32, (x, y)) are overwritten
 * by d_values (device [n][q] float) after every step, after the blackbody
 * walls (a source on a wall cell wins), and now and at every later
 * initialisation.  An isotropic blackbody source at T has values w_i T; a
 * flux source the values of wlbm_flux_distribution.  The arrays stay the
 * caller's and must remain valid and unchanged while set; n = 0 removes the
 * sources.  Waits for the stream (the cells are checked on the host:
 * WLBM_EINVAL for a cell outside the lattice or listed twice). */
wlbm_status wlbm_set_sources(wlbm_lattice* lat, int32_t n, const int32_t* d_cells,
                             const float* d_values);

/* Angle-dependent grid speed (Sec. 2.3: the TAS can impose any
 * direction-dependent velocity): host [q] speeds v_i in (0, 1] cells per step
 * (NULL: 1 for all, the isotropic TAS).  Direction i then hops iff
 * |P_i + s_i|^2 <= (v_i n + 1)^2 at step n (float64; the integer rule for
 * v_i = 1).  The relaxation weight is unchanged.  Only at step 0
 * (WLBM_ESTATE otherwise). */
wlbm_status wlbm_set_speeds(wlbm_lattice* lat, const double* speeds);

/* Change the blackbody wall temperatures (Sec. 2.6 allows time-dependent
 * boundary values).  Takes effect from the next step. */
wlbm_status wlbm_set_wall_temperatures(wlbm_lattice* lat, double t_x_lo, double t_x_hi,
                                       double t_y_lo, double t_y_hi);

/* Number of trailing steps of each wlbm_step call over which the heat flux is
 * accumulated for wlbm_read_heat_flux(..., averaged = 1); 0 disables it
 * (default).  Sec. 3.4 averages the flux over ten steps.  The per-cell sums
 * are kept in float64 (a float32 sum over a million steps can be off by
 * 1e-3 of its value).  Steps of a window run several per launch as other
 * steps do (the launch adds the flux of each of its window steps, with the
 * bits of single steps). */
wlbm_status wlbm_set_flux_window(wlbm_lattice* lat, int32_t window);

/* Advance nsteps >= 0 time steps of the worm-LBM: for every cell and
 * direction, BGK relaxation towards w_i sum_j e_j with the corrected weight
 * and streaming along the worm path with TAS pauses (Eq. algorithm,
 * Eq. worm-paths), followed by the wall conditions.  The step count after
 * the call must stay below 2^31. */
wlbm_status wlbm_step(wlbm_lattice* lat, int64_t nsteps);

/* Pseudo-temperature T = sum_i e_i (Eq. pseudo-T, linear gray model) into a
 * device [ny][nx] array. */
wlbm_status wlbm_read_temperature(wlbm_lattice* lat, float* d_T);

/* d_T += scale * T (device [ny][nx]): superposition of uncoupled gray runs
 * (the multigray approach of Sec. 2.2), one call per band. */
wlbm_status wlbm_accumulate_temperature(wlbm_lattice* lat, double scale, float* d_T);

/* Heat flux q = sum_i e_i s_i (Eq. q_corr, v_g = 1) into device [ny][nx]
 * arrays.  averaged = 0: the current state.  averaged = 1: the mean over the
 * trailing flux window of the last wlbm_step call (WLBM_ESTATE if that call
 * ran fewer steps than the window, or no window is set). */
wlbm_status wlbm_read_heat_flux(wlbm_lattice* lat, float* d_qx, float* d_qy, int32_t averaged);

/* Copy all populations into a device [q][ny][nx] array. */
wlbm_status wlbm_read_populations(wlbm_lattice* lat, float* d_e);

/* Totals over the lattice, accumulated in float64 in a fixed order (so the
 * result is reproducible): energy = sum_x T(x), with T = E = sum_i e_i
 * (Sec. 2.2 Eq. lbm-energy-density, Eq. pseudo-T in the linear gray model),
 * and qx_sum, qy_sum = sum_x q(x), q = sum_i e_i s_i (Eq. q_corr).
 * Waits for the stream.  WLBM_ENONFINITE if any of them is not finite.
 * Output pointers may be NULL. */
wlbm_status wlbm_read_totals(wlbm_lattice* lat, double* energy, double* qx_sum, double* qy_sum);

/* For callers that cannot allocate or wait (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the totals of
 * wlbm_read_totals, written in stream order to the caller's device buffer
 * d_totals ([3] float64: energy, qx_sum, qy_sum), with no host wait and no
 * finiteness check.  Same kernels and summation order as wlbm_read_totals,
 * so the values are identical.  The float64 block partials live in a fixed
 * array of the library (24 KiB per GPU, looked up at wlbm_create and held
 * until the process ends) instead of the lattice workspace; the reduction
 * uses at most its 1024 partials whatever the lattice size, so no size is
 * refused.  Every call on one GPU shares that array: calls that overlap on
 * one GPU (different streams, or threads) race and must be ordered by the
 * caller.  Nothing needs clearing between calls (each call writes every
 * partial it reads).  The call allocates nothing and calls no allocating
 * routine. */
wlbm_status wlbm_read_totals_noalloc(wlbm_lattice* lat, double* d_totals);

/* Mean heat flux over the columns x0 <= x < x1 and all rows, summed in
 * float64 in a fixed order: of the trailing flux window of the last
 * wlbm_step call (averaged = 1; WLBM_ESTATE without a complete window) or of
 * the current state (averaged = 0).  Sec. 3.5 takes the in-plane flux of a
 * film from such averages (over ten steps, as stated in Sec. 3.4).  Waits for the stream.  Outputs may be NULL. */
wlbm_status wlbm_read_flux_mean(wlbm_lattice* lat, int32_t x0, int32_t x1, int32_t averaged,
                                double* qx_mean, double* qy_mean);

/* Host-side tables, valid without a GPU (they need only the parameters). */

/* Unit vectors (sx, sy) and weights w of the q directions, host [q] arrays
 * (any may be NULL): evenly spaced directions with weights 1/Q (Sec. 2.2), or
 * the D2Q[M x 8] ring set with the angular-gap weights of Sec. 2.4
 * Eq. weight.  These weights set the equilibrium w_i E of Eq. lbm-energy-
 * weighting and the imposed DDEDs of every boundary (Sec. 2.6). */
wlbm_status wlbm_get_directions(const wlbm_params* p, double* sx, double* sy, double* w);

/* Grid-MFP correction Lambda_corr = Q / sum_i c_i (Eq. W-correction-factor-
 * gereralized), W = 1/MFP and the corrected weight (Eq. W-correction). */
wlbm_status wlbm_get_constants(const wlbm_params* p, double* lambda_corr, double* w,
                               double* w_corr);

/* DDEDs of a flux boundary or source (Sec. 2.6, Eq. lbm-heat-flux) into a host
 * [q] array: the paper asks for the DDEDs to be prescribed uniquely; this is
 * the distribution linear in the direction, e_i = w_i (T + s_i . a), whose
 * energy sum_i e_i is T and whose flux sum_i e_i s_i is (qx, qy)
 * (a = M^-1 q, M = sum_i w_i s_i s_i^T; for evenly spaced directions
 * e_i = w_i (T + 2 q . s_i)).  Host only. */
wlbm_status wlbm_flux_distribution(const wlbm_params* p, double T, double qx, double qy,
                                   double* e);

/* Worm/TAS schedule of steps step0+1 .. step0+n into a host [n][q] int8 array
 * (speeds: host [q] grid speeds as for wlbm_set_speeds, or NULL for 1):
 * the D2Q8 move 1..8 (E, N, W, S, NE, NW, SW, SE) pending for each direction,
 * positive if the DDED hops on that step, negative if it pauses (Sec. 2.3
 * Eq. algorithm, Sec. 2.5 Eq. worm-paths).  If pos is not NULL it receives
 * the host [n][q][2] int64 worm positions after each step. */
wlbm_status wlbm_get_schedule(const wlbm_params* p, const double* speeds, int64_t step0,
                              int64_t n, int8_t* moves, int64_t* pos);

/* ---- Saved states (checkpoints) ------------------------------------------
 * A state is the lattice's padded population planes followed by its padded
 * E plane, wlbm_state_bytes bytes, in device memory owned by the caller.  Its
 * internal layout is not part of this interface; buffers move between calls
 * of this library only, for lattices created with the same parameters. */

/* Bytes of one saved state (a multiple of 256). */
wlbm_status wlbm_state_bytes(const wlbm_lattice* lat, size_t* bytes);

/* Copy the current state into d_buf (at least wlbm_state_bytes bytes), in
 * stream order. */
wlbm_status wlbm_save_state(wlbm_lattice* lat, void* d_buf, size_t bytes);

/* Make d_buf the current state and `step` the current step count (the
 * schedule continues from that step; step must be the step the state was
 * saved at for the result to be the same run).  In stream order. */
wlbm_status wlbm_load_state(wlbm_lattice* lat, const void* d_buf, size_t bytes, int64_t step);

/* As wlbm_step, and the state after each step is kept: step k (1-based) of
 * this call writes its output directly into slot k-1 of d_tape, slot j at
 * d_tape + j * slot_bytes (256-byte aligned, slot_bytes a multiple of 256 and
 * at least wlbm_state_bytes).  The tape must be zero-filled before its first
 * use: the library writes only the ghost copies of periodic edges, and the
 * ghost frame of other edges must read zero.  The last slot is also copied
 * into the lattice's current state. */
wlbm_status wlbm_step_tape(wlbm_lattice* lat, int64_t nsteps, void* d_tape, size_t slot_bytes);

/* Temperatures T = sum_i e_i at n probe cells: d_cells is a device [n][2]
 * int32 array of (x, y), d_T a device [n] float array (NaN for a cell outside
 * the lattice). */
wlbm_status wlbm_read_probes(wlbm_lattice* lat, int32_t n, const int32_t* d_cells, float* d_T);

/* ---- Adjoint (reverse mode) ----------------------------------------------
 * Gradients of a loss L of probe temperatures T^m(p) with respect to the
 * per-cell mean free path, the initial temperature field and the blackbody
 * wall temperatures, for periodic and blackbody edges.
 *
 * For a fixed relaxation field a time step is affine in the populations
 * (Sec. 2.3, Eq. algorithm; Sec. 2.6 for the wall overwrite), so the adjoint
 * lam^m = dL/de^m obeys lam^{m-1} = A_m^T lam^m + dL/de^{m-1}, with lam zero at
 * blackbody cells after their contribution to the wall gradient is taken.
 * The reverse pass runs from step M down to 0:
 *   wlbm_adjoint_begin(lat, ws, bytes, M);
 *   at every loss step m (from M downwards): wlbm_adjoint_seed(dL/dT^m(p)),
 *   then wlbm_adjoint_steps(lat, n, states, slot) to go from m to m - n,
 *   where the states e^{m-n} .. e^{m-1} of the forward run (saved with
 *   wlbm_save_state or wlbm_step_tape) sit in consecutive slots;
 *   wlbm_adjoint_read at step 0.
 * The adjoint workspace is caller-owned device memory of wlbm_adjoint_bytes
 * bytes that must stay valid until the reverse pass is over; the lattice's
 * forward state is not used or changed by the reverse pass. */

/* Bytes of the adjoint workspace. */
wlbm_status wlbm_adjoint_bytes(const wlbm_lattice* lat, size_t* bytes);

/* Start a reverse pass at forward step `step` (the last step of the run):
 * clears the workspace (256-byte aligned) in stream order, sets lam = 0 and
 * zeroes the gradient accumulators.  WLBM_EINVAL for diffuse walls. */
wlbm_status wlbm_adjoint_begin(wlbm_lattice* lat, void* d_ws, size_t bytes, int64_t step);

/* Add dL/dT^m at probe cells for the current adjoint step m: d_cells is a
 * device [n][2] int32 array of (x, y), d_dT a device [n] float array.  Every
 * population of the cell receives the value (T = sum_i e_i); at a blackbody
 * cell it goes to the wall gradient.  Repeated cells add up.  A cell outside
 * the lattice is skipped and reported as WLBM_EINVAL by wlbm_adjoint_read. */
wlbm_status wlbm_adjoint_seed(wlbm_lattice* lat, int32_t n, const int32_t* d_cells,
                              const float* d_dT);

/* Take n reverse steps, from adjoint step m to m - n (0 <= n <= m).  Reverse
 * step k needs the forward state e^{k-1}: the states of steps m - n .. m - 1
 * are read from slots 0 .. n-1 of d_states (256-byte aligned, slot_bytes a
 * multiple of 256, at least wlbm_state_bytes).  The lattice's relaxation
 * field must be the one of the forward run. */
wlbm_status wlbm_adjoint_steps(wlbm_lattice* lat, int64_t n, const void* d_states,
                               size_t slot_bytes);

/* Gradients so far (complete at adjoint step 0); each output may be NULL.
 * d_g_mfp: device [ny][nx] float, dL/dMFP per cell (the relaxation time in
 * lattice units; through Eq. W-correction and W = 1/MFP).  d_g_T0: device
 * [ny][nx] float, sum_i w_i lam_i at the current step, i.e. dL/dT0 at step 0
 * (e_i^0 = w_i T0).  g_walls: host [4] double, dL/dT of the x_lo, x_hi, y_lo,
 * y_hi blackbody walls (x walls own the corners; 0 for other edges).  Waits
 * for the stream. */
wlbm_status wlbm_adjoint_read(wlbm_lattice* lat, float* d_g_mfp, float* d_g_T0, double* g_walls);

/* Current adjoint step m, or -1 when no reverse pass was begun. */
int64_t wlbm_adjoint_step_index(const wlbm_lattice* lat);

/* ---- Launch configuration and autotuning ---------------------------------
 * The step kernel splits the q directions of each cell over 1, 2 or 4
 * waves.  The per-cell sum E is added in the same order for every split
 * (sums of 8-direction batches, in batch order), so all splits, the batched
 * step and the multi-step kernels give identical bits. */

/* Set the split (0: library default for q; else 1, 2 or 4 with q a multiple
 * of 8 * split).  Takes effect from the next step. */
wlbm_status wlbm_set_dir_split(wlbm_lattice* lat, int32_t split);

/* Current split, or -1 for NULL. */
int32_t wlbm_get_dir_split(const wlbm_lattice* lat);

/* Time steps that wlbm_step advances per kernel launch on this lattice as
 * it stands (edges, q, per-cell field, sources, step_fusion): 1 for the
 * single-step kernel, else 2 .. 4 (steps left over where calls and schedule
 * chunks do not divide evenly still run single steps).  The
 * automatic choice (step_fusion = 1) is four, and two for lattices with
 * walls and q above 64 or a per-cell field, and for q above 128 (measured
 * fastest on MI355X).  -1 for NULL. */
int32_t wlbm_get_steps_per_launch(const wlbm_lattice* lat);

/* Output rows per block of the kernel that advances k = 2, 3 or 4 steps per
 * launch, for the lattice's current weight mode (uniform or per-cell field):
 * the height fixed by wlbm_set_block_rows or chosen by wlbm_tune_block_rows,
 * else the library's launch model's pick (the height whose blocks fill the
 * device in the fewest row iterations, from the kernel's occupancy and the
 * number of compute units; on a lattice with walls among blocks of at most
 * 18 row iterations, R + 2 (k - 1) <= 18, which measured faster there).
 * wlbm_step never times anything itself.  0 if
 * the lattice runs one step per launch (see step_fusion), -1 for NULL or k
 * outside 2 .. 4.  Results do not depend on the height. */
int32_t wlbm_get_block_rows(const wlbm_lattice* lat, int32_t k);

/* Fix the output rows per block of the k-step kernel (k = 2 .. 4) for the
 * lattice's current weight mode: rows + 2 (k - 1) a multiple of 3, 1 .. 62;
 * 0 returns to the launch model's pick.  Results do not depend on it. */
wlbm_status wlbm_set_block_rows(wlbm_lattice* lat, int32_t k, int32_t rows);

/* Time every candidate block height of the k-step kernel (k = 2 .. 4) on the
 * current state, `launches` launches of k steps each (1 .. 1000, after two
 * warm-up launches, best of two passes), keep the fastest and return it in
 * *rows (may be NULL).  The state and step count are saved in d_state
 * (wlbm_state_bytes bytes) and restored after each trial, so the lattice
 * ends where it started; the flux-window sums are not touched.  Waits for
 * the stream (not capturable).  WLBM_EINVAL if the lattice runs one step per
 * launch, or fewer than k (periodic x edges with diffuse y walls run at most
 * two). */
wlbm_status wlbm_tune_block_rows(wlbm_lattice* lat, void* d_state, size_t bytes, int32_t k,
                                 int32_t launches, int32_t* rows);

/* Time `steps` steps (1 .. 10000, after 2 warm-up steps, one step per launch:
 * the split is the single-step kernel's) with each valid split on the
 * current state and keep the fastest.  The state and step count
 * are saved in d_state (wlbm_state_bytes bytes) and restored after each
 * trial, so the lattice ends where it started; the flux-window sums are not
 * touched.  ms_by_split (host [3], may be NULL) receives the time per step of
 * splits 1, 2, 4 (-1 where not valid); *chosen (may be NULL) the split kept.
 * Waits for the stream. */
wlbm_status wlbm_autotune(wlbm_lattice* lat, void* d_state, size_t bytes, int32_t steps,
                          float* ms_by_split, int32_t* chosen);

/* ---- Batches ----------------------------------------------------------------
 * Several lattices at the same step, with the same split, per-cell field use,
 * schedule chunk and flux window, are advanced together: one kernel launch
 * per time step covers the tiles of all of them.  Sizes, edges, wall
 * temperatures, relaxation weights, q, direction sets and grid speeds may
 * differ: lattices with the same q, set and speeds share one schedule (it
 * depends only on the directions and the step), each such group has its own
 * schedule ring in the batch workspace.  Each step gives the same result as
 * wlbm_step on each lattice. */

/* Bytes of device workspace for a batch of these n lattices (1 .. 4096). */
wlbm_status wlbm_batch_bytes(wlbm_lattice* const* lats, int32_t n, size_t* bytes);

/* Create a batch over the n lattices (the handles stay owned by the caller
 * and must outlive the batch) in the caller's workspace (256-byte aligned).
 * Batch work is enqueued on `stream`; the caller orders it with the work of
 * the lattices' own streams (e.g. by using one stream for both). */
wlbm_status wlbm_batch_create(wlbm_lattice* const* lats, int32_t n, void* d_ws, size_t bytes,
                              void* stream, wlbm_batch** out);

/* Advance every lattice of the batch nsteps steps, as wlbm_step would (their
 * step counts, buffers and flux windows are updated).  Wall temperatures and
 * fields are read from the lattices at each call; a member whose q,
 * direction set or grid speeds no longer match its group's is refused
 * (WLBM_EINVAL: create the batch again).  When every member takes the
 * multi-step kernels and all have one q, one launch advances all of them by
 * the fewest steps per launch that any member allows
 * (wlbm_get_steps_per_launch), each member with its own block height
 * (wlbm_get_block_rows); otherwise one kernel launch per step (see
 * wlbm_batch_set_graphs).  Results do not depend on either. */
wlbm_status wlbm_batch_step(wlbm_batch* batch, int64_t nsteps);

/* Time steps one launch of wlbm_batch_step advances every member (the fewest
 * any member allows when all take the multi-step kernels with one q), or 1
 * when the batch runs one step per launch; -1 for NULL. */
int32_t wlbm_batch_get_steps_per_launch(const wlbm_batch* batch);

/* Time every candidate block height of the batch's multi-step launches, one
 * height for all members, on the members' current states: `launches`
 * launches (1 .. 1000) after two warm-up launches, best of two passes; keep
 * the fastest for every member (as wlbm_set_block_rows would) and return it
 * in *rows (may be NULL).  The states and step counts are saved in d_states
 * (256-byte aligned, at least the sum of the members' wlbm_state_bytes, each
 * rounded up to 256 bytes; the members' slots in member order) and restored
 * after every trial, so the members end where they started; flux-window sums
 * are not touched.  Everything runs on the batch's stream, which the call
 * waits for.  Without it each member keeps its own height, picked by the
 * launch model as if it filled the GPU alone.  WLBM_EINVAL if the batch runs
 * one step per launch. */
wlbm_status wlbm_batch_tune_block_rows(wlbm_batch* batch, void* d_states, size_t bytes,
                                       int32_t launches, int32_t* rows);

/* on = 1: each whole schedule chunk (sched_chunk steps, when that is even)
 * with no flux-window step and no sources runs as one launch of a HIP graph
 * of its per-step launches, captured on first use for each of the two
 * schedule-ring slots (and again after a change of split or per-cell field
 * use); the kernels, and the bits, are those of step-by-step launches.
 * on = 0 (the default): one launch per step.  Other values are rejected
 * (WLBM_EINVAL). */
wlbm_status wlbm_batch_set_graphs(wlbm_batch* batch, int32_t on);

/* Release the batch after waiting for its stream.  NULL is accepted. */
wlbm_status wlbm_batch_destroy(wlbm_batch* batch);

/* Steps taken since creation (or -1 for NULL). */
int64_t wlbm_step_count(const wlbm_lattice* lat);

/* Message of the last failing call on this thread ("" if none). */
const char* wlbm_last_error(void);

/* Release the handle and its pinned host memory after waiting for its stream.
 * The workspace may be reused afterwards.  NULL is accepted. */
wlbm_status wlbm_destroy(wlbm_lattice* lat);

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif

#endif /* WORMLBM_H */
