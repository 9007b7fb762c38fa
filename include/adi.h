/*
 * adi.h -- C ABI of libadi, an MI355X (gfx950) implementation of the
 * alternating-direction-implicit (ADI) solver for the axisymmetric heat
 * equation in a layered cylinder, after A. Ayriyan and J. Busa Jr.,
 * "Parallel Algorithm for Numerical Solution of Heat Equation in Complex
 * Cylindrical Domain" (arXiv 1912.03744), plus the batched design-sweep path
 * and the learned surrogate built on it.
 *
 * Conventions
 *  - Every call returns an adi_status; nothing throws or aborts across the
 *    ABI.  adi_last_error() gives a thread-local message for the last failure.
 *  - Fields are double, row-major with r fastest: cell (i, j) of an nr x nz
 *    grid is element j*nr + i.  Region ids: 0 cooler, 1 inner insulator,
 *    2 heater, 3 outer insulator, 4 terminal, 255 outside the domain.
 *  - The library owns every device buffer it allocates (hipMalloc, or the
 *    caller's allocator set with adi_set_allocator) and frees it in the
 *    matching destroy call.  Host buffers belong to the caller and are only
 *    read or written during the call.
 *  - Work is enqueued on the HIP stream given at creation; NULL makes the
 *    handle create (and later destroy) a non-blocking stream of its own, so
 *    that its steps can be captured into HIP graphs.  Calls that return host
 *    data synchronise that stream.
 *    Asynchronous failures (non-finite values, energy-balance violations) are
 *    latched on the device and reported by the next synchronising call.
 *  - A handle is bound to one stream and is not thread-safe.
 */
#ifndef ADI_H
#define ADI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADI_OK = 0,
  ADI_EINVAL = -1,       /* invalid argument (message says which) */
  ADI_ENOMEM = -2,       /* device or host allocation failed */
  ADI_EDEVICE = -3,      /* a HIP runtime call failed */
  ADI_ESTATE = -4,       /* call not allowed in the handle's current state */
  ADI_ENONFINITE = -5,   /* a NaN/Inf appeared in the field or an input */
  ADI_EBALANCE = -6,     /* the discrete energy identity was violated */
  ADI_EUNSUPPORTED = -7  /* combination the compiled library does not support */
} adi_status;

/* Time integrator.
 * ADI_PR: Peaceman-Rachford half steps of Sec. 3, eq. 8-9: r implicit / z
 *   explicit over tau/2, then z implicit / r explicit over tau/2; the source
 *   enters both half steps.
 * ADI_LOD_BE: locally one-dimensional backward Euler (Yanenko splitting, cited
 *   in Sec. 3): r implicit over tau with the source, then z implicit over tau. */
typedef enum { ADI_PR = 0, ADI_LOD_BE = 1 } adi_scheme;

/* Storage of the right-hand sides carried between sweeps (the field T is
 * always stored by rows, r fastest):
 *   ADI_LAYOUT_ROWS    by rows, like T; any grid size;
 *   ADI_LAYOUT_STRIPS  strips of 4 columns, each strip a contiguous run of
 *                      rows of 4 values, so that both sweeps move whole
 *                      cache lines; nr <= 2048 and nz <= 3072;
 *   ADI_LAYOUT_RESIDENT  by rows between calls, but every run of steps
 *                      between energy checks runs in one launch of a single
 *                      workgroup that keeps the right-hand side in LDS (lines
 *                      solved by two-ended Thomas elimination, two lanes per
 *                      line); for small grids: 3 <= nr, nz <= 512 and
 *                      nz (nr + 1) + 8 (3 nr + 4 nz) doubles within 160 KB
 *                      (64 x 160 takes 136 KB).  Check steps run on the rows
 *                      kernels. */
typedef enum { ADI_LAYOUT_ROWS = 0, ADI_LAYOUT_STRIPS = 1, ADI_LAYOUT_RESIDENT = 2 } adi_layout;

/* Geometry of Fig. 1 (Sec. 2): cooler r < r0 for z < zmax; inner insulator
 * r0 <= r < r1, heater r1 <= r < r2, outer insulator r2 <= r < rmax, all three
 * for z < z0; terminal slab zmax <= z < ztop over the whole radius; cells with
 * r >= r0 and z0 <= z < zmax are outside the domain.  Requires
 * 0 < r0 <= r1 <= r2 <= rmax and 0 < z0 <= zmax <= ztop.
 * Grid (eq. 7): cell-centred, nr x nz cells (1 <= nr, nz; nr*nz < 2^31).
 * r_faces / z_faces: optional monotone face coordinates (nr+1 / nz+1 values,
 * first 0, last rmax / ztop), copied at creation; NULL gives the uniform grid
 * r_face[i] = rmax*i/nr, r_centre[i] = (i+0.5)*rmax/nr (same in z with ztop).
 * A cell belongs to the region containing its centre. */
typedef struct {
  double r0, r1, r2, rmax;
  double z0, zmax, ztop;
  int32_t nr, nz;
  const double* r_faces;
  const double* z_faces;
} adi_geometry;

/* Boundary films (eq. 6 generalised to Robin): face classes 0 = bottom z = 0,
 * 1 = outer r = rmax, 2 = top z = ztop, 3 = faces against cells outside the
 * domain.  The flux out of cell c through such a face is g (T_c - t_inf) with
 * g = 1/(d_c/(2 k_c) + 1/h): h = 0 is an insulated face, h = INFINITY fixes
 * the face temperature to t_inf.  The axis r = 0 never carries flux.
 * Requires h >= 0 (INFINITY allowed) and finite t_inf. */
typedef struct {
  double h[4];
  double t_inf[4];
} adi_bc;

typedef struct adi_problem_s* adi_problem;
typedef struct adi_batch_s* adi_batch;
typedef struct adi_mlp_s* adi_mlp;

/* Energy bookkeeping (2 pi dropped): E = sum rho c T V over active cells with
 * V = r_c dr dz; source_power = sum Q V; boundary_flow = heat flow out through
 * all boundary faces at the current field; residual = largest relative
 * violation of the per-step energy identity seen by the periodic checks
 * (0 if none ran); checks = number of periodic checks run. */
typedef struct {
  double E, E0, source_power, boundary_flow, residual, time;
  int64_t steps, checks;
} adi_energy_report;

/* ------------------------------------------------------------ problems -- */

/* Create a single-instance problem.  hip_stream: a hipStream_t (may be NULL).
 * Allocates the field and work buffers on the current HIP device.
 * Errors: ADI_EINVAL (geometry/bc), ADI_ENOMEM, ADI_EDEVICE. */
adi_status adi_create_problem(const adi_geometry* g, const adi_bc* bc, adi_scheme scheme,
                              void* hip_stream, adi_problem* out);

/* Per-region conductivity k[5] and volumetric heat capacity rho_c[5]
 * (eq. 1 with constant coefficients).  Both > 0 and finite. */
adi_status adi_set_materials(adi_problem p, const double k[5], const double rho_c[5]);

/* Per-region volumetric source Q[5] (eq. 2 with a constant source); finite. */
adi_status adi_set_sources(adi_problem p, const double q[5]);

/* Set the field: host_T (nz*nr doubles, values outside the domain ignored) or,
 * if host_T is NULL, the uniform initial condition T0 of eq. 5.  Resets the
 * step counter, the time and E0. */
adi_status adi_set_field(adi_problem p, const double* host_T, double T0);

/* Advance nsteps >= 0 steps of size dt > 0 (asynchronous on the stream).
 * Requires materials and sources (else ADI_ESTATE).  Line solves use the
 * factor tables of the current (dt, materials); they are rebuilt on the
 * device when either changes. */
adi_status adi_step(adi_problem p, double dt, int64_t nsteps);

/* Run the discrete energy-identity check every `every` steps (0 = never) and
 * latch ADI_EBALANCE when the relative residual exceeds tol (> 0). */
adi_status adi_set_check(adi_problem p, int32_t every, double tol);

/* Copy the field to host_out (count must equal nz*nr); cells outside the
 * domain read as NaN.  Synchronises; returns a latched error if any. */
adi_status adi_read_field(adi_problem p, double* host_out, size_t count);

/* Enqueue a device-to-device copy of the field (nz*nr doubles, cells outside
 * the domain hold 0) into dev_out. */
adi_status adi_read_field_device(adi_problem p, void* dev_out);

/* Region id per cell (count = nz*nr), computed on the device.  Synchronises. */
adi_status adi_read_region_map(adi_problem p, uint8_t* host_out, size_t count);

/* Temperature profile along one row, resampled at r_k = (k+0.5)*rmax/npts by
 * linear interpolation between cell centres (constant beyond the first and
 * last centre).  which = 0: top row (outer face of the terminal); which = 1:
 * first row inside the terminal (contact face).  The row must lie inside the
 * domain everywhere (ADI_EINVAL otherwise).  Synchronises. */
adi_status adi_read_profile(adi_problem p, int32_t which, int32_t npts, double* host_out);

/* Energy report of the current field.  Synchronises. */
adi_status adi_energy(adi_problem p, adi_energy_report* out);

/* Kernel timing for the roofline report: nlaunch half-step pairs (r sweep,
 * then z sweep, each reading what the other has just written, as in a time
 * step) on the problem's side buffers and stream, every launch carrying HIP
 * start and end events of its own dispatch; returns the mean duration per
 * launch of each direction in ms.  Under ADI_LAYOUT_RESIDENT: nlaunch steps
 * in one launch on a copy of the carried right-hand side, *ms_r = the time per
 * step (launch included) and *ms_z = 0.  The field and the carried
 * right-hand side are left unchanged.  Synchronises. */
adi_status adi_time_sweeps(adi_problem p, double dt, int32_t nlaunch, float* ms_r, float* ms_z);

/* Launch shape of the line solves (advanced; the autotuner uses it).
 * dir 0 = r lines, 1 = z lines.  chunk: cells per lane and line; a wave's
 * lanes form lines_per_wave slots x (64/lines_per_wave) chunks; a line spans
 * waves_per_line waves; each lane handles lines_per_lane lines; a workgroup
 * runs groups_per_block line groups.  (64/lines_per_wave)*waves_per_line*chunk
 * must cover the line length.  Only compiled shapes are accepted
 * (ADI_EUNSUPPORTED otherwise); see adi_layout_shapes: the shape must
 * belong to the problem's layout. */
adi_status adi_set_launch(adi_problem p, int32_t dir, int32_t chunk, int32_t lines_per_wave,
                          int32_t waves_per_line, int32_t lines_per_lane, int32_t groups_per_block);
adi_status adi_get_launch(adi_problem p, int32_t dir, int32_t* chunk, int32_t* lines_per_wave,
                          int32_t* waves_per_line, int32_t* lines_per_lane, int32_t* groups_per_block);

/* Launch shapes compiled into the library for the rows layout: writes up to
 * max_shapes records (chunk, lines_per_wave, waves_per_line, lines_per_lane,
 * groups_per_block) to out (5*max_shapes int32) and the number of shapes to
 * *count. */
adi_status adi_launch_shapes(int32_t* out, int32_t max_shapes, int32_t* count);

/* Same for a layout and direction (dir 0 = r, 1 = z).  Strip-layout shapes
 * are (chunk, 1, waves, 4, 1): one line slot per wave, 4 lines per lane.
 * ADI_LAYOUT_RESIDENT has one fixed shape and lists none (*count = 0); its
 * check steps use the rows shapes set with adi_set_launch. */
adi_status adi_layout_shapes(int32_t layout, int32_t dir, int32_t* out, int32_t max_shapes, int32_t* count);

/* Choose the right-hand-side layout (adi_layout); resets both launch shapes
 * to the layout's defaults.  Results do not depend on the layout beyond
 * rounding order (the same tables and arithmetic per line).  Synchronises.
 * ADI_EUNSUPPORTED if the grid exceeds the layout's kernels. */
adi_status adi_set_layout(adi_problem p, int32_t layout);
adi_status adi_get_layout(adi_problem p, int32_t* layout);

/* Wait until all work enqueued on the problem's stream has finished. */
adi_status adi_sync(adi_problem p);

/* Graphs in adi_step: with steps = K > 0, adi_step replays captured HIP
 * graphs of K steps and of every power of two below K (each run of steps
 * between energy checks as whole graphs, largest first), captured together
 * on the first call after the tables or the check pattern change; 0 = plain
 * launches.  K <= 4096. */
adi_status adi_set_graph_steps(adi_problem p, int32_t steps);

void adi_destroy(adi_problem p);

/* ---------------------------------------------- nonlinear method path -- */

/* The paper's method with temperature-dependent coefficients (Sec. 2-4):
 * lambda(T), rho c_V(T) and the source amplitude chi(T) I^2/S_C per region,
 * each half step of eq. 8-9 solved by the simple iteration of eq. 12 (r
 * implicit, laws and source at the iterate, Lambda_z at the current layer)
 * and eq. 14 (z implicit, laws at the iterate, rho c_V, Lambda_r and the
 * source at T-bar), stopped by the max-norm rule of eq. 13
 * (max |T^{s+1} - T^s| over the cells of the domain < eps); a half step that
 * has not stopped after iter_max solves fails, and the step is retried from
 * the same T with tau/2 (end of Sec. 3).  Face conductivities take each
 * side's lambda at the mean of the two cell temperatures and combine the
 * half cells in series; a film uses lambda at the cell's own temperature.
 * The source of both half steps is evaluated at t + tau/2 through the pulse
 * p(t) of eq. 2-4.  These calls use the problem's geometry, films and field;
 * the constant materials and sources of adi_set_materials / adi_set_sources
 * do not enter.  Lines of at most 3072 cells (ADI_EUNSUPPORTED otherwise). */

/* Laws per region (5 regions x 4 coefficients, region-major): value =
 * c0 + c1 T + c2 T^2 + c3 T^3.  lam: conductivity, cap: volumetric heat
 * capacity, src: source amplitude.  Finite coefficients (ADI_ENONFINITE);
 * the laws must stay positive (lam, cap) over the temperatures reached. */
adi_status adi_set_laws(adi_problem p, const double lam[20], const double cap[20], const double src[20]);

/* Normalised source p(t) (eq. 2): kind 0 constant 1; kind 1 the rectangular
 * pulse train of eq. 3; kind 2 the erf-smoothed switching of eq. 4.  params:
 * t_per, t_src, t_trs, xi, zeta with 0 < t_trs <= t_src, t_src + t_trs <=
 * t_per, zeta > 0 (kind 0: only t_src, t_trs > 0 are checked; the step rule
 * of adi_set_step_rule reads t_src and t_trs for every kind); NULL allowed
 * for kind 0 (keeps the previous values, initially 0.1, 0.01, 1e-4, 4, 2). */
adi_status adi_set_pulse(adi_problem p, int32_t kind, const double params[5]);

/* Stop rule and retries: eps > 0 of eq. 13, iter_max in [1, 64] solves per
 * half step, tau_min > 0 (a run fails once halving goes below it).
 * Defaults 1e-6, 10, 1e-12. */
adi_status adi_set_iteration(adi_problem p, double eps, int32_t iter_max, double tau_min);

/* Step rule of Sec. 4: each step starts with tau = t_trs/tau_trs_div inside
 * a transition of the source (the first t_trs after a switch-on or a
 * switch-off) and t_src/tau_src_div elsewhere, and ends no later than the
 * next switch point, transition end or t_end (constant source: t_src/
 * tau_src_div throughout).  periodic_tol > 0: at every period start the
 * field is compared with the previous period start's, and the run stops
 * once the max-norm change is below periodic_tol (0: never).  Defaults
 * 1000, 100, 0. */
adi_status adi_set_step_rule(adi_problem p, double tau_trs_div, double tau_src_div, double periodic_tol);

/* One step attempt of size tau from the problem's current time, without
 * the step rule and without halving.  *accepted (nullable): 1 if both
 * iterations stopped (the field and time then advance), else 0 (the field
 * is unchanged).  solves (nullable, 2): solves of each half step (-1: did
 * not stop, 0: not run).  changes (nullable, 2): the change norm that
 * decided each half.  Synchronises.  ADI_ESTATE before adi_set_laws;
 * ADI_EDEVICE as for adi_nl_run. */
adi_status adi_nl_step(adi_problem p, double tau, int32_t* accepted, int32_t solves[2], double changes[2]);

typedef struct {
  double t;            /* model time reached */
  int64_t steps;       /* accepted steps */
  int64_t rejected;    /* attempts retried with half the step */
  int64_t solves_r;    /* line-system solves of the r half steps (accepted steps) */
  int64_t solves_z;    /* same for the z half steps */
  int32_t periodic;    /* 1 if the periodic-regime stop ended the run */
  double min_margin;   /* smallest |change - bound| / bound over every stop
                          decision (eq. 13 and periodic): how far the run's
                          decisions were from a tie */
} adi_nl_report;

/* The time loop of Sec. 4 from the problem's current time up to t_end (or
 * the periodic stop, or max_steps accepted steps), on the device in one
 * persistent cooperative kernel per 4096 attempts.  host_log (nullable,
 * 4*log_cap doubles): (t before, tau, solves_r, solves_z) of the first
 * log_cap accepted steps.  out (nullable) receives the report.
 * Synchronises.  ADI_EINVAL if halving went below tau_min (the field then
 * holds the last accepted step), ADI_EDEVICE if a grid-wide wait of the
 * kernel ran out (every wave leaves at its next wait; the problem's time
 * is unchanged, its field undefined until adi_set_field).  A wait polls at
 * most about 3e7 times (about a second); the environment variable
 * ADI_NL_WAIT_POLLS, read at each call, sets another bound (0: abort at the
 * first wait that would poll), so that callers can exercise this path. */
adi_status adi_nl_run(adi_problem p, double t_end, int64_t max_steps, double* host_log, int64_t log_cap,
                      adi_nl_report* out);

/* ------------------------------------------------------- ragged batch -- */

/* A batch of n independent instances (the design sweep): instance i has its
 * own geometry geoms[i] (uniform grid, 3 <= nr <= 192, 3 <= nz <= 480;
 * face arrays are not supported here) and films bcs[i].  All instances are
 * advanced together, in one of two ways chosen by adi_batch_set_launch: one
 * persistent kernel launch, where each workgroup takes the next instance
 * from an atomic queue (largest grids first), builds its geometry and factor
 * tables, runs the whole time loop and takes the next; or batched sweep
 * launches, one per half step over all instances (one per z chunk shape),
 * with one single-wave workgroup per block of 4 lines of any instance.
 * Errors: ADI_EINVAL, ADI_EUNSUPPORTED (grid or face arrays), ADI_ENOMEM. */
adi_status adi_create_batch(int32_t n, const adi_geometry* geoms, const adi_bc* bcs, adi_scheme scheme,
                            void* hip_stream, adi_batch* out);

/* Per-instance materials and sources, n*5 values each (instance-major):
 * k > 0, rho_c > 0, finite q (eq. 1-2 with constant coefficients). */
adi_status adi_batch_set_materials(adi_batch b, const double* k, const double* rho_c, const double* q);

/* Uniform initial temperature per instance (n values; NULL = all 0). */
adi_status adi_batch_set_initial(adi_batch b, const double* T0);

/* Launch shape of the batch (the autotuner uses it): lines per lane (1 or
 * 2: right-hand sides by rows, line slots of 16 or 32 chunks; 4: right-hand
 * sides in strips of 4 columns, one wave per block of 4 lines), waves per
 * workgroup (4 or 8: the persistent kernel; 1, with 4 lines per lane: the
 * batched sweep launches, each instance keeping its own right-hand sides and
 * scratch), resident workgroups per compute unit (1..8; persistent kernel
 * only).  ADI_EUNSUPPORTED for shapes not compiled. */
adi_status adi_batch_set_launch(adi_batch b, int32_t lines_per_lane, int32_t waves_per_block,
                                int32_t blocks_per_cu);

/* Compiled shapes of the z lines in the batched sweep launches, by z class:
 * the instances whose columns have up to 192, 256, 320 or 512 rows are
 * classes 0..3 (one z launch per class and half step).  Shape `variant` of
 * a class puts each block of 4 columns on a workgroup of *waves waves of 64
 * chunks of *cells cells (the line solve of Sec. 3-4 split by the partition
 * method); *max_rows receives the class's longest column.  Variant 0 is the
 * default.  Needs no device.  ADI_EINVAL for a class or variant out of range
 * (the outputs are then left unchanged). */
adi_status adi_batch_zshape_info(int32_t zclass, int32_t variant, int32_t* waves, int32_t* cells,
                                 int32_t* max_rows);

/* Use shape `variant` (see adi_batch_zshape_info) for the z lines of class
 * zclass in the batched sweep launches, from the next adi_batch_step on
 * (the autotuner picks one per class).  Results do not depend on the shape
 * beyond rounding.  ADI_EINVAL for a class or variant out of range. */
adi_status adi_batch_set_zshape(adi_batch b, int32_t zclass, int32_t variant);

/* Advance every instance nsteps steps of size dt from its initial field
 * (each call starts again from the initial fields), recording the outer
 * terminal-face profile (top row resampled at r_k = (k+0.5)*rmax/npts, as in
 * adi_read_profile) after every snapshot_every-th step (0 = none).
 * dev_profiles: NULL, or a device buffer of the caller (at least n * nsnap *
 * npts doubles, nsnap = nsteps/snapshot_every, instance-major, then
 * snapshot, then point) that receives the snapshots instead of the batch's
 * own buffer, e.g. a torch tensor; it must stay allocated until the work of
 * this call has finished.  npts is an argument of this call (not only of
 * the read) because the snapshots are resampled on the device as they are
 * taken.  Enqueued on the batch's stream as captured HIP graphs: one for the
 * persistent kernel (queue reset + kernel), or, for the batched sweep
 * launches, one per 256 steps (the instance set-up in the first); returns
 * without waiting. */
adi_status adi_batch_step(adi_batch b, double dt, int64_t nsteps, int32_t snapshot_every, int32_t npts,
                          double* dev_profiles);

/* Wait for the batch's stream. */
adi_status adi_batch_sync(adi_batch b);

/* Profiles of the last adi_batch_step, from the batch's own buffer or the
 * caller's dev_profiles: npts must equal that call's npts; count = n *
 * (nsteps/snapshot_every) * npts doubles, instance-major, then snapshot,
 * then point.  Synchronises. */
adi_status adi_batch_read_profiles(adi_batch b, int32_t npts, double* host_out, size_t count);

/* Final field of instance i (nz*nr doubles, r fastest; cells outside the
 * domain hold 0).  Synchronises. */
adi_status adi_batch_read_field(adi_batch b, int32_t i, double* host_out, size_t count);

/* Total cells over all instances, snapshots per instance of the last step,
 * workgroups: persistent workgroups launched, or the r-sweep workgroups of
 * one step for the batched sweep launches. */
adi_status adi_batch_info(adi_batch b, int64_t* total_cells, int32_t* nsnap, int32_t* workgroups);

/* Cells inside the domain (not masked) summed over all instances. */
adi_status adi_batch_active_cells(adi_batch b, int64_t* active);

/* Run adi_batch_step(b, dt, nsteps, 0, 64, NULL) reps times back to back,
 * bracketed by HIP events on the batch's stream, and return the mean
 * milliseconds per call (launch shape as set; fields end as after one call).
 * Synchronises.  Used by the autotuner and the benchmark. */
adi_status adi_batch_time(adi_batch b, double dt, int64_t nsteps, int32_t reps, float* ms_out);

void adi_batch_destroy(adi_batch b);

/* ---------------------------------------------------- learned surrogate -- */

/* Multilayer perceptron x -> gelu(x W_1 + b_1) -> ... -> h W_out + b_out with
 * gelu(u) = u Phi(u) (erf form).  widths[0] inputs (1..64), then nwidths-1
 * layer widths (multiples of 64, <= 4096); at most 8 layers.  Weights are
 * initialised from `seed` (He-normal, zero biases).  Products run on bf16
 * matrix cores with fp32 accumulation; hidden activations are kept in bf16,
 * the output and pre-activations in fp32; fp32 master weights and Adam
 * (beta 0.9/0.999, eps 1e-8).  The flat parameter vector holds, layer by
 * layer, W_l ([n_in x n_out] row-major) then b_l. */
adi_status adi_mlp_create(const int32_t* widths, int32_t nwidths, uint64_t seed, void* hip_stream,
                          adi_mlp* out);
adi_status adi_mlp_num_params(adi_mlp m, int64_t* n);

/* Input encoding applied on the device: x' = (x - shift) * scale per feature
 * (widths[0] values each). */
adi_status adi_mlp_set_scaling(adi_mlp m, const float* shift, const float* scale);

/* Parameters as fp32 host arrays (count = number of parameters).  set resets
 * the optimiser state. */
adi_status adi_mlp_get_params(adi_mlp m, float* host_out, int64_t count);
adi_status adi_mlp_set_params(adi_mlp m, const float* host_in, int64_t count);

/* y = network(x): dev_x [batch x widths[0]] fp32 and dev_y [batch x
 * widths[last]] fp32 are device pointers; batch is a multiple of 64.
 * Asynchronous on the network's stream. */
adi_status adi_mlp_forward(adi_mlp m, const float* dev_x, int64_t batch, float* dev_y);

/* Wait until all work enqueued on the network's stream has finished. */
adi_status adi_mlp_sync(adi_mlp m);

/* Mean-squared-error loss against dev_t and its gradient w.r.t. every
 * parameter (copied to host_grads, nullable); loss_out (host, nullable).
 * Synchronises. */
adi_status adi_mlp_gradients(adi_mlp m, const float* dev_x, const float* dev_t, int64_t batch,
                             float* host_grads, float* loss_out);

/* One training step: forward, backward, Adam with learning rate lr.  If
 * loss_out is not NULL the loss before the update is written there (and the
 * call synchronises). */
adi_status adi_mlp_train_step(adi_mlp m, const float* dev_x, const float* dev_t, int64_t batch, float lr,
                              float* loss_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * network output as adi_mlp_forward (bit for bit: the same products and
 * epilogues), with the encoded input and the hidden activations kept in a
 * fixed work area of ADI_MLP_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends, and the output written
 * straight into dev_y.  Allocates nothing.  The area takes
 * 2 * batch * (64 + 2 * w) bytes, w the widest hidden layer (at most 14,528
 * rows for 256-wide layers): larger batches fail with ADI_EINVAL.  Every
 * call on one GPU uses the same area: calls ordered on one stream are safe,
 * calls that overlap in time on one GPU (other streams or threads) race.
 * Asynchronous on the network's stream; the inputs and dev_y must stay
 * allocated until that work has finished. */
#define ADI_MLP_NOALLOC_SCRATCH_BYTES (16u << 20)
adi_status adi_mlp_forward_noalloc(adi_mlp m, const float* dev_x, int64_t batch, float* dev_y);

void adi_mlp_destroy(adi_mlp m);

/* Screening reductions of the surrogate's design sweep, on the device.
 * dev_pred: [members][n][nout] fp32 network outputs, for each design the
 * shape of its scaled terminal-face profile (outputs 0..63) and its
 * standardised log scale (outputs 64..nout-1, averaged): member m's profile
 * is y_k = exp(mu + sd * scale) * shape_k, the ensemble's ybar_k the mean
 * over the members.  Per design: dev_peak = max_k ybar_k * qt (dev_qt:
 * n values, e.g. Q t to turn y into a temperature; NULL: 1), dev_dis = the
 * disagreement max_k |y_first - y_last| / max(max_k ybar_k, floor_),
 * dev_bound_ok = 1 if every ybar_k <= 1 + 1e-3 (the maximum principle of
 * the scaled profile).  64 < nout <= 4096.  Asynchronous on hip_stream. */
adi_status adi_screen_profiles(const float* dev_pred, int32_t members, int64_t n, int32_t nout, double mu,
                               double sd, double floor_, const double* dev_qt, double* dev_peak, double* dev_dis,
                               uint8_t* dev_bound_ok, void* hip_stream);

/* Indices of the k largest of n device doubles (1 <= k <= n; NaN below
 * every number; of equal values the lower indices first), into dev_idx (k
 * int64): first those above the k-th largest value in ascending index
 * order, then those equal to it, in ascending index order.  Radix
 * selection on the device (eight 8-bit passes) and an order-keeping
 * compaction; work buffers from the library's allocator.  Synchronises
 * hip_stream. */
adi_status adi_top_k(const double* dev_vals, int64_t n, int32_t k, int64_t* dev_idx, void* hip_stream);

/* ---------------------------------------------------------- utilities -- */

/* Device-memory hook (for a caller's caching allocator, e.g. PyTorch's):
 * alloc(bytes, ctx) returns a device pointer aligned to 256 bytes, or NULL
 * when out of memory (the calling entry point then fails with ADI_ENOMEM);
 * free_fn(ptr, ctx) takes back a block alloc returned.  From this call on,
 * every device allocation of the library (problems, batches, networks) goes
 * through the hook; both NULL restores hipMalloc / hipFree.  Each block is
 * returned to the free function that was set when it was allocated, after
 * the device has finished every queued use of it (the library synchronises
 * the device first, as hipFree does).  Process-wide; the hook functions may
 * be called from any thread that calls the library.  Errors: ADI_EINVAL if
 * exactly one of alloc, free_fn is NULL. */
typedef void* (*adi_alloc_fn)(size_t bytes, void* ctx);
typedef void (*adi_free_fn)(void* ptr, void* ctx);
adi_status adi_set_allocator(adi_alloc_fn alloc, adi_free_fn free_fn, void* ctx);

const char* adi_status_string(adi_status s);
const char* adi_last_error(void);
/* Library version string. */
const char* adi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ADI_H */
