/*
 * snrt.h -- C ABI of the MI355X explicit S_N transport step.
 *
 * The library advances the discrete-ordinates system of arXiv 2505.17284
 * (Sec. 4.1, eq. eq_sn_2d: M ordinates on the upper hemisphere, weights summing
 * to 2 pi, isotropic scattering through phi = sum_l w_l psi_l, isotropic source)
 * with the upwind finite-volume balance of Sec. 4.2 (eqs. eq_sn_2d_eqn_fv,
 * eq_upwind1stOrder) on a uniform Cartesian grid of square cells, first-order
 * or minmod-limited second-order reconstruction, ghost-cell boundaries (end of
 * Sec. 4.2), and forward Euler or Heun's method (Sec. 4.3, eq. eq_ODE) with
 * dt = T / N_t, N_t = ceil(T / (CFL h) - 1e-9) (Sec. 5.1.3). Along the way it
 * accumulates the quantities of interest of Sec. 3.1.2 / 3.2.2: particle mass,
 * absorption per tally region, outflow and inflow through rectangle boundaries,
 * instantaneous and integrated over time.
 *
 * Conventions
 *  - Every call returns sn_status; SN_OK is 0. Nothing throws across the ABI.
 *    The text of the last failure on the calling thread is sn_last_error().
 *  - Host input arrays belong to the caller and are read (and copied) only
 *    during the call that receives them.
 *  - Device buffers belong to the caller (the Python layer allocates them with
 *    PyTorch) and are lent to a plan by sn_plan_bind; the library never frees
 *    them. The plan owns only host memory and HIP events.
 *  - `stream` arguments are hipStream_t values passed as void* (NULL = the
 *    legacy default stream). Calls that launch work are asynchronous unless
 *    documented as synchronising; asynchronous device faults are reported as
 *    SN_ERR_DEVICE by the next synchronising call.
 *  - A plan is not thread-safe: one thread at a time may call into it.
 */
#ifndef SNRT_H
#define SNRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SN_MAX_TALLIES 8   /* absorption tally regions */
#define SN_MAX_RECTS 4     /* outflow/inflow rectangles */
#define SN_MAX_FLUENCE_BLOCKS 1024 /* blocks of sn_plan_fluence_functionals */
#define SN_MAX_PROBES 8              /* space-time probes */
#define SN_MAX_WINDOWS 4096          /* time windows of the probes */
#define SN_MAX_PROBE_CELLS (1 << 20) /* cells of all probes together */
#define SN_MAX_REGIONS 256 /* material regions (uint8 ids) */
#define SN_MAX_ORDINATES 4096

typedef int32_t sn_status;
#define SN_OK 0
#define SN_ERR_INVALID 1     /* argument or problem statement rejected */
#define SN_ERR_OOM 2         /* host allocation failed, or buffers too small */
#define SN_ERR_DEVICE 3      /* a HIP call failed */
#define SN_ERR_UNSUPPORTED 4 /* valid request the library does not implement */
#define SN_ERR_NONFINITE 5   /* a QoI became NaN or infinite */
#define SN_ERR_BUSY 6        /* admission refused: over the memory budget */
#define SN_ERR_STATE 7       /* call out of order (e.g. run before bind/init) */

/* Boundary kinds per side, sides ordered W (x = x0), E, S (y = y0), N. */
#define SN_BC_VACUUM 0  /* ghost value 0 */
#define SN_BC_INFLOW 1  /* isotropic inflow value inflow[side] */
#define SN_BC_REFLECT 2 /* ghost = mirror ordinate's value in the boundary cell */

#define SN_EULER 0
#define SN_HEUN 1

#define SN_F32 0  /* psi stored as IEEE binary32 */
#define SN_BF16 1 /* psi stored as bfloat16, math in FP32; every stored value is
                   * rounded stochastically (unbiased) with reproducible bits
                   * drawn from (stage, ordinate, cell) */

/* One cell of a space-time probe (see sn_problem). */
typedef struct sn_probe_cell {
    int32_t cell;  /* interior index j * nx + i */
    int32_t probe; /* 0 .. n_probes-1 */
    double weight; /* the cell's share of the probe's average */
} sn_probe_cell;

/* A problem statement (Sec. 4.1 with the benchmark data of Sec. 3).
 *
 *  nx, ny, h      grid of nx * ny square cells of side h > 0; cell (i, j),
 *                 i along x, covers [i h, (i+1) h] x [j h, (j+1) h] relative to
 *                 the lower-left corner.
 *  M, xi, eta, w  ordinates: direction cosines along x and y and weights, [M]
 *                 each; sum w must equal 2 pi to 1e-10 relative (Sec. 4.1).
 *  mirror_x/_y    [M] index of the ordinate with xi (eta) negated and equal
 *                 weight; required when a side is SN_BC_REFLECT (checked
 *                 bit-exactly), otherwise may be NULL.
 *  region         [ny][nx] row-major material id of every cell, < n_regions.
 *  sigma_a/s, q   [n_regions] absorption and scattering cross-sections
 *                 (>= 0, finite) and isotropic source per ordinate (finite).
 *  tally          [n_regions] absorption tally id (< n_tallies <= 8).
 *  bc, inflow     boundary kind and inflow value per side (W, E, S, N).
 *  order          1 (first-order upwind), 2 (minmod MUSCL) or 3 (Green-Gauss
 *                 gradient with the Venkatakrishnan limiter, eq. eq_V_limiter;
 *                 its ghost cells hold the side's ghost value for every
 *                 ordinate); boundary faces are first order.
 *  stepper        SN_EULER or SN_HEUN.
 *  cfl, t_end     dt = t_end / N_t with N_t = ceil(t_end / (cfl h) - 1e-9).
 *  rects          [n_rects][4] = (i0, j0, i1, j1), half-open cell ranges
 *                 0 <= i0 < i1 <= nx, 0 <= j0 < j1 <= ny; the outflow and
 *                 inflow through each rectangle's boundary are QoIs.
 *  psi_dtype      SN_F32 or SN_BF16.
 *  n_probes, n_windows, n_probe_cells, probe_cells
 *                 space-time probes (Hohlraum QoI-1, Sec. 3.2.2): probe p
 *                 averages phi = sum_k w_k psi_k, J_x = sum_k w_k xi_k psi_k and
 *                 J_y = sum_k w_k eta_k psi_k over its cells, weighted by
 *                 probe_cells[].weight (the cell's share of the probe region,
 *                 e.g. area inside a ball over the ball's area), and over each
 *                 of n_windows equal windows of [0, t_end]: the time integral
 *                 (the stepper's rule) divided by the window's length. A step
 *                 counts in the window holding its start time, floor(step *
 *                 n_windows / N_t); steps past N_t count nowhere.
 *                 0 <= n_probes <= SN_MAX_PROBES; 1 <= n_windows <=
 *                 SN_MAX_WINDOWS when n_probes > 0; probe_cells[n_probe_cells]
 *                 (n_probe_cells <= SN_MAX_PROBE_CELLS) may be NULL when 0.
 *                 The stage kernels sum the probes over tiles of 128 columns
 *                 by rows_per_wave x waves rows (8 by default): plan creation
 *                 fails with SN_ERR_UNSUPPORTED when a tile holds more probe
 *                 cells than fit 64 lanes of 8, a lane's cells all of one
 *                 probe (at least 448 fit: in the default 8-row tiles, the
 *                 cells of one ball of radius 30 h).
 *  fluence        1: also accumulate the fluence Phi = int_0^t phi dt per cell
 *                 in FP64, with the stepper's time rule (Euler dt phi(psi^n);
 *                 Heun dt/2 (phi(psi^n) + phi(psi^(1)))); the Hohlraum QoI-3
 *                 to QoI-6 (Sec. 3.2.2) are functionals of sigma_a Phi. Costs
 *                 8 nx ny bytes of scratch and 20 bytes of traffic per cell and
 *                 stage. 0: off.
 */
typedef struct sn_problem {
    int32_t nx, ny;
    double h;
    int32_t M;
    const double *xi, *eta, *w;
    const int32_t *mirror_x, *mirror_y;
    const uint8_t *region;
    int32_t n_regions;
    const double *sigma_a, *sigma_s, *q;
    const uint8_t *tally;
    int32_t n_tallies;
    int32_t bc[4];
    double inflow[4];
    int32_t order;
    int32_t stepper;
    double cfl, t_end;
    int32_t n_rects;
    const int32_t *rects;
    int32_t psi_dtype;
    int32_t fluence;
    int32_t n_probes, n_windows, n_probe_cells;
    const struct sn_probe_cell *probe_cells;
} sn_problem;

/* Sizes and derived constants of a plan. psi_bytes is the size of ONE angular
 * flux buffer; a plan needs two (A and B) plus one scratch buffer, each
 * 256-byte aligned. Each ordinate's plane in a psi buffer holds the nx * ny
 * cells inside a frame of two ghost cells, x fastest, rows of `pitch`
 * elements (pitch >= nx + 4); sn_plan_read_psi returns the plain
 * [M][ny][nx] array. */
typedef struct sn_plan_info {
    int32_t n_steps;   /* N_t */
    double dt;
    int32_t nx, ny, M, pitch;
    int32_t n_groups;  /* ordinate groups of the update stage (Euler, Heun
                        * stage 1): phi partials per cell it writes */
    int32_t group_size;      /* ordinates per workgroup of the update stage */
    int32_t rows_per_wave;   /* grid rows per wavefront */
    int32_t waves_per_group; /* wavefronts per workgroup, stacked along y */
    int32_t n_workgroups;    /* workgroups of one stage launch */
    uint64_t psi_bytes;
    uint64_t scratch_bytes;
    int32_t psi_dtype;
    int32_t step;      /* steps taken so far */
    int32_t n_groups_average;     /* the same for Heun's averaging stage */
    int32_t group_size_average;
    int32_t n_workgroups_average;
} sn_plan_info;

/* QoIs of the current state (instantaneous) and their time integrals over
 * [0, t], integrated with the rule of the stepper: Euler dt q(psi^n); Heun
 * dt/2 (q(psi^n) + q(psi^(1))). balance_residual = mass(t) - [mass(0) +
 * int (source + inflow_domain - outflow_domain - sum absorption) dt], where
 * rectangle 0 is taken as the domain boundary when it covers the whole grid
 * (0 otherwise). */
typedef struct sn_qoi {
    int64_t step;
    double t;
    int32_t n_tallies, n_rects;
    double mass, source;
    double absorption[SN_MAX_TALLIES];
    double outflow[SN_MAX_RECTS];
    double inflow[SN_MAX_RECTS];
    double int_mass, int_source;
    double int_absorption[SN_MAX_TALLIES];
    double int_outflow[SN_MAX_RECTS];
    double int_inflow[SN_MAX_RECTS];
    double balance_residual;
    int32_t nonfinite; /* 1 if any QoI became NaN or infinite */
} sn_qoi;

typedef struct sn_plan sn_plan;

/* Validate a problem statement and build a plan (host only; no device work).
 * Copies every input array. Returns SN_ERR_INVALID with the reason in
 * sn_last_error() for a statement the method does not define. */
sn_status sn_plan_create(const sn_problem *problem, sn_plan **out);

/* Same, with an explicit launch shape (0 = library default for each):
 * group_size ordinates per workgroup (both stages), rows_per_wave grid rows
 * per wavefront (2 or 4), waves_per_group compute wavefronts per workgroup
 * (4 or 8; one more wavefront stages rows for them). Returns
 * SN_ERR_UNSUPPORTED for a shape the library was not compiled for. */
sn_status sn_plan_create_tuned(const sn_problem *problem, int32_t group_size,
                               int32_t rows_per_wave, int32_t waves_per_group,
                               sn_plan **out);

/* Same, with separate ordinates per workgroup for the update stage (Euler,
 * Heun stage 1, and the QoI pass) and for Heun's averaging stage, whose
 * workgroups stream psi^n as well (0 = library default for each). */
sn_status sn_plan_create_shaped(const sn_problem *problem, int32_t group_size_update,
                                int32_t group_size_average, int32_t rows_per_wave,
                                int32_t waves_per_group, sn_plan **out);

sn_status sn_plan_get_info(const sn_plan *plan, sn_plan_info *out);

/* Lend device buffers: psi_a and psi_b of info.psi_bytes each, scratch of
 * info.scratch_bytes; all 256-byte aligned, non-overlapping, valid until the
 * plan is destroyed or rebound. */
sn_status sn_plan_bind(sn_plan *plan, void *psi_a, void *psi_b, void *scratch);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): the same as
 * sn_plan_bind, with the scratch taken from an area of SN_STATIC_SCRATCH_BYTES
 * that the library keeps in the memory of every device it is loaded on (held
 * until the process ends) instead of a caller buffer. psi_a and psi_b are the
 * caller's, as for sn_plan_bind. The area belongs to the device current at
 * this call. Allocates nothing: no device allocation or free, and no
 * allocating library routine.
 *  - SN_ERR_UNSUPPORTED when the plan's scratch_bytes (sn_plan_get_info)
 *    exceed SN_STATIC_SCRATCH_BYTES: bind caller-owned scratch instead.
 *  - SN_ERR_BUSY while another plan is bound to the same device's area: the
 *    area holds one plan's tables, QoI accumulators and phi at a time; that
 *    plan must be destroyed or bound elsewhere first. The area keeps what the
 *    last plan left in it; sn_plan_init resets everything a solve reads
 *    before writing it.
 *  - Work of one plan on two streams that overlaps on the device races on the
 *    area, as it does on caller scratch.
 * Rebinding the plan (either call) or destroying it frees the area for other
 * plans. */
#define SN_STATIC_SCRATCH_BYTES (64 << 20)
sn_status sn_plan_bind_static(sn_plan *plan, void *psi_a, void *psi_b);

/* Upload the plan's tables, set psi to psi0 (host [M][ny][nx] float32, or
 * NULL for psi0 = 0 as in both benchmarks), reset step and QoI integrals.
 * Asynchronous on `stream`; psi0 is copied before the call returns. */
sn_status sn_plan_init(sn_plan *plan, const float *psi0, void *stream);

/* Advance min(n_steps, N_t - step) time steps. Asynchronous. */
sn_status sn_plan_run(sn_plan *plan, int32_t n_steps, void *stream);

/* Advance exactly n_steps (may go past N_t; used for timing). Asynchronous. */
sn_status sn_plan_run_unbounded(sn_plan *plan, int32_t n_steps, void *stream);

/* QoIs of the current state and the integrals so far. Synchronises `stream`.
 * Returns SN_ERR_NONFINITE (with *out filled) if any QoI is not finite. */
sn_status sn_plan_qoi(sn_plan *plan, sn_qoi *out, void *stream);

/* Copy the current psi to host [M][ny][nx] float32 (BF16 widened exactly).
 * Synchronises `stream`. */
sn_status sn_plan_read_psi(const sn_plan *plan, float *host_out, void *stream);

/* Copy the current scalar flux phi = sum_k w_k psi_k to host [ny][nx]
 * float32 (the FP32 value the next stage uses). Synchronises `stream`. */
sn_status sn_plan_read_phi(const sn_plan *plan, float *host_out, void *stream);

/* Copy the probes' window averages (sn_problem.n_probes) accumulated since
 * sn_plan_init to host [n_windows][n_probes][3] float64 = (phi, J_x, J_y);
 * windows not reached yet hold their partial integral over the window's
 * full length. Synchronises `stream`. SN_ERR_STATE if the plan has no
 * probes. */
sn_status sn_plan_read_probes(const sn_plan *plan, double *host_out, void *stream);

/* Copy the fluence Phi (sn_problem.fluence) accumulated since sn_plan_init
 * to host [ny][nx] float64. Synchronises `stream`. SN_ERR_STATE if the plan
 * does not accumulate it. */
sn_status sn_plan_read_fluence(const sn_plan *plan, double *host_out, void *stream);

/* One piece of an integral of a = sigma_a Phi over a set made of cells: the
 * piece's value is the mean of a over cells cell_a and cell_b (interior
 * indices j * nx + i; equal for a piece inside one cell, the two cells that
 * share a face for a piece of a line along that face), and it enters its
 * set's integral with `weight` (the piece's area or length divided by the
 * set's, so that a set's weights sum to 1). */
typedef struct sn_fluence_piece {
    int32_t cell_a, cell_b;
    double weight;
} sn_fluence_piece;

/* Block and line functionals of the fluence (Hohlraum QoI-3 to QoI-6,
 * Sec. 3.2.2), computed on the device in FP64 in a fixed order. All three
 * arrays are DEVICE memory owned by the caller (the library allocates
 * nothing):
 *  pieces[n_pieces] sorted by set; set g holds pieces [set_start[g],
 *  set_start[g + 1]) of set_start[n_blocks + 2]: sets 0 .. n_blocks-1 are
 *  the blocks g_i, set n_blocks is the line L; 1 <= n_blocks <=
 *  SN_MAX_FLUENCE_BLOCKS.
 *  out[4 + n_blocks] receives
 *    out[0] A_G = (1/n_blocks) sum_i A_i   with A_i = sum_{p in g_i} w_p a_p
 *    out[1] V_G = (1/n_blocks) sum_i (A_G - A_i)^2
 *    out[2] A_L = sum_{p in L} w_p a_p
 *    out[3] V_L = sum_{p in L} w_p (A_L - a_p)^2
 *    out[4 + i] = A_i,
 *  where a_p is the piece's value (sn_fluence_piece). Uses the fluence as it
 *  stands after the work queued on `stream`; synchronises `stream`.
 * SN_ERR_STATE if the plan does not accumulate the fluence; SN_ERR_INVALID
 * (out filled with NaN) when the kernel finds a cell index out of range, a
 * non-finite weight, or set_start not non-decreasing from 0 to n_pieces. */
sn_status sn_plan_fluence_functionals(const sn_plan *plan, const sn_fluence_piece *pieces,
                                      int32_t n_pieces, const int32_t *set_start,
                                      int32_t n_blocks, double *out, void *stream);

/* Capture `steps_per_graph` steps (even, >= 2; 0 disables) into a hipGraph
 * and replay it in sn_plan_run. */
sn_status sn_plan_use_graph(sn_plan *plan, int32_t steps_per_graph);

/* Per-kernel timing: when on, sn_plan_run records HIP events around every
 * stage launch on the launch stream. sn_plan_kernel_ms returns the summed
 * milliseconds and launch counts per kernel kind: index 0 = Euler stage,
 * 1 = Heun stage 1, 2 = Heun stage 2, 3 = QoI finalize. Synchronises. */
sn_status sn_plan_set_timing(sn_plan *plan, int32_t on);
sn_status sn_plan_kernel_ms(sn_plan *plan, double ms[4], int64_t counts[4]);

void sn_plan_destroy(sn_plan *plan);

/* ------------------------------------------------------------------ batches
 * Many independent solves advanced together (the batched uncertainty-
 * quantification and serving workloads built on the benchmarks of Sec. 3 with
 * the parameter draws of Sec. 3.1.3, DP-2): every admitted plan keeps its own
 * state in its own device buffers. Each stage of the unfinished plans that
 * are too small to fill the GPU on their own runs as one batched launch whose
 * workgroups step over the concatenated tiles of those instances (one
 * workgroup per tile by default, or a persistent grid, see
 * workgroups_per_cu), followed by one batched QoI/phi finalize; plans with at
 * least direct_min_workgroups workgroups per stage take their stages as
 * launches of their own in the same run. Per plan the arithmetic is that of
 * sn_plan_run, so a plan's results are the same alone and in any mix (bit
 * for bit), reading its QoIs mid-run included.
 *
 * Ownership: the batch owns host state only. Its device tables live in a
 * caller-provided workspace of sn_batch_workspace_bytes(opts) bytes (256-byte
 * aligned, valid until sn_batch_destroy). Admitted plans stay owned by the
 * caller and must not be run, rebound, re-initialised or destroyed while
 * admitted. The batch never allocates device memory. */
typedef struct sn_batch_opts {
    int32_t max_instances;     /* slots, 1 .. 4096 */
    int32_t max_steps_per_run; /* most steps one sn_batch_run takes, 1 .. 256 */
    int32_t order, stepper, psi_dtype; /* every admitted plan must match */
    int32_t rows_per_wave, waves_per_group; /* launch shape of every admitted
                                             * plan (0 = library default) */
    uint64_t hbm_budget_bytes; /* admitted plans' 2 psi_bytes + scratch_bytes
                                * may not exceed this (0 = unlimited) */
    int32_t use_graph;         /* 1: each run's launches are captured in a
                                * hipGraph, replayed while the set and the
                                * active pattern are unchanged */
    int32_t workgroups_per_cu; /* stage launches: 0 = one workgroup per tile
                                * (default), > 0 = a persistent grid of that
                                * many workgroups per compute unit striding
                                * over the tiles, -1 = a persistent grid of as
                                * many as are resident at once */
    uint64_t cache_group_bytes; /* > 0: plans whose two psi buffers fit this
                                 * size are packed into groups of at most this
                                 * many bytes that take their steps of a run
                                 * back to back (cache reuse, fewer workgroups
                                 * per launch); 0 (default): every unfinished
                                 * plan takes each stage in one launch */
    int32_t direct_min_workgroups; /* plans with at least this many workgroups
                                    * per stage fill the GPU on their own and
                                    * take their stages as launches of their
                                    * own (kernel arguments, no instance
                                    * lookup); smaller plans share the batched
                                    * launch. 0 = 2 per compute unit, -1 = never */
} sn_batch_opts;

typedef struct sn_batch_info {
    int32_t n_admitted;        /* occupied slots */
    int32_t n_unfinished;      /* admitted plans with step < N_t */
    uint64_t bytes_admitted;   /* sum of the admitted plans' footprints */
    uint64_t hbm_budget_bytes;
    int64_t launches;          /* batched stage launches issued so far */
    int64_t graph_replays;     /* runs served by replaying a captured graph */
} sn_batch_info;

typedef struct sn_batch sn_batch;

/* Workspace bytes for these options. SN_ERR_INVALID on bad options. */
sn_status sn_batch_workspace_bytes(const sn_batch_opts *opts, uint64_t *bytes);

/* Host-only set-up (plus one query of the current device's compute units). */
sn_status sn_batch_create(const sn_batch_opts *opts, void *workspace, sn_batch **out);

/* Footprint of a plan in HBM: 2 psi_bytes + scratch_bytes. */
sn_status sn_plan_footprint(const sn_plan *plan, uint64_t *bytes);

/* Admit a bound and initialised plan into a free slot. SN_ERR_BUSY when no
 * slot is free or the budget would be exceeded; SN_ERR_INVALID when its order,
 * stepper, storage type or launch shape differs from the batch's. Uploads the
 * plan's launch tables (synchronous copy). */
sn_status sn_batch_admit(sn_batch *batch, sn_plan *plan, int32_t *slot);

/* Advance every admitted plan with step < N_t by min(n_steps, N_t - step)
 * steps, 1 <= n_steps <= max_steps_per_run. Asynchronous on `stream`. */
sn_status sn_batch_run(sn_batch *batch, int32_t n_steps, void *stream);

/* Per-slot step quota: in every later sn_batch_run the slot advances at most
 * `steps` steps (1 .. max_steps_per_run; 0 removes the quota;
 * SN_STEPS_PAUSED keeps the slot's state where it is until the quota is set
 * again). A scheduler uses it to share the GPU by work rather than by steps,
 * or to give the oldest request full runs and let later ones fill in. */
#define SN_STEPS_PAUSED (-1)
sn_status sn_batch_set_steps(sn_batch *batch, int32_t slot, int32_t steps);

/* Host view of a slot: done = (step == N_t). The QoIs of the plan come from
 * sn_plan_qoi on the plan itself (synchronising). */
sn_status sn_batch_status(const sn_batch *batch, int32_t slot, int32_t *done, int64_t *step);

/* Free a slot; the plan is the caller's again (in whatever state it reached). */
sn_status sn_batch_retire(sn_batch *batch, int32_t slot);

sn_status sn_batch_get_info(const sn_batch *batch, sn_batch_info *out);

void sn_batch_destroy(sn_batch *batch);

const char *sn_status_str(sn_status s);
const char *sn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SNRT_H */
