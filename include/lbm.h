/*
 * lbm.h -- C-ABI of the MI355X (gfx950) D2Q9 Shan-Chen lattice Boltzmann
 * library (libsclbm.so).
 *
 * Method: the pseudopotential multiphase lattice Boltzmann step of Li & Zhang,
 * "Physics-Informed Neural Networks for Enhanced Interface Preservation in
 * Lattice Boltzmann Multiphase Simulations", arXiv 2504.10539:
 *   - Sec. II-A, Eq. (1): f_i(x + e_i, t + 1) = f_i(x, t) + Omega_i + F_i,
 *     with a pseudopotential interaction force; read here as D2Q9,
 *     psi = 1 - exp(-rho), F = -G psi(x) sum_i w_i psi(x + e_i) e_i, BGK
 *     collision towards the equilibrium at the force-shifted velocity
 *     u_eq = sum_i f_i e_i / rho + tau F / rho, and periodic streaming;
 *   - Sec. III-A: droplet in a square periodic domain;
 *   - Sec. II-D Eqs. (9)-(13), Sec. IV-E Eqs. (14)-(16): interface metrics.
 *
 * Conventions shared by every entry point:
 *   - Velocities e0 = (0,0); e1..e4 = (1,0) (0,1) (-1,0) (0,-1);
 *     e5..e8 = (1,1) (-1,1) (-1,-1) (1,-1); weights 4/9, 1/9, 1/36.
 *   - Arrays a caller reads or writes are plane-major, x fastest: population
 *     states (lbm_get_state / lbm_set_state) have element (i, y, x) at
 *     i*nx*ny + y*nx + x, fields (lbm_moments) element (y, x) at y*nx + x.
 *     The layout inside the two population buffers is private to the
 *     library (row-interleaved: row y of population i at (9 y + i) nx).
 *   - "State at step t" means the pre-collision populations f_i(x, t).
 *   - Device pointers are HIP device addresses (e.g. torch tensors on the
 *     GPU).  The library never allocates, frees or retains device memory
 *     beyond the lifetime rules stated per call; every buffer is the
 *     caller's.  Host pointers are read during the call only, unless stated.
 *   - Work is enqueued on the caller's HIP stream given at creation and is
 *     asynchronous unless a call says it synchronises.  Errors from
 *     asynchronous work surface at the next synchronising call.
 *   - Every call returns an lbm_status; on failure lbm_last_error() gives a
 *     thread-local message.  No C++ exception crosses this boundary.
 */
#ifndef SCLBM_LBM_H
#define SCLBM_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;

#define LBM_OK 0
#define LBM_EINVAL (-1)    /* invalid argument, or state misuse */
#define LBM_ENOMEM (-2)    /* a caller buffer is too small, or a request can never fit the pool */
#define LBM_EDEVICE (-3)   /* a HIP runtime call failed */
#define LBM_PENDING (-4)   /* lbm_poll: the request has not finished */
#define LBM_EUNSTABLE (-5) /* non-finite populations or non-positive density */
#define LBM_ENOTFOUND (-6) /* unknown or already-collected ticket */
#define LBM_EBUSY (-7)     /* the context is driven by a batch or server */

/* Population storage. */
#define LBM_F32 0          /* FP32 populations, 36 bytes per cell per buffer */
#define LBM_F16_SHIFTED 1  /* FP16 h_i = f_i - w_i rho0 (the FP32 difference,
                              then rounded to nearest even), read back as
                              float(h_i) + w_i rho0; 18 bytes per cell per
                              buffer; arithmetic stays FP32 */
#define LBM_F16_CELL 2     /* FP16 shifted per cell: the nine values a cell x
                              stores hold A_i(x) - w_i rhohat(x) (rounded
                              once to nearest even from the exact value), with
                              rhohat(x) = half(rho) of that cell stored in a
                              tenth FP16 plane; read back as rhohat w_i + h_i
                              rounded once.  20 bytes per cell per buffer, 40
                              bytes moved per lattice update */
#define LBM_F16_MOMENT 3   /* FP16 with exact conserved moments: a cell x stores
                              the record of the nine values A_i(x) it wrote -
                              its density rho (the record's mass) and the
                              momentum jx, jy of the A_i in FP32, and A_3 .. A_8
                              as h_i = half(A_i - w_i rho) (rounded once from
                              the exact value) - read back as
                              A_i = rho w_i + h_i (i >= 3), A_1 and A_2 from the
                              momentum, A_0 = rho - (the other eight).  Mass and
                              momentum pass between cells at FP32 rounding;
                              only non-conserved moments round to half
                              precision.  24 bytes per cell per buffer, 48
                              bytes moved per lattice update (24 with two
                              steps per launch).  Tile shapes: strips, and
                              two-step shapes of width <= threads - 8 (no
                              paired-column shapes) */

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;
typedef struct lbm_server lbm_server;

/* Simulation parameters (Sec. III-A: square periodic domain, tau, g). */
typedef struct lbm_params {
  int32_t nx, ny;   /* grid size, periodic in x and y; 1 <= nx, ny <= 65536 */
  double G;         /* interaction strength (negative for attraction), finite */
  double tau;       /* BGK relaxation time, tau > 0.5 */
  int32_t storage;  /* LBM_F32, LBM_F16_SHIFTED, LBM_F16_CELL or LBM_F16_MOMENT */
  double rho0;      /* LBM_F16_SHIFTED's shift density (finite, >= 0); ignored otherwise */
} lbm_params;

/* Droplet initial condition (Sec. III-A).  For each cell (x, y):
 *   rho = rho_g + (rho_l - rho_g) max_k s_k + eta,
 *   s_k = 0.5 (1 - tanh((r_k - R_k) / width)),
 * r_k the minimum-image distance, in a periodic frame of period_x x period_y
 * cells, from the integer point (origin_x + x, origin_y + y) to droplet k's
 * centre; eta = noise_amp (2u - 1), u in [0, 1) the top 53 bits of the
 * (gy * period_x + gx)-th output of SplitMix64 seeded with `seed`
 * (gx, gy the cell's frame coordinates).  period 0 means the grid itself and
 * requires origin 0; the grid must lie inside the frame (origin + nx <=
 * period_x, origin + ny <= period_y).  The fluid starts at rest:
 * f_i = w_i rho. */
typedef struct lbm_init {
  double rho_l, rho_g;   /* liquid and gas densities */
  double width;          /* tanh width (> 0) */
  double noise_amp;      /* >= 0 */
  uint64_t seed;
  int64_t period_x, period_y;
  int64_t origin_x, origin_y;
} lbm_init;

/* Interface metrics and conservation diagnostics of the state at `step`,
 * evaluated in FP64 on the GPU from the stored populations. */
typedef struct lbm_metrics {
  double W;         /* Eq. (9): fraction of cells with |grad rho| > 0.01 */
  double Gmax;      /* Eq. (10): max |grad rho| */
  double drho;      /* Eq. (11): rho_max - rho_min */
  double W_eff;     /* Eqs. (12),(14): sum |grad rho| / (Gmax nx ny); 0 if Gmax = 0 */
  double E_int;     /* Eqs. (13),(15): sum |grad rho|^2 */
  double rho_max, rho_min;
  double sum_grad;  /* sum |grad rho| */
  double mass;      /* sum_x sum_i f_i */
  double mom_x, mom_y; /* sum_x sum_i f_i e_i */
  int64_t n_above;  /* number of cells with |grad rho| > 0.01 */
  int64_t step;     /* time step t of the state */
  int32_t finite;   /* 1 if every population is finite and every rho > 0 */
  int32_t reserved;
} lbm_metrics;

/* ------------------------------------------------------------ single run */

/* Sizes the caller must allocate for one run: `pop_bytes` for EACH of the two
 * population buffers (9 * nx * ny * 4 for LBM_F32, * 2 for LBM_F16_SHIFTED,
 * 10 * nx * ny * 2 for LBM_F16_CELL, 24 * nx * ny for LBM_F16_MOMENT),
 * and `work_bytes` of device workspace (tile tables and reduction partials).
 * Either output pointer may be NULL.  LBM_EINVAL for invalid parameters. */
lbm_status lbm_buffer_bytes(const lbm_params* p, size_t* pop_bytes, size_t* work_bytes);

/* Creates a run over caller-owned device buffers popA, popB (each
 * >= pop_bytes, 256-byte aligned) and `work` (>= work_bytes, 256-byte
 * aligned), all borrowed until lbm_destroy.  `hip_stream` is the caller's
 * hipStream_t (NULL = the default stream).  The state is undefined until
 * lbm_init_droplets or lbm_set_state.  Picks the tile shape from the tuning
 * cache when one applies (see lbm_autotune), else a default.
 * Errors: LBM_EINVAL (parameters, NULL or misaligned pointers), LBM_ENOMEM
 * (a buffer is smaller than required), LBM_EDEVICE. */
lbm_status lbm_create(const lbm_params* p, void* popA, void* popB, size_t pop_bytes,
                      void* work, size_t work_bytes, void* hip_stream, lbm_ctx** out);

/* Releases host state.  Never frees caller memory.  Synchronises the stream. */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* Writes the droplet initial condition (see lbm_init) as the state at t = 0.
 * `drops` is a host array of n x 3 doubles (cx, cy, R), copied during the
 * call; n = 0 gives a uniform rho_g plus noise.  Uses the second population
 * buffer as scratch (8 bytes per cell for rho, then the droplet list), so n
 * is limited to (pop_bytes - 8 nx ny) / 24; LBM_EINVAL beyond that or for
 * bad lbm_init fields.  Synchronises the stream. */
lbm_status lbm_init_droplets(lbm_ctx* ctx, const double* drops, int32_t n, const lbm_init* ip);

/* Enqueues n >= 0 time steps (Eq. (1)): one fused pull-stream, force and
 * collide kernel launch per step, per two steps with a two-step tile shape
 * (plus one single-step launch when n is odd) or per three with a three-step
 * shape (plus one two-step or one single-step launch for the steps left
 * over), alternating the two buffers.
 * Returns after enqueue.  LBM_EBUSY if the context belongs to a live batch. */
lbm_status lbm_step_n(lbm_ctx* ctx, int64_t n);

/* Advances n >= 0 steps like lbm_step_n and records the interface metrics of
 * every `every`-th state on the way (the time series of Sec. IV's evolution
 * runs): the states at step counts t0, t0 + every, ... below t0 + n, where t0
 * is lbm_step_count at the call, ceil(n / every) records in all, written to
 * out[0 ..] (host array of `capacity` records; *count receives the number
 * written).  Each record is computed inside the launch that advances that
 * state, from the populations it pulls, with the FP64 arithmetic of
 * lbm_interface_metrics (rho summed in FP64 in index order, Eq. (16) with
 * periodic wrap): n_above, G_max, rho_max and rho_min equal what
 * lbm_interface_metrics reports for that state, and the sums agree up to FP64
 * summation order.  The step itself is bitwise the one lbm_step_n takes.  The
 * metrics of the final state t0 + n are not included (lbm_interface_metrics
 * gives them).  Synchronises.  LBM_EINVAL if every < 1 or capacity <
 * ceil(n / every); LBM_EBUSY for a member of a live batch. */
lbm_status lbm_step_series(lbm_ctx* ctx, int64_t n, int32_t every, lbm_metrics* out,
                           int32_t capacity, int32_t* count);

/* Writes the macroscopic fields of the current state into caller device
 * arrays of nx * ny floats: rho = sum_i f_i and the half-force-corrected
 * velocity u = (sum_i f_i e_i + F / 2) / rho (the density and velocity fields
 * that Sec. II-B, Eq. (2), takes as the fluid variables).  Any pointer may be NULL.
 * FP32.  Uses the idle population buffer as scratch.  Asynchronous. */
lbm_status lbm_moments(lbm_ctx* ctx, float* rho, float* ux, float* uy);

/* Computes the interface metrics (Eqs. (9)-(16), periodic central
 * differences) and the conservation sums of the current state in FP64 on the
 * GPU; deterministic for a fixed tile shape.  Synchronises the stream and
 * fills the host struct.  Uses the idle population buffer as scratch. */
lbm_status lbm_interface_metrics(lbm_ctx* ctx, lbm_metrics* out);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops that must not allocate, harnesses that forbid it): the metrics of
 * lbm_interface_metrics, computed by the same kernels, written as one
 * lbm_metrics record to `out`, caller device memory (8-byte aligned), without
 * waiting for the stream.  Nothing is allocated: the FP64 density goes into the
 * idle population buffer, as in lbm_interface_metrics, and the reduction
 * partials into a static device array of 2048 partial records (264 KiB per
 * GPU the library runs on, held until the process ends) instead of the
 * run's workspace; the pass never needs more than 2048 records (LBM_ENOMEM
 * if it ever would).  The array is shared by every call on one GPU: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller.  The record equals what lbm_interface_metrics
 * reports for the same state.  Asynchronous. */
lbm_status lbm_interface_metrics_noalloc(lbm_ctx* ctx, lbm_metrics* out);

/* Copies the current state out as 9 planes of nx * ny FP32 pre-collision
 * populations f_i(x, t) into a caller device buffer (FP16 storage is widened
 * exactly as the step kernel reads it).  With lbm_set_state it forks runs
 * from one common state, as the protocol of Sec. III-C continues the pure
 * LBM run and the coupled run from the same initialised droplet.
 * Asynchronous. */
lbm_status lbm_get_state(lbm_ctx* ctx, float* f);

/* Replaces the current state with caller-supplied FP32 populations (same
 * layout as lbm_get_state), rounded to the storage type; the step counter is
 * kept (the fork of Sec. III-C).  Asynchronous. */
lbm_status lbm_set_state(lbm_ctx* ctx, const float* f);

/* Number of time steps taken since the last init / set_state-free creation. */
int64_t lbm_step_count(const lbm_ctx* ctx);

/* Tile shapes of the step kernel.  Shape k (0 <= k < lbm_tile_count()) is a
 * strip of `width` columns marched over `rows` rows by `threads` threads with
 * `prefetch` rows of loads in flight, each thread holding `cells` cells of a
 * row.  paired = 0: the psi halo of a row is shared through LDS (any grid
 * width).  paired = 1: each lane holds two adjacent cells and takes its
 * column neighbours from the adjacent lanes of its wavefront; such shapes
 * need an even nx >= 128 (lbm_set_tile returns LBM_EINVAL otherwise).
 * steps = 2: one launch advances the strip two time steps, the intermediate
 * populations kept on chip (rounded to the storage type as a store would
 * round them); such a strip reads three halo columns on each side of its
 * `width`, which is threads - 6 or a multiple of 16 below that (strips that
 * start and end on 64-byte boundaries in FP32), and a grid no wider than
 * `threads` is marched as one periodic strip with no halo columns.  steps =
 * 3 (LBM_F32 only): the same over three time steps, five halo columns on
 * each side (`width` a multiple of 16, at most threads - 10).  rows = 0:
 * balanced bands, whose height is chosen per grid so that a launch is about
 * two rounds of the workgroups the device holds at once (lbm_tile_layout
 * gives it).  LBM_F16_MOMENT runs strip shapes (steps = 1, paired = 0) and
 * two-step shapes of at most threads - 8 columns; lbm_set_tile refuses the
 * shapes a storage type does not run with LBM_EINVAL.  Every valid shape
 * computes bitwise the same result; only speed differs.  Any output pointer
 * may be NULL; k out of range is LBM_EINVAL. */
int32_t lbm_tile_count(void);
lbm_status lbm_tile_describe(int32_t k, int32_t* width, int32_t* rows, int32_t* threads,
                             int32_t* prefetch, int32_t* cells, int32_t* paired, int32_t* steps);
/* Band height (*rows) and number of work items (*items) of tile shape k on a
 * grid with these parameters.  For a balanced shape the height depends on
 * the step kernel's occupancy on the current device.  Either output may be
 * NULL; invalid parameters or k out of range are LBM_EINVAL. */
lbm_status lbm_tile_layout(const lbm_params* p, int32_t k, int32_t* rows, int32_t* items);
/* The built-in tile shape a run with these parameters starts with when the
 * tuning cache has no entry for it (*k; measured defaults by storage type and
 * grid size).  Invalid parameters are LBM_EINVAL. */
lbm_status lbm_default_tile(const lbm_params* p, int32_t* k);
lbm_status lbm_set_tile(lbm_ctx* ctx, int32_t k);
int32_t lbm_get_tile(const lbm_ctx* ctx);

/* Times every tile shape on this run's grid (each shape `reps` launches,
 * reading the current buffer and writing the idle one, so the state is not
 * changed), selects the fastest per time step, and records it in the tuning cache
 * (a JSON file named by the SCLBM_TUNE_CACHE environment variable; no file
 * if unset) keyed by device architecture, storage and grid size; entries
 * written for another tile table are ignored.
 * Synchronises.  *best (may be NULL) receives the chosen shape. */
lbm_status lbm_autotune(lbm_ctx* ctx, int32_t reps, int32_t* best);

/* lbm_autotune timed as the run steps: the state is first copied to
 * `scratch` (caller-owned device memory of at least lbm_buffer_bytes'
 * pop_bytes, 256-byte aligned, borrowed for the call), each shape then
 * advances the run `reps` launches with the buffers alternating (every
 * launch reads what the previous one wrote), and afterwards the state, the
 * buffer holding it and the step count are restored.  On grids whose two
 * buffers fit the GPU's caches, repeated launches over one unchanged buffer
 * run faster than stepping does, and by a different amount per shape; this
 * entry point measures what stepping costs.  Same selection and tuning cache
 * as lbm_autotune.  LBM_EINVAL for a NULL or unaligned scratch, LBM_ENOMEM
 * when scratch_bytes is too small.  Synchronises. */
lbm_status lbm_autotune_stepping(lbm_ctx* ctx, int32_t reps, void* scratch, size_t scratch_bytes,
                                 int32_t* best);

/* ------------------------------------------------------------ batched runs */

/* Workspace needed to advance the n contexts together. */
lbm_status lbm_batch_work_bytes(lbm_ctx* const* ctxs, int32_t n, size_t* bytes);

/* Groups n >= 1 contexts created on the same stream into one batch that
 * advances all of them with one persistent multi-instance kernel launch per
 * time step (one per storage type present), `steps_per_graph` steps captured
 * in a HIP graph and replayed.  Each storage type uses the step shape of its
 * widest member's tile: with a two-step shape, one launch per two steps and a
 * single-step launch for a member's odd last step of a replay; with a
 * three-step shape (LBM_F32), one launch per three steps and a two-step or a
 * single-step launch for the steps a member has left over in a replay.  The
 * per-cell arithmetic is the same code as lbm_step_n, so every member's
 * result is bitwise the one it would have alone.  The contexts are borrowed and must not be stepped on their own
 * (LBM_EBUSY) until lbm_batch_destroy; metrics, moments and state copies on a
 * member stay valid.  `work` is a caller device buffer of >=
 * lbm_batch_work_bytes bytes. */
lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int32_t n, void* work, size_t work_bytes,
                            int32_t steps_per_graph, lbm_batch** out);

/* Enqueues n time steps of every member.  Asynchronous. */
lbm_status lbm_batch_step_n(lbm_batch* b, int64_t n);

/* Times every tile shape on the whole batch (each shape `reps` launches in
 * which every member reads its current buffer and writes its idle one, so no
 * state changes) and rebuilds the batch's graph with the fastest shape for
 * all members; members' own single-run tile shapes are left as they are.
 * Synchronises.  *best (may be NULL) receives the chosen shape. */
lbm_status lbm_batch_autotune(lbm_batch* b, int32_t reps, int32_t* best);

/* Releases the batch (synchronises the stream); members become free again. */
lbm_status lbm_batch_destroy(lbm_batch* b);

/* ------------------------------------------------------------ serving */

#define LBM_POLICY_CONTINUOUS 0  /* continuous batching: admit while memory and slots allow */
#define LBM_POLICY_FIFO 1        /* plain path: one simulation at a time, its own tile shape */

typedef struct lbm_server_opts {
  int32_t policy;          /* LBM_POLICY_CONTINUOUS or LBM_POLICY_FIFO */
  int32_t steps_per_tick;  /* time steps per scheduling tick (graph length), >= 1 */
  int32_t max_slots;       /* maximum resident simulations, >= 1 */
  int32_t fake_executor;   /* 1: host-only virtual executor, no GPU work (tests) */
  double fake_mlups;       /* virtual executor speed in MLUPS when fake_executor = 1 */
} lbm_server_opts;

/* One droplet simulation request.  Host arrays are copied by lbm_submit. */
typedef struct lbm_request {
  lbm_params params;
  lbm_init init;
  const double* drops;     /* n_drops x 3 (cx, cy, R) */
  int32_t n_drops;
  int32_t reserved;
  int64_t steps;           /* >= 0 */
  float* rho_out;          /* optional device array nx*ny: final rho (FP32); NULL to skip */
  float* f_out;            /* optional device array 9*nx*ny: final state (FP32); NULL to skip */
} lbm_request;

typedef struct lbm_result {
  lbm_metrics metrics;     /* metrics of the final state */
  double t_submit, t_admit, t_done; /* seconds on the server clock */
  int64_t ticket;
} lbm_result;

typedef struct lbm_server_stats {
  int64_t submitted, admitted, completed, failed, queued, resident;
  int64_t ticks;
  double lattice_updates;  /* sum over requests completed with LBM_OK of nx*ny*steps */
  size_t pool_bytes;       /* bytes of the pool available to requests (the
                              continuous policy keeps its batch tables in the
                              rest) */
  size_t pool_in_use, pool_high_water;
  int64_t unstable;        /* requests completed with LBM_EUNSTABLE (also in failed) */
  int64_t retired_early;   /* of those, retired before their last step */
  double unstable_updates; /* lattice updates the unstable requests advanced */
} lbm_server_stats;

/* Starts a serving loop on a scheduler thread.  `pool` (caller device buffer
 * of pool_bytes, 256-byte aligned) is the HBM budget: each admitted request's
 * two population buffers and workspace are carved out of it and returned on
 * completion; the continuous policy keeps its batch tables at the top of the
 * pool (lbm_server_stats.pool_bytes gives what is left for requests).
 * Requests are admitted first-come first-served, except that a request that
 * does not fit yet may be passed by a later one that does.  Admitted requests
 * are initialised and advanced together.  A run whose step kernels meet a cell
 * with a non-finite or non-positive density is retired within a tick or two,
 * before its last step, and completes with LBM_EUNSTABLE (its result's
 * metrics.step is where it stopped).  With fake_executor = 1, pool may be
 * NULL and no GPU is used; a request whose starting density is not positive
 * then stands for an unstable run and is retired after its first tick. */
lbm_status lbm_server_create(void* pool, size_t pool_bytes, void* hip_stream,
                             const lbm_server_opts* opts, lbm_server** out);

/* Queues a request; thread-safe.  LBM_EINVAL for bad parameters (checked
 * before any host array is read: n_drops must fit the grid's scratch, as in
 * lbm_init_droplets), LBM_ENOMEM if the request alone exceeds the pool's
 * capacity for requests, LBM_EDEVICE if the scheduler has stopped on an
 * internal error. */
lbm_status lbm_submit(lbm_server* s, const lbm_request* r, uint64_t* ticket);

/* Non-blocking: LBM_PENDING, or LBM_OK / LBM_EUNSTABLE with *out filled (the
 * ticket is then released; a second poll gives LBM_ENOTFOUND). */
lbm_status lbm_poll(lbm_server* s, uint64_t ticket, lbm_result* out);

/* Blocks until every submitted request has finished (results stay pollable). */
lbm_status lbm_server_drain(lbm_server* s);

lbm_status lbm_server_get_stats(lbm_server* s, lbm_server_stats* out);

/* Seconds on the server's monotonic clock (the clock of lbm_result). */
double lbm_server_clock(const lbm_server* s);

/* Stops the scheduler after draining, then releases host state. */
lbm_status lbm_server_destroy(lbm_server* s);

/* ------------------------------------------------------------ PINN surrogate */

/* The network of Sec. III-B: inputs (x, y), hidden layers of 64, 128, 128
 * and 64 neurons with tanh, a linear output layer giving (rho, u_x, u_y)
 * (Sec. II-B, Eq. (2)).  Its parameters are one device array of
 * LBM_PINN_PARAMS FP32 values: for each layer l = 1..5 in order, W_l
 * row-major with shape (out, in) (a layer maps h to W_l h + b_l), then b_l.
 * The input of cell (x, y) is its centre scaled to (-1, 1):
 * ((2 x + 1) / nx - 1, (2 y + 1) / ny - 1).  Layers 2 to 4 run on the matrix
 * cores with their weights and inputs rounded to FP16 and FP32 accumulation;
 * layers 1 and 5 and tanh are FP32.  The hidden activations are rounded to
 * FP16 between layers, so an output differs from the same network in exact
 * arithmetic by at most ||W_5|| (2^-11 sqrt(64) + ||W_4|| (2^-11 sqrt(128) +
 * ||W_3|| (2^-11 sqrt(128) + ||W_2|| 2^-11 sqrt(64)))) (spectral norms of the
 * FP16-rounded weights) plus FP32 rounding. */
#define LBM_PINN_PARAMS 33475

/* The network's fields at every cell of the run's grid: rho_N, u_x and u_y
 * into caller device arrays of nx * ny floats (row-major; any may be NULL).
 * `params` is a device array of LBM_PINN_PARAMS floats (4-byte aligned).
 * Does not touch the state.  Asynchronous. */
lbm_status lbm_pinn_infer(lbm_ctx* ctx, const float* params, float* rho, float* ux, float* uy);

/* The correction of Sec. II-C, applied to the current state at its interface
 * cells: the cells with |grad rho| > 0.01 (Eq. (9), the Eq. (16) gradient
 * with periodic wrap, rho in FP64 from the stored populations).  On such a
 * cell, with rho and u = sum_i f_i e_i / rho of its populations and the
 * network's rho_N, u_N: rho' = rho + beta (rho_N - rho), u' = u + beta
 * (u_N - u), and f_i becomes f_i + f_eq_i(rho', u') - f_eq_i(rho, u) (FP32),
 * stored back in the run's storage form; every other cell is left bitwise as
 * it was.  beta in [0, 1].  `mask` (optional caller device array of nx * ny
 * bytes) receives 1 for the corrected cells, 0 elsewhere.  Uses the idle
 * population buffer as scratch.  LBM_EINVAL for LBM_F16_MOMENT (its records
 * hold no single value per population to rewrite), a bad beta or a NULL or
 * misaligned params; LBM_EBUSY for a member of a live batch.
 * Asynchronous. */
lbm_status lbm_pinn_correct(lbm_ctx* ctx, const float* params, double beta, uint8_t* mask);

/* ------------------------------------------------------------ measurement */

/* Device-to-device copy of `bytes` (multiple of 16) with a plain streaming
 * kernel, on `hip_stream`: the achievable-bandwidth reference for the step
 * kernel's roofline.  Asynchronous. */
lbm_status lbm_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* Thread-local description of the last failure in this thread. */
const char* lbm_last_error(void);

/* Library version string. */
const char* lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SCLBM_LBM_H */
