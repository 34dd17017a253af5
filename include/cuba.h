/*
 * cuba.h -- C ABI of libcuba.so, an MI355X (gfx950) implementation of the
 * per-time-step particle-in-cell Boltzmann update of "CuBA - a CUDA
 * implementation of BAMPS" (Cardoso, Bicudo, Eilhauer, Bouras;
 * arXiv:1208.0961).
 *
 * The method (Sec. 2 of the paper): a massless gluon gas is represented by
 * test particles with position r and momentum p in a box with reflecting
 * walls, divided into cells of volume V_cell = dx dy dz.  One step of length
 * dt
 *   1. free-streams every particle, x <- x + (p_x / E) dt with E = |p|
 *      (Eq. (2), c = 1), likewise y and z;
 *   2. reflects it elastically at the six walls (mirror the overshoot, flip
 *      the normal momentum component);
 *   3. bins the particles into cells;
 *   4. tests every pair (a < b) of particles in the same cell for a binary
 *      collision with probability P22 = v_rel sigma / r_test * dt / V_cell,
 *      v_rel = s / (2 E1 E2) (Eq. (3) with the test-particle rescaling);
 *      a particle scatters at most once per step: pairs are taken in
 *      lexicographic order of their canonical indices and skipped when a
 *      member has already scattered in the step;
 *   5. gives each accepted pair an isotropic direction in its CM frame with
 *      |p*| = sqrt(s)/2 and boosts back to the lab.
 *
 * Determinism contract.  Within a cell, particles are ordered by id (the
 * index in the arrays given to cuba_init); pair (a, b) of an n-particle
 * cell c has index k = a (2n - a - 1) / 2 + (b - a - 1).  Its acceptance
 * uniform is u = ((w1:w0) >> 11) 2^-53 of the Philox4x32-10 block with
 * counter (k, c, t, 0) and key (seed low word, seed high word), t the step
 * index; the outgoing direction takes cos(theta) = 2 U53(w0, w1) - 1 and
 * phi = 2 pi U53(w2, w3) of the block with counter (k, c, t, 1), and the
 * lower index a takes +n.  Cell ids are x-major: c = (ix ny + iy) nz + iz,
 * i_d = min(floor(x_d / dx_d), n_d - 1).  Given the same state, step index
 * and seed, cell indices, the canonical order, the candidate and accepted
 * pairs, positions, and the momenta of particles that did not scatter are
 * bit-identical to any correct implementation of this contract; scattered
 * momenta agree to rounding of sin and cos (|dp| <= 1e-12 (Ea + Eb)).
 *
 * Conventions for every function below.
 *  - Units: fm for lengths, GeV for momenta, c = 1.
 *  - "device" pointers are HIP device allocations owned by the caller;
 *    "host" pointers are ordinary host memory.  The library allocates no
 *    device memory: all of its device state lives in the caller's
 *    workspace (or, for cuba_init_static only, in one fixed array per GPU
 *    that the library's code object holds).  It allocates only the small
 *    host-side context.
 *  - stream arguments are hipStream_t values passed as void* (NULL: the
 *    null stream).  All device work of a context is issued on its stream,
 *    asynchronously; errors raised by the device (a cell holding more than
 *    CUBA_MAX_CELL_PARTICLES particles, a trace buffer too small) are
 *    reported by the next cuba_sync.
 *  - A context is not thread-safe; one context per stream.
 *  - Return values: CUBA_OK (0) or a negative CUBA_E* code; cuba_strerror
 *    names the code and cuba_last_error() gives the detail of the most
 *    recent failure on the calling thread.
 */
#ifndef CUBA_H
#define CUBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CUBA_OK 0
#define CUBA_EINVAL -1  /* invalid parameters or arguments                 */
#define CUBA_ERANGE -2  /* a particle outside the box, a non-finite value,
                           |p| = 0, or a cell holding more particles than
                           CUBA_MAX_CELL_PARTICLES                          */
#define CUBA_ENOMEM -3  /* workspace (or trace buffer) too small           */
#define CUBA_EDEVICE -4 /* HIP runtime error; see cuba_last_error()         */

/* Largest cuba_params.cell_capacity (the slots of a cell's block; the
 * collision kernels hold a block's ids in LDS).  Not a limit on how many
 * particles a cell may hold: those past the block are kept in a spill
 * region (sized for every particle of the context) and the cell is stepped
 * by a kernel for such cells. */
#define CUBA_MAX_CELL_CAPACITY 1024

/* Most particles one cell may hold: the pair index k < n (n - 1) / 2 of the
 * determinism contract is one 32-bit word of the Philox counter (it fits up
 * to 92 682 members; the bound stays one lower).  A cell
 * holding more has its collisions skipped (its particles still stream) and
 * the next cuba_sync reports CUBA_ERANGE. */
#define CUBA_MAX_CELL_PARTICLES 92681

typedef struct cuba_ctx cuba_ctx;

/* Problem definition (Sec. 2; the step-size rule is from Sec. 5). */
typedef struct {
  double box[3];    /* Lx, Ly, Lz [fm] > 0; walls at 0 and L_d on each axis */
  int32_t cells[3]; /* nx, ny, nz >= 1; dx_d = L_d / n_d (FP64)             */
  double sigma;     /* total isotropic cross section [fm^2], >= 0           */
  double r_test;    /* test particles per physical particle, > 0            */
  double dt;        /* time step [fm/c], 0 < dt < min_d dx_d                */
  uint64_t seed;    /* Philox key: key[0] = low 32 bits, key[1] = high      */
  uint32_t step0;   /* index t of the first step (0, or t when resuming)    */
  int32_t cell_capacity; /* slots of each cell's block in the workspace, in
                            [1, CUBA_MAX_CELL_CAPACITY]; 0 selects twice the
                            mean occupancy n / cells + 32, rounded up to 32
                            (cuba_suggest_cell_capacity sizes it from the
                            initial state instead).  A layout choice, not a
                            limit: a cell receiving more keeps the surplus
                            in the spill region and is stepped (slower,
                            same result) by the kernel for such cells.     */
} cuba_params;

/* Bytes of device workspace cuba_init needs for n particles with these
 * parameters (for admission by memory footprint): two state buffers of
 * cells x cell_capacity slots of 52 bytes, each with n spill slots (56
 * bytes each, with the cell tag), scratch of 12 bytes per particle for
 * stepping overflowing cells, and per-cell bookkeeping.  Returns 0 if the parameters
 * are invalid.  The workspace must be 256-byte aligned. */
size_t cuba_workspace_bytes(const cuba_params *params, int64_t n);

/* Slots per cell suited to an initial state, counted on the device: twice
 * the largest occupancy of any cell (positions x, y, z: device arrays of n
 * doubles, binned as Sec. 2 bins them; non-finite positions are skipped)
 * plus 32, rounded up to 32, within [64, CUBA_MAX_CELL_CAPACITY]; written
 * to *cap for params.cell_capacity.  scratch: device memory of at least
 * cuba_capacity_scratch_bytes(params), 256-byte aligned, owned by the
 * caller.  Runs on stream and waits for it (a set-up call, not part of a
 * step).  Errors: CUBA_EINVAL for invalid parameters, NULL arrays with
 * n > 0, a NULL cap or too small a scratch; CUBA_EDEVICE. */
size_t cuba_capacity_scratch_bytes(const cuba_params *params);
int cuba_suggest_cell_capacity(const cuba_params *params, int64_t n, const double *x,
                               const double *y, const double *z, void *scratch,
                               size_t scratch_bytes, void *stream, int32_t *cap);

/* Creates a context.  x..pz are device arrays of n doubles (particle id =
 * array index), copied into the workspace; they may be freed once the
 * stream has passed this call.  workspace: device memory of ws_bytes >=
 * cuba_workspace_bytes(params, n), owned by the caller and used by the
 * context until cuba_destroy.  Validates the parameters (CUBA_EINVAL:
 * non-finite or non-positive box, cells, r_test or dt; sigma < 0;
 * dt >= min dx_d; 2 K > 1 with K = sigma / r_test * dt / V_cell, which
 * would let P22 exceed 1) and the particles (CUBA_ERANGE: outside
 * [0, L_d], non-finite, |p| = 0; this check synchronizes the stream), then
 * bins the initial state.  On success *out receives the context. */
int cuba_init(cuba_ctx **out, const cuba_params *params, int64_t n,
              const double *x, const double *y, const double *z,
              const double *px, const double *py, const double *pz,
              void *workspace, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * cuba_init, with the same validation and errors, but the context lives in
 * a workspace the library holds, CUBA_STATIC_WORKSPACE_BYTES of device
 * memory per GPU (allocated with the library's code when it first runs on
 * that GPU and held until the process ends), and a context object the
 * library holds; the call allocates no device memory and no context.  The caller
 * still passes the initial state (device arrays as for cuba_init).
 * CUBA_ENOMEM when cuba_workspace_bytes(params, n) exceeds
 * CUBA_STATIC_WORKSPACE_BYTES.  Every call on a GPU reuses that GPU's
 * workspace and context object: a call ends the previous context set up by
 * this function on the same GPU (its handle must no longer be used), and
 * calls or steps that overlap on one GPU (other threads, other streams)
 * race.  cuba_destroy of the handle only ends its stage timing.  The
 * workspace's contents are those the last call left; this call clears what
 * must start at zero. */
#define CUBA_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int cuba_init_static(cuba_ctx **out, const cuba_params *params, int64_t n,
                     const double *x, const double *y, const double *z,
                     const double *px, const double *py, const double *pz,
                     void *stream);

/* Advances the state by nsteps >= 0 steps, asynchronously on the stream.
 * Step indices continue from params->step0.  Internally one kernel per
 * step does the collisions of step t and the streaming and binning of step
 * t+1; a call issues nsteps + 1 launches, so advancing many steps per call
 * is cheaper than one step per call. */
int cuba_step(cuba_ctx *ctx, int32_t nsteps);

/* Lab-frame energy and x-momentum density profiles over the nx slabs of
 * cells along x, of the current state (Fig. 2 of the paper shows the
 * energy density): T00[ix] = sum_{particles in slab} E / (r_test dx Ly Lz),
 * T0x[ix] = sum p_x / (same) [GeV/fm^3].  T00, T0x: device arrays of nx
 * doubles.  Sums run in the (unspecified) storage order. */
int cuba_observe(cuba_ctx *ctx, double *T00, double *T0x);

/* Moments of the current state over the nx slabs along x, for the approach
 * to ideal hydrodynamics as sigma grows (Sec. 5, Fig. 3).  out: device array
 * of 6 nx doubles, rows in this order:
 *   T00, T0x  as cuba_observe;
 *   Txx = sum p_x^2 / E / (r_test dx Ly Lz)              [GeV/fm^3];
 *   n   = count / (r_test dx Ly Lz)                      [fm^-3];
 *   e, v: the slab's rest frame, T^mu_nu u^nu = e u^mu with u = gamma (1, v)
 *         on the t-x block (transverse flow neglected):
 *         a = T00 + Txx, b = 2|T0x|, d = max((a - b)(a + b), 0),
 *         e = ((T00 - Txx) + sqrt(d)) / 2, v = T0x / (e + Txx) (0 if e + Txx
 *         is 0), evaluated in this order.
 * Errors: CUBA_EINVAL for NULL. */
int cuba_observe_moments(cuba_ctx *ctx, double *out);

/* Copies the current state into device arrays of n doubles in id order. */
int cuba_get_state(cuba_ctx *ctx, double *x, double *y, double *z,
                   double *px, double *py, double *pz);

/* One step with a record of its decisions, for parity checks.  All arrays
 * are device memory owned by the caller; a NULL array is not written.
 *   cell    [n]      cell of each particle (by id) after this step's binning
 *   perm    [n]      ids in canonical (cell, id) order
 *   offsets [C+1]    start of each cell in perm (C = nx ny nz)
 *   cand    [3*cand_cap]   (cell, a, b) of every pair with u < P22 judged on
 *                          the momenta before the cell's collisions, in
 *                          unspecified order
 *   claim   [3*claim_cap]  (cell, a, b) of the pairs that scattered,
 *                          unspecified order
 *   counts  [2]      number of candidates and claims (written even when
 *                    they exceed the capacities; then cuba_sync reports
 *                    CUBA_ENOMEM and only the first *_cap are stored) */
typedef struct {
  uint32_t *cell;
  uint32_t *perm;
  uint32_t *offsets;
  uint32_t *cand;
  int64_t cand_cap;
  uint32_t *claim;
  int64_t claim_cap;
  uint32_t *counts;
} cuba_trace;

int cuba_trace_step(cuba_ctx *ctx, const cuba_trace *trace);

/* Waits for the context's stream and reports device-side errors raised
 * since the last cuba_sync (CUBA_ERANGE, CUBA_ENOMEM) or CUBA_EDEVICE. */
int cuba_sync(cuba_ctx *ctx);

/* Lanes per cell of the collision and binning kernels (a launch shape; the
 * results are bit-identical for every setting).  0: one wave64 per cell,
 * whatever its occupancy.  8, 16, 32 or 64: each wave takes 64 / lanes
 * consecutive cells with one particle per lane, which serves sparse cells
 * without a mostly idle wave each; cells holding more particles than lanes
 * are stepped by the whole wave in a second kernel (a wave per 64 cells, or
 * a wave per cell once the initial state has more than one such cell in 64).
 * 1 (packed): each wave takes 64 consecutive cells and packs whole cells, in
 * order, into units of at most 64 particles, one particle per lane, testing
 * pairs with the Philox filter first and the exact test in compacted rows;
 * cells of more than 64 particles go to the second kernel.  For sparse
 * boxes and boxes of dense and sparse regions.  128: a workgroup of two
 * waves per cell, which split its pair tests (the first wave claims every
 * accepted pair in increasing pair order); for boxes of fewer cells than the
 * chip has SIMDs.  cuba_init chooses from the initial occupancy and
 * K = sigma / r_test * dt / V_cell: 128 below 1024 cells if at least half of
 * them hold more than 32 particles, else 0 below 16384 cells (launch-bound
 * steps), else 1 if at most 0.2 % of the cells hold more than 64 particles
 * and the mean occupancy is at most 8 (at most 12 if 2K >= 0.01), else the
 * smallest of 8, 16, 32 that all but 0.2 % of the cells fit, else 1 if at
 * least a quarter of the cells hold at most 8 particles and at most 0.2 %
 * more than 64, else 0.  Errors: CUBA_EINVAL for NULL or any other value.
 * For an event in a batch use cuba_batch_set_cell_lanes (which takes
 * neither 1 nor 128). */
int cuba_set_cell_lanes(cuba_ctx *ctx, int32_t lanes);
int cuba_get_cell_lanes(const cuba_ctx *ctx, int32_t *lanes);

/* Variable time step (Sec. 6 names a variable dt as the method's next
 * step).  dt [fm/c] replaces cuba_params.dt for every step issued after
 * the call, in streaming (Eq. (2)) and in K = sigma / r_test * dt / V_cell
 * of Eq. (3); the step index keeps counting, so the random numbers of step
 * t are those of a run with a fixed dt.  Validated as at init: finite,
 * 0 < dt < every cell edge (Sec. 5) and 2K <= 1.  Errors: CUBA_EINVAL (the
 * old dt stays), CUBA_EDEVICE.  Asynchronous on the context's stream. */
int cuba_set_dt(cuba_ctx *ctx, double dt);
int cuba_get_dt(const cuba_ctx *ctx, double *dt);

/* Index of the next step, number of particles, number of cells. */
int cuba_info(const cuba_ctx *ctx, uint32_t *next_step, int64_t *n,
              int64_t *n_cells);

/* Cumulative work and decision counts since cuba_init (synchronizes the
 * stream): out[0] pair tests (sum over cells of n(n-1)/2 per step),
 * out[1] candidate pairs (u < P22), out[2] scatterings (claimed pairs). */
int cuba_counters(cuba_ctx *ctx, uint64_t out[3]);

/* Stage timing.  cuba_timing_begin makes the following steps and
 * observations record two HIP events on the context's stream for each
 * launch, for at most max_launches launches: on the kernel's own dispatch
 * where the stage is one kernel (so they read its duration), else around
 * the stage's kernels.  cuba_timing_end waits for the stream and writes,
 * per stage, the summed duration in ms and the number of launches timed.
 * Stages (index into the arrays):
 *   0 bin      stream + reflect + bin (first step of a cuba_step call)
 *   1 step     fused: pair tests, claims and kinematics of step t, then
 *              stream + reflect + bin of step t+1
 *   2 collide  pair tests, claims and kinematics (last step of a call)
 *   3 observe  slab profiles
 *   4 offsets  compact cell offsets (cuba_trace_step only)
 * Events are host-side runtime objects; no device memory is allocated. */
#define CUBA_NUM_STAGES 5
int cuba_timing_begin(cuba_ctx *ctx, int32_t max_launches);
/* As cuba_timing_begin, but of the fused-step launches (stage 1, the one a
 * run repeats) only every step_every-th is timed, starting with the first;
 * the others run with no events.  Events between launches delay the next
 * launch by a few microseconds, so a run that times every launch runs
 * slower than an untimed one; sampling keeps that out of the run while the
 * average duration still comes from its own launches.  (A collision launch
 * that is one kernel carries its events on its own dispatch, so they read
 * the kernel's duration; other launches are bracketed by two events.)
 * Errors: CUBA_EINVAL for NULL, max_launches < 1 or step_every < 1. */
int cuba_timing_begin_sampled(cuba_ctx *ctx, int32_t max_launches, int32_t step_every);
int cuba_timing_end(cuba_ctx *ctx, double stage_ms[CUBA_NUM_STAGES],
                    int64_t stage_launches[CUBA_NUM_STAGES]);

/* Frees the host context; the caller's workspace is not touched. */
void cuba_destroy(cuba_ctx *ctx);

/* Name of an error code; detail of the calling thread's last failure. */
const char *cuba_strerror(int code);
const char *cuba_last_error(void);

/* Identification of the loaded library: "sources <h>; <arch>", where <h>
 * is the first 16 hex digits of a SHA-256 over the library's source files
 * and build flags, fixed when the library was compiled ("unknown" if the
 * build did not supply it).  A static string; never NULL. */
const char *cuba_build_info(void);

/* ------------------------------------------------------------------------
 * Batches: many independent events (each a cuba_ctx with its own
 * parameters, seed, step index and workspace) advanced together, one
 * kernel launch per step for all of them.  Work items are runs of
 * `cells per item` consecutive cells of one event; each event's result is
 * bit-identical to running it alone with cuba_step (same per-cell code,
 * same keys and step indices).  All device work runs on the batch's
 * stream; the events' own calls (cuba_observe, cuba_get_state,
 * cuba_counters, cuba_info) may be used through cuba_batch_slot.
 * ------------------------------------------------------------------------ */
typedef struct cuba_batch cuba_batch;

/* Device bytes of the batch's event table for max_slots slots (0 unless
 * 1 <= max_slots <= 65535). */
size_t cuba_batch_workspace_bytes(int32_t max_slots);

/* Creates a batch.  workspace: device memory of ws_bytes >=
 * cuba_batch_workspace_bytes(max_slots), 256-byte aligned, owned by the
 * caller.  max_slots: 1 .. 65535, else CUBA_EINVAL.  stream: hipStream_t (must not be NULL if graphs are enabled).
 * The batch also creates one stream of its own (default priority), on which
 * the kernels of a step that are independent of the small-cell kernel run
 * concurrently, joined back into `stream` before the next step, and two
 * pinned host buffers through which a changed event table is uploaded
 * without waiting for the stream. */
int cuba_batch_create(cuba_batch **out, int32_t max_slots, void *workspace,
                      size_t ws_bytes, void *stream);

/* Admits an event into a free slot: as cuba_init (same arguments, same
 * validation and errors; synchronizes the batch stream), on the batch's
 * stream.  The event joins the next cuba_batch_step. */
int cuba_batch_admit(cuba_batch *b, int32_t slot, const cuba_params *params,
                     int64_t n, const double *x, const double *y,
                     const double *z, const double *px, const double *py,
                     const double *pz, void *workspace, size_t ws_bytes);

/* As cuba_batch_admit, without waiting for the stream: for a serving loop
 * that admits requests while earlier steps still run.  The initial state is
 * not checked on the host; a particle outside [0, L], non-finite or with
 * |p| = 0 is reported by cuba_batch_sync with this slot.  lanes: the event's
 * lanes per cell (0, 8, 16, 32 or 64, as cuba_batch_set_cell_lanes; the
 * synchronous admission chooses it from the initial occupancy, which this
 * call does not read back).  Errors: as cuba_batch_admit, CUBA_EINVAL for
 * other lanes. */
int cuba_batch_admit_async(cuba_batch *b, int32_t slot, const cuba_params *params,
                           int64_t n, const double *x, const double *y,
                           const double *z, const double *px, const double *py,
                           const double *pz, void *workspace, size_t ws_bytes,
                           int32_t lanes);

/* Frees a slot, without waiting for the stream: the steps already queued
 * still run on the event's workspace, which the caller may reuse in stream
 * order (e.g. through a stream-ordered allocator on the batch's stream) or
 * after cuba_batch_sync. */
int cuba_batch_retire(cuba_batch *b, int32_t slot);

/* The context of an occupied slot, or NULL.  Owned by the batch. */
cuba_ctx *cuba_batch_slot(cuba_batch *b, int32_t slot);

/* Holds an admitted event out of the batch's steps (active = 0) or lets it
 * take part again (active != 0; every event is admitted active).  A held event
 * keeps its state and step index and may be observed; a scheduler uses
 * this to run the events with the least remaining work first.  A change
 * takes effect at the next cuba_batch_step, which then rebuilds the event
 * table (and recaptures its graphs).  Errors: CUBA_EINVAL for an empty
 * slot. */
int cuba_batch_set_active(cuba_batch *b, int32_t slot, int32_t active);

/* Observation inside runs (the T00 and T0x profiles of Fig. 2, as
 * cuba_batch_observe computes them): after each step s of the slot's
 * event with (s + 1) % every == 0, the collision launch of that step
 * writes the event's per-cell sums and a launch after it writes the
 * profiles to row ((s + 1) / every) % rows of out, a device array of
 * rows x 2 x cells[0] doubles (per row: T00, then T0x), in stream order.
 * So a run of cuba_batch_step need not end at an observation.  The steps
 * of a run observe whatever step they fall on, the last one included.
 * every = 0 turns it off.  out is owned by the caller and must outlive
 * the runs that write it.  Takes effect at the next cuba_batch_step
 * (which rebuilds the event table); retiring the slot turns it off.
 * Errors: CUBA_EINVAL for an empty slot, every < 0, or every > 0 with a
 * NULL out or rows < 1. */
int cuba_batch_set_observe(cuba_batch *b, int32_t slot, int32_t every, double *out,
                           int32_t rows);

/* Cells per binning work item of a slot's event (default: about 64
 * particles per item, at most 64 cells; 64 cells for events with lanes per
 * cell > 0); set by the autotuner.  The collision kernels take fixed units:
 * a cell per wave, or 64 / lanes cells per wave with lanes per cell > 0. */
int cuba_batch_set_cells_per_item(cuba_batch *b, int32_t slot, int32_t cells);

/* The profiles of a slot's event (as cuba_observe on cuba_batch_slot(b, slot),
 * enqueued on the batch stream after the steps issued so far).  T00, T0x:
 * device f64[nx] each.  Errors: CUBA_EINVAL for an empty slot or NULL. */
int cuba_batch_observe(cuba_batch *b, int32_t slot, double *T00, double *T0x);

/* The moments of a slot's event (as cuba_observe_moments), on the batch
 * stream.  out: device f64[6 nx]. */
int cuba_batch_observe_moments(cuba_batch *b, int32_t slot, double *out);

/* Lanes per cell of a slot's event (as cuba_set_cell_lanes).  The default
 * is cuba_init's choice without its 8-lane fallback for boxes of dense and
 * sparse regions (a batch steps oversize cells a wave per 64 cells); set by
 * the autotuner. */
int cuba_batch_set_cell_lanes(cuba_batch *b, int32_t slot, int32_t lanes);

/* A slot's time step (as cuba_set_dt) from its next cuba_batch_step on.
 * Errors: CUBA_EINVAL for an empty slot or a dt cuba_set_dt rejects. */
int cuba_batch_set_dt(cuba_batch *b, int32_t slot, double dt);

/* Launch shape: persistent_waves > 0 runs the binning kernel on that many
 * persistent waves taking work items with a grid stride (0: one wave per
 * item); use_graphs != 0 captures each run of n steps as a hipGraph (cached
 * per n, rebuilt after admissions, retirements and setting changes). */
int cuba_batch_set_launch(cuba_batch *b, int32_t persistent_waves,
                          int32_t use_graphs);

/* Advances every admitted event that is not held (cuba_batch_set_active)
 * by nsteps steps (asynchronous). */
int cuba_batch_step(cuba_batch *b, int32_t nsteps);

/* Waits for the stream and reports the device error of the first event
 * (in slot order) that has one, with its slot in *bad_slot (else -1), and
 * clears it; other events' errors stay pending and are reported by the
 * following calls, one per call, so a caller can retire each failing event
 * and go on with the rest. */
int cuba_batch_sync(cuba_batch *b, int32_t *bad_slot);

/* Stage timing of the following non-graph runs, as cuba_timing_begin/end
 * (stages 0 bin, 1 step, 2 collide). */
int cuba_batch_timing_begin(cuba_batch *b, int32_t max_launches);
int cuba_batch_timing_end(cuba_batch *b, double stage_ms[CUBA_NUM_STAGES],
                          int64_t stage_launches[CUBA_NUM_STAGES]);

/* Destroys the batch and its events' contexts (not the workspaces). */
void cuba_batch_destroy(cuba_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* CUBA_H */
