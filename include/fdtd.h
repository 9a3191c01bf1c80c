/*
 * fdtd.h -- C interface of the MI355X FDTD S-parameter library.
 *
 * The library runs the time-domain part of the transmission-line
 * characterization workflow of Sawant et al. (arXiv 2208.04371, Sec. II-A):
 * a 3-D Yee leapfrog with per-edge permittivity/conductivity coefficients,
 * PEC conductors, convolutional-PML absorbing layers, a soft excitation on
 * the port plane, and per-step port voltage/current integrals accumulated
 * into FP64 running DFTs; plus the FP64 host post-processing of those
 * spectra into S*, S referred to 50 ohm, Z_r, the overall Z0 and the phase
 * delay (eqs. 1, 2, 5-8).
 *
 * Conventions used by every call
 *  - Return value: an fdtd_status (0 = FDTD_OK, negative on error).  No C++
 *    exception crosses this interface.  fdtd_last_error() gives a message
 *    for the last failing call on a plan or batch.
 *  - Host arrays passed in are owned by the caller and copied during the
 *    call; no host pointer is kept after a call returns.
 *  - Device memory is owned by the caller: the library states how many bytes
 *    it needs (fdtd_plan_workspace_size), the caller allocates one block and
 *    hands it over (fdtd_plan_bind).  The library never allocates device
 *    memory itself and never frees the caller's block.
 *  - "stream" arguments are hipStream_t values passed as void* (NULL = the
 *    null stream).  Calls that launch work are asynchronous on that stream
 *    unless they say otherwise.
 *  - A plan is not thread-safe; distinct plans are independent.
 *  - Grid: nx*ny*nz cells, nodes (i, j, k) with i in [0, nx] etc.  Yee
 *    staggering: Ex(i+1/2, j, k), Ey(i, j+1/2, k), Ez(i, j, k+1/2) on edges,
 *    Hx(i, j+1/2, k+1/2), Hy(i+1/2, j, k+1/2), Hz(i+1/2, j+1/2, k) on faces.
 *    A component with node index (i, j, k) is stored at that index.
 *  - Host field arrays exchanged with the library are FP64, dense,
 *    (nz+1)*(ny+1)*(nx+1) values, x fastest.
 */
#ifndef FDTD_H
#define FDTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdtd_plan fdtd_plan;
typedef struct fdtd_batch fdtd_batch;

typedef int32_t fdtd_status;
enum {
    FDTD_OK = 0,
    FDTD_E_INVALID_ARG = -1,  /* an argument is out of range or inconsistent */
    FDTD_E_STATE = -2,        /* call made in the wrong order (e.g. run before bind) */
    FDTD_E_UNSUPPORTED = -3,  /* valid request this build does not implement */
    FDTD_E_HIP = -4,          /* a HIP runtime call failed; message has the hipError_t */
    FDTD_E_NOMEM = -5,        /* host allocation failed or workspace too small */
    FDTD_E_DIVERGED = -6      /* non-finite values found in the results */
};

enum { FDTD_FP32 = 0, FDTD_FP64 = 1 };              /* field precision */
enum { FDTD_SI = 0, FDTD_NORMALIZED = 1 };          /* NORMALIZED: c = eps0 = mu0 = 1 */
enum { FDTD_KERNEL_PLAIN = 0, FDTD_KERNEL_FUSED = 1 };
enum { FDTD_FACE_PEC = 0, FDTD_FACE_CPML = 1 };
enum { FDTD_WAVE_NONE = 0, FDTD_WAVE_GAUSSIAN_STEPS = 1, FDTD_WAVE_GAUSS_SINE = 2,
       FDTD_WAVE_DIFF_GAUSSIAN = 3, FDTD_WAVE_SAMPLED = 4 };
enum { FDTD_EX = 0, FDTD_EY = 1, FDTD_EZ = 2, FDTD_HX = 3, FDTD_HY = 4, FDTD_HZ = 5 };

/* Grid and run options.  The time step is courant / (c sqrt(dx^-2 + dy^-2 +
 * dz^-2)), i.e. courant is the fraction of the 3-D Yee stability limit
 * (the paper runs at 0.9, Sec. II-B and Sec. III).  kernel = FUSED needs
 * precision = FP32. */
typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;          /* metres (SI) or grid units (NORMALIZED) */
    double courant;
    int32_t precision;          /* FDTD_FP32 or FDTD_FP64 */
    int32_t units;              /* FDTD_SI or FDTD_NORMALIZED */
    int32_t kernel;             /* FDTD_KERNEL_PLAIN or FDTD_KERNEL_FUSED */
} fdtd_grid;

/* One entry of the material table.  Non-magnetic media only (the paper's
 * oxide, silicon and metals, Sec. II-B, Sec. III). */
typedef struct {
    double eps_r;               /* relative permittivity, > 0 */
    double sigma;               /* conductivity, S/m (or normalized), >= 0 */
    int32_t is_pec;             /* nonzero: perfect electric conductor */
} fdtd_material;

/* Domain faces in the order x-, x+, y-, y+, z-, z+.  A CPML face carries a
 * convolutional PML of cells[f] cells backed by PEC (the paper puts a PML on
 * every face except the PEC ground, Sec. II-A).  Profiles (Roden-Gedney
 * CPML, polynomial grading of order m from the inner interface):
 * sigma = sigma_max (rho/d)^m, kappa = 1 + (kappa_max - 1)(rho/d)^m,
 * alpha = alpha_max (1 - rho/d); sigma_max <= 0 selects 0.8 (m+1)/(eta0 d_axis). */
typedef struct {
    int32_t face[6];
    int32_t cells[6];
    double m, sigma_max, kappa_max, alpha_max;
} fdtd_boundary;

/* A port on the plane x = i (node index), inward direction dir = +1 (+x) or
 * -1.  The strip occupies cells y in [y0, y1), z in [z0, z1); the ground is
 * the z = 0 face.  Voltage (eq. 4): minus the integral of Ez over the nodes
 * j in [y0, y1] (trapezoidal in y) and edges k in [0, z0), divided by the
 * strip width.  Current (eq. 4): the closed integral of H around the strip
 * on the H-node rectangle half a cell outside the metal, counter-clockwise
 * seen from +x, averaged over the planes x = i - 1/2 and x = i + 1/2 and
 * multiplied by dir.  The contour must lie inside the grid. */
typedef struct {
    int32_t i;
    int32_t dir;
    int32_t y0, y1, z0, z1;
} fdtd_port;

/* Soft source added to Ez on the inclusive node box (i0, i1, j0, j1, k0, k1)
 * after every E update: Ez += s(t_{n+1}) (eq. 3 and the soft-source remark
 * after it).  Waveforms, with t the time of the new E level:
 *   GAUSSIAN_STEPS: s = A exp(-((n+1 - t0)/width)^2), t0 and width in steps;
 *   GAUSS_SINE:     s = A exp(-((t-t0)/tau)^2) sin(2 pi fc (t-t0)),
 *                   tau = 2 sqrt(ln 1000) / (pi bandwidth);
 *   DIFF_GAUSSIAN:  s = A (-2 (t-t0)/width) exp(-((t-t0)/width)^2)  (eq. 3);
 *   SAMPLED:        s = A samples[n] at level n+1 (0 past the last sample),
 *                   any pulse given point by point, see
 *                   fdtd_plan_set_source_samples.
 * t0 <= 0 selects three pulse widths (tau or width). */
typedef struct {
    int32_t kind;
    int32_t box[6];
    double t0, width, fc, bandwidth, amplitude;
} fdtd_source;

/* ---- plan construction (host only, no GPU work) ------------------------ */

/* Create an empty plan for a grid.  *out receives the plan.
 * Errors: INVALID_ARG for fewer than 2 cells along an axis, more than 2^34
 * cells, non-positive spacings or courant, unknown enums; UNSUPPORTED for
 * FUSED with FP64 (a FUSED grid whose field arrays would reach 4 GiB is
 * refused with UNSUPPORTED when the plan is finalized). */
fdtd_status fdtd_plan_create(const fdtd_grid *grid, fdtd_plan **out);

/* Material map: cells[nz][ny][nx] (x fastest) indexes table[0..n-1].
 * Errors: INVALID_ARG on a NULL array, n outside [1, 256], an id >= n or a
 * material with eps_r <= 0 or sigma < 0. */
fdtd_status fdtd_plan_set_materials(fdtd_plan *plan, const uint8_t *cells,
                                    const fdtd_material *table, int32_t n);

/* Boundary kinds and CPML parameters.  Default: every face PEC.
 * Errors: INVALID_ARG on unknown face kinds, negative cells, layers that
 * overlap along an axis, m < 0 or kappa_max < 1. */
fdtd_status fdtd_plan_set_boundary(fdtd_plan *plan, const fdtd_boundary *b);

/* Add a voltage/current port (see fdtd_port); *id receives its probe index.
 * Errors: INVALID_ARG when the planes, surface or contour leave the grid. */
fdtd_status fdtd_plan_add_port(fdtd_plan *plan, const fdtd_port *port, int32_t *id);

/* Add a point probe that records one field component at node (i, j, k) as
 * its "voltage" signal (its current signal is zero); *id receives its probe
 * index.  Errors: INVALID_ARG outside the component's index range. */
fdtd_status fdtd_plan_add_point_probe(fdtd_plan *plan, int32_t comp, int32_t i, int32_t j,
                                      int32_t k, int32_t *id);

/* Set the soft source (see fdtd_source).  Errors: INVALID_ARG for a box
 * outside [0,nx)x[0,ny]x[0,nz) or bad waveform parameters. */
fdtd_status fdtd_plan_set_source(fdtd_plan *plan, const fdtd_source *src);

/* Samples of a SAMPLED source: samples[m] (FP64, n values, host memory,
 * copied) is added at E level m + 1.  Before the plan is finalized (the
 * first fdtd_plan_workspace_size); a plan whose source is SAMPLED cannot be
 * finalized without them (STATE).  Errors: INVALID_ARG for NULL samples or
 * n < 1. */
fdtd_status fdtd_plan_set_source_samples(fdtd_plan *plan, const double *samples, int64_t n);

/* Analysis frequencies (Hz or normalized), nf in [1, 4096]. */
fdtd_status fdtd_plan_set_frequencies(fdtd_plan *plan, const double *f, int32_t nf);

/* Finalize the plan (per-edge coefficients, absorbing-layer profiles, probe
 * tables) and report the device workspace it needs in *bytes.  After this
 * call the plan's description can no longer change. */
fdtd_status fdtd_plan_workspace_size(fdtd_plan *plan, size_t *bytes);

/* Time step of the plan (seconds or normalized).  Needs a finalized plan. */
fdtd_status fdtd_plan_get_dt(const fdtd_plan *plan, double *dt);

/* ---- device binding and stepping -------------------------------------- */

/* Bind a caller-allocated device block of at least the workspace size
 * (256-byte aligned), upload the static tables and clear the state.
 * Synchronous.  Errors: STATE if not finalized, NOMEM if too small,
 * INVALID_ARG if misaligned, HIP on runtime failure. */
fdtd_status fdtd_plan_bind(fdtd_plan *plan, void *dptr, size_t bytes, void *stream);

/* Zero the fields, absorbing-layer state, probe histories and DFT
 * accumulators, and rewind the step counter to 0.  Asynchronous. */
fdtd_status fdtd_reset(fdtd_plan *plan, void *stream);

/* Advance nsteps leapfrog steps (nsteps >= 0), sampling every probe after
 * every step and accumulating the running DFTs:
 *   F_V(f) = sum_n V^n exp(-j 2 pi f n dt) dt,
 *   F_I(f) = sum_n I^{n-1/2} exp(-j 2 pi f (n-1/2) dt) dt,   n = 1, 2, ...
 * Resumable: a second call continues where the first stopped.  Asynchronous.
 * Errors: STATE if not bound (or bound into a batch). */
fdtd_status fdtd_run(fdtd_plan *plan, int64_t nsteps, void *stream);

/* fdtd_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid it): the same
 * steps, probe samples and DFT folds with the same kernels and bitwise the
 * same results, and it calls no hipMalloc, hipFree or allocating library
 * routine.  The probe history ring (the FP64 staging between each step's
 * port sums and the DFT fold) lives in a static device array of the library,
 * NOALLOC_RING_BYTES = 262144 bytes per GPU (held until the process ends),
 * instead of the plan's workspace; the caller's bound workspace still holds
 * the fields, auxiliaries and DFT accumulators.  The ring takes
 * nprobe * 2 * 512 * 8 bytes, so plans of up to 32 probes fit.  Every call
 * on one GPU shares that GPU's ring, which keeps the last call's contents
 * (each call writes every slot before reading it and folds all its samples
 * into the accumulators before it returns): calls that overlap on one GPU
 * (plans run concurrently on several streams or host threads) race and
 * must be serialized by the caller.  Run the plan with the device it was
 * bound on current.  The kernel timer (fdtd_plan_set_timing) does not cover
 * these calls.  Asynchronous.  Errors: STATE if not bound, bound into a
 * batch, or another device is current; INVALID_ARG if the plan's ring
 * exceeds the static ring (more than 32 probes); HIP if the ring's address
 * could not be obtained. */
fdtd_status fdtd_run_noalloc(fdtd_plan *plan, int64_t nsteps, void *stream);

/* Number of completed steps. */
fdtd_status fdtd_get_step(const fdtd_plan *plan, int64_t *step);

/* Copy the DFTs of one probe to the host as interleaved (re, im) FP64:
 * V[2*nf], I[2*nf] (either may be NULL).  Synchronizes the stream.
 * Errors: INVALID_ARG for a bad probe index; DIVERGED if a value is not
 * finite. */
fdtd_status fdtd_get_spectra(fdtd_plan *plan, int32_t probe, double *V, double *I,
                             void *stream);

/* Copy one field component to/from a dense FP64 host array (see the top of
 * this file).  Synchronizes the stream.  write_field is for initial
 * conditions; values outside the component's computed index range are
 * ignored on write and returned as 0 on read. */
fdtd_status fdtd_read_field(fdtd_plan *plan, int32_t comp, double *host, void *stream);
fdtd_status fdtd_write_field(fdtd_plan *plan, int32_t comp, const double *host, void *stream);

/* Checkpoint: the whole mutable state (fields, absorbing-layer state, probe
 * histories, DFT accumulators, step counter) as an opaque host blob of
 * fdtd_checkpoint_size bytes.  save/load synchronize the stream.  Loading a
 * checkpoint and running on gives results bitwise equal to an uninterrupted
 * run.  Errors: NOMEM if the blob is too small, INVALID_ARG if it belongs to
 * a different plan shape. */
fdtd_status fdtd_checkpoint_size(const fdtd_plan *plan, size_t *bytes);
fdtd_status fdtd_checkpoint_save(fdtd_plan *plan, void *host, size_t bytes, void *stream);
fdtd_status fdtd_checkpoint_load(fdtd_plan *plan, const void *host, size_t bytes, void *stream);

/* Message for the last failing call on this plan ("" if none).  Owned by
 * the plan, valid until its next call. */
const char *fdtd_last_error(const fdtd_plan *plan);

/* Release the plan's host state.  The caller still owns (and frees) the
 * device block it bound.  NULL is ignored. */
void fdtd_plan_destroy(fdtd_plan *plan);

/* ---- batches: many plans stepped together ------------------------------ */

/* Group n >= 1 finalized, unbound FP32 FUSED plans (shapes may differ) so
 * that one launch per step advances all of them: the per-port excitations
 * of one S-matrix and geometry variants of one sweep (the per-port run
 * protocol of Sec. II-A).  The batch keeps pointers to the plans; they must
 * outlive it.  Errors: INVALID_ARG, STATE, UNSUPPORTED (not FP32 FUSED). */
fdtd_status fdtd_batch_create(fdtd_plan *const *plans, int32_t n, fdtd_batch **out);

/* Workspace for all plans of the batch plus the shared launch tables. */
fdtd_status fdtd_batch_workspace_size(fdtd_batch *batch, size_t *bytes);

/* Bind one device block for the whole batch (each plan gets its own slice,
 * after which fdtd_get_spectra/read_field work on the member plans).
 * Synchronous. */
fdtd_status fdtd_batch_bind(fdtd_batch *batch, void *dptr, size_t bytes, void *stream);

/* Reset every member plan. */
fdtd_status fdtd_batch_reset(fdtd_batch *batch, void *stream);

/* Advance every member plan by nsteps steps: in lockstep, or group after
 * group when the batch is grouped (fdtd_batch_set_group_bytes); either way
 * all members are at the same step when the call returns.  Asynchronous.
 * After a failure the member states are undefined until fdtd_batch_reset. */
fdtd_status fdtd_batch_run(fdtd_batch *batch, int64_t nsteps, void *stream);

/* Choose the tile height (2, 4, 8, 12, 16 rows), z-chunk (4, 8, 16, 32, 64
 * planes) and tile order (automatic or 16, see fdtd_batch_set_tile_order) of the
 * batched kernel by timing each candidate
 * for `trial_steps` steps; the member states are reset afterwards.  When the
 * member workspaces exceed the group budget (fdtd_batch_set_group_bytes), the
 * schedule is chosen too: every shape is timed grouped and in lockstep (all
 * members in one launch pair per step), and a lockstep win puts the batch in
 * one group (fdtd_batch_get_groups then returns 1) until the next
 * set_group_bytes.  A grouped trial runs each group's steps in turn, so
 * trial_steps of 50 or more keep the refill of the memory-side cache at
 * each group's start from weighing on it.
 * cache_path (may be NULL) names a JSON file keyed by GPU architecture and
 * member grid shapes: a hit applies the stored choice without timing
 * (*best_index = -1), a miss stores the winner.  Synchronous.  *best_index
 * receives the index of the chosen candidate in (schedule, rows, z-chunk,
 * order) lexicographic order, the configured schedule first (50
 * candidates per schedule).  Any choice gives the same results bit for
 * bit.  On a
 * failure the launch shape is the last one tried and the member states are
 * undefined until fdtd_batch_reset. */
fdtd_status fdtd_batch_autotune(fdtd_batch *batch, int32_t trial_steps, const char *cache_path,
                                void *stream, int32_t *best_index);

/* Launch configuration of the fused kernel: tile rows per block (2, 4, 8,
 * 12 or 16; a block is 64 x rows threads) and the number of z planes one block
 * marches through (1..64).  set returns INVALID_ARG for other values.  The
 * default (at creation, and after fdtd_batch_set_group_bytes while neither
 * set_config nor the autotuner has chosen one) is 8 rows and the longest
 * z-chunk of 16, 8 or 4 planes that still yields at least 2048 tiles in one
 * launch (of the largest group when the batch is grouped). */
fdtd_status fdtd_batch_get_config(const fdtd_batch *batch, int32_t *tile_rows,
                                  int32_t *zchunk);
fdtd_status fdtd_batch_set_config(fdtd_batch *batch, int32_t tile_rows, int32_t zchunk);

/* State budget of the batch schedule.  When the member workspaces add up
 * to more than `bytes`, the members are split, in their order, into groups
 * of consecutive members whose workspaces fit it (a larger member forms a
 * group alone), and fdtd_batch_run advances one group at a time by nsteps:
 * each group's state then stays in the GPU's memory-side cache for its
 * whole span instead of streaming from HBM every step.  Otherwise (or with
 * bytes = 0) all members step in lockstep, one launch pair per step.
 * Default 256 MiB (the MI355X memory-side cache).  Results do not depend on
 * the schedule; between fdtd_batch_run calls all members are at the same
 * step.  Kernel timing counts the launches of each group as steps.  get
 * returns the number of groups (1 = lockstep). */
fdtd_status fdtd_batch_set_group_bytes(fdtd_batch *batch, uint64_t bytes);
/* (set_group_bytes, set_config and set_tile_order on a bound batch rewrite
 * its launch tables through the null stream and wait for the copy: call them
 * between runs, not while a run of the batch may still execute on another
 * stream.) */
fdtd_status fdtd_batch_get_groups(const fdtd_batch *batch, int32_t *ngroups);

/* Order in which the blocks of a fused launch take their tiles.  The GPU
 * deals blocks to its 8 XCDs (each with its own L2) in turn.  0: each XCD
 * takes one contiguous run of the tiles, so neighbouring tiles share its L2
 * (best while the state fits the 256 MB memory-side cache); k in [1, 4096]:
 * runs of k tiles go to the XCDs in turn, so all XCDs stream one region of
 * the grid at a time (better once the state streams from HBM); -1
 * (default): automatic, 0 for a workspace of at most 256 MiB, else 16.  The
 * order changes timing only, never results.  get returns the setting and
 * the order launches use (*used, from the workspace size once known). */
fdtd_status fdtd_batch_set_tile_order(fdtd_batch *batch, int32_t order);

/* Streaming (non-temporal) stores of the fields a fused launch writes.  The
 * outputs of a step are read again only by the next step: once the state
 * exceeds the 256 MB memory-side cache, caching them evicts the inputs still
 * to be read (1024x512x256: 1484 against 1538 us per step), while for a
 * state inside that cache they would push next step's inputs out of it
 * (400x120x80: 77 against 56 us).  Not far above the cache size much of
 * the state still hits it and the outcome depends on the grid (a 296 MiB
 * microstrip gains 5 %, sweep grids of 289 and 308 MiB lose heavily).
 * mode: 1 on, 0 off, -1 (default) automatic, on for a launch whose
 * workspace (a batch: its group's) exceeds 512 MiB.  It applies to the
 * single-level launches; the two-level pass (fdtd_plan_set_temporal) always
 * stores through the cache, since its 60-cell rows do not start on 128-byte
 * lines and the cache merges the partial lines of neighbouring tiles.
 * Results do not depend on it.  INVALID_ARG for other modes.  The plan getter
 * returns the setting and (*used) the mode its launches use, from the
 * workspace size once known. */
fdtd_status fdtd_batch_set_stream_stores(fdtd_batch *batch, int32_t mode);
fdtd_status fdtd_batch_get_tile_order(const fdtd_batch *batch, int32_t *order, int32_t *used);

/* Message of the batch's last failed call; with batch == NULL, of the last
 * failed fdtd_batch_create on the calling thread. */
const char *fdtd_batch_last_error(const fdtd_batch *batch);
void fdtd_batch_destroy(fdtd_batch *batch);

/* Launch configuration of a single FUSED plan (same meaning as for a batch). */
fdtd_status fdtd_plan_get_config(const fdtd_plan *plan, int32_t *tile_rows, int32_t *zchunk);
fdtd_status fdtd_plan_set_config(fdtd_plan *plan, int32_t tile_rows, int32_t zchunk);
fdtd_status fdtd_plan_set_tile_order(fdtd_plan *plan, int32_t order);
fdtd_status fdtd_plan_get_tile_order(const fdtd_plan *plan, int32_t *order, int32_t *used);
fdtd_status fdtd_plan_set_stream_stores(fdtd_plan *plan, int32_t mode);
fdtd_status fdtd_plan_get_stream_stores(const fdtd_plan *plan, int32_t *mode, int32_t *used);

/* Two-level (temporally blocked) steps of a FUSED plan.  Tiles whose cells
 * lie at least two cells away from every absorbing layer then advance two
 * leapfrog steps per pass over the grid (level n read once, level n+2 written
 * once, level n+1 recomputed on a two-cell halo and kept on chip), while the
 * other tiles take the two steps one at a time; the plan keeps a third field
 * buffer for the intermediate level of those tiles.  This halves the field
 * traffic of the interior tiles, which is what bounds the step on grids far
 * larger than the memory-side cache.  The update formulas, their rounding,
 * the sampling and so the results are bitwise those of single steps.  Runs
 * of an odd number of steps end with a single step.
 * set_temporal: mode 1 on, 0 off, -1 (default) automatic: on when the plan's
 * state with two buffers would exceed 512 MiB and its default launch shape
 * leaves two-level tiles.  Before the plan is finalized (STATE after);
 * INVALID_ARG for other modes; UNSUPPORTED for mode 1 on a PLAIN plan.
 * Such plans cannot join a batch.
 * set_temporal_config: the two-level tiles are 60 cells in x, tile_rows
 * (8, 10 or 13) in y and zchunk (4..256) planes in z; default 13 x 32.
 * It also makes the plan take two-level passes again where the autotuner
 * chose single steps (depth 1, fdtd_plan_autotune).
 * INVALID_ARG for other values.  Takes effect at the next run.
 * get_temporal: the mode, whether the plan takes two-level passes (*used:
 * finalized with the third buffer, depth 2), the tile shape and the number
 * of two-level tiles of the current launch shape (0 if none or if *used is
 * 0; then every step is single).  Any output may be NULL. */
fdtd_status fdtd_plan_set_temporal(fdtd_plan *plan, int32_t mode);
fdtd_status fdtd_plan_set_temporal_config(fdtd_plan *plan, int32_t tile_rows, int32_t zchunk);
fdtd_status fdtd_plan_get_temporal(const fdtd_plan *plan, int32_t *mode, int32_t *used,
                                   int32_t *tile_rows, int32_t *zchunk, int32_t *tiles);

/* fdtd_batch_autotune for one bound FUSED plan that is not in a batch: the
 * same candidates, timing and cache (a plan and a one-member batch of the
 * same grid shape share a cache entry).  A plan finalized with two-level
 * steps (fdtd_plan_set_temporal) is also tuned in its temporal-block depth:
 * a second stage keeps the winning (rows, z-chunk, order) and times
 * two-level passes with tiles of 8, 10 or 13 rows and z-chunks of 8, 16, 32
 * or 64 planes (12 candidates, in that lexicographic order), then single
 * steps only (depth 1); *best_index = i1 + 50 * i2 with i1 the first stage's
 * index and i2 < 13 the second's.  Such plans have cache entries of their
 * own, which also hold the depth and the two-level tile shape.  Any choice
 * gives the same results bit for bit.
 * The plan is reset afterwards unless
 * the shape came from the cache.  STATE if unbound or in a batch,
 * UNSUPPORTED for the plain kernels, INVALID_ARG for trial_steps < 1.  On a
 * failure the launch shape is the last one tried and the state is undefined
 * until fdtd_reset.  Synchronous. */
fdtd_status fdtd_plan_autotune(fdtd_plan *plan, int32_t trial_steps, const char *cache_path,
                               void *stream, int32_t *best_index);

/* ---- kernel timing ----------------------------------------------------- */

/* enable = n >= 1: the steps of each run (the field-update launches of a
 * plan or batch) are timed by HIP events on the run stream in windows of n
 * consecutive steps, one event pair per window (a run's last window may be
 * shorter); ..._get_kernel_time returns the summed window time and the
 * number of steps it covers (and synchronizes the stream).  n = 1 brackets
 * each step alone.  A window's time includes the gaps between its launches
 * and any probe or DFT launch between its steps.  0 disables; a negative
 * value is INVALID_ARG.  Setting clears the totals.  An event pair costs
 * the host about as much as a 400x120x80 step takes on the GPU and adds its
 * own latency on the GPU, so n = 1 slows such short steps; windows of 16
 * steps keep that cost out of the measurement. */
fdtd_status fdtd_plan_set_timing(fdtd_plan *plan, int32_t enable);
fdtd_status fdtd_plan_get_kernel_time(fdtd_plan *plan, double *ms, int64_t *launches);
fdtd_status fdtd_batch_set_timing(fdtd_batch *batch, int32_t enable);
fdtd_status fdtd_batch_get_kernel_time(fdtd_batch *batch, double *ms, int64_t *launches);

/* ---- post-processing (host, FP64, no plan needed) ---------------------- */

/* Network parameters of an np-port from the per-port run protocol of
 * Sec. II-A.  All complex arrays are interleaved (re, im) FP64:
 *   f[nf]                   analysis frequencies
 *   Vinc[np][nf], Iinc[np][nf]  V and I spectra at port j in the run that
 *                           drives port j on a locally uniform line
 *   Vtot[np][np][nf]        Vtot[j][i]: V spectrum at port i in the run that
 *                           drives port j on the full circuit
 * Outputs (any may be NULL):
 *   S_star[nf][np][np]      eq. 1: S*_jj = (Vtot_jj - Vinc_j)/Vinc_j,
 *                           S*_ij = Vtot_ji / Vinc_j * sqrt(Zr_j / Zr_i)
 *                           (principal root)
 *   S[nf][np][np]           eqs. 5-6 referred to z_ref, read as
 *                           B = (Z' - Zr)(Z' + conj Zr)^-1,
 *                           A = G'^-1 G (I - conj B),
 *                           S = A^-1 (S* - conj B)(I - B S*)^-1 conj A,
 *                           G = diag(|Re Zr|^-1/2), G' = z_ref^-1/2, Z' = z_ref
 *   Zr[nf][np]              eq. 2: Zr_j = Vinc_j / Iinc_j
 *   Z0[nf]                  np == 2 only: Z from the power waves of S* at Zr
 *                           (Kurokawa), ABCD from Z, Z0 = sqrt(B/C) with
 *                           Re Z0 >= 0 (the ABCD step of Sec. II-A)
 *   tau[nf][np][np]         eq. 8 for i != j (0 on the diagonal):
 *                           -theta/(2 pi f) with theta the phase unwrapped
 *                           along f and shifted by the multiple of 2 pi
 *                           that puts its straight-line extension through
 *                           the two lowest frequencies nearest 0 at f = 0
 * Errors: INVALID_ARG for np outside [1, 16], nf < 1 or NULL inputs;
 * DIVERGED if a matrix to invert is singular or a value is not finite. */
fdtd_status fdtd_sparams(int32_t np, int32_t nf, const double *f, const double *Vinc,
                         const double *Iinc, const double *Vtot, double z_ref,
                         double *S_star, double *S, double *Zr, double *Z0, double *tau);

/* ---- measurement support ------------------------------------------------ */

/* Copy `bytes` from src to dst, both device memory, on `stream`
 * (asynchronous).  A plain streaming copy: every byte read once and written
 * once, so its rate is the practical memory-bandwidth ceiling of the GPU
 * and its memory counters calibrate those of the field update.  Both
 * pointers and `bytes` must be multiples of 16 and the ranges must not
 * overlap (INVALID_ARG otherwise); HIP if the launch fails.  Not part of
 * the method. */
fdtd_status fdtd_device_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Text for a status code. */
const char *fdtd_status_string(fdtd_status s);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_H */
