/*
 * cm.h -- C ABI of libcm, batched simulation of stochastic cognitive models
 * on AMD Instinct MI355X (gfx950).
 *
 * The library runs many independent stochastic runs of one model across a
 * grid of parameter or control settings, as in the grid evaluation of the
 * Distill paper (arXiv 2110.15425, Sec. 3.6: every grid point is an
 * independent evaluation with its own random stream), reduces them to
 * outcome histograms and per-setting statistics (Sec. 2.1: modellers want
 * outcome distributions across parameter settings) and scores the grid,
 * picking the best allocation with a random tie-break (Sec. 2.1, Sec. 3.3).
 *
 * Data layout follows Sec. 3.3: read-only parameters are separated from
 * per-run state (which never leaves the GPU's registers), inputs and
 * outputs are flat arrays, and string keys become the enum offsets below.
 *
 * Conventions for every entry point:
 *  - No C++ types and no exceptions cross the ABI.  Every call returns a
 *    cm_status; on anything but CM_OK a message is available from
 *    cm_last_error() (thread-local) and output contents are undefined.
 *  - Arguments are validated in full before anything is enqueued: a
 *    rejected call has launched nothing.
 *  - The caller owns all memory.  "DEVICE" pointers are HIP device
 *    allocations on the handle's device, 8-byte aligned; the workspace is
 *    256-byte aligned.  "HOST" pointers are read during the call only.
 *  - Launches are asynchronous on the caller's HIP stream and ordered on it;
 *    buffers must stay alive until the stream has passed the launch.
 *  - The library allocates no device memory on the launch path.
 *
 * Determinism: for a fixed model, sweep and precision every integer output
 * is independent of launch geometry, tuning and batching: random numbers
 * are keyed by (seed, setting, trial, step) and all reductions are integer
 * additions.
 */
#ifndef CM_H
#define CM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* cm_model.abi_version must equal this.  2: cm_tuning gained tail_sweeps
 * and the cm_queue_* device work queue was added. */
#define CM_ABI_VERSION 2u

typedef struct cm_handle cm_handle;

typedef enum {
  CM_OK = 0,
  CM_E_INVALID = 1,     /* an argument violates the contract */
  CM_E_BUDGET = 2,      /* workspace too small / request exceeds the budget */
  CM_E_DEVICE = 3,      /* a HIP call failed; cm_last_error() has its text */
  CM_E_UNSUPPORTED = 4, /* valid, but this kind/precision combination is not built */
  CM_E_BUSY = 5         /* the serving queue is full; retry after cm_poll */
} cm_status;

/* Mechanism families (the DDM and LCA of Sec. 4.4; the logistic transfer and
 * weight-matrix projections of Sec. 3.4.2). */
typedef enum {
  CM_DDM = 0,          /* drift-diffusion, Euler-Maruyama, bounds +-theta */
  CM_CONFLICT_LCA = 1, /* two-pathway logistic network -> 2-unit leaky competing accumulator */
  CM_RATE_RNN = 2,     /* n-unit logistic recurrent rate network with a 2-unit readout */
  CM_CONFLICT_LOOP = 3 /* the conflict LCA under closed-loop control re-optimised every step */
} cm_kind;

/* Arithmetic modes.  CM_FP64: everything in double.  CM_FP32_STEP: normals,
 * drive and increments in float, accumulators and threshold tests in
 * double.  CM_BF16_PROJ (rate network only): CM_FP32_STEP plus the
 * recurrent projection on bf16 matrix cores with float accumulation. */
typedef enum { CM_FP64 = 0, CM_FP32_STEP = 1, CM_BF16_PROJ = 2 } cm_precision;

/* Parameter offsets into cm_model.params, one table per kind. */
enum { CM_DDM_DT = 0, CM_DDM_DRIFT, CM_DDM_NOISE, CM_DDM_THRESH, CM_DDM_START,
       CM_DDM_T0, CM_DDM_NPARAM };
enum { CM_LCA_DT = 0, CM_LCA_LEAK, CM_LCA_COMP, CM_LCA_NOISE, CM_LCA_THRESH,
       CM_LCA_OFFSET, CM_LCA_HID_GAIN, CM_LCA_HID_BIAS, CM_LCA_NONNEG, CM_LCA_T0,
       CM_LCA_NPARAM };
enum { CM_RNN_DT = 0, CM_RNN_NOISE, CM_RNN_THRESH, CM_RNN_INPUT_GAIN, CM_RNN_T0,
       CM_RNN_NPARAM };
/* Closed loop: the conflict LCA's parameters, then the control search.
 * Before every step the control node scores each allocation (c_A, c_B) of
 * the L x L grid of levels a_i = A_max i / (L - 1) (A_max when L = 1) by M
 * one-step look-aheads, each on its own random stream, as
 * COST * (c_A^2 + c_B^2) - mean over samples of the change in x_c - x_w
 * (c the correct response of the trial's stimulus), takes the lowest score
 * (exact ties: a random pick) and runs the step with it on the run's own
 * stream: the control loop nested in every time step of the predator-prey
 * model (Distill, Sec. 2.1), allocations and samples evaluated in parallel
 * (Sec. 3.6).  Requires 1 <= L, M <= 4096 integers and L*L*M < 2^30.  A run
 * is also flagged when its best and second-best scores differ by less than
 * flag_eps without being equal. */
enum { CM_LOOP_LEVELS = CM_LCA_NPARAM, CM_LOOP_AMAX, CM_LOOP_SAMPLES, CM_LOOP_COST,
       CM_LOOP_NPARAM };

/* Per-setting statistics, CM_NSTAT uint64 words per setting. */
enum { CM_ST_DEC0 = 0, CM_ST_DEC1, CM_ST_UNDEC, CM_ST_CORRECT, CM_ST_SUMN0,
       CM_ST_SUMN1, CM_ST_SUMSQ0, CM_ST_SUMSQ1, CM_ST_FLAGGED, CM_NSTAT };

/*
 * The model.
 *  kind, precision  cm_kind, cm_precision.
 *  n_units          DDM 1; conflict LCA and its closed loop 2; rate network n,
 *                   64 <= n <= 256, n a multiple of 64.
 *  n_stimuli        DDM 1; conflict LCA 9 (pairs (a, b) of one-hot inputs,
 *                   trial t uses stimulus t mod 9, as the trial loop of
 *                   Sec. 2.2 cycles through its input list); rate network 1.
 *  n_signals        signals per grid setting.  DDM 0 or 1 (overrides the
 *                   drift); conflict LCA 0 or 2 (control gains c_A, c_B,
 *                   1 when absent); closed loop 0 or 1 (overrides the
 *                   control-cost weight); rate network 0 or 1 (overrides
 *                   the input gain).
 *  params           HOST, n_params doubles in the kind's enum order.
 *  weights          DEVICE, row-major blocks.  Conflict LCA and loop: W_A[4x3],
 *                   W_B[4x3], O_A[2x4], O_B[2x4] (40 doubles).  Rate
 *                   network: W[n x n] then R[2 x n].  DDM: unused (NULL).
 */
typedef struct {
  uint32_t abi_version; /* CM_ABI_VERSION */
  uint32_t kind, precision, n_units, n_stimuli, n_signals;
  const double *params;
  uint32_t n_params;
  const double *weights;
  uint64_t n_weights;
} cm_model;

/*
 * The sweep: n_settings grid points x trials runs each.
 *  grid       DEVICE [n_settings x n_signals] doubles, NULL if n_signals == 0.
 *  trials     runs per setting, 1 <= trials < 2^31.
 *  seed       64-bit key of every random stream.
 *  max_steps  step cap N >= 1; a run that has not crossed by step N is
 *             undecided (choice -1).
 *  n_bins     histogram bins B, 1 <= B <= N; a run deciding at step n goes
 *             to bin floor((n-1) B / N).
 *  reward, cost  score[s] = reward * correct[s]/trials - cost * sum_k c_k^2;
 *             both 0: no score.
 *  flag_eps   a run is flagged when a compared quantity came within this
 *             distance of its threshold (or, at a decision, the two
 *             accumulators within it of each other).
 */
typedef struct {
  const double *grid;
  uint64_t n_settings;
  uint64_t trials, seed;
  uint32_t max_steps, n_bins;
  double reward, cost;
  double flag_eps;
} cm_sweep;

/*
 * Outputs, all DEVICE, caller-allocated; the library zero-fills them.
 *  hist     [n_settings][2][n_bins] uint64: decided runs per choice and bin.
 *  stats    [n_settings][CM_NSTAT] uint64.
 *  score    [n_settings] double, or NULL (required when reward/cost != 0).
 *  best     [2] int64 {argmax setting, number of tied settings}, or NULL.
 *  run_*    optional per-run dumps indexed setting * trials + trial:
 *           choice (-1 undecided), decision step, flag, final state
 *           (DDM x; LCA x0 x1; rate network y0 y1 then x[n]).
 */
typedef struct {
  uint64_t *hist;
  uint64_t *stats;
  double *score;
  int64_t *best;
  int8_t *run_choice;
  uint32_t *run_step;
  uint8_t *run_flag;
  double *run_state;
} cm_result;

/* Launch-shape knobs; 0 in a field means "let the library choose".  The
 * register-use versus occupancy trade-off the Distill paper measures on its
 * GPU kernels (Sec. 6.3) is what these choose between; cm_get_tuning
 * reports the stored values (runs_per_lane 0 = size-dependent).
 *  block          threads per workgroup of the lane kernels: 256, or 512 or
 *                 1024 for the DDM and conflict-LCA lane kernels (a larger
 *                 workgroup packs more unfinished runs together while its
 *                 chunk drains; it takes block x runs_per_lane runs and
 *                 stages block x ~64 bytes of LDS).  Other values, and other
 *                 kinds: CM_E_UNSUPPORTED.  The time-course variant runs 256.
 *  runs_per_lane  lane-per-run kernels: runs handed to a workgroup per lane
 *                 (0: chosen per launch from the run count, 2..8).
 *  steps_per_sync lane-per-run kernels: steps between refills of finished
 *                 lanes (1..64; the DDM counts step pairs).  Defaults: 16
 *                 steps (LCA), 8 pairs (DDM).
 *  tile_rows      rate network: runs per workgroup tile, one 16-column
 *                 matrix-core tile; only 16 is supported (the 256-unit
 *                 network's W fragments fill the registers of a wider tile).
 *  lanes_per_run  DDM only: 1 (one lane per run), 64 (one wavefront per
 *                 run, 128 steps per prefix scan; runs_per_lane then counts
 *                 runs per wavefront) or 0 (per launch: 64 when every sweep
 *                 of the launch has at most 2^20 runs, else 1).  The
 *                 wavefront form runs 8 wavefronts per workgroup when the
 *                 launch has at most 2^17 runs, else 4 (the block knob
 *                 does not apply to it).
 *  waves_per_simd DDM and conflict LCA, one lane per run: 0 (the compiler's
 *                 register allocation), or 4 or 8: the kernel built with its
 *                 registers capped so that 4 or 8 wavefronts fit on each
 *                 SIMD -- the register use versus occupancy study of the
 *                 paper's GPU kernels (Sec. 6.3); a cap below the kernel's
 *                 own use spills or recomputes values.  Other values:
 *                 CM_E_UNSUPPORTED.  The time-course variant ignores it.
 *  tail_sweeps    DDM and conflict LCA, one lane per run: the last
 *                 tail_sweeps sweeps of a launch (cm_launch's one sweep
 *                 included) take chunks of half the runs -- twice as many
 *                 workgroups, each half as long -- so that the launch's
 *                 last workgroups end closer together (0..12; 0: none).
 *                 Other kinds: 0 only (else CM_E_UNSUPPORTED).  The
 *                 time-course variant ignores it.
 * Results do not depend on these choices. */
typedef struct {
  uint32_t block, runs_per_lane, steps_per_sync, tile_rows, lanes_per_run, waves_per_simd;
  uint32_t tail_sweeps;
} cm_tuning;

/* Pure host checks of a model/sweep pair (the rules above and the kind's
 * parameter ranges: dt > 0, noise >= 0, thresholds > 0, |start| < theta,
 * shapes); touches no device.  This is the framework's sanitization check
 * before a run (Distill, Sec. 2.2) and the type and shape extraction that
 * follows from it (Sec. 3.1): shapes and parameters are fixed once, for the
 * whole sweep, before any simulation work.  Every launch entry point runs
 * the same checks first.  CM_E_INVALID or CM_E_UNSUPPORTED with the reason
 * in cm_last_error(). */
cm_status cm_validate(const cm_model *model, const cm_sweep *sweep);

/* Workspace bytes a launch of this model/sweep needs (host only): the
 * correct-response table, the conflict network's drive per (setting,
 * stimulus) -- the loop-invariant work hoisted out of the step loop
 * (Sec. 3.5) -- and the rate network's W in matrix-core fragment order.
 * The caller allocates it (256-byte aligned) and may reuse it for any
 * launch whose model and sweep need no more; the library writes it on the
 * stream and it must not be shared by launches that may run concurrently. */
cm_status cm_workspace_bytes(const cm_model *model, const cm_sweep *sweep, uint64_t *bytes);

/* A handle is bound to one HIP device (device_ordinal; CM_E_INVALID when
 * out of range) and holds that device's properties, the tuning table and
 * the serving slots; *out receives it.  It is the host-side state that the
 * paper's generated code keeps between evaluations of a model (compiled
 * once, then invoked for every grid point: Sec. 3.6, Sec. 3.7): here the
 * launch shapes chosen for the device, never model data or results.  Launches through a handle run on
 * its device.  cm_destroy waits for work on the handle's serving slots,
 * then releases the handle; NULL is accepted.  Several threads may launch
 * through one handle while kernel timing (cm_profile) is off; the tuning
 * table, timing and serving queue must be used from one thread.
 * cm_set_tuning stores the launch shape for one (kind, precision) pair
 * (fields as in cm_tuning; 0 = default), CM_E_INVALID or CM_E_UNSUPPORTED
 * for values outside the ranges above; it changes launch shapes only,
 * never results.  cm_get_tuning reports the stored values. */
cm_status cm_create(int device_ordinal, cm_handle **out);
cm_status cm_destroy(cm_handle *h);
cm_status cm_set_tuning(cm_handle *h, uint32_t kind, uint32_t precision, const cm_tuning *t);
cm_status cm_get_tuning(cm_handle *h, uint32_t kind, uint32_t precision, cm_tuning *t);

/* One sweep, stream-ordered on hip_stream (a hipStream_t, NULL = default):
 * the trial loop of Sec. 2.2 (trials per setting, trial t using stimulus
 * t mod n_stimuli, each run stepped until its end-of-trial condition or the
 * cap) for every setting of the grid, evaluated in parallel with an
 * independent random stream per run (Sec. 3.6), reduced to the outcome
 * histograms modellers study (Sec. 2.1) and scored with the best allocation
 * picked at random among ties (Sec. 2.1, Sec. 3.3).
 * Enqueues: output zero-fill, drive precompute (conflict LCA; the
 * loop-invariant work of Sec. 3.5), the simulation kernel, the score/argmax
 * kernel when scoring is requested.  Errors: CM_E_INVALID for a bad
 * argument (also a NULL handle or unaligned pointer), CM_E_BUDGET when
 * workspace_bytes is below cm_workspace_bytes, CM_E_UNSUPPORTED for a
 * precision the kind lacks, CM_E_DEVICE when a HIP call fails. */
cm_status cm_launch(cm_handle *h, const cm_model *model, const cm_sweep *sweep,
                    const cm_result *result, void *workspace, uint64_t workspace_bytes,
                    void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cm_launch
 * with the library's own scratch array as the workspace, so the caller
 * passes only the model, sweep, outputs and stream.  The array is a static
 * device array of CM_SCRATCH_BYTES on every device the library runs on,
 * held until the process ends; its device address is looked up once per
 * device by the first cm_create on it.  This call allocates nothing: no
 * device memory, no events (cm_profile does not time it), no host heap on
 * success.  Results equal cm_launch's for the same arguments.
 * Errors: those of cm_launch; CM_E_BUDGET when cm_workspace_bytes of the
 * model and sweep exceeds CM_SCRATCH_BYTES (a conflict-LCA grid of more
 * than 29,125 settings, a closed loop of more than 166 levels).
 * Every call on a device shares that device's one array, which keeps the
 * last call's tables: calls that may overlap on one device (other streams,
 * other threads, other handles) race and must be ordered by the caller.
 * Nothing in the array needs to start at zero: each launch writes the tables
 * it reads before reading them, on the same stream. */
#define CM_SCRATCH_BYTES (4u << 20)
cm_status cm_launch_scratch(cm_handle *h, const cm_model *model, const cm_sweep *sweep,
                            const cm_result *result, void *hip_stream);

/* Several sweeps in one call, stream-ordered on hip_stream.  Entry i uses
 * models[i], sweeps[i], results[i] and workspaces[i] (workspace_bytes[i]
 * bytes); every entry is validated before anything is enqueued.  Sweeps of
 * the lane-per-run kinds (DDM, conflict LCA) that share a kind and precision
 * run in one simulation launch of up to 12 sweeps: the grid evaluation of
 * Sec. 3.6 extended over several grids of different sizes and run lengths,
 * so small sweeps fill the GPU together.  Results are identical to separate
 * cm_launch calls. */
cm_status cm_launch_batch(cm_handle *h, uint32_t n, const cm_model *models,
                          const cm_sweep *sweeps, const cm_result *results,
                          void *const *workspaces, const uint64_t *workspace_bytes,
                          void *hip_stream);

/* cm_launch_batch replayed from a HIP graph the handle keeps: the first call
 * with a given argument set captures the batch's launches on a stream of the
 * library's own and instantiates them; a later call whose arguments are all
 * equal -- every struct field, every pointer, the parameter values behind
 * `params`, and the handle's tuning -- launches that graph on hip_stream, one
 * launch instead of a preparation, simulation and score launch per group
 * (the batching of many evaluations into few launches, Sec. 3.6, carried to
 * the launch sequence itself).  Results are those of cm_launch_batch: the
 * graph re-zeroes the outputs with its preparation kernels, never with
 * memset nodes.  A graph holds the buffers' addresses, so its entry must not
 * be replayed after the buffers are freed; cm_graph_clear drops every graph,
 * and at most CM_GRAPH_CACHE are kept (the least recently used goes first).
 * The graph is launched untimed (cm_profile sees no simulation launch).
 * Errors as for cm_launch_batch, or CM_E_DEVICE when capture, instantiation
 * or the graph launch fails. */
#define CM_GRAPH_CACHE 16u
cm_status cm_launch_graph(cm_handle *h, uint32_t n, const cm_model *models,
                          const cm_sweep *sweeps, const cm_result *results,
                          void *const *workspaces, const uint64_t *workspace_bytes,
                          void *hip_stream);
cm_status cm_graph_clear(cm_handle *h);

/* Time course: what cm_launch computes, plus ensemble statistics of the state
 * over time -- the dynamics modellers study beside final outcomes (Distill,
 * Sec. 1 and 2.1), including the conflict energy of the two mutually
 * inhibiting response units that the Stroop model tracks (Sec. 4.4).  At
 * every sample step n = every*k, k = 1..K with K = max_steps / every, the runs
 * of a setting whose decision step is n or later contribute their state after
 * step n.  timecourse (DEVICE, 8-byte aligned, [n_settings][K][6] int64,
 * zero-filled by the call) receives per (setting, k): the count of
 * contributing runs, then the sums of q(x0), q(x1), q(x0*x0), q(x1*x1) and
 * q(comp*(x0*x1)) with q(v) = v*2^32 rounded to nearest even and clamped to
 * +-2^62, summed modulo 2^64 (integer sums: independent of run order and
 * launch shape).  The DDM has one unit (x1 = 0).  Kinds CM_DDM and
 * CM_CONFLICT_LCA, precisions FP64 and FP32_STEP; 1 <= every <= max_steps.
 * The launch rounds the tuned steps_per_sync to a multiple of the sampling
 * interval (in step pairs for the DDM) when the interval is at most 64 of
 * those units, so that the runs of a wavefront sample together. */
cm_status cm_launch_timecourse(cm_handle *h, const cm_model *model, const cm_sweep *sweep,
                               const cm_result *result, uint32_t every, int64_t *timecourse,
                               void *workspace, uint64_t workspace_bytes, void *hip_stream);

/* Ablation: the same sweep executed node by node, the GPU analogue of the
 * Distill paper's per-node compilation (Sec. 6.2): each step runs as separate
 * kernels for the random numbers, the accumulator update and the threshold
 * test with compaction of the active runs, with run state in HBM and the host
 * driving the step loop (it synchronises on the stream every 16 steps to
 * stop early when no run is left).  DDM and conflict LCA only, at most
 * 2^32 - 1 runs (n_settings x trials; the node kernels index runs with 32
 * bits; CM_E_INVALID beyond).  Results are identical to cm_launch.  The
 * workspace must hold cm_unfused_workspace_bytes bytes (about 50 bytes per
 * run). */
cm_status cm_unfused_workspace_bytes(const cm_model *model, const cm_sweep *sweep,
                                     uint64_t *bytes);
cm_status cm_launch_unfused(cm_handle *h, const cm_model *model, const cm_sweep *sweep,
                            const cm_result *result, void *workspace, uint64_t workspace_bytes,
                            void *hip_stream);

/* Exact first-passage distribution of the discretised DDM, without sampling:
 * the Distill paper notes the DDM has an analytical solution that can replace
 * thousands of simulated runs (Sec. 1, Sec. 4.4).  For each setting the
 * survivor mass of the walk x_n = x_{n-1} + a + b z on n_cells cells of
 * (-theta, theta) is propagated with the exact Gaussian step kernel (the first
 * step from the start point, later steps from cell centres; error O(h^2) in
 * the cell width h), one workgroup per setting.  first_passage (DEVICE,
 * [n_settings][2][max_steps] doubles) receives the probability of deciding
 * for choice c (0 lower, 1 upper bound) at step n in [s][c][n-1].
 * Propagation stops once the survivor mass is below tol (the rest is 0).
 * Requires kind CM_DDM, noise > 0, 16 <= n_cells <= 1300; trials, seed and
 * precision are not used. */
cm_status cm_ddm_density(cm_handle *h, const cm_model *model, const cm_sweep *sweep,
                         uint32_t n_cells, double tol, double *first_passage, void *hip_stream);

/* Serving queue: asynchronous submission of batches on the handle's own
 * streams ("slots"), for a server that admits simulation requests while
 * others are still on the GPU.  Runs are independent and keyed by their own
 * (seed, setting, trial, step), so a request computes the same outputs
 * whatever else is in flight (Sec. 3.6).
 *
 * cm_serve_config creates n_slots streams (1..64, default priority) and an
 * event per slot; it fails with CM_E_BUSY while a slot holds unfinished work.
 * The first cm_submit on a handle creates 4 slots if none exist.
 *
 * cm_submit enqueues cm_launch_batch of entries 0..n-1 on a free slot and, when
 * host is not NULL, copies of each entry's hist, stats, score and best into
 * host[i]'s buffers (NULL fields skipped; sizes as in cm_result).  Host
 * buffers should be pinned (hipHostMalloc) for the copies to be
 * asynchronous.  producer_stream (a hipStream_t or NULL for none) is the
 * stream that wrote the inputs: the slot first waits for all work enqueued
 * on it so far.  *ticket receives a positive ticket.  CM_E_BUSY: every slot
 * holds unfinished work (nothing was enqueued; retry after cm_poll reports a
 * completion).  Other errors are those of cm_launch_batch; nothing is then
 * enqueued.  Device buffers and host buffers must stay alive until cm_poll
 * reports the ticket done.
 *
 * cm_poll sets *done to 1 once all work of the ticket, copies included, has
 * finished (the host buffers then hold the results), else to 0; it never
 * waits.  Unknown tickets (0 or not yet issued) give CM_E_INVALID.
 * A handle's queue is not thread-safe: submit and poll from one thread. */
typedef struct {
  uint64_t *hist;  /* HOST [n_settings][2][n_bins] or NULL */
  uint64_t *stats; /* HOST [n_settings][CM_NSTAT] or NULL */
  double *score;   /* HOST [n_settings] or NULL */
  int64_t *best;   /* HOST [2] or NULL */
} cm_host_result;
cm_status cm_serve_config(cm_handle *h, uint32_t n_slots);
cm_status cm_submit(cm_handle *h, uint32_t n, const cm_model *models, const cm_sweep *sweeps,
                    const cm_result *results, void *const *workspaces,
                    const uint64_t *workspace_bytes, const cm_host_result *host,
                    void *producer_stream, uint64_t *ticket);
cm_status cm_poll(cm_handle *h, uint64_t ticket, int *done);

/* Device work queue of the serving path: one persistent simulation kernel
 * that takes the work of many requests from a queue, so requests that arrive
 * while others run join the work on the device without a launch of their
 * own (the continuous batching of evaluations of Sec. 3.6, fed
 * continuously).  The host publishes each request as a ring entry and a
 * descriptor in pinned host memory the queue allocates at creation; one
 * workgroup at a time copies new entries into device memory, and workgroups
 * claim the requests' items with a fetch-and-add on a device counter.  A
 * request's items are its preparation pieces (output zero-fill and tables,
 * as cm_launch's preparation kernel computes them) followed by its chunks,
 * each run as one workgroup of cm_launch's kernel would run it once the
 * pieces are done; the workgroup that finishes the last chunk scores the
 * sweep (when it is scored) and marks the request done in host memory.
 * Results equal cm_launch's for the same sweep with a 256-thread workgroup;
 * a request's outputs are complete once cm_queue_poll reports it done.
 *  cm_queue_create  kind CM_CONFLICT_LCA, precision CM_FP64 or
 *                   CM_FP32_STEP (else CM_E_UNSUPPORTED); slots: requests
 *                   in flight (1..4096); groups_per_cu: persistent
 *                   workgroups per compute unit (1..4; the rest of the GPU
 *                   stays free for other streams' kernels); idle_us: the
 *                   kernel ends after this long without an item (100 us ..
 *                   10 s) and is launched again by the next submit or poll.
 *                   Allocates the queue's pinned host memory, a small
 *                   device block (counters and copies of the ring and the
 *                   descriptors) and two streams of its own, for the kernel
 *                   and for the host copies (default priority).
 *  cm_queue_submit  validates like cm_launch, waits until the work enqueued
 *                   so far on producer_stream is finished (NULL: no
 *                   producer; the uploads of the sweep's inputs go there),
 *                   then publishes the request and returns a ticket.  host
 *                   (or NULL): pinned host buffers (hipHostMalloc; others
 *                   give CM_E_INVALID) that receive copies of hist, stats,
 *                   score and best (NULL fields skipped, sizes as in
 *                   cm_result), enqueued on the queue's copy stream by the
 *                   first cm_queue_poll that finds the request done on the
 *                   device.
 *                   CM_E_BUSY when no slot is free, or when max(512,
 *                   4 slots) requests have been published since the oldest
 *                   unfinished one (nothing is published then).  The
 *                   buffers must stay allocated until the ticket is done.
 *  cm_queue_poll    *done = 1 once the request's outputs (and, for a scored
 *                   sweep, its scores) are complete, and its host copies
 *                   with them; the ticket is then retired.  It never waits.
 *                   CM_E_INVALID for an unknown ticket.
 *  cm_queue_destroy asks the kernel to stop, waits until it has ended and
 *                   frees the queue.  A running kernel first finishes the
 *                   items already copied to the device; requests that
 *                   cm_queue_poll has not reported done are abandoned
 *                   (their outputs may be incomplete; their tickets are
 *                   void), and their buffers must stay allocated until
 *                   cm_queue_destroy returns.
 * A queue is not thread-safe: submit, poll and destroy from one thread. */
typedef struct cm_queue cm_queue;
cm_status cm_queue_create(cm_handle *h, uint32_t kind, uint32_t precision, uint32_t slots,
                          uint32_t groups_per_cu, uint32_t idle_us, cm_queue **out);
cm_status cm_queue_submit(cm_queue *q, const cm_model *model, const cm_sweep *sweep,
                          const cm_result *result, void *workspace, uint64_t workspace_bytes,
                          const cm_host_result *host, void *producer_stream, uint64_t *ticket);
cm_status cm_queue_poll(cm_queue *q, uint64_t ticket, int *done);
cm_status cm_queue_destroy(cm_queue *q);

/* Measured ceiling of the lane kernels' step: `lanes` lanes (a multiple of
 * 256) each run `steps` steps of the model's random numbers (one Philox
 * block per step, per two steps for the DDM, and its Box-Muller pair) and
 * state update, from the start state, with no threshold tests, refills or
 * histogram work; out (DEVICE, [lanes] doubles) receives each lane's final
 * first unit.  steps * lanes / time is the step rate the instruction mix
 * itself reaches on the device: the empirical roofline against which a
 * sweep's rate is compared.  Kinds CM_DDM and CM_CONFLICT_LCA, precisions
 * CM_FP64 and CM_FP32_STEP; only the model's parameters are read. */
cm_status cm_ceiling(cm_handle *h, const cm_model *model, uint32_t steps, uint64_t lanes,
                     double *out, void *hip_stream);

/* Kernel timing.  While enabled, every cm_launch brackets its simulation
 * kernel with a pair of HIP events on the launch stream.  cm_profile_read
 * waits for the recorded events, returns the summed kernel time in
 * milliseconds and the number of timed launches since profiling was
 * enabled, and keeps profiling on.  Enabling again resets the totals. */
cm_status cm_profile(cm_handle *h, int enable);
cm_status cm_profile_read(cm_handle *h, double *sim_ms, uint64_t *launches);

/* Text of the last failure on this thread ("" if none).  The paper's
 * generated code reports no errors of its own; this is the error channel of
 * a C boundary that lets no exception cross it.  The pointer stays valid
 * until the next failing call on the same thread. */
const char *cm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
