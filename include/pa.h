/*
 * pa.h -- C ABI of the MI355X population-annealing Max-Cut engine.
 *
 * Problem (paper arXiv 2510.21105, section 1, eq. (1)): given an undirected
 * graph with weights w_ij, find x in {-1,+1}^N maximising
 *     cut(x) = 1/2 * sum_{i<j} w_ij (1 - x_i x_j).
 * Section 2: this is the ground state of the Ising energy with couplings
 * J_ij = -w_ij, E(x) = sum_{i<j} w_ij x_i x_j, and cut = (W_tot - E) / 2 with
 * W_tot = sum_{i<j} w_ij.
 * Method (abstract, section 3): population annealing Monte Carlo with
 * adaptive control of stochasticity and periodic non-local moves. The
 * paper names these parts without defining them; the exact integer rules
 * implemented here (Philox4x32-10 draws, fixed-point Metropolis thresholds,
 * systematic resampling, noise levels, Houdayer cluster moves) are spelled
 * out with pa_run below and in the project's design notes.
 *
 * Conventions for every call:
 *  - Every function returns pa_status; PA_OK is 0 and errors are negative.
 *    No C++ exception crosses this boundary. On error, pa_last_error()
 *    returns a thread-local, NUL-terminated description that stays valid
 *    until the next call on the same thread.
 *  - Host pointers are read during the call only (inputs are copied).
 *  - Device memory is never allocated by the library: pa_run works inside a
 *    caller-owned device workspace and on a caller-owned HIP stream.
 *  - Nodes are 0-based; the paper's variable v is node v-1.
 */
#ifndef PA_H
#define PA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PA_OK = 0,
    PA_EINVAL = -1,     /* malformed graph, schedule or argument          */
    PA_ERANGE = -2,     /* a size or count outside the supported range    */
    PA_EWORKSPACE = -3, /* workspace missing, too small or misaligned     */
    PA_EDEVICE = -4,    /* HIP runtime error (text in pa_last_error)      */
    PA_ESTATE = -5,     /* call out of order, e.g. results before a run   */
    PA_EABORTED = -6    /* the run stopped at the step set by pa_set_fault_step */
} pa_status;

/* Opaque solver: one validated graph. Owned by the caller from pa_create
 * until pa_destroy. Not thread-safe: one thread at a time per solver. */
typedef struct pa_solver pa_solver;

/* Annealing schedule. All pointers are host memory, copied by pa_run. */
typedef struct {
    int32_t n_steps;          /* K >= 1 temperature steps                         */
    const double *beta;       /* K inverse temperatures: finite, >= 0, non-decreasing */
    int32_t sweeps_per_step;  /* S, 1..65535 Metropolis sweeps per step           */
    const int32_t *order;     /* NULL = nodes 0..N-1; else a permutation of 0..N-1 */
    int32_t as_enable;        /* adaptive stochasticity: 0 off, 1 on              */
    int32_t as_stall_steps;   /* steps without a new best before raising the level, >= 1 */
    int32_t as_max_level;     /* highest noise level, 0..15                       */
    int32_t as_frozen_inv;    /* raise only if frozen_inv * uphill_accepts < uphill_attempts, >= 1 */
    double as_gamma;          /* level l sweeps at beta_k * gamma^l, 0 < gamma <= 1 */
    int32_t nl_period;        /* non-local cluster moves every nl_period steps, 0 = off;
                                 the kind is nl_kind below                       */
    int32_t sweep_kernel;     /* 0 = automatic; 1 = one node per lane over byte spin
                                 records (max degree <= 127); 2 = one replica per lane
                                 over bit spin words. Results never depend on it.  */
    int32_t tile_replicas;    /* replicas per workgroup, 0 = automatic; kernel 1 takes
                                 4, 8 or 16, kernel 2 takes 16, 32 or 64. Results
                                 never depend on it.                              */
    int32_t wg_threads;       /* threads per sweep workgroup, 0 = automatic, else a
                                 multiple of 64 in [64, 1024]. Results never depend on it. */
    int32_t record;           /* bit 0: keep per-step copy counts; bit 1: keep the
                                 initial population (both for pa_get_* below)     */
    int32_t nl_kind;          /* kind of non-local move (the paper names the moves, section
                                 3, without defining them):
                                 0 = Houdayer cluster move on the replica pairs
                                     (p, p + R/2), R even: the connected component of a
                                     random node of the set where the two disagree is
                                     flipped in both;
                                 1 = single-replica Wolff cluster update of every
                                     replica at the step's sweep temperature beta' =
                                     beta_k gamma^l: a bond with w_ij x_i x_j < 0 is
                                     activated with probability 1 - exp(-2 beta'), and
                                     the active-bond component of a random node flips. */
    int32_t beta_adapt;       /* 0: step k sweeps at beta[k] (K steps). 1: adaptive steps:
                                 beta[] is an evenly spaced grid; each step sweeps at the
                                 current grid point g and then moves to g + j for the
                                 largest j in [1, min(adapt_jump, K-1-g)] whose resampling
                                 weights W_r = floor(2^32 exp(-((beta[j] - beta[0])
                                 (E_r - E_min)))) keep (sum W)^2 / (R sum W^2) >=
                                 adapt_num / adapt_den (decided in exact integers; j = 1
                                 if none), resampling with those weights. On an evenly
                                 spaced grid beta[j] - beta[0] is the increase
                                 beta[g+j] - beta[g] of the jump wherever it starts, so
                                 the reweighting is the population-annealing one; a grid
                                 whose spacings differ by more than 1e-9 of the mean
                                 spacing plus 8 ulps of the largest |beta| is refused
                                 with PA_EINVAL. The run ends after the step at the last
                                 grid point (at most K steps; later steps are empty).
                                 The paper adapts the annealing without defining how
                                 (section 3); this is one definition. pa_run then looks
                                 every 64 steps, with a stream synchronisation, whether
                                 the run has ended, and enqueues no further steps once
                                 it has.                                          */
    int32_t adapt_jump;       /* 1..64, largest jump in grid points (beta_adapt = 1)  */
    int32_t adapt_num, adapt_den; /* target, 0 <= adapt_num <= adapt_den <= 65536, den >= 1 */
    int32_t field_bits;       /* 0 = no check; 8 or 16: refuse the run with PA_ERANGE
                                 unless every local field h_i = sum_j w_ij x_j (|h_i| is
                                 at most the degree of i) fits a signed integer of that
                                 many bits, for a caller that keeps fields (such as
                                 those of pa_get_population) in that width; other
                                 values give PA_EINVAL. The device keeps no fields, so
                                 this is a check only: results never depend on it. */
} pa_schedule;

/* Text of the last error on this thread ("" if none). */
const char *pa_last_error(void);

/*
 * Validate and keep a graph (host only; no device call).
 *   n        number of nodes, 2 <= n <= 32767
 *   row_ptr  n+1 int32, row_ptr[0] = 0, non-decreasing
 *   col      row_ptr[n] int32 neighbour ids in [0, n)
 *   w        row_ptr[n] int8 weights, each -1 or +1 (the G-set's binary
 *            signed or unsigned weights, paper section 1)
 * The CSR must be symmetric (j in row i with weight w iff i in row j with
 * weight w), without self loops or repeated neighbours, and every node needs
 * degree <= 4096. Errors: PA_EINVAL (malformed), PA_ERANGE (sizes).
 */
pa_status pa_create(pa_solver **out, int32_t n, const int32_t *row_ptr,
                    const int32_t *col, const int8_t *w);

/* Release the solver (NULL is accepted). The workspace of its last run is
 * the caller's and is not touched. */
pa_status pa_destroy(pa_solver *s);

/* Graph facts: n, nnz (directed entries), W_tot = sum_{i<j} w_ij, max degree. */
pa_status pa_graph_info(const pa_solver *s, int64_t out[4]);

/* Device workspace bytes pa_run needs for this schedule and population R.
 * The workspace must be 256-byte aligned. */
pa_status pa_workspace_bytes(const pa_solver *s, const pa_schedule *sch, int32_t R,
                             size_t *bytes);

/*
 * Run population annealing with R replicas (1 <= R <= 32768; even when
 * nl_period > 0 and nl_kind = 0), 64-bit seed and instance id (0..65535). Asynchronous on
 * `stream` (a hipStream_t; NULL is the default stream) inside `workspace`
 * (device memory of at least pa_workspace_bytes, 256-byte aligned). The
 * workspace holds the results and must stay untouched until the last
 * pa_best_* / pa_get_* call for this run. Every output is a pure function of
 * (graph, schedule except sweep_kernel, tile_replicas and wg_threads, R, seed,
 * instance).
 *
 * Per step k = 0..K-1 (all integer on the device; g = k unless beta_adapt):
 *   1. S sweeps over `order`; for node i of replica r:
 *      m = -x_i h_i with h_i = sum_j w_ij x_j; accept iff m <= 0 or
 *      draw(0, s, k, i, r) < floor(2^32 exp(-(beta_g gamma^l * 2m))); the best
 *      configuration is tracked after every sweep.
 *   2. Every nl_period steps: the non-local move of kind nl_kind (Houdayer
 *      cluster move on replica pairs, or a Wolff update of every replica),
 *      then a best check.
 *   3. Noise level update (adaptive stochasticity).
 *   4. If g < K-1: weights floor(2^32 exp(-((beta_{k+1}-beta_k)(E_r-E_min))))
 *      (adaptive steps: of the chosen jump), systematic resampling back to R
 *      replicas.
 * draw(tag, s, k, i, r) is word (r & 3) of Philox4x32-10 with key
 * (lo32 seed, hi32 seed) and counter (i, s | tag << 16, k, (r >> 2) | instance << 16).
 *
 * Errors: PA_EINVAL (a malformed schedule field), PA_ERANGE (a count out of
 * range: R, instance, sweeps_per_step, as_max_level; or a graph whose spin
 * state does not fit a workgroup's LDS: every graph with +1 weights fits, a
 * graph with -1 weights fits up to 32,511 nodes at max degree <= 127 and
 * about 23,500 nodes above),
 * PA_EWORKSPACE (workspace short or misaligned), PA_EDEVICE (HIP error; text
 * in pa_last_error). All checks happen before any device work is enqueued.
 */
pa_status pa_run(pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed,
                 uint32_t instance, void *workspace, size_t workspace_bytes, void *stream);

/* Bytes of the static device workspace of pa_run_static (64 MiB). */
#define PA_STATIC_SCRATCH_BYTES (64u << 20)

/*
 * pa_run for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * run, with the same results, enqueued on `stream`, but inside a workspace
 * the library holds as a static device array of PA_STATIC_SCRATCH_BYTES per
 * GPU (kept until the process ends) instead of one the caller passes. It
 * calls no hipMalloc, hipHostMalloc, hipFree or other allocating device
 * routine: the host inputs are copied from pageable host memory, and run
 * timing (pa_set_timing) is not recorded. The first call on a device looks
 * up the array's address there (hipGetSymbolAddress).
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents: the results of this run stay readable through the pa_best_* /
 * pa_get_* / pa_checkpoint_save calls of this solver only until the next
 * pa_run_static on the same GPU (from any solver) starts, and calls that
 * overlap on one GPU (other streams, other threads, or this run still in
 * flight) race on the array; the caller orders them. pa_run_steps cannot
 * continue such a run.
 * Errors: as pa_run; PA_EWORKSPACE when the run needs more than
 * PA_STATIC_SCRATCH_BYTES (pa_workspace_bytes gives the need), PA_EDEVICE
 * when the array's address cannot be taken.
 */
pa_status pa_run_static(pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed,
                        uint32_t instance, void *stream);

/*
 * Steps [k_begin, k_end) of the same run as pa_run (0 <= k_begin <= k_end <=
 * K), for schedules too long for one call and for checkpoints. k_begin = 0
 * starts the run (initial population) in `workspace`; k_begin > 0 continues
 * the run that this solver holds in the same workspace, which must have
 * reached exactly step k_begin with the same graph, schedule (launch-shape
 * fields aside), R, seed and instance, either through earlier pa_run_steps
 * calls or pa_checkpoint_load. Splitting a run into ranges gives results
 * identical to one pa_run. The best and statistics calls report the steps
 * run so far; pa_get_population returns the population that the next step
 * starts from (after resampling). Errors as pa_run, plus PA_EINVAL for a bad
 * range, PA_ESTATE when there is no such run to continue (wrong step, other
 * schedule, R, seed or instance) and PA_EWORKSPACE for another workspace.
 * A stream other than the previous call's is ordered after it by a host
 * synchronisation.
 */
pa_status pa_run_steps(pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed,
                       uint32_t instance, int32_t k_begin, int32_t k_end, void *workspace,
                       size_t workspace_bytes, void *stream);

/*
 * Checkpoints (runs of many hours, paper section 3, need them): the complete
 * state between two steps, as a host byte blob. Counter-based draws make a
 * restored run continue exactly as the uninterrupted one.
 *   pa_checkpoint_bytes  size of the blob for the solver's current run.
 *   pa_checkpoint_save   writes it into caller memory `out` (at least that
 *                        many bytes); synchronises the run's stream. The blob
 *                        holds the population (with the pending resampling
 *                        applied), energies, noise-level state, best
 *                        configuration and its record, the per-step
 *                        statistics of the steps run, and the recorded copy
 *                        counts / initial population, plus a header with the
 *                        next step and a hash of graph, schedule (launch-shape
 *                        fields aside), R, seed and instance.
 *   pa_checkpoint_load   prepares `workspace` for that run (as pa_run would)
 *                        and restores the state from `in`; synchronises
 *                        `stream`. Continue with pa_run_steps(k, K) where k
 *                        is the saved next step. The launch shape may differ
 *                        from the saved run's.
 * Errors: PA_EINVAL for null pointers, a short buffer, or a blob of another
 * library version, graph, schedule, R, seed or instance (checked before any
 * device call); PA_ESTATE when the solver has no run to save; as pa_run for
 * the workspace and device.
 */
pa_status pa_checkpoint_bytes(const pa_solver *s, size_t *bytes);
pa_status pa_checkpoint_save(pa_solver *s, void *out, size_t bytes);
pa_status pa_checkpoint_load(pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed,
                             uint32_t instance, const void *in, size_t bytes, void *workspace,
                             size_t workspace_bytes, void *stream);

/* One run of a batch: the arguments of pa_run. */
typedef struct {
    pa_solver *solver;          /* distinct solver per run */
    const pa_schedule *schedule;
    int32_t R;
    uint64_t seed;
    uint32_t instance;
    void *workspace;            /* as for pa_run: 256-byte aligned device memory */
    size_t workspace_bytes;
} pa_batch_run;

/*
 * Many independent runs sharing the device (for instance a mix of graphs and
 * population sizes whose single runs leave compute units idle): run i is
 * enqueued as pa_run would on streams[i % n_streams], so runs on different
 * streams overlap on the device while each keeps the results of the same run
 * alone, bit for bit. When a run has adaptive steps (beta_adapt = 1, whose
 * host waits for the device every 64 steps), every run is started first and
 * the steps are then enqueued in chunks of 64, one chunk of each run in turn,
 * so that no run's wait holds back the others. Asynchronous like pa_run
 * (apart from those waits); the per-solver result calls synchronise the
 * run's stream. Solvers must be distinct and each run needs its own
 * workspace. Returns PA_OK, or the status of the first run that fails (its
 * index is in pa_last_error); the runs before it stay enqueued and valid (in
 * a chunked batch the others stay valid part-way, resumable with
 * pa_run_steps). PA_EINVAL for a null array, count < 1, n_streams < 1 or a
 * solver used twice.
 */
pa_status pa_run_batch(const pa_batch_run *runs, int32_t count, void *const *streams,
                       int32_t n_streams);

/* One run of a fused batch: the arguments of pa_run without workspace and
 * stream. */
typedef struct {
    pa_solver *solver;                /* distinct solver per run */
    const pa_schedule *schedule;      /* launch-shape fields are ignored */
    int32_t R;
    uint64_t seed;
    uint32_t instance;
} pa_fused_entry;

/* Opaque fused batch: runs planned to share kernel launches. */
typedef struct pa_fused pa_fused;

/*
 * Many runs sharing kernel launches (for instance dozens of uneven graphs and
 * population sizes, most of which alone leave compute units idle). Runs are
 * grouped by record mode (graphs with only +1 weights, graphs with -1
 * weights) and graph size (below 1,500, 3,000 and 5,000 nodes, and larger);
 * step k of a whole group is one sweep launch, whose workgroups each take one
 * replica tile of one run from a work list, and one epilogue launch with one
 * workgroup per run. Groups run concurrently, each on a stream of its own
 * forked from and joined back to the caller's. Every run gives exactly the
 * results of pa_run with the same arguments (any launch shape), and after
 * pa_fused_run its solver answers the pa_best_* / pa_get_* /
 * pa_checkpoint_save calls as after pa_run; pa_run_steps cannot continue it.
 *
 *   pa_fused_create   validates and plans the runs (host only; the schedules,
 *                     orders and arrays are copied). Each run must be a valid
 *                     pa_run on its solver with nl_period = 0 and beta_adapt =
 *                     0, maximum degree <= 127 and no inverse temperature whose
 *                     acceptance rounds to 1 for some uphill moves only.
 *                     Solvers must be distinct and outlive the batch.
 *   pa_fused_workspace_bytes  device bytes the batch needs (every run's state
 *                     and the batch's own argument and work-list tables).
 *   pa_fused_tune     measures, per group, each candidate launch shape (4, 8
 *                     or 16 replicas per workgroup x 64, 128, 256 or 512
 *                     threads, where the group's graphs fit LDS) on the
 *                     first probe_steps (1..64) steps of the group's runs
 *                     inside `workspace` (two probes each), and keeps the
 *                     fastest. Synchronous (it waits for the probes); leaves
 *                     no valid results. Without it a default shape is used:
 *                     8 replicas per workgroup and the smallest thread count
 *                     that needs no more rounds per sweep than 512 threads.
 *   pa_fused_run      enqueues the whole batch on `stream`: each run's setup
 *                     (inputs, initial population), then the step loop of
 *                     every group, captured once into a HIP graph (for this
 *                     workspace address and these shapes) and launched on
 *                     `stream`. Asynchronous; the results live in `workspace`
 *                     (256-byte aligned, at least pa_fused_workspace_bytes),
 *                     which must stay untouched until the last result call.
 *   pa_fused_set_graph  1 (default): step loop as a HIP graph; 0: the same
 *                     launches enqueued directly (for comparison).
 *   pa_fused_info     per group 8 int64 {record mode (0 +1 weights, 2 signed
 *                     graphs with sign-bit entries), runs, replicas per
 *                     workgroup, threads, offset entries (1) or record
 *                     indices (0), sweep workgroups per step, sweep LDS bytes,
 *                     measured femtoseconds per attempt (0 untuned)} for up to
 *                     max_groups groups into `out` (NULL: count only), and
 *                     the number of groups into *groups.
 *   pa_fused_destroy  releases the batch (NULL accepted); the solvers keep
 *                     their results.
 * Errors: PA_EINVAL (null arguments, a run that cannot share launches, a
 * solver used twice, a bad probe count), the errors of pa_run for each run
 * (the run index is in pa_last_error), PA_EWORKSPACE, PA_EDEVICE.
 */
pa_status pa_fused_create(pa_fused **out, const pa_fused_entry *runs, int32_t count);
pa_status pa_fused_workspace_bytes(const pa_fused *f, size_t *bytes);
pa_status pa_fused_tune(pa_fused *f, void *workspace, size_t workspace_bytes, void *stream,
                        int32_t probe_steps);
pa_status pa_fused_run(pa_fused *f, void *workspace, size_t workspace_bytes, void *stream);
pa_status pa_fused_set_graph(pa_fused *f, int32_t on);
pa_status pa_fused_info(const pa_fused *f, int64_t *out, int32_t max_groups, int32_t *groups);
pa_status pa_fused_destroy(pa_fused *f);

/* Opaque pool of resident runs advanced together (continuous batching). */
typedef struct pa_pool pa_pool;

/*
 * A pool of runs sharing the device as they come and go (serving): the pool
 * works inside a caller-owned device region (its HBM budget) and admits
 * submitted runs in arrival order, without overtaking, as their state fits
 * the memory left. Admitted runs of one launch shape (record mode, tile
 * width, entry form, threads, LDS occupancy class) form a lane with a stream
 * of its own; each iteration of a lane advances all its runs by one
 * temperature step, each at its own step: one sweep launch over the replica
 * tiles of those runs and one epilogue launch with a workgroup per run.
 * Lanes progress independently. A run's population stays resident on the
 * device from admission to release. Every run gives exactly the results of
 * pa_run with the same arguments (GPU tests compare with the oracle).
 *
 *   pa_pool_create    over `workspace` (256-byte aligned device memory,
 *                     kept by the caller until pa_pool_destroy); about 10 MB
 *                     of it hold the lanes' argument tables, the rest the
 *                     runs. Host only.
 *   pa_pool_submit    queues a run (a valid pa_run with nl_period = 0 and
 *                     beta_adapt = 0, maximum degree <= 127; inputs copied)
 *                     and returns its ticket. PA_EWORKSPACE if it can never
 *                     fit the pool; PA_EINVAL if its solver already has an
 *                     unreleased run in the pool.
 *   pa_pool_cancel    drops a run that is still waiting (PA_ESTATE if it was
 *                     admitted).
 *   pa_pool_advance   admits what fits (setting it up on `stream`, always
 *                     the same stream for a pool), then enqueues up to
 *                     `iterations` (1..1024) iterations of every lane on the
 *                     lane's stream, rebuilding a lane's argument tables only
 *                     when runs join or leave it; a lane with two batches
 *                     still in flight is skipped this call. *done = lane
 *                     iterations enqueued (0: nothing to step now).
 *                     Asynchronous; never waits for a busy lane.
 *   pa_pool_poll      tickets of runs that have finished since the last poll
 *                     (up to cap); their solvers answer the pa_best_* /
 *                     pa_get_* calls as after pa_run, until released.
 *   pa_pool_release   returns a finished run's memory to the pool; its
 *                     solver's results are gone afterwards (PA_ESTATE before
 *                     its last step was enqueued).
 *   pa_pool_info      {waiting, stepping, finished and not released, bytes
 *                     in use, bytes for runs, iterations so far}.
 *   pa_pool_destroy   waits for the pool's stream and releases the pool.
 * Solvers must outlive their runs in the pool.
 */
pa_status pa_pool_create(pa_pool **out, void *workspace, size_t workspace_bytes);
pa_status pa_pool_submit(pa_pool *p, const pa_fused_entry *run, int64_t *ticket);
pa_status pa_pool_cancel(pa_pool *p, int64_t ticket);
pa_status pa_pool_advance(pa_pool *p, void *stream, int32_t iterations, int32_t *done);
pa_status pa_pool_poll(pa_pool *p, int64_t *tickets, int32_t cap, int32_t *count);
pa_status pa_pool_release(pa_pool *p, int64_t ticket);
pa_status pa_pool_info(const pa_pool *p, int64_t out[6]);
pa_status pa_pool_destroy(pa_pool *p);

/*
 * Test hook: the fixed-point tables a run with this schedule uses, dense, as
 * little-endian u64 into caller memory `out` (NULL: only *bytes is set):
 *   thresholds [K][L][d_max + 1], L = as_max_level + 1 with adaptive
 *     stochasticity else 1: entry m = floor(2^32 exp(-(beta_k gamma^l * 2m)))
 *     for m >= 1 (gamma^l as l successive FP64 products) and 2^32 for m = 0;
 *   weights [K - 1][e_span + 1]: entry n = floor(2^32 exp(-(beta_{k+1} -
 *     beta_k) n)); with beta_adapt = 1 instead [J][e_span + 1], J =
 *     min(adapt_jump, K - 1), row j - 1 for beta_j - beta_0.
 * *bytes = 8 (K L (d_max + 1) + (K - 1 or J)(e_span + 1)). PA_EINVAL for a bad
 * schedule (as for pa_run) or negative sizes, PA_ERANGE when
 * d_max > 4096, e_span > 2^26 or *bytes is too small for a non-NULL `out`.
 */
pa_status pa_build_tables(const pa_schedule *sch, int32_t d_max, int32_t e_span, void *out,
                          size_t *bytes);

/* Best cut found by the last run: cut = (W_tot - E) / 2 (eq. (1)) and its
 * Ising energy E. Synchronises the run's stream. PA_ESTATE before a run. */
pa_status pa_best_cut(pa_solver *s, int64_t *cut, int32_t *energy);

/* Where the best was found: {E, step, sweep, replica}; step -1 means the
 * initial population, sweep == S means right after a non-local move. */
pa_status pa_best_info(pa_solver *s, int64_t out[4]);

/* Best configuration, n int8 values in {-1,+1} (caller-allocated). */
pa_status pa_best_config(pa_solver *s, int8_t *x);

/* Best configuration in the paper's hexadecimal format (section 3): digit p
 * holds variables 4p+1..4p+4, most significant bit first, bit 1 = spin +1,
 * zero-padded to a multiple of 4 variables. Needs len >= ceil(n/4) + 1. */
pa_status pa_best_config_hex(pa_solver *s, char *buf, size_t len);

/* Final population of the last run: x (R*n int8, replica-major, +-1), the
 * local fields h (R*n int16, replica-major: h_i = sum_j w_ij x_j, so that
 * E = (1/2) sum_i x_i h_i, eq. (1) up to the constant W_tot) and E (R int32).
 * The device keeps no fields: h is computed on the host from x. Any pointer
 * may be NULL. Synchronises the stream. */
pa_status pa_get_population(pa_solver *s, int8_t *x, int16_t *h, int32_t *E);

/* Initial population (R*n int8); needs schedule.record bit 1. */
pa_status pa_get_initial_population(pa_solver *s, int8_t *x);

/* Fields per step in pa_get_step_stats (and per row of the statistics in a
 * checkpoint). */
#define PA_STAT_FIELDS 10

/* Per-step records: K * PA_STAT_FIELDS int64, row k = step k, into caller
 * memory `out` (exactly that many values are written). Fields of a row:
 *   0  E_min: lowest energy after the step's sweeps and non-local move,
 *      before resampling
 *   1  E_sum: sum of the R energies at the same point
 *   2  uphill attempts (m > 0) during the step's sweeps
 *   3  uphill accepts
 *   4  noise level used by the step's sweeps (0 without adaptive
 *      stochasticity)
 *   5  best E after the step
 *   6  replicas with at least one copy in the resampling (0 on the last step)
 *   7  weight sum S of the resampling (0 on the last step)
 *   8  grid point g whose inverse temperature the step swept at (= k unless
 *      beta_adapt)
 *   9  grid points advanced after the step (1 unless beta_adapt; 0 on the
 *      last step)
 * Rows of steps that did not run (an adaptive run that ended early, or a
 * range not yet run) are 0. Synchronises the run's stream. */
pa_status pa_get_step_stats(pa_solver *s, int64_t *out);

/* Copy counts n_r of every resampling, K*R int32 (row K-1 is zero); needs
 * schedule.record bit 0. */
pa_status pa_get_counts(pa_solver *s, int32_t *out);

/* Launch facts of the last run: {sweep kernel (1 or 2), replicas per
 * workgroup, threads per workgroup, workgroups per sweep launch, dynamic LDS
 * bytes per workgroup, dependency levels per sweep, workgroup rounds per
 * sweep (kernel 1) or longest wave pass stream (kernel 2), sweep launches}. */
pa_status pa_get_launch_info(pa_solver *s, int64_t out[8]);

/* Timing mode for measurement. every = 0: off (the default); every = n >= 1:
 * runs started after this call record HIP events on the run's stream around
 * the sweep-kernel launch of every step k with k mod n = 0 (n = 1: every
 * launch; a larger n keeps the events' own cost out of most steps).
 * pa_get_sweep_time then returns the summed time of the timed sweep
 * launches in ms and their number (synchronising the stream). Results are
 * unchanged. Errors: PA_EINVAL for every < 0; pa_get_sweep_time returns
 * PA_ESTATE when the run was not timed. */
pa_status pa_set_timing(pa_solver *s, int32_t every);

/*
 * Fault injection for tests of failure handling and recovery. k >= 0: the
 * next call on this solver that would enqueue step k (pa_run, pa_run_steps,
 * pa_run_static) stops before it:
 * steps before k are enqueued as usual, the call synchronises its stream and
 * returns PA_EABORTED, and the solver holds the run after k steps, as if
 * pa_run_steps had been called for [0, k) -- pa_checkpoint_save and
 * pa_run_steps from step k work on it, and continuing gives the results of
 * an uninterrupted run. The hook fires once, then clears itself; k = -1
 * clears it. Batched, fused and pooled runs ignore it. Errors: PA_EINVAL for
 * k < -1 or a null solver.
 */
pa_status pa_set_fault_step(pa_solver *s, int32_t k);
pa_status pa_get_sweep_time(pa_solver *s, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* PA_H */
