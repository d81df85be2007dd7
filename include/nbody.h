/*
 * nbody.h -- C ABI of the MI355X (gfx950) Hermite 6th-order block-step N-body
 * library (libnbody.so).
 *
 * The method is the direct N-body scheme of Goz et al., "Astrophysical code
 * migration into Exascale Era" (section "Code implementation": Hermite 6th-order
 * integrator, double precision for inter-particle distances and accelerations,
 * an extended-precision float-float alternative; section "Performance results":
 * the O(N^2) evaluation as the dominant kernel). The paper prints no formula; the
 * formulas used are the standard 6th-order Hermite scheme (Nitadori & Makino 2008)
 * with power-of-two block steps (Makino 1991; Aarseth 2003). Each call below names
 * the step of the block-step cycle it performs:
 *
 *     nb_active    -> next block time and the bodies due at it
 *     nb_predict   -> Taylor prediction of every body to that time
 *     nb_evaluate  -> acceleration, jerk, snap, potential of the due bodies (O(N_act N))
 *     nb_correct   -> 6th-order Hermite corrector of the due bodies
 *     nb_timesteps -> new power-of-two steps of the due bodies
 *     nb_energy    -> total energy (diagnostic, O(N^2))
 *
 * Conventions
 *   - Device pointers ("d_") are HIP device addresses on the context's device;
 *     host pointers ("h_") are ordinary host memory.
 *   - Vectors are structure-of-arrays, component-major: x[k*n + i], k = 0, 1, 2.
 *   - Time is an int64 tick count; one tick is 2^dt_min_log2 time units. A body on
 *     level k has step 2^(dt_max_log2 - k). Units: G = 1.
 *   - Evaluation results are out[c*n_act + q], c = 0..9 = ax ay az jx jy jz sx sy sz
 *     phi, for the q-th entry of the index list.
 *   - Index lists are int32, strictly ascending, each in [0, n).
 *
 * Ownership: the caller owns all device memory. nb_create carves every device
 * array the library uses out of one caller-provided workspace, which must stay
 * valid until nb_destroy. The library owns only the host-side context (and a few
 * bytes of pinned host memory for results). It never allocates device memory.
 *
 * Ordering: every call is enqueued on the stream given in nb_params and returns
 * without waiting, except nb_active, nb_step, nb_energy and nb_get_state, which
 * wait for the stream (they return values to the host). Input arrays passed to an
 * asynchronous call must stay valid until the stream reaches it.
 *
 * Times: an int64 tick count rather than a double, so block times compare and
 * divide exactly (a body's time is always a multiple of its power-of-two step).
 *
 * Errors: no C++ exception crosses this boundary; every call returns an
 * nb_status and nb_last_error() gives a message. NB_ERR_SPACE is the status for a
 * workspace (or the fixed device array of nb_evaluate_static) too small for the
 * request; the library never allocates, so it never runs out of memory itself. Argument errors found on the
 * host are returned at once. Errors found by kernels (an index out of range, a
 * non-finite corrector result, a step below dt_min) are latched in a device word
 * and returned by the next waiting call, which then clears the word.
 * One host thread at a time may use a context.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nb_ctx nb_ctx; /* opaque, library-owned host object */

typedef enum {
    NB_OK = 0,
    NB_ERR_ARG = 1,     /* a bad argument (host check) or a bad index (device check) */
    NB_ERR_SPACE = 2,   /* workspace smaller than nb_workspace_bytes() */
    NB_ERR_DEVICE = 3,  /* a HIP runtime error */
    NB_ERR_STATE = 4,   /* calls out of order (e.g. nb_correct without nb_evaluate) */
    NB_ERR_NUMERIC = 5  /* non-finite values, or a body needs a step below dt_min */
} nb_status;

typedef enum {
    NB_FP64 = 0,  /* everything in IEEE binary64 */
    NB_SPLIT = 1  /* evaluation: float-float differences, FP32 algebra, FP64 sums */
} nb_precision;

/* nb_params.flags: nb_start also evaluates the exact third derivative of every
 * body's acceleration (crackle, nb_evaluate_crackle) and stores it as c, instead of
 * starting from c = 0; it enters the first step's predictions. Adds 104 bytes per
 * body to the workspace. */
#define NB_FLAG_START_CRACKLE 1

typedef struct {
    int64_t n;            /* number of bodies, 1 <= n <= 2^30 */
    double eps;           /* Plummer softening length, >= 0 */
    double eta;           /* accuracy parameter of the 6th-order step criterion (> 0) */
    double eta_init;      /* accuracy parameter of the initial-step rule (> 0) */
    int32_t dt_max_log2;  /* largest step 2^dt_max_log2 */
    int32_t dt_min_log2;  /* tick size and smallest step 2^dt_min_log2;
                             0 <= dt_max_log2 - dt_min_log2 <= 62 */
    int32_t precision;    /* nb_precision of nb_evaluate */
    int32_t flags;        /* 0 or NB_FLAG_START_CRACKLE */
    int64_t partial_slots;/* capacity of the partial-sum buffer in units of 10 doubles
                             (j-split x active body); 0 = default: max(4n, 2^20), raised
                             for FP64 and 8192 <= n <= 65536 to what the symmetric full
                             evaluation needs: 1 + 768 U + 384 nb (nb - 1) slots with
                             nb = ceil(n / 768) and U = P nb (nb + 1) / 2 units, P the parts
                             per block (2 to 12); about n^2 / 500 */
    void *stream;         /* hipStream_t for every launch; NULL = the null stream */
} nb_params;

/* A view of the full body state, for nb_set_state (read) and nb_get_state
 * (written). Every pointer is a device address; NULL fields are skipped.
 * Shapes: m, a4n, a5n, phi, tick, level: [n]; x, v, a, j, s, c: [3][n]. */
typedef struct {
    double *m;      /* masses */
    double *x, *v;  /* position, velocity at the body's own time */
    double *a, *j, *s; /* acceleration, jerk, snap at the body's own time */
    double *c;      /* third derivative of a (interpolated by the corrector) */
    double *a4n, *a5n; /* |4th| and |5th| derivative of a (from the corrector) */
    double *phi;    /* potential from the body's last evaluation (read-only) */
    int64_t *tick;  /* the body's own time, in ticks */
    int32_t *level; /* the body's step level */
} nb_state;

/* Bookkeeping (no passage of the method): the device memory of a context.
 * Size in bytes of the device workspace a context with these parameters needs.
 * Returns NB_ERR_ARG for invalid parameters. Touches no device. */
nb_status nb_workspace_bytes(const nb_params *p, size_t *h_bytes);

/* Create a context over d_workspace (device memory of at least
 * nb_workspace_bytes() bytes, 256-byte aligned, owned by the caller). The state is
 * zero until nb_set_state. Returns NB_ERR_SPACE if the workspace is too small. */
nb_status nb_create(const nb_params *p, void *d_workspace, size_t bytes, nb_ctx **out);

/* Destroy a context (NULL is accepted). Waits for its stream. Does not free the
 * workspace. */
void nb_destroy(nb_ctx *ctx);

/* Message of the last error on this context ("" if none). Valid until the next call. */
const char *nb_last_error(const nb_ctx *ctx);

/* Bookkeeping (no passage of the method): state in and out of the workspace.
 * Load a state. m, x and v are required. a, j, s, c, a4n, a5n default to 0, tick to
 * tick0 for every body and level to 0 when NULL. If tick is NULL the state is
 * "synchronised at tick0" and nb_start may be called; a full state (tick and
 * level given) resumes a run exactly (checkpoint restore). Asynchronous. */
nb_status nb_set_state(nb_ctx *ctx, const nb_state *src, int64_t tick0);

/* Load only the time bookkeeping: every body's own time d_tick[n] (ticks) and step
 * level d_level[n] (device arrays); positions, velocities and derivatives are
 * kept. Used to re-arm a block schedule (for instance to make every body due at
 * the same time) without reloading the physical state. Asynchronous. */
nb_status nb_set_times(nb_ctx *ctx, const int64_t *d_tick, const int32_t *d_level);

/* Copy the state into the non-NULL fields of dst (device arrays). Waits. */
nb_status nb_get_state(nb_ctx *ctx, const nb_state *dst);

/* Passage: the start of the 6th-order Hermite scheme named in the paper's section
 * "Code implementation" (the paper gives no start rule; this is the initial-step rule
 * Delta0 = eta_init min(|a|/|j|, sqrt(|a|/|s|)) with power-of-two quantisation).
 * Hermite start-up on a synchronised state: two evaluations of every body (the
 * first gives a and j, the second s with the predicted accelerations set to the
 * first a), c = 0, then the initial-step rule for every body. Asynchronous; a
 * non-finite result (e.g. two bodies at one place with eps = 0) is reported by the
 * next waiting call as NB_ERR_NUMERIC. */
nb_status nb_start(nb_ctx *ctx);

/* Passage: the block time steps of the paper's section "Code implementation"
 * (individual power-of-two steps; Makino 1991). Split out of nb_timesteps so the
 * active list is a device array that the other calls take as they are.
 * Block-step selection: tick_next = min over bodies of (tick + step) and the
 * ascending list of bodies with tick + step == tick_next, written to d_idx_out
 * (capacity n). Returns the count in *h_n_act and the time in *h_tick_next. Waits. */
nb_status nb_active(nb_ctx *ctx, int32_t *d_idx_out, int64_t *h_n_act,
                    int64_t *h_tick_next);

/* Passage: the predictor of the 6th-order Hermite scheme (section "Code
 * implementation"; Nitadori & Makino 2008): x, v, a extrapolated by their Taylor
 * series up to the interpolated third derivative of a.
 * Predict every body to tick (>= every body's own time) with its Taylor series
 * up to the third derivative of a; the result feeds nb_evaluate. Asynchronous. */
nb_status nb_predict(nb_ctx *ctx, int64_t tick);

/* Copy the predicted positions, velocities and accelerations of the last
 * nb_predict into [3][n] device arrays (NULL skipped). Asynchronous. */
nb_status nb_get_predicted(nb_ctx *ctx, double *d_xp, double *d_vp, double *d_ap);

/* Passage: the O(N^2) force evaluation the paper's section "Performance results"
 * measures, in double precision for distances and accelerations or in the
 * extended-precision (float-float) variant of section "Code implementation"; the
 * pairwise acceleration, jerk and snap of the 6th-order Hermite scheme (Nitadori &
 * Makino 2008) with Plummer softening.
 * Acceleration, jerk, snap and potential of the n_act bodies d_idx against all
 * n predicted bodies (self pair excluded), in the precision chosen at
 * nb_create. In FP64, when every body is active (n_act = n >= 8192) and the
 * partial-sum buffer holds its partial sums (the default capacity does up to
 * n = 65536), each pair is computed once and added to both bodies (the terms are
 * antisymmetric in the pair apart from the masses); otherwise each active body sums
 * over all bodies. Both agree with the exact sums to FP64 rounding. The result is kept for nb_correct and, if d_out is not NULL, also
 * written to d_out[10][n_act]. n_act = 0 is a no-op. Asynchronous. */
nb_status nb_evaluate(nb_ctx *ctx, const int32_t *d_idx, int64_t n_act, double *d_out);

/* The evaluation extended by one derivative (FP64 in either precision): for the
 * active bodies idx, acceleration, jerk, snap, crackle and potential,
 *   C = m3 jj - 9 alpha S - 9 beta J - 3 gamma A,
 *   gamma = (3 v.a + r.jj) / R + alpha (3 beta - 4 alpha^2),
 * the time derivative of the snap term along the relative motion with jerk jj (the
 * derivative chain of the 6th-order Hermite scheme of the paper's section "Code
 * implementation", continued one order). The bodies' jerks are predicted to the
 * time of the last nb_predict (jp = j + h s + h^2/2 c). Output d_out[13][n_act]:
 * a(3), j(3), s(3), crackle(3), phi. Needs a prior nb_predict (NB_ERR_STATE);
 * idx as nb_evaluate. Does not feed nb_correct. Stream-ordered. */
nb_status nb_evaluate_crackle(nb_ctx *c, const int32_t *d_idx, int64_t n_act, double *d_out);

/* Size of the device memory nb_evaluate_static uses: a file-scope array that each
 * GPU the library runs on holds until the process ends. */
#define NB_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the evaluation of
 * nb_evaluate (FP64) without a context or workspace. It allocates nothing: its
 * j-records and partial sums live in the library's fixed device array of
 * NB_STATIC_SCRATCH_BYTES bytes.
 *   n bodies with masses d_m[n] and predicted positions, velocities and
 *   accelerations d_xp, d_vp, d_ap ([3][n] component-major, device); softening
 *   eps >= 0; the active bodies d_idx[n_act] (int32, device, each in [0, n)); the
 *   result d_out[10][n_act] (device; the layout of nb_evaluate's output).
 *   stream: hipStream_t, NULL = the null stream. Stream-ordered, returns without
 *   waiting; every kernel it enqueues is a plain kernel launch (no memset), so the
 *   call can be captured into a HIP graph.
 * It takes the one-sided evaluation kernels with the launch shapes of nb_evaluate
 * (default table and partial-sum capacity), so for n_act < n its result is bitwise
 * that of nb_evaluate on a context of n bodies; for n_act = n nb_evaluate may take
 * the pairwise-symmetric kernel instead, and the two agree to the FP64 rounding of
 * the sums.
 * Errors: NB_ERR_ARG for n outside [1, 2^30], n_act outside [0, n], eps < 0 or a
 * NULL pointer; NB_ERR_SPACE (nothing enqueued) when the j-records (80 n bytes)
 * plus the partial sums of the launch shape (80 S n_act bytes) do not fit the array;
 * NB_ERR_DEVICE for a HIP error. It cannot wait for the device, so an index outside
 * [0, n) is not returned as a status: every value of d_out is then NaN.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (two streams, or two host threads) race and give undefined results. */
nb_status nb_evaluate_static(int64_t n, const double *d_m, const double *d_xp, const double *d_vp,
                             const double *d_ap, double eps, const int32_t *d_idx, int64_t n_act,
                             double *d_out, void *stream);

/* Supply the evaluation of the bodies d_idx from outside instead of nb_evaluate:
 * d_in[10][n_act] (same layout as nb_evaluate's output) becomes the result that
 * the next nb_correct with the same d_idx and n_act uses. This is how partial sums
 * computed elsewhere (another device's share of the j-bodies, after a sum over
 * devices) enter the corrector. Asynchronous. */
nb_status nb_set_evaluation(nb_ctx *ctx, const int32_t *d_idx, int64_t n_act,
                            const double *d_in);

/* Launch shape of nb_evaluate, for tuning and tests: h_cfg = {ipl, waves per
 * workgroup, tile, j-splits S (>= 1)}. Three kernel families:
 *   - ipl = 1 or 2 active bodies per lane (each lane sweeps every record of its
 *     j-split, read from LDS as wave-wide broadcasts), (waves, tile) one of (1, 64),
 *     (1, 128), (2, 128), (1, 256), (2, 256), (4, 256) with tile the LDS tile in bodies;
 *   - FP64 only, for small active sets: ipl = -Pmax, Pmax a power of two <= 64: a wave
 *     holds P = min(Pmax, the power of two >= n_act) active bodies on 64 / P lanes
 *     each (lane w of a body takes records w, w + 64/P, ... of the split, and the
 *     lane sums are combined by a fixed butterfly); waves 1; tile 64 (LDS tiles of 64
 *     records) or 0 (records read straight from memory);
 *   - FP64 only, the group kernel: ipl = -Pmax with Pmax a power of two <= 128 and
 *     waves 4 or 8: every wave of a workgroup holds the same group of G = min(Pmax,
 *     the power of two >= n_act) active bodies (64 / G lanes each; G = 128: two per
 *     lane) and the waves share the split's records; tile 256 (LDS tiles; raises G to
 *     at least waves x 64 / 256) or 0 (records read straight from memory). When the
 *     last workgroup of a group can add the S partial sums cheaply (S x G x 10 at
 *     most 24 per thread), it does so in the same launch.
 * All zeros (or h_cfg NULL) returns to the launch table. The shape never changes
 * results beyond FP64 rounding of the split sums. Host-only; returns NB_ERR_ARG for an
 * unsupported combination. h_shape_out (may be NULL; 7 int32) receives the shape the
 * next call with n_act bodies will use: {ipl (for the small-set and group kernels:
 * -P or -G), waves, tile, jchunk, splits, iblocks (groups), fused (1: the splits are
 * added inside the evaluation launch)}; for the pairwise-symmetric kernel {0, waves,
 * 64, records per unit, claimed units and pieces, workgroups, 0}. */
nb_status nb_eval_config(nb_ctx *ctx, const int32_t *h_cfg, int64_t n_act,
                         int32_t *h_shape_out);

/* Launch-shape table of nb_evaluate, as produced by the tuner
 * (paper_1812_00367_amd/tune.py): nrows rows of five int32 {n_act_max, ipl, waves
 * per workgroup, tile, target waves}, n_act_max strictly increasing. A call with
 * n_act bodies uses the first row with n_act <= n_act_max (the last row also covers
 * larger sets); the target sets the j-split count S ~ target / (waves along the
 * active bodies). Supported shapes are those listed for nb_eval_config. nrows = 0
 * restores the built-in table. A forced shape from nb_eval_config takes precedence.
 * Host-only. */
nb_status nb_eval_table(nb_ctx *ctx, const int32_t *h_rows, int32_t nrows);

/* Passage: the corrector of the 6th-order Hermite scheme (section "Code
 * implementation"; Nitadori & Makino 2008), with the third to fifth derivatives of a
 * from the quintic through (a, j, s) at both ends of the step.
 * Hermite 6th-order corrector of the bodies of the last nb_evaluate (same d_idx,
 * n_act) to tick, using that evaluation. Updates x, v, a, j, s, c, a4n, a5n and
 * sets their time to tick. Asynchronous. The kernel checks that d_idx is strictly
 * ascending (a body listed twice would be corrected twice): otherwise the next
 * waiting call returns NB_ERR_ARG and the listed bodies' state is undefined. */
nb_status nb_correct(nb_ctx *ctx, const int32_t *d_idx, int64_t n_act, int64_t tick);

/* Passage: the block time steps of section "Code implementation": the generalised
 * Aarseth criterion of order 6, Delta = eta [(sqrt(|a||s|) + |j|) / (sqrt(|a3||a5|) +
 * |a4|)]^(1/3) (Nitadori & Makino 2008), quantised to powers of two with the block
 * rules of Makino 1991 and Aarseth 2003. The next active list is not returned here
 * but by nb_active.
 * New step levels of the bodies d_idx at their current time: the 6th-order
 * criterion and the block rules (init = 0), or the initial-step rule (init = 1).
 * Asynchronous; a body needing a step below dt_min is reported by the next
 * waiting call as NB_ERR_NUMERIC. */
nb_status nb_timesteps(nb_ctx *ctx, const int32_t *d_idx, int64_t n_act, int init);

/* Passage: one cycle of the block-step scheme of section "Code implementation".
 * One whole block step: nb_active, nb_predict, nb_evaluate, nb_correct and
 * nb_timesteps in order, with the active list kept in the workspace. Returns the
 * step's time and size. If tick_limit >= 0 and the next block time is beyond it,
 * nothing is done and *h_n_act is 0. Waits (after selecting the active set). */
nb_status nb_step(nb_ctx *ctx, int64_t tick_limit, int64_t *h_n_act, int64_t *h_tick_next);

/* Passage: the energy diagnostic of a direct N-body code (the paper reports no energy
 * error; this is the softened total energy used to check the integration).
 * Total energy at tick: every body is predicted to tick (this overwrites the
 * predicted state), then E_kin = sum m v^2 / 2 and
 * E_pot = -1/2 sum_i sum_{j != i} m_i m_j / sqrt(r^2 + eps^2). Waits. */
nb_status nb_energy(nb_ctx *ctx, int64_t tick, double *h_ekin, double *h_epot);

/* ------------------------------------------------------------ batches ----
 * Many independent systems ("jobs") of uneven size resident in one workspace and
 * advanced together (block steps as in the paper's section "Code implementation").
 * A batch step gives each job its own next block step (its own block time and
 * active set, as nb_step does for one system) with four kernel launches for all
 * jobs and no host work in between: active sets; prediction, with the work split
 * built beside it; one persistent evaluation over work items (job, i-tile of up to
 * 128 active bodies, j-chunk) of three item classes (two in split precision); and a
 * per-body pass that sums the partials in a fixed order, corrects and sets the new
 * levels. A
 * job's split depends only on its own (n, n_act) and the batch constants, so its
 * results are bitwise the same alone and in any mix of jobs.
 * Jobs are admitted into a fixed pool of bodies (first fit): nb_batch_add fails with
 * NB_ERR_SPACE when the pool or the job table has no room, which is the admission
 * control of a serving loop. Every call waits for the stream before it returns. */
typedef struct nb_batch nb_batch; /* opaque, library-owned host object */

typedef struct {
    int64_t capacity;      /* bodies in the pool, 1 <= capacity <= 2^30 */
    int32_t max_jobs;      /* job-table size, 1 <= max_jobs <= 65536 */
    int32_t precision;     /* nb_precision of the evaluation */
    double eps, eta, eta_init;        /* as in nb_params, shared by every job */
    int32_t dt_max_log2, dt_min_log2; /* as in nb_params */
    int32_t jchunk;        /* j-records per lane of a work item (multiple of 64; 0 = 64):
                              sets a job's j-chunks, S = ceil(n / (jchunk f min(W, 16)))
                              where W lanes share an active body (W = 64 / next power of two
                              >= n_act for n_act < 64, else 1) and f is the factor of the
                              job's item class below */
    int32_t items_per_job; /* at most this many work items per job and step come from
                              j-chunks (an upper bound on S i-tiles; 0 = 2048, <= 16384) */
    int32_t chunk_tile;    /* factor f of a job with 9 <= n_act < 128 (tile items; and of a
                              split-precision job with n_act >= 9): 0 = 2, <= 64 */
    int32_t chunk_wide;    /* factor f of an FP64 job with n_act >= 128 (wide items, 128
                              active bodies each): 0 = 4, <= 64 */
    int32_t chunk_direct;  /* factor f of a job with n_act <= 8 (direct items): 0 = 1, <= 64 */
    int64_t partial_slots; /* partial-sum buffer in (j-chunk x active body) units; raised to
                              the bound every step fits, 2 capacity + 128 (items_per_job + 1)
                              max_jobs; 0 = that bound */
    void *stream;          /* hipStream_t for every launch; NULL = the null stream */
} nb_batch_params;

/* Workspace bytes for a batch; NB_ERR_ARG for invalid parameters. No device use. */
nb_status nb_batch_workspace_bytes(const nb_batch_params *p, size_t *h_bytes);

/* Create a batch over d_workspace (caller-owned, 256-byte aligned, at least
 * nb_batch_workspace_bytes()). The library allocates no device memory; it keeps a
 * few small pinned host buffers for staging. */
nb_status nb_batch_create(const nb_batch_params *p, void *d_workspace, size_t bytes,
                          nb_batch **out);

/* Destroy a batch (NULL accepted). Waits for its stream. */
void nb_batch_destroy(nb_batch *b);

/* Message of the last error on this batch. */
const char *nb_batch_last_error(const nb_batch *b);

/* Admit a job of n bodies whose state is src (device arrays of this job's size,
 * as for nb_set_state; m, x, v required) and which runs until tick_end. Without
 * src->tick the job starts synchronised at tick0 and the Hermite start-up (two
 * evaluations and the initial-step rule, as nb_start) runs for it alone; with a
 * full state it resumes exactly. Writes the job id to *h_job. NB_ERR_SPACE (and
 * no change) when the pool has no free range of n bodies, the job table is full,
 * or one evaluation of this job would not fit the work buffers. */
nb_status nb_batch_add(nb_batch *b, int64_t n, const nb_state *src, int64_t tick0,
                       int64_t tick_end, int32_t *h_job);

/* Remove a job and free its bodies for later admissions. */
nb_status nb_batch_remove(nb_batch *b, int32_t job);

/* One block step of every job whose next block time is not beyond its tick_end.
 * Host outputs indexed by job id (arrays of max_jobs entries, each may be NULL):
 * the number of bodies the job advanced (0: finished, failed or not present), its
 * next block time (a finished or failed job keeps the last one computed), and its
 * error word (0 ok; 1 a non-finite start-up evaluation or corrector value;
 * 2 a body needs a step below dt_min; 3 an inconsistent time or level). A job with
 * a non-zero error word is not stepped again; the other jobs are unaffected.
 * *h_interactions = the sum over jobs of n_act x n. */
nb_status nb_batch_step(nb_batch *b, int64_t *h_n_act, int64_t *h_tick_next,
                        int32_t *h_job_err, int64_t *h_interactions);

/* `steps` batch steps enqueued back to back with no host work or wait in between,
 * then one wait. Outputs as nb_batch_step for the last step (a job that has finished
 * reports n_act 0); *h_interactions and *h_steps = interactions and batch steps in
 * which some job advanced, over the call. */
nb_status nb_batch_run(nb_batch *b, int32_t steps, int64_t *h_n_act, int64_t *h_tick_next,
                       int32_t *h_job_err, int64_t *h_interactions, int64_t *h_steps);

/* Copy a job's state into the non-NULL fields of dst (device arrays of the job's
 * size, layouts as nb_get_state). */
nb_status nb_batch_get(nb_batch *b, int32_t job, const nb_state *dst);

/* Energy of one job at tick (its bodies are predicted to tick first). */
nb_status nb_batch_energy(nb_batch *b, int32_t job, int64_t tick, double *h_ekin,
                          double *h_epot);

/* Pool offset and size of a job. Host-only. */
nb_status nb_batch_info(const nb_batch *b, int32_t job, int64_t *h_offset, int64_t *h_n);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
