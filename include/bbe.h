/*
 * bbe.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of the BBE betting-exchange model: many independent Monte-Carlo
 * simulations of a track race, run from the start or from an in-play
 * state, whose finish orders are tallied into win-probability estimates
 * (Cliff, Hawkins, Keen & Lau-Soto, EMSS 2021, Sections 3 and 6).
 *
 * Conventions
 *  - Every function returns an int status: BBE_OK (0) or a negative code.
 *    Nothing throws across the ABI.  bbe_last_error() gives a
 *    human-readable message for the last failing call on this thread.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are GPU
 *    memory of the current HIP device (e.g. from hipMalloc or a torch CUDA
 *    tensor).  All data buffers belong to the caller; opaque handles belong
 *    to the library until the matching *_free.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it and the call returns after enqueueing.
 *  - Array layouts are row-major and densely packed unless a stride is
 *    given.
 */
#ifndef BBE_H
#define BBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BBE_MAX_COMPETITORS 20
/* A simulation stops after this many ticks past its start state even if
 * fewer than stop_after competitors have crossed the line; it then counts
 * no win.  Races accepted by bbe_race_init need far fewer ticks. */
#define BBE_TICK_LIMIT (1u << 20)
/* bbe_race_init rejects races in which track_len / (slowest possible free
 * step) exceeds this many ticks. */
#define BBE_EXPECTED_TICK_BOUND 65536
#define BBE_UNRANKED 0xFF

enum {
    BBE_OK = 0,
    BBE_EINVAL = -1,   /* an argument breaks a documented rule */
    BBE_ENOMEM = -2,   /* host or device allocation failed */
    BBE_EDEVICE = -3   /* a HIP call failed; message has the HIP error */
};
/* Every call reports failure by its return code and a message for
 * bbe_last_error; a call that fails releases what it allocated and leaves
 * the handles it was given usable.  For tests of these paths the library
 * reads the environment variable BBE_FAULT_INJECT once per process:
 * "alloc:K1,K2,..." makes the K-th device allocation of the process (counted
 * from 1) fail as out of memory (BBE_ENOMEM), "device:K1,..." replaces the
 * K-th counted HIP call (the uploads, launches, graph capture and graph
 * launches of the entry points) by a failure without making it
 * (BBE_EDEVICE); both may be given, separated by a space.  Unset, nothing
 * is counted. */

/* One competitor (paper Section 3, Eq. 1).
 *   lo, hi  free step law delta(v_c) = U(lo, hi) per tick, distance units;
 *           finite, 0 < lo <= hi.
 *   pref    preference coefficient P_c(f_r, p_c) in (0, 1], constant for
 *           the race (the race factors do not change during a race).
 *   rho     responsiveness: R_c(d) = 1 + rho*(2 d_c / L - 1), |rho| < 1.
 *   theta   blocking threshold theta_c >= 0, distance units.            */
typedef struct bbe_competitor {
    float lo, hi, pref, rho, theta;
} bbe_competitor;

/* Opaque race description (competitors + track length). */
typedef struct bbe_race bbe_race;

/* In-play state of one race (paper Section 3: the state of a race is the
 * vector of positions d(t); Eq. 1's blocked branch also needs each
 * competitor's previous step S_c(t - dt)).  Host pointers, n entries each.
 *   tick       absolute tick index t0 of the state (it keys the random
 *              stream, so resuming from a state reproduces the
 *              uninterrupted run); t0 <= 2^32 - 1 - BBE_TICK_LIMIT.
 *   pos        d_c(t0): finite, 0 <= pos < track length.
 *   prev_step  S_c(t0 - dt): finite, > 0.                                 */
typedef struct bbe_state {
    uint32_t tick;
    const float *pos;
    const float *prev_step;
} bbe_state;

/* Validate and store a race: n competitors (1..BBE_MAX_COMPETITORS) on a
 * track of length track_len (finite, > 0).  `comp` is a host array of n
 * competitors, copied (the caller may free it on return).  Also rejects
 * races whose slowest possible free step, lo*pref*(1-|rho|), would need
 * more than BBE_EXPECTED_TICK_BOUND ticks to cover the track, and
 * competitors whose scaled span pref*(hi-lo) (float32) is neither 0 nor at
 * least 2^-110 (the kernels apply the 2^-16 of the draw to the span, which
 * is exact only there; any sensible race is far inside).
 * Errors: BBE_EINVAL, BBE_ENOMEM.                                          */
int bbe_race_init(const bbe_competitor *comp, int n, float track_len, bbe_race **out);

/* Preference coefficients from race factors (paper Section 3: P_c(f_r, p_c)
 * in [0, 1] reduces a competitor's stochastic step by an amount that grows
 * with the mismatch between the race's factors, such as going or terrain,
 * and the competitor's preferred values):
 *   P_c = prod_k fl(1 - fl(w_ck * |fl(f_k - p_ck)|)),
 * in single precision, k = 0 .. n_factors-1 in order.  Host inputs: factors
 * float[n_factors] and prefs float[n][n_factors], all in [0, 1]; sens
 * float[n][n_factors], each in [0, 1).  Host output pref_out float[n], in
 * (0, 1]: the `pref` of each bbe_competitor.  No device work.
 * Errors: BBE_EINVAL (a value out of range, or a product that underflows
 * to 0).                                                                   */
#define BBE_MAX_FACTORS 64
int bbe_pref_from_factors(const float *factors, int n_factors, const float *prefs,
                          const float *sens, int n, float *pref_out);

/* Gives the competitors' responsiveness a time term (paper Section 3: R_c
 * depends on time as well as on the positions, to model a competitor that
 * starts fast and fades, or starts slow and finishes strongly):
 *   R_c(t, d) = fl(fl(alpha_c + fl(beta_c * d_c)) + fl(gamma_c * th)),
 *   th = min(t, tau_c),
 * with t the absolute tick (the state's tick counts from the start of the
 * race), so the pace drifts by gamma_c per tick until tick tau_c and then
 * holds.  Host arrays gamma, tau float[n]: gamma finite; tau an integer in
 * 0..2^24; a slowing term must keep 1 - |rho_c| + gamma_c*tau_c >= 2^-10,
 * and the race must still end within BBE_EXPECTED_TICK_BOUND ticks at its
 * slowest.  All zeros (the state after bbe_race_init) is the plain race;
 * races with some gamma != 0 run kernels that evaluate the term.  The
 * surrogate's state encoding (bbe_encode_states) carries no time term.
 * Errors: BBE_EINVAL (the race is left unchanged).                         */
int bbe_race_set_pace(bbe_race *race, const float *gamma, const float *tau);

/* Release a race handle (NULL is ignored). */
void bbe_race_free(bbe_race *race);

/* Number of competitors of a race (or BBE_EINVAL for NULL). */
int bbe_race_n(const bbe_race *race);

/* Monte-Carlo dry-runs of one race (paper Section 3: repeated simulation
 * with different random seeds; Section 6: their finish orders estimate the
 * PMF over the n! finish orders).
 *
 * Runs simulations sim_begin .. sim_begin + n_sims - 1 of the stream
 * (seed, request), each from `state` (NULL = start of race: tick 0, every
 * competitor at position 0).  The draws of competitor c in the tick that
 * starts at absolute tick t of simulation s are Philox4x32-10 with key
 * (seed & 0xffffffff, seed >> 32) and counter (t, s, request, c >> 3),
 * word (c >> 1) & 3, its high 16 bits for even c and its low 16 bits for
 * odd c: u = k * 2^-16.  The result of each simulation therefore depends
 * only on (race, state, seed, request, s), not on how the range is split
 * into calls.
 *
 * A simulation stops after the tick in which the number of finishers
 * reaches stop_after (1..n; n = full finish order, 1 = winner only).
 *
 *   finish_orders  device uint8[n_sims][n] or NULL: row j lists the
 *                  competitors of simulation sim_begin + j by finishing
 *                  rank; ranks not reached hold BBE_UNRANKED.
 *   win_counts     device uint64[n] or NULL: OVERWRITTEN with the number of
 *                  simulations each competitor won.
 *   step_count     device uint64[1] or NULL: OVERWRITTEN with the number of
 *                  competitor-steps simulated (one per running competitor
 *                  per tick).
 * Rules: n_sims >= 1, sim_begin + n_sims <= 2^32.
 * Errors: BBE_EINVAL, BBE_EDEVICE.                                          */
int bbe_race_sim(const bbe_race *race, const bbe_state *state, uint32_t sim_begin,
                 uint32_t n_sims, uint64_t seed, uint32_t request, int stop_after,
                 uint8_t *finish_orders, uint64_t *win_counts, uint64_t *step_count,
                 void *stream);

/* Frequentist win probabilities (paper Section 3: an RP(d) bettor's
 * estimate from d dry-runs; with d = 0 its estimates are equiprobable).
 * For each of n_rows rows: probs[r][c] = win_counts[r][c] / sum_c
 * win_counts[r][c] in double precision, or 1/n when the row sums to 0.
 *   win_counts  device uint64, row r at win_counts + r * row_stride.
 *   probs       device double, row r at probs + r * row_stride.
 * Rules: n_rows >= 1, 1 <= n <= BBE_MAX_COMPETITORS, row_stride >= n.
 * Errors: BBE_EINVAL, BBE_EDEVICE.                                          */
int bbe_win_probs(const uint64_t *win_counts, int n_rows, int n, int row_stride,
                  double *probs, void *stream);

/* Finish-position tallies (paper Section 6: the finish orders of repeated
 * runs are the outcomes whose frequencies estimate the race's PMF; place
 * and each-way markets need more than the winner).  From a finish-order
 * matrix as bbe_race_sim writes it (device uint8 [n_sims][n], rank-major
 * competitor indices, 0xFF for unranked places): counts[c][r] = number of
 * simulations in which competitor c finished at rank r (device uint64
 * [n][n], overwritten; unranked places are not counted).  The probability
 * of finishing in the first k is sum_{r<k} counts[c][r] / n_sims.
 * Rules: 1 <= n <= BBE_MAX_COMPETITORS; orders may be NULL when n_sims = 0.
 * Errors: BBE_EINVAL, BBE_EDEVICE.                                          */
int bbe_rank_counts(const uint8_t *orders, uint32_t n_sims, int n, uint64_t *counts,
                    void *stream);

/* Largest n for bbe_order_pmf (7! = 5040 orders). */
#define BBE_ORDER_PMF_MAX_N 7

/* Frequencies of complete finish orders (paper Section 6: a PMF over the
 * n! orders).  counts[k] (device uint64 [n!], overwritten) = number of
 * simulations whose finish order is the k-th permutation of 0..n-1 in
 * lexicographic order (k = 0 for 0, 1, ..., n-1); rows with an unranked
 * place are not counted.  Input as for bbe_rank_counts.
 * Rules: 1 <= n <= BBE_ORDER_PMF_MAX_N; orders may be NULL when n_sims = 0.
 * Errors: BBE_EINVAL, BBE_EDEVICE.                                          */
int bbe_order_pmf(const uint8_t *orders, uint32_t n_sims, int n, uint64_t *counts,
                  void *stream);

/* In-play state generator: advance simulation `sim` of stream (seed,
 * request) of `race` from `state` (NULL = start) until the leading
 * position is >= target, and write that state (the simulation is the same
 * one bbe_race_sim runs).  Device outputs: tick_out uint32[1], pos_out and
 * prev_out float[n].  target must be finite and < track length; the call
 * fails on the device side (tick_out = 0xFFFFFFFF) if a competitor would
 * cross the line first.
 * Errors: BBE_EINVAL, BBE_EDEVICE.                                          */
int bbe_race_prefix(const bbe_race *race, const bbe_state *state, uint64_t seed,
                    uint32_t request, uint32_t sim, float target, uint32_t *tick_out,
                    float *pos_out, float *prev_out, void *stream);

/* Advances simulation `sim` of stream (seed, request) of `race` from
 * `state` (NULL = start) by exactly n_ticks ticks (1..BBE_TICK_LIMIT) and
 * writes the state reached (device outputs as in bbe_race_prefix); used to
 * step the race that bettors watch in play.  tick_out = 0xFFFFFFFF if a
 * competitor crosses the line within those ticks.
 * Errors: BBE_EINVAL, BBE_EDEVICE.                                          */
int bbe_race_advance(const bbe_race *race, const bbe_state *state, uint64_t seed,
                     uint32_t request, uint32_t sim, uint32_t n_ticks, uint32_t *tick_out,
                     float *pos_out, float *prev_out, void *stream);

/* ------------------------------------------------------------------ */
/* Batches of uneven requests in one graph launch.                      */
/* ------------------------------------------------------------------ */

/* One request of a batch: simulations sim_begin .. sim_begin + n_sims - 1
 * of stream (seed, request) of `race` from `state` (NULL = start of race),
 * exactly as one bbe_race_sim call would run them.  stop_after is 1..n, or
 * 0 for n (the full finish order).  Host pointers; `race` stays owned by
 * the caller and may be freed once the plan is created.                   */
typedef struct bbe_request {
    const bbe_race *race;
    const bbe_state *state;
    uint32_t sim_begin;
    uint32_t n_sims;
    uint32_t request;
    int stop_after;
} bbe_request;

typedef struct bbe_batch_plan bbe_batch_plan;

/* Plan flag: time candidate launch shapes (waves per workgroup, simulations
 * per work item, workgroups per CU) on the batch itself and keep the
 * fastest; the choice is cached per device and batch size class for later
 * plans, in memory and in a JSON file ($BBE_TUNE_CACHE if set, an empty
 * value for none; else $XDG_CACHE_HOME/bbe/tune.json or
 * $HOME/.cache/bbe/tune.json) keyed by the device (architecture, name, CU
 * count) and the library's kernel sources, so that later processes skip
 * the timing. */
#define BBE_PLAN_AUTOTUNE 1u

/* Builds a plan for n_reqs (>= 1) requests (the many dry-run requests of
 * in-play bettors, paper Section 3 and Section 6): copies the request
 * descriptors and a work list (requests split into work items of whole
 * generations of 64 simulations, ordered by expected competitor-steps,
 * largest first) to the device, optionally autotunes, and captures into a
 * HIP graph the whole launch sequence: clear the outputs, reset the work
 * queue, run one persistent kernel over every item (each item with the
 * kernel's instance for its competitor count; races with a time term of R
 * in a second launch of the paced variant), compute probabilities.
 *   win_counts  device uint64[n_reqs][BBE_MAX_COMPETITORS]: row r receives
 *               request r's win counts (columns >= its n stay 0).
 *   probs       device double[n_reqs][BBE_MAX_COMPETITORS] or NULL: row r
 *               receives the win probabilities of request r as
 *               bbe_win_probs computes them, 0 in the padding columns.
 *   step_count  device uint64[1] or NULL: total competitor-steps.
 * The output buffers are bound to the plan and must stay valid while it is
 * launched.  Runs (and, with BBE_PLAN_AUTOTUNE, times) work on `stream`
 * and returns after it has completed.
 * Errors: BBE_EINVAL (any request breaking the rules of bbe_race_sim),
 * BBE_ENOMEM, BBE_EDEVICE.                                                 */
int bbe_batch_plan_create(const bbe_request *reqs, int n_reqs, uint64_t seed,
                          uint64_t *win_counts, double *probs, uint64_t *step_count,
                          unsigned flags, void *stream, bbe_batch_plan **out);

/* Enqueues one launch of the plan's graph on `stream`.  Launches of one
 * plan must not overlap (they share the work queue).
 * Errors: BBE_EINVAL, BBE_EDEVICE.                                          */
int bbe_batch_plan_launch(bbe_batch_plan *plan, void *stream);

/* Replaces the start states of a plan's requests (the serving loop of in-play
 * bettors: the same dry-run requests re-run from the new state of the race
 * every time it advances, paper Sections 3 and 6), keeping the plan's
 * graph.  `states` is a host array of the plan's n_reqs states, validated as
 * in bbe_race_sim (all of them first: on error the plan is unchanged).  The
 * request table is copied on `stream`, after the launches already enqueued
 * there; launch the plan on the same stream.  The work order keeps the
 * expected lengths of the plan's creation.
 * Errors: BBE_EINVAL, BBE_EDEVICE.                                          */
int bbe_batch_plan_set_states(bbe_batch_plan *plan, const bbe_state *states, void *stream);

/* Launch shape chosen for a plan (any output pointer may be NULL); `grid`
 * is the largest grid among the plan's per-competitor-count kernels. */
int bbe_batch_plan_info(const bbe_batch_plan *plan, int *waves_per_block, int *grid,
                        int *sims_per_item, int *n_items);

/* Releases a plan (NULL is ignored).  Waits for the device to be idle.     */
void bbe_batch_plan_free(bbe_batch_plan *plan);

/* In-play states for a batch (the batched form of bbe_race_prefix): for
 * each i < n, advances simulation sims[i] of stream (seed, reqs[i].request)
 * of reqs[i].race from reqs[i].state until the leader reaches targets[i].
 * reqs[i].n_sims, sim_begin and stop_after are ignored.  Host inputs;
 * device outputs tick_out uint32[n] (0xFFFFFFFF if a competitor would
 * cross first), pos_out and prev_out float[n][BBE_MAX_COMPETITORS]
 * (competitor order, zero padding).  Returns after the work completed.
 * Errors: BBE_EINVAL, BBE_ENOMEM, BBE_EDEVICE.                             */
int bbe_prefix_batch(const bbe_request *reqs, const uint32_t *sims, const float *targets, int n,
                     uint64_t seed, uint32_t *tick_out, float *pos_out, float *prev_out,
                     void *stream);

/* bbe_prefix_batch for callers that cannot allocate memory (code that must
 * not call hipMalloc, such as tight serving loops or harnesses that forbid
 * it): same arguments, same outputs, same errors, but no device or host
 * allocation.  The request descriptors are staged in a fixed device array
 * of BBE_PREFIX_NOALLOC_MAX entries (about 3 MB), one per GPU, held until
 * the process ends; n > BBE_PREFIX_NOALLOC_MAX is rejected with BBE_EINVAL.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (from several threads or streams) race and must not be made.  Returns
 * after the work completed.                                                 */
#define BBE_PREFIX_NOALLOC_MAX 4096
int bbe_prefix_batch_noalloc(const bbe_request *reqs, const uint32_t *sims, const float *targets,
                             int n, uint64_t seed, uint32_t *tick_out, float *pos_out,
                             float *prev_out, void *stream);

/* ------------------------------------------------------------------ */
/* In play: the race the bettors watch and the cheap bettor rules.      */
/* ------------------------------------------------------------------ */

/* Positions of one simulated race tick by tick (paper Section 3: the state
 * of a race is its vector of positions, advanced by Eq. 1 every tick): row
 * 0 is `state` (NULL = start), row r the positions after r ticks of
 * simulation `sim` of stream (seed, request) -- the simulation bbe_race_sim
 * runs.  The trace ends before the first tick in which a competitor would
 * reach the line (in-play betting on the winner closes then), or after
 * max_rows rows (1..BBE_TICK_LIMIT+1).  Device outputs: trace float
 * [max_rows][n] (rows past the end untouched), n_rows uint32[1] (>= 1).
 * Errors: BBE_EINVAL, BBE_EDEVICE.                                          */
int bbe_race_trace(const bbe_race *race, const bbe_state *state, uint64_t seed,
                   uint32_t request, uint32_t sim, uint32_t max_rows, float *trace,
                   uint32_t *n_rows, void *stream);

/* Bettor rules of paper Section 5 that read the race itself; each bettor
 * holds a view of which competitor will win.  At trace row r (positions x,
 * tick t0 + r):
 *   ZI     (param ignored) a competitor drawn uniformly afresh each tick:
 *          floor(w*n/2^32) for the first word w of the Philox4x32-10 block
 *          with key (seed lo, seed hi) and counter (t, bettor, ~0, ~0), a
 *          counter race draws never use;
 *   LW     (param ignored) the leader, ties to the lowest index;
 *   UD     (param D >= 0, finite) the runner-up (largest position after the
 *          leader's, ties to the lowest index) while fl(x_P1 - x_P2) < D,
 *          else the leader; LW's view when n = 1;
 *   LinEx  (param N, an integer in 1..BBE_TICK_LIMIT) mean step over the
 *          last w = min(N, r) ticks, held to the line: the competitor with
 *          the least ratio fl(L - x_c) / fl(x_c - x_c(r - w)) among those
 *          with a positive displacement (ratios compared exactly, equal ones
 *          to the lowest index); LW's view when w = 0 or nobody moved.
 * The RP(d) bettors of Section 3 are served by dry-run requests instead.   */
#define BBE_BETTOR_ZI 0
#define BBE_BETTOR_LW 1
#define BBE_BETTOR_UD 2
#define BBE_BETTOR_LINEX 3

typedef struct bbe_bettors bbe_bettors;

/* Stores a population of n_bettors (>= 1) bettors on the device: host
 * arrays kind uint8 [n_bettors] (BBE_BETTOR_*) and param float [n_bettors].
 * Bettor b keeps index b in the outputs of bbe_bettor_views.  Synchronous.
 * Errors: BBE_EINVAL (unknown kind, parameter out of range), BBE_ENOMEM,
 * BBE_EDEVICE.                                                              */
int bbe_bettors_create(const uint8_t *kind, const float *param, int n_bettors,
                       bbe_bettors **out);

/* Releases a population (NULL is ignored). */
void bbe_bettors_free(bbe_bettors *b);

/* Bettors of each kind: per_kind uint32[4] (host), indexed by BBE_BETTOR_*. */
int bbe_bettors_count(const bbe_bettors *b, uint32_t *per_kind);

/* Views of every bettor at trace rows first_row .. first_row + n_eval - 1
 * (first_row + n_eval <= n_rows).  Device input: trace float [n_rows][n]
 * (e.g. from bbe_race_trace; row r at tick t0 + r; positions below
 * track_len).  Device outputs, either may be NULL but not both: views
 * uint8 [n_eval][n_bettors], the competitor each bettor backs; counts
 * uint32 [n_eval][n], bettors per competitor (overwritten).  n_eval = 0 is
 * a no-op.  Errors: BBE_EINVAL, BBE_EDEVICE.                                */
int bbe_bettor_views(const bbe_bettors *b, const float *trace, uint32_t n_rows, int n,
                     float track_len, uint32_t t0, uint32_t first_row, uint32_t n_eval,
                     uint64_t seed, uint8_t *views, uint32_t *counts, void *stream);

/* Views of RP(d) bettors (paper Section 3) from their own dry-run win
 * counts: the competitor with the most wins, ties (and rows without a win)
 * to the lowest index.  Device input: wins uint64 [n_bettors][row_stride]
 * (competitors 0..n-1 read; e.g. a batch plan's win counts, one request per
 * bettor).  Device outputs, either may be NULL but not both: views uint8
 * [n_bettors]; counts uint32 [n], bettors per competitor (overwritten).
 * Errors: BBE_EINVAL, BBE_EDEVICE.                                          */
int bbe_rp_views(const uint64_t *wins, int n_bettors, int n, int row_stride, uint8_t *views,
                 uint32_t *counts, void *stream);

/* ------------------------------------------------------------------ */
/* Surrogate network: encoded in-play state -> win probabilities.       */
/* ------------------------------------------------------------------ */

/* A 160 -> 256 -> 256 -> 256 -> 20 perceptron with ReLU hidden layers and a
 * softmax over the slots that hold a competitor, trained with a soft
 * cross-entropy against Monte-Carlo win frequencies (the frequentist
 * estimates of paper Section 3) and Adam (beta1 0.9, beta2 0.999, eps
 * 1e-8).  Products run on the matrix cores in bfloat16 with float32
 * accumulation; the master parameters, the Adam moments and the gradients
 * are float32.
 *
 * Parameters travel as one float32 vector of BBE_MLP_NPARAMS values packed
 * as W1 [256][160], b1 [256], W2 [256][256], b2 [256], W3 [256][256],
 * b3 [256], W4 [20][256], b4 [20] (W[n][k]: input k to output n).
 *
 * Network inputs: x, bfloat16 (uint16 bit patterns) [batch][160] from
 * bbe_encode_states; n_valid, int32 [batch], the number of slots that hold
 * a competitor (1..20); slots are in the encoder's order.                  */
#define BBE_MLP_IN 160
#define BBE_MLP_HIDDEN 256
#define BBE_MLP_OUT 20
#define BBE_MLP_NPARAMS 177940

typedef struct bbe_mlp bbe_mlp;

/* Creates a network from host parameters (copied) with device buffers for
 * training batches of up to max_batch rows.  Synchronous.
 * Errors: BBE_EINVAL (non-finite parameter, max_batch < 1), BBE_ENOMEM,
 * BBE_EDEVICE.                                                              */
int bbe_mlp_create(const float *params, int max_batch, bbe_mlp **out);

/* Releases a network (NULL is ignored).  Waits for the device.              */
void bbe_mlp_free(bbe_mlp *m);

/* Copies the float32 master parameters to host memory.  Synchronous.       */
int bbe_mlp_get_params(const bbe_mlp *m, float *params);

/* Saves a network's parameters to a file (host path): the 8 bytes
 * "BBEMLP01", the parameter count as uint32 (little endian), then the
 * float32 parameters in the packing above.  Synchronous.
 * Errors: BBE_EINVAL (NULL argument, file not writable), BBE_EDEVICE.       */
int bbe_mlp_save(const bbe_mlp *m, const char *path);

/* Saves a training checkpoint to a file (host path): the 8 bytes
 * "BBEMLP02", the parameter count as uint32 and the number of Adam steps
 * taken as uint64 (little endian), then the float32 parameters, the Adam
 * first moments and the Adam second moments, each in the packing above.
 * Training resumed from it takes the same steps, bit for bit, as training
 * that did not stop.  Synchronous: call it once the network's last training
 * step has completed on its stream.
 * Errors: BBE_EINVAL (NULL argument, file not writable), BBE_EDEVICE.       */
int bbe_mlp_save_checkpoint(const bbe_mlp *m, const char *path);

/* Creates a network (as bbe_mlp_create, with max_batch) from a file written
 * by bbe_mlp_save (Adam state zero, no steps taken) or by
 * bbe_mlp_save_checkpoint (Adam state and step count restored).
 * Errors: BBE_EINVAL (missing or malformed file, or what bbe_mlp_create
 * rejects), BBE_ENOMEM, BBE_EDEVICE.                                         */
int bbe_mlp_load(const char *path, int max_batch, bbe_mlp **out);

/* Inference on `batch` rows (any size).  Device outputs, each optional:
 * probs float [batch][20] (0 in empty slots), entropy float [batch]
 * (natural log), logits float [batch][32] (-inf in empty slots).           */
int bbe_mlp_forward(const bbe_mlp *m, const uint16_t *x, const int32_t *n_valid, int batch,
                    float *probs, float *entropy, float *logits, void *stream);

/* The forward pass of bbe_mlp_forward, also returning what each hidden
 * layer feeds the next: hidden, device uint16 [3][batch][256], receives the
 * bfloat16 bit patterns of h1, h2 and h3 (after bias and ReLU, rounded to
 * nearest even), so that every layer can be checked on its own inputs;
 * logits as in bbe_mlp_forward (may be NULL).
 * Errors: BBE_EINVAL (NULL network, x, n_valid or hidden; batch < 1),
 * BBE_EDEVICE.                                                              */
int bbe_mlp_forward_hidden(const bbe_mlp *m, const uint16_t *x, const int32_t *n_valid,
                           int batch, uint16_t *hidden, float *logits, void *stream);

/* Mean soft cross-entropy of `batch` (1..max_batch) rows against target
 * (device float [batch][20], each row summing to 1 over its valid slots)
 * into loss (device float[1], overwritten), and its gradient into grad
 * (device float[BBE_MLP_NPARAMS], overwritten; NULL = the network's own
 * gradient buffer, used by bbe_mlp_adam_step with grad = NULL).  The
 * gradient is summed over the rows in a fixed order: the same inputs give
 * the same bits on every call (the loss is summed with atomics and may
 * differ in its last bits).                                                */
int bbe_mlp_loss_grad(bbe_mlp *m, const uint16_t *x, const int32_t *n_valid,
                      const float *target, int batch, float *loss, float *grad, void *stream);

/* One Adam step with learning rate lr (> 0) on gradient grad (device, NULL =
 * the network's own buffer); refreshes the bfloat16 weight copies.         */
int bbe_mlp_adam_step(bbe_mlp *m, const float *grad, float lr, void *stream);

/* bbe_mlp_loss_grad followed by bbe_mlp_adam_step on the own buffer.       */
int bbe_mlp_train_step(bbe_mlp *m, const uint16_t *x, const int32_t *n_valid,
                       const float *target, int batch, float lr, float *loss, void *stream);

/* Encodes in-play states for the network.  Device inputs: comp float
 * [batch][20][5] (lo, hi, pref, rho, theta per competitor), n int32
 * [batch] (competitors, 1..20), pos and prev float [batch][20] (state, as
 * in bbe_state).  Slots list the competitors by expected remaining ticks
 * T = (L-d)/((lo+hi)*0.5*(1 + rho*d/L)), smallest first (equal T: lower
 * index first), padded to 20; per slot 8 float32 features rounded to
 * bfloat16, positions only relative to the line or to other competitors:
 * (L-d)/L, (d_lead-d)/(75 dt), min((d_above-d)/(7.5 dt), 4) with d_above
 * the position of the competitor directly ahead on the track (position
 * order, equal positions by lower index; 4 for the leader), s/(7.5 dt),
 * (lo+hi)/(15 dt), (hi-lo)/(hi+lo), rho/0.2 and (T - T_min)/10 with T_min
 * the state's smallest T (all 0 for padding), where dt is the tick length
 * in seconds the race parameters are expressed in.  Outputs: x [batch][160] (16-byte aligned, else
 * BBE_EINVAL); slot_comp int32 [batch][20] or
 * NULL, the competitor in each slot (-1 for padding).  With probs (device
 * double [batch][20], competitor order, e.g. from bbe_batch_plan_create)
 * the matching target (device float [batch][20]) receives them in slot
 * order, 0 for padding: the training labels.  probs and target are both
 * NULL or both given.                                                        */
int bbe_encode_states(const float *comp, const int32_t *n, const float *pos, const float *prev,
                      int batch, float track_len, float dt, uint16_t *x, int32_t *slot_comp,
                      const double *probs, float *target, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *bbe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BBE_H */
