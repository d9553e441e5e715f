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
 * more than BBE_EXPECTED_TICK_BOUND ticks to cover the track.
 * Errors: BBE_EINVAL, BBE_ENOMEM.                                          */
int bbe_race_init(const bbe_competitor *comp, int n, float track_len, bbe_race **out);

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
 * (seed & 0xffffffff, seed >> 32) and counter (t, s, request, c >> 2),
 * word c & 3.  The result of each simulation therefore depends only on
 * (race, state, seed, request, s), not on how the range is split into
 * calls.
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

/* Message of the last failing call on this thread ("" if none). */
const char *bbe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BBE_H */
