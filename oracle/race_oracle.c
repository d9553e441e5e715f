/*
 * race_oracle.c -- plain, slow, obviously-correct CPU oracle of the BBE
 * track-race model (Cliff, Hawkins, Keen & Lau-Soto, "Implementing the BBE
 * Agent-Based Model of a Sports-Betting Exchange", EMSS 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * source, header or constant table with the GPU library: every formula here
 * is written out again from the paper and from the published Philox
 * definition.
 *
 * What is computed (paper Section 3 and Eq. 1):
 *   - a race is n competitors on a 1-D track of length L; the state is the
 *     vector of positions d(t) (Section 3 takes it as the race's state);
 *   - each tick every running competitor advances by S_c(t) > 0 computed from
 *     the start-of-tick state (Section 3, d_c(t+dt) = d_c(t) + S_c(t));
 *   - S_c follows Eq. 1: R_c * P_c * delta(v_c) when the nearest competitor
 *     strictly ahead is farther than theta_c, else R_c * delta_min, where
 *     delta_min is the smaller of the previous steps of c and of that
 *     competitor (text right after Eq. 1);
 *   - a competitor finishes when d_c >= L (Section 3, race end rule);
 *   - repeated seeded runs give finish orders, tallied into frequentist win
 *     probabilities (Section 3 on RP(d) bettors; Section 6 on the PMF over
 *     the n! finish orders).
 *
 * Readings of points the paper leaves open (each is listed with its reason
 * in the design notes of the repository):
 *   delta(v_c) = U(lo, hi); P_c is a per-race constant folded into the
 *   bounds: P_c*U(lo,hi) = U(P_c*lo, P_c*hi), evaluated as
 *   elo + espan*u with elo = fl(P*lo), espan = fl(P*fl(hi-lo)).
 *   R_c(d) = 1 + rho_c*(2 d_c/L - 1) = alpha_c + beta_c*d_c with
 *   alpha_c = fl(1-rho_c), beta_c = fl(2 rho_c / L), evaluated on the
 *   competitor's own start-of-tick position; R_c may also depend on time
 *   (Section 3 writes R_c(t, d)): R = fl(fl(alpha + fl(beta*d)) +
 *   fl(gamma*th)) with th = min(t, tau) for the absolute tick t, so the
 *   pace drifts by gamma per tick until tick tau and then holds.  gamma = 0
 *   (the default) adds +0 and leaves R unchanged.
 *   The nearest competitor ahead is the running competitor i != c with the
 *   smallest position d_i > d_c, the lowest index among equal positions;
 *   the gap is fl(d_i - d_c).  Nobody ahead means an infinite gap.
 *   Blocked iff gap <= theta_c.
 *   Competitors that crossed the line in an earlier tick are no longer
 *   running: they take no step and block nobody.
 *   Same-tick finishers are ordered by the crossing fraction
 *   fl((L - d_old)/S), then by index.  A simulation stops after the tick in
 *   which the number of finishers reaches stop_after (every competitor that
 *   crossed during that tick is ranked).
 *   Draws: Philox4x32-10 with key (seed_lo, seed_hi) and counter
 *   (t, sim, request, c>>3); word w = out[(c>>1)&3]; its high half
 *   k = w >> 16 for even c, its low half k = w & 0xffff for odd c;
 *   u = k * 2^-16.
 *
 * All single-precision arithmetic is written one rounding per operation and
 * must be compiled with -ffp-contract=off (no fused multiply-add).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_N 20
#define ORC_TICK_LIMIT (1u << 20)      /* hard stop, ticks after t0 */
#define ORC_EXPECTED_TICK_BOUND 65536.0 /* validation bound on L / min step */

enum { ORC_OK = 0, ORC_EINVAL = -1 };

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, "Parallel random
 * numbers: as easy as 1, 2, 3").  Round: two 32x32->64 products of the
 * even counter words with the two multipliers; the high halves are xored
 * with the odd words and the round key; the key is bumped by the two
 * Weyl constants between rounds.                                        */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The uniform draw of competitor c at tick t of simulation `sim`: one
 * 16-bit half of a Philox word, so one Philox block serves 8 competitors.
 * 16 bits resolve the free step (elo + espan*u) to espan/65536, about the
 * spacing of float32 positions near the finish of a 2000-unit track.
 * levels == 0: the full 16-bit draw.  levels == K (a power of two): the
 * draw truncated to K equally spaced levels {0, 1/K, ..., (K-1)/K}; used
 * only by the tests that compare against exact enumeration.             */
static float draw_u(uint64_t seed, uint32_t t, uint32_t sim, uint32_t request,
                    int c, uint32_t levels)
{
    uint32_t ctr[4] = { t, sim, request, (uint32_t)c >> 3 };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    uint32_t w = out[(c >> 1) & 3];
    uint32_t m = (c & 1) ? (w & 0xffffu) : (w >> 16);   /* 16 bits */
    if (levels == 0)
        return (float)m * 0x1p-16f;
    int lg = 0;
    while ((1u << lg) < levels) ++lg;
    return (float)(m >> (16 - lg)) / (float)levels;
}

/* ------------------------------------------------------------------ */
/* Race description with the derived per-competitor constants.         */
/* ------------------------------------------------------------------ */
typedef struct {
    int n;
    float L;
    float elo[ORC_MAX_N], espan[ORC_MAX_N];
    float alpha[ORC_MAX_N], beta[ORC_MAX_N];
    float theta[ORC_MAX_N];
    float gamma[ORC_MAX_N], tau[ORC_MAX_N];
} orc_race;

/* comp is [n][7] = {lo, hi, pref, rho, theta, gamma, tau} per competitor;
 * gamma and tau give R_c its dependence on time (below).                */
static int race_setup(int n, float L, const float *comp, orc_race *r)
{
    if (n < 1 || n > ORC_MAX_N) return ORC_EINVAL;
    if (!isfinite(L) || !(L > 0.0f)) return ORC_EINVAL;
    if (!comp) return ORC_EINVAL;
    r->n = n;
    r->L = L;
    for (int c = 0; c < n; ++c) {
        const float *q = comp + 7 * c;
        float lo = q[0], hi = q[1], pref = q[2], rho = q[3], theta = q[4];
        float gamma = q[5], tau = q[6];
        if (!isfinite(lo) || !isfinite(hi) || !isfinite(pref) || !isfinite(rho) ||
            !isfinite(theta) || !isfinite(gamma) || !isfinite(tau))
            return ORC_EINVAL;
        if (!(tau >= 0.0f) || tau > 16777216.0f || tau != floorf(tau)) return ORC_EINVAL;
        if (!(lo > 0.0f) || !(hi >= lo)) return ORC_EINVAL;
        if (!(pref > 0.0f) || !(pref <= 1.0f)) return ORC_EINVAL;
        if (!(fabsf(rho) < 1.0f)) return ORC_EINVAL;
        if (!(theta >= 0.0f)) return ORC_EINVAL;
        float span = hi - lo;
        r->elo[c] = pref * lo;
        r->espan[c] = pref * span;
        r->alpha[c] = 1.0f - rho;
        r->beta[c] = (2.0f * rho) / L;
        r->theta[c] = theta;
        r->gamma[c] = gamma;
        r->tau[c] = tau;
        /* S > 0 keeps the race finite: R is at least 1 - |rho| + min(0,
         * gamma*tau) over d in [0, L) and all t; a slowing time term must
         * leave it at least 2^-10.  Bound how long the race can take.     */
        double slow = (double)gamma * (double)tau;
        double r_min = 1.0 - fabs((double)rho) + (slow < 0.0 ? slow : 0.0);
        if (slow < 0.0 && !(r_min >= 0x1p-10)) return ORC_EINVAL;
        double min_step = (double)r->elo[c] * r_min;
        if (!(min_step > 0.0) || (double)L / min_step > ORC_EXPECTED_TICK_BOUND)
            return ORC_EINVAL;
    }
    return ORC_OK;
}

static int state_check(const orc_race *r, uint32_t t0, const float *pos, const float *prev)
{
    if (t0 > 0xFFFFFFFFu - ORC_TICK_LIMIT) return ORC_EINVAL;
    if (!pos) return ORC_OK; /* start of race */
    for (int c = 0; c < r->n; ++c) {
        if (!isfinite(pos[c]) || pos[c] < 0.0f || !(pos[c] < r->L)) return ORC_EINVAL;
        if (!prev || !isfinite(prev[c]) || !(prev[c] > 0.0f)) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Eq. 1 for every running competitor, from the start-of-tick state     */
/* (d, s).  The draw source is explicit `draws` (one row of n, for this */
/* tick) when non-NULL, else Philox at absolute tick t.  `used`         */
/* (optional) marks which draws were consumed.                          */
/* ------------------------------------------------------------------ */
static void tick_steps(const orc_race *r, const float *d, const float *s, const int *running,
                       uint32_t t, uint64_t seed, uint32_t request, uint32_t sim,
                       uint32_t levels, const float *draws, uint8_t *used, float *S)
{
    const int n = r->n;
    for (int c = 0; c < n; ++c) {
        if (!running[c]) continue;
        /* nearest running competitor strictly ahead: the smallest position
         * greater than d_c, the lowest index among equal positions */
        int ahead = -1;
        for (int i = 0; i < n; ++i) {
            if (i == c || !running[i]) continue;
            if (d[i] > d[c] && (ahead < 0 || d[i] < d[ahead])) ahead = i;
        }
        float gap = ahead >= 0 ? d[ahead] - d[c] : INFINITY;
        float s_ahead = ahead >= 0 ? s[ahead] : 0.0f;
        /* R_c(t, d) = alpha + beta*d_c + gamma*min(t, tau): the own-position
         * term, plus a time term frozen after tick tau (zero when gamma = 0) */
        float th = fminf((float)t, r->tau[c]);
        float R = (r->alpha[c] + r->beta[c] * d[c]) + r->gamma[c] * th;
        if (gap > r->theta[c]) {
            float u;
            if (draws) {
                u = draws[c];
                if (used) used[c] = 1;
            } else {
                u = draw_u(seed, t, sim, request, c, levels);
            }
            float x = r->elo[c] + r->espan[c] * u;
            S[c] = R * x;
        } else {
            float dmin = fminf(s[c], s_ahead);
            S[c] = R * dmin;
        }
    }
}

/* ------------------------------------------------------------------ */
/* One simulated race.                                                  */
/* Draw source: explicit `draws` ([max_ticks][n], relative tick) when   */
/* non-NULL, else Philox.  `used` (optional, [max_ticks][n]) marks the  */
/* draws the path consumed; `trace` (optional, [max_ticks][n]) receives */
/* the positions after every tick.  Returns the number of ranked        */
/* finishers, or -1 when explicit draws ran out.                        */
/* ------------------------------------------------------------------ */
static int simulate(const orc_race *r, uint32_t t0, const float *pos0, const float *prev0,
                    uint64_t seed, uint32_t request, uint32_t sim, int stop_after,
                    uint32_t levels, const float *draws, int max_ticks, uint8_t *used,
                    float *trace, uint8_t *order, uint64_t *steps_out)
{
    const int n = r->n;
    float d[ORC_MAX_N], s[ORC_MAX_N], S[ORC_MAX_N], frac[ORC_MAX_N];
    int running[ORC_MAX_N], crossed[ORC_MAX_N];
    int nfin = 0;
    uint64_t steps = 0;
    uint32_t t = t0;

    for (int c = 0; c < n; ++c) {
        d[c] = pos0 ? pos0[c] : 0.0f;
        s[c] = prev0 ? prev0[c] : 0.0f;
        running[c] = 1;
        order[c] = 0xFF;
    }

    while (nfin < stop_after) {
        uint32_t rel = t - t0;
        if (rel >= ORC_TICK_LIMIT) break;
        if (draws && (int)rel >= max_ticks) return -1;

        /* Eq. 1 for every running competitor, from the start-of-tick state. */
        tick_steps(r, d, s, running, t, seed, request, sim, levels,
                   draws ? draws + (size_t)rel * n : NULL,
                   used ? used + (size_t)rel * n : NULL, S);

        /* Synchronous update; detect crossings of the finish line. */
        int ncross = 0;
        for (int c = 0; c < n; ++c) {
            crossed[c] = 0;
            if (!running[c]) continue;
            float dn = d[c] + S[c];
            if (dn >= r->L) {
                crossed[c] = 1;
                frac[c] = (r->L - d[c]) / S[c];
                ++ncross;
            }
            d[c] = dn;
            s[c] = S[c];
            ++steps;
        }

        if (trace)
            for (int c = 0; c < n; ++c) trace[(size_t)rel * n + c] = d[c];

        /* Rank this tick's finishers by (fraction, index). */
        while (ncross > 0) {
            int best = -1;
            for (int c = 0; c < n; ++c) {
                if (!crossed[c]) continue;
                if (best < 0 || frac[c] < frac[best]) best = c;
            }
            order[nfin++] = (uint8_t)best;
            crossed[best] = 0;
            running[best] = 0;
            --ncross;
        }
        ++t;
    }
    if (steps_out) *steps_out = steps;
    return nfin;
}

/* ------------------------------------------------------------------ */
/* Exported entry points (host pointers).                               */
/* ------------------------------------------------------------------ */

/* Monte-Carlo: sims [sim_begin, sim_begin+n_sims).  orders [n_sims][n]
 * (0xFF = unranked) or NULL; wins [n] overwritten, or NULL; steps: total
 * competitor-steps, or NULL.  threads > 1 splits the sims over OpenMP
 * threads (results do not depend on it).                                */
int orc_race_sim(int n, float L, const float *comp, uint32_t t0, const float *pos,
                 const float *prev, uint32_t sim_begin, uint32_t n_sims, uint64_t seed,
                 uint32_t request, int stop_after, uint32_t levels, uint8_t *orders,
                 uint64_t *wins, uint64_t *steps, int threads)
{
    orc_race r;
    if (race_setup(n, L, comp, &r) != ORC_OK) return ORC_EINVAL;
    if (!pos) t0 = 0;
    if (state_check(&r, t0, pos, prev) != ORC_OK) return ORC_EINVAL;
    if (n_sims == 0 || (uint64_t)sim_begin + n_sims > 0x100000000ull) return ORC_EINVAL;
    if (stop_after < 1 || stop_after > n) return ORC_EINVAL;
    if (levels != 0 && (levels > (1u << 16) || (levels & (levels - 1)) != 0)) return ORC_EINVAL;
    if (threads < 1) threads = 1;

    uint64_t w[ORC_MAX_N];
    memset(w, 0, sizeof w);
    uint64_t total = 0;

#pragma omp parallel for num_threads(threads) schedule(dynamic, 64) reduction(+ : w[:ORC_MAX_N], total)
    for (int64_t j = 0; j < (int64_t)n_sims; ++j) {
        uint8_t ord[ORC_MAX_N];
        uint64_t st = 0;
        int nf = simulate(&r, t0, pos, prev, seed, request, sim_begin + (uint32_t)j,
                          stop_after, levels, NULL, 0, NULL, NULL, ord, &st);
        if (nf > 0) w[ord[0]] += 1;
        total += st;
        if (orders) memcpy(orders + (size_t)j * n, ord, (size_t)n);
    }
    if (wins)
        for (int c = 0; c < n; ++c) wins[c] = w[c];
    if (steps) *steps = total;
    return ORC_OK;
}

/* The same race driven by explicit draws: n_seq sequences, each
 * [max_ticks][n] draws indexed by (tick - t0, competitor).  orders
 * [n_seq][n]; used (optional) [n_seq][max_ticks][n] marks consumed draws;
 * trace (optional) [n_seq][max_ticks][n] receives positions after each
 * tick (untouched past the end of a race).
 * Returns ORC_EINVAL if a sequence needs more than max_ticks ticks.      */
int orc_race_draws(int n, float L, const float *comp, uint32_t t0, const float *pos,
                   const float *prev, int stop_after, int n_seq, int max_ticks,
                   const float *draws, uint8_t *orders, uint8_t *used, float *trace)
{
    orc_race r;
    if (race_setup(n, L, comp, &r) != ORC_OK) return ORC_EINVAL;
    if (!pos) t0 = 0;
    if (state_check(&r, t0, pos, prev) != ORC_OK) return ORC_EINVAL;
    if (stop_after < 1 || stop_after > n || n_seq < 0 || max_ticks < 1 || !draws || !orders)
        return ORC_EINVAL;
    for (int q = 0; q < n_seq; ++q) {
        const float *dq = draws + (size_t)q * max_ticks * n;
        uint8_t *uq = used ? used + (size_t)q * max_ticks * n : NULL;
        if (uq) memset(uq, 0, (size_t)max_ticks * n);
        float *tq = trace ? trace + (size_t)q * max_ticks * n : NULL;
        int nf = simulate(&r, t0, pos, prev, 0, 0, 0, stop_after, 0, dq, max_ticks, uq, tq,
                          orders + (size_t)q * n, NULL);
        if (nf < 0) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* In-play state generator: advance simulation `sim` of `request` from the
 * given state (pos == NULL: start of race) tick by tick until the leading
 * position is >= target, and return that state (tick, positions, previous
 * steps).  Nobody may cross the line before that (ORC_EINVAL otherwise).
 * With target <= the current leading position the input state is
 * returned unchanged.                                                    */
int orc_race_prefix(int n, float L, const float *comp, uint32_t t0, const float *pos,
                    const float *prev, uint64_t seed, uint32_t request, uint32_t sim,
                    float target, uint32_t *t_out, float *pos_out, float *prev_out)
{
    orc_race r;
    if (race_setup(n, L, comp, &r) != ORC_OK) return ORC_EINVAL;
    if (!pos) t0 = 0;
    if (state_check(&r, t0, pos, prev) != ORC_OK) return ORC_EINVAL;
    if (!isfinite(target) || !(target < L) || !t_out || !pos_out || !prev_out)
        return ORC_EINVAL;

    float d[ORC_MAX_N], s[ORC_MAX_N], S[ORC_MAX_N];
    int all_running[ORC_MAX_N];
    for (int c = 0; c < n; ++c) {
        d[c] = pos ? pos[c] : 0.0f;
        s[c] = pos ? prev[c] : 0.0f;
        all_running[c] = 1;
    }
    uint32_t t = t0;
    for (;;) {
        float lead = d[0];
        for (int c = 1; c < n; ++c)
            if (d[c] > lead) lead = d[c];
        if (lead >= target) break;
        if (t - t0 >= ORC_TICK_LIMIT) return ORC_EINVAL;
        tick_steps(&r, d, s, all_running, t, seed, request, sim, 0, NULL, NULL, S);
        for (int c = 0; c < n; ++c) {
            d[c] = d[c] + S[c];
            s[c] = S[c];
            if (d[c] >= L) return ORC_EINVAL;
        }
        ++t;
    }
    *t_out = t;
    for (int c = 0; c < n; ++c) {
        pos_out[c] = d[c];
        prev_out[c] = s[c];
    }
    return ORC_OK;
}

/* Positions of one simulated race tick by tick: row 0 is the given state
 * (pos == NULL: the start), row r the positions after r ticks of
 * simulation `sim` of `request`.  The trace ends before the first tick in
 * which some competitor reaches the line (in-play betting on the winner
 * closes then, Section 3), or after max_rows rows.  trace [max_rows][n];
 * *rows_out = rows written (>= 1).                                        */
int orc_race_trace(int n, float L, const float *comp, uint32_t t0, const float *pos,
                   const float *prev, uint64_t seed, uint32_t request, uint32_t sim,
                   uint32_t max_rows, float *trace, uint32_t *rows_out)
{
    orc_race r;
    if (race_setup(n, L, comp, &r) != ORC_OK) return ORC_EINVAL;
    if (!pos) t0 = 0;
    if (state_check(&r, t0, pos, prev) != ORC_OK) return ORC_EINVAL;
    if (max_rows < 1 || max_rows > ORC_TICK_LIMIT + 1 || !trace || !rows_out)
        return ORC_EINVAL;

    float d[ORC_MAX_N], s[ORC_MAX_N], S[ORC_MAX_N];
    int all_running[ORC_MAX_N];
    for (int c = 0; c < n; ++c) {
        d[c] = pos ? pos[c] : 0.0f;
        s[c] = pos ? prev[c] : 0.0f;
        all_running[c] = 1;
        trace[c] = d[c];
    }
    uint32_t rows = 1;
    uint32_t t = t0;
    while (rows < max_rows) {
        tick_steps(&r, d, s, all_running, t, seed, request, sim, 0, NULL, NULL, S);
        int crosses = 0;
        for (int c = 0; c < n; ++c)
            if (d[c] + S[c] >= L) crosses = 1;
        if (crosses) break;
        for (int c = 0; c < n; ++c) {
            d[c] = d[c] + S[c];
            s[c] = S[c];
            trace[(size_t)rows * n + c] = d[c];
        }
        ++rows;
        ++t;
    }
    *rows_out = rows;
    return ORC_OK;
}

/* Frequentist win probabilities: p_c = wins_c / sum(wins) in double;
 * with no recorded win every competitor gets 1/n (an RP(0) bettor holds
 * equiprobable estimates, Section 3).                                    */
int orc_win_probs(const uint64_t *wins, int n, double *probs)
{
    if (!wins || !probs || n < 1 || n > ORC_MAX_N) return ORC_EINVAL;
    uint64_t tot = 0;
    for (int c = 0; c < n; ++c) tot += wins[c];
    for (int c = 0; c < n; ++c)
        probs[c] = tot ? (double)wins[c] / (double)tot : 1.0 / (double)n;
    return ORC_OK;
}

int orc_max_competitors(void) { return ORC_MAX_N; }
uint32_t orc_tick_limit(void) { return ORC_TICK_LIMIT; }
