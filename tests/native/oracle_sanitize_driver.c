/* Runs the oracle's entry points on inputs read from a file and writes their
 * outputs to another, so that tests/test_oracle_sanitizers.py can build the
 * oracle with the address and undefined-behaviour sanitizers and compare
 * what that build computes with the plain build.  Every buffer is allocated
 * at exactly the size the entry point is told, so an access past it is
 * reported.
 *
 * Input (little-endian): int32 n, float L, float comp[7 n] (lo, hi, pref,
 *   rho, theta, gamma, tau per competitor), uint32 t0,
 *   int32 has_state, float pos[n], float prev[n], uint32 sim_begin,
 *   uint32 n_sims, uint64 seed, uint32 request, int32 stop_after,
 *   float target, uint32 max_rows.
 * Output: int32 rc, uint8 orders[n_sims n], uint64 wins[n], uint64 steps
 *   (orc_race_sim); int32 rc, uint32 tick, float pos[n], float prev[n]
 *   (orc_race_prefix); int32 rc, uint32 rows, float trace[rows n]
 *   (orc_race_trace); int32 rc, double probs[n] (orc_win_probs of wins).  */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_race_sim(int n, float L, const float *comp, uint32_t t0, const float *pos,
                 const float *prev, uint32_t sim_begin, uint32_t n_sims, uint64_t seed,
                 uint32_t request, int stop_after, uint32_t levels, uint8_t *orders,
                 uint64_t *wins, uint64_t *steps, int threads);
int orc_race_prefix(int n, float L, const float *comp, uint32_t t0, const float *pos,
                    const float *prev, uint64_t seed, uint32_t request, uint32_t sim,
                    float target, uint32_t *t_out, float *pos_out, float *prev_out);
int orc_race_trace(int n, float L, const float *comp, uint32_t t0, const float *pos,
                   const float *prev, uint64_t seed, uint32_t request, uint32_t sim,
                   uint32_t max_rows, float *trace, uint32_t *rows_out);
int orc_win_probs(const uint64_t *wins, int n, double *probs);

static void rd(FILE *f, void *p, size_t bytes)
{
    if (fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
}

static void wr(FILE *f, const void *p, size_t bytes)
{
    if (bytes && fwrite(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short output\n");
        exit(2);
    }
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 2;
    }
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int32_t n, has_state, stop_after;
    float L, target;
    uint32_t t0, sim_begin, n_sims, request, max_rows;
    uint64_t seed;
    rd(in, &n, 4);
    if (n < 1 || n > 20) return 2;
    rd(in, &L, 4);
    float *comp = malloc(sizeof(float) * 7 * (size_t)n);
    float *pos = malloc(sizeof(float) * (size_t)n);
    float *prev = malloc(sizeof(float) * (size_t)n);
    rd(in, comp, sizeof(float) * 7 * (size_t)n);
    rd(in, &t0, 4);
    rd(in, &has_state, 4);
    rd(in, pos, sizeof(float) * (size_t)n);
    rd(in, prev, sizeof(float) * (size_t)n);
    rd(in, &sim_begin, 4);
    rd(in, &n_sims, 4);
    rd(in, &seed, 8);
    rd(in, &request, 4);
    rd(in, &stop_after, 4);
    rd(in, &target, 4);
    rd(in, &max_rows, 4);
    fclose(in);
    const float *sp = has_state ? pos : NULL, *sv = has_state ? prev : NULL;

    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    uint8_t *orders = malloc((size_t)n_sims * (size_t)n);
    uint64_t *wins = malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t steps = 0;
    int32_t rc = orc_race_sim(n, L, comp, t0, sp, sv, sim_begin, n_sims, seed, request,
                              stop_after, 0, orders, wins, &steps, 1);
    wr(out, &rc, 4);
    wr(out, orders, (size_t)n_sims * (size_t)n);
    wr(out, wins, sizeof(uint64_t) * (size_t)n);
    wr(out, &steps, 8);

    uint32_t tick = 0;
    float *p_out = malloc(sizeof(float) * (size_t)n);
    float *s_out = malloc(sizeof(float) * (size_t)n);
    rc = orc_race_prefix(n, L, comp, t0, sp, sv, seed, request, 0, target, &tick, p_out, s_out);
    wr(out, &rc, 4);
    wr(out, &tick, 4);
    wr(out, p_out, sizeof(float) * (size_t)n);
    wr(out, s_out, sizeof(float) * (size_t)n);

    uint32_t rows = 0;
    float *trace = malloc(sizeof(float) * (size_t)max_rows * (size_t)n);
    rc = orc_race_trace(n, L, comp, t0, sp, sv, seed, request, 0, max_rows, trace, &rows);
    wr(out, &rc, 4);
    wr(out, &rows, 4);
    wr(out, trace, sizeof(float) * (size_t)rows * (size_t)n);

    double *probs = malloc(sizeof(double) * (size_t)n);
    rc = orc_win_probs(wins, n, probs);
    wr(out, &rc, 4);
    wr(out, probs, sizeof(double) * (size_t)n);
    fclose(out);

    free(comp);
    free(pos);
    free(prev);
    free(orders);
    free(wins);
    free(p_out);
    free(s_out);
    free(trace);
    free(probs);
    return 0;
}
