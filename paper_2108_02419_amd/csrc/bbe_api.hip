// bbe_api.hip -- the C ABI declared in include/bbe.h: argument validation,
// race handles, per-race constants, launch configuration and errors.
#include "../../include/bbe.h"
#include "kernels.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#define BBE_API extern "C" __attribute__((visibility("default")))

struct bbe_race {
    int n;
    float L;
    bbe_competitor comp[BBE_MAX_COMPETITORS];
    bbe::RaceConst rc;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return BBE_OK;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(BBE_EDEVICE, "%s: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
}

uint32_t f32_bits(float x) {
    uint32_t b;
    std::memcpy(&b, &x, 4);
    return b;
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

// Validates one competitor and fills its derived constants.
int setup_competitor(const bbe_competitor& c, float L, int idx, bbe::RaceConst& rc) {
    if (!std::isfinite(c.lo) || !std::isfinite(c.hi) || !std::isfinite(c.pref) ||
        !std::isfinite(c.rho) || !std::isfinite(c.theta))
        return fail(BBE_EINVAL, "competitor %d: non-finite parameter", idx);
    if (!(c.lo > 0.0f)) return fail(BBE_EINVAL, "competitor %d: lo must be > 0", idx);
    if (!(c.hi >= c.lo)) return fail(BBE_EINVAL, "competitor %d: hi must be >= lo", idx);
    if (!(c.pref > 0.0f && c.pref <= 1.0f))
        return fail(BBE_EINVAL, "competitor %d: pref must be in (0, 1]", idx);
    if (!(std::fabs(c.rho) < 1.0f)) return fail(BBE_EINVAL, "competitor %d: |rho| must be < 1", idx);
    if (!(c.theta >= 0.0f)) return fail(BBE_EINVAL, "competitor %d: theta must be >= 0", idx);
    // One rounding per operation (the library is built with -ffp-contract=off).
    float span = c.hi - c.lo;
    float elo = c.pref * c.lo;
    float espan = c.pref * span;
    float two_rho = 2.0f * c.rho;
    float alpha = 1.0f - c.rho;
    float beta = two_rho / L;
    rc.elo[idx] = elo;
    rc.espan[idx] = espan;
    rc.alpha[idx] = alpha;
    rc.beta[idx] = beta;
    rc.theta_bits[idx] = f32_bits(c.theta);
    double slowest = (double)elo * (1.0 - std::fabs((double)c.rho));
    if (!(slowest > 0.0) || (double)L / slowest > (double)BBE_EXPECTED_TICK_BOUND)
        return fail(BBE_EINVAL,
                    "competitor %d: slowest free step %.3g needs more than %d ticks to cover "
                    "the track",
                    idx, slowest, BBE_EXPECTED_TICK_BOUND);
    return BBE_OK;
}

int check_state(const bbe_race* r, const bbe_state* st, float* d0, float* s0, uint32_t* t0) {
    if (!st) {
        for (int c = 0; c < r->n; ++c) d0[c] = s0[c] = 0.0f;
        *t0 = 0;
        return BBE_OK;
    }
    if (st->tick > 0xFFFFFFFFu - BBE_TICK_LIMIT)
        return fail(BBE_EINVAL, "state tick %u too large", st->tick);
    if (!st->pos || !st->prev_step) return fail(BBE_EINVAL, "state needs pos and prev_step");
    for (int c = 0; c < r->n; ++c) {
        float p = st->pos[c], q = st->prev_step[c];
        if (!std::isfinite(p) || p < 0.0f || !(p < r->L))
            return fail(BBE_EINVAL, "state: pos[%d] must be finite and in [0, L)", c);
        if (!std::isfinite(q) || !(q > 0.0f))
            return fail(BBE_EINVAL, "state: prev_step[%d] must be finite and > 0", c);
        d0[c] = p;
        s0[c] = q;
    }
    *t0 = st->tick;
    return BBE_OK;
}

}  // namespace

BBE_API const char* bbe_last_error(void) { return g_err.c_str(); }

BBE_API int bbe_race_init(const bbe_competitor* comp, int n, float track_len, bbe_race** out) {
    if (!out) return fail(BBE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!comp) return fail(BBE_EINVAL, "comp is NULL");
    if (n < 1 || n > BBE_MAX_COMPETITORS)
        return fail(BBE_EINVAL, "n = %d outside 1..%d", n, BBE_MAX_COMPETITORS);
    if (!std::isfinite(track_len) || !(track_len > 0.0f))
        return fail(BBE_EINVAL, "track_len must be finite and > 0");
    bbe_race* r = new (std::nothrow) bbe_race();
    if (!r) return fail(BBE_ENOMEM, "out of host memory");
    r->n = n;
    r->L = track_len;
    r->rc.n = n;
    r->rc.L = track_len;
    for (int c = 0; c < n; ++c) {
        r->comp[c] = comp[c];
        int rc = setup_competitor(comp[c], track_len, c, r->rc);
        if (rc != BBE_OK) {
            delete r;
            return rc;
        }
    }
    *out = r;
    return ok();
}

BBE_API void bbe_race_free(bbe_race* race) { delete race; }

BBE_API int bbe_race_n(const bbe_race* race) {
    if (!race) return fail(BBE_EINVAL, "race is NULL");
    return race->n;
}

BBE_API int bbe_race_sim(const bbe_race* race, const bbe_state* state, uint32_t sim_begin,
                         uint32_t n_sims, uint64_t seed, uint32_t request, int stop_after,
                         uint8_t* finish_orders, uint64_t* win_counts, uint64_t* step_count,
                         void* stream) {
    if (!race) return fail(BBE_EINVAL, "race is NULL");
    if (n_sims == 0) return fail(BBE_EINVAL, "n_sims must be >= 1");
    if ((uint64_t)sim_begin + n_sims > 0x100000000ull)
        return fail(BBE_EINVAL, "sim_begin + n_sims exceeds 2^32");
    if (stop_after < 1 || stop_after > race->n)
        return fail(BBE_EINVAL, "stop_after = %d outside 1..%d", stop_after, race->n);
    bbe::SimArgs a;
    std::memset(&a, 0, sizeof a);
    a.rc = race->rc;
    int rc = check_state(race, state, a.d0, a.s0, &a.t0);
    if (rc != BBE_OK) return rc;
    a.sim_begin = sim_begin;
    a.n_sims = n_sims;
    a.request = request;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.stop_after = stop_after;
    a.orders = finish_orders;
    a.wins = reinterpret_cast<unsigned long long*>(win_counts);
    a.steps = reinterpret_cast<unsigned long long*>(step_count);

    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (a.wins && (e = bbe::launch_zero_u64(a.wins, race->n, s)) != hipSuccess)
        return hip_fail(e, "zeroing win_counts");
    if (a.steps && (e = bbe::launch_zero_u64(a.steps, 1, s)) != hipSuccess)
        return hip_fail(e, "zeroing step_count");

    const int block = bbe::mc_block_size();
    uint64_t need = ((uint64_t)n_sims + block - 1) / block;
    uint64_t resident = (uint64_t)bbe::mc_blocks_per_cu(race->n) * device_cus();
    int grid = (int)(need < resident ? need : resident);
    if ((e = bbe::launch_race_mc(a, grid, s)) != hipSuccess)
        return hip_fail(e, "launching race_mc_kernel");
    return ok();
}

BBE_API int bbe_win_probs(const uint64_t* win_counts, int n_rows, int n, int row_stride,
                          double* probs, void* stream) {
    if (!win_counts || !probs) return fail(BBE_EINVAL, "NULL buffer");
    if (n_rows < 1) return fail(BBE_EINVAL, "n_rows must be >= 1");
    if (n < 1 || n > BBE_MAX_COMPETITORS) return fail(BBE_EINVAL, "n = %d outside 1..%d", n,
                                                      BBE_MAX_COMPETITORS);
    if (row_stride < n) return fail(BBE_EINVAL, "row_stride must be >= n");
    hipError_t e = bbe::launch_win_probs(reinterpret_cast<const unsigned long long*>(win_counts),
                                         n_rows, n, row_stride, probs,
                                         static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "launching win_probs_kernel");
    return ok();
}

BBE_API int bbe_race_prefix(const bbe_race* race, const bbe_state* state, uint64_t seed,
                            uint32_t request, uint32_t sim, float target, uint32_t* tick_out,
                            float* pos_out, float* prev_out, void* stream) {
    if (!race) return fail(BBE_EINVAL, "race is NULL");
    if (!tick_out || !pos_out || !prev_out) return fail(BBE_EINVAL, "NULL output");
    if (!std::isfinite(target) || !(target < race->L))
        return fail(BBE_EINVAL, "target must be finite and < track length");
    bbe::PrefixArgs a;
    std::memset(&a, 0, sizeof a);
    a.rc = race->rc;
    int rc = check_state(race, state, a.d0, a.s0, &a.t0);
    if (rc != BBE_OK) return rc;
    a.request = request;
    a.sim = sim;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.target = target;
    a.tick_out = tick_out;
    a.pos_out = pos_out;
    a.prev_out = prev_out;
    hipError_t e = bbe::launch_race_prefix(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "launching race_prefix_kernel");
    return ok();
}
