// bbe_api.hip -- the C ABI declared in include/bbe.h: argument validation,
// race handles, per-race constants, launch configuration and errors.
#include "abi_internal.hpp"

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <new>
#include <vector>

namespace bbe_abi {
thread_local std::string g_err;

namespace {

// The calls BBE_FAULT_INJECT names, per kind (sorted), and the running
// count of each kind's calls.
struct FaultPlan {
    std::vector<uint64_t> at[2];
    std::atomic<uint64_t> count[2];

    FaultPlan() {
        count[0] = 0;
        count[1] = 0;
        const char* env = std::getenv("BBE_FAULT_INJECT");
        if (!env) return;
        std::string spec(env);
        size_t pos = 0;
        while (pos < spec.size()) {
            size_t end = spec.find(' ', pos);
            if (end == std::string::npos) end = spec.size();
            std::string item = spec.substr(pos, end - pos);
            pos = end + 1;
            size_t colon = item.find(':');
            if (colon == std::string::npos) continue;
            std::string kind = item.substr(0, colon);
            int k = kind == "alloc" ? kFaultAlloc : kind == "device" ? kFaultDevice : -1;
            if (k < 0) continue;
            const char* p = item.c_str() + colon + 1;
            while (*p) {
                char* e = nullptr;
                unsigned long long v = std::strtoull(p, &e, 10);
                if (e == p) break;
                if (v > 0) at[k].push_back(v);
                p = (*e == ',') ? e + 1 : e;
                if (*e != ',') break;
            }
            std::sort(at[k].begin(), at[k].end());
        }
    }
};

FaultPlan& fault_plan() {
    static FaultPlan plan;
    return plan;
}

}  // namespace

bool fault(FaultKind kind) {
    FaultPlan& plan = fault_plan();
    const std::vector<uint64_t>& at = plan.at[kind];
    if (at.empty()) return false;
    const uint64_t n = plan.count[kind].fetch_add(1, std::memory_order_relaxed) + 1;
    return std::binary_search(at.begin(), at.end(), n);
}

}  // namespace bbe_abi

using namespace bbe_abi;

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

BBE_API int bbe_race_set_pace(bbe_race* race, const float* gamma, const float* tau) {
    if (!race) return fail(BBE_EINVAL, "race is NULL");
    if (!gamma || !tau) return fail(BBE_EINVAL, "NULL argument");
    for (int c = 0; c < race->n; ++c) {
        if (!std::isfinite(gamma[c])) return fail(BBE_EINVAL, "competitor %d: gamma not finite", c);
        if (!(tau[c] >= 0.0f && tau[c] <= 16777216.0f) || tau[c] != std::floor(tau[c]))
            return fail(BBE_EINVAL, "competitor %d: tau must be an integer in 0..2^24", c);
        const double slow = (double)gamma[c] * (double)tau[c];
        const double r_min = 1.0 - std::fabs((double)race->comp[c].rho) + (slow < 0.0 ? slow : 0.0);
        if (slow < 0.0 && !(r_min >= 0x1p-10))
            return fail(BBE_EINVAL, "competitor %d: the time term takes R below 2^-10", c);
        const double slowest = (double)race->rc.elo[c] * r_min;
        if (!(slowest > 0.0) || (double)race->L / slowest > (double)BBE_EXPECTED_TICK_BOUND)
            return fail(BBE_EINVAL,
                        "competitor %d: slowest free step %.3g needs more than %d ticks to "
                        "cover the track",
                        c, slowest, BBE_EXPECTED_TICK_BOUND);
    }
    int paced = 0;
    for (int c = 0; c < race->n; ++c) {
        race->pace.gamma[c] = gamma[c];
        race->pace.tau[c] = tau[c];
        if (gamma[c] != 0.0f) paced = 1;
    }
    race->pace.paced = paced;
    return ok();
}

BBE_API int bbe_pref_from_factors(const float* factors, int n_factors, const float* prefs,
                                  const float* sens, int n, float* pref_out) {
    if (!factors || !prefs || !sens || !pref_out) return fail(BBE_EINVAL, "NULL argument");
    if (n < 1 || n > BBE_MAX_COMPETITORS)
        return fail(BBE_EINVAL, "n must be in 1..%d", BBE_MAX_COMPETITORS);
    if (n_factors < 1 || n_factors > BBE_MAX_FACTORS)
        return fail(BBE_EINVAL, "n_factors must be in 1..%d", BBE_MAX_FACTORS);
    auto unit = [](float v) { return std::isfinite(v) && v >= 0.0f && v <= 1.0f; };
    for (int k = 0; k < n_factors; ++k)
        if (!unit(factors[k])) return fail(BBE_EINVAL, "factor %d must be in [0, 1]", k);
    for (int i = 0; i < n * n_factors; ++i) {
        if (!unit(prefs[i])) return fail(BBE_EINVAL, "preference %d must be in [0, 1]", i);
        if (!(std::isfinite(sens[i]) && sens[i] >= 0.0f && sens[i] < 1.0f))
            return fail(BBE_EINVAL, "sensitivity %d must be in [0, 1)", i);
    }
    for (int c = 0; c < n; ++c) {
        // one rounding per operation, factors in order
        float P = 1.0f;
        for (int k = 0; k < n_factors; ++k) {
            const float mismatch = std::fabs(factors[k] - prefs[c * n_factors + k]);
            const float wm = sens[c * n_factors + k] * mismatch;
            const float term = 1.0f - wm;
            P = P * term;
        }
        if (!(P > 0.0f)) return fail(BBE_EINVAL, "competitor %d: P underflows to 0", c);
        pref_out[c] = P;
    }
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
    a.pace = race->pace;
    int rc = check_state(race, state, a.d0, a.s0, a.id0, &a.t0);
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
    if (a.wins && (e = BBE_HIP(bbe::launch_zero_u64(a.wins, race->n, s))) != hipSuccess)
        return hip_fail(e, "zeroing win_counts");
    if (a.steps && (e = BBE_HIP(bbe::launch_zero_u64(a.steps, 1, s))) != hipSuccess)
        return hip_fail(e, "zeroing step_count");

    const int block = bbe::mc_block_size();
    uint64_t need = ((uint64_t)n_sims + block - 1) / block;
    uint64_t resident = (uint64_t)bbe::mc_blocks_per_cu(race->n, race->pace.paced != 0) * device_cus();
    int grid = (int)(need < resident ? need : resident);
    if ((e = BBE_HIP(bbe::launch_race_mc(a, grid, s))) != hipSuccess)
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
    hipError_t e = BBE_HIP(bbe::launch_win_probs(
        reinterpret_cast<const unsigned long long*>(win_counts), n_rows, n, row_stride, probs,
        static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching win_probs_kernel");
    return ok();
}

BBE_API int bbe_rank_counts(const uint8_t* orders, uint32_t n_sims, int n, uint64_t* counts,
                            void* stream) {
    if (n < 1 || n > BBE_MAX_COMPETITORS)
        return fail(BBE_EINVAL, "n = %d outside 1..%d", n, BBE_MAX_COMPETITORS);
    if (!counts || (!orders && n_sims > 0)) return fail(BBE_EINVAL, "NULL buffer");
    hipError_t e = BBE_HIP(bbe::launch_rank_counts(
        orders, n_sims, n, reinterpret_cast<unsigned long long*>(counts),
        static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching rank_counts_kernel");
    return ok();
}

BBE_API int bbe_order_pmf(const uint8_t* orders, uint32_t n_sims, int n, uint64_t* counts,
                          void* stream) {
    if (n < 1 || n > BBE_ORDER_PMF_MAX_N)
        return fail(BBE_EINVAL, "n = %d outside 1..%d", n, BBE_ORDER_PMF_MAX_N);
    if (!counts || (!orders && n_sims > 0)) return fail(BBE_EINVAL, "NULL buffer");
    int n_fact = 1;
    for (int k = 2; k <= n; ++k) n_fact *= k;
    hipError_t e = BBE_HIP(bbe::launch_order_pmf(
        orders, n_sims, n, n_fact, reinterpret_cast<unsigned long long*>(counts),
        static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching order_pmf_kernel");
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
    a.pace = race->pace;
    int rc = check_state(race, state, a.d0, a.s0, a.id0, &a.t0);
    if (rc != BBE_OK) return rc;
    a.request = request;
    a.sim = sim;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.target = target;
    a.max_ticks = 0xFFFFFFFFu;
    a.tick_out = tick_out;
    a.pos_out = pos_out;
    a.prev_out = prev_out;
    hipError_t e = BBE_HIP(bbe::launch_race_prefix(a, static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching race_prefix_kernel");
    return ok();
}

BBE_API int bbe_race_advance(const bbe_race* race, const bbe_state* state, uint64_t seed,
                             uint32_t request, uint32_t sim, uint32_t n_ticks, uint32_t* tick_out,
                             float* pos_out, float* prev_out, void* stream) {
    if (!race) return fail(BBE_EINVAL, "race is NULL");
    if (!tick_out || !pos_out || !prev_out) return fail(BBE_EINVAL, "NULL output");
    if (n_ticks < 1 || n_ticks > BBE_TICK_LIMIT)
        return fail(BBE_EINVAL, "n_ticks must be in 1..BBE_TICK_LIMIT");
    bbe::PrefixArgs a;
    std::memset(&a, 0, sizeof a);
    a.rc = race->rc;
    a.pace = race->pace;
    int rc = check_state(race, state, a.d0, a.s0, a.id0, &a.t0);
    if (rc != BBE_OK) return rc;
    a.request = request;
    a.sim = sim;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.target = __builtin_inff();
    a.max_ticks = n_ticks;
    a.tick_out = tick_out;
    a.pos_out = pos_out;
    a.prev_out = prev_out;
    hipError_t e = BBE_HIP(bbe::launch_race_prefix(a, static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching race_prefix_kernel");
    return ok();
}
