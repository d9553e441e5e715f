// bbe_bettors.hip -- C ABI of the in-play side: the race trace and the
// cheap bettor populations (paper Sections 3 and 5).
#include "abi_internal.hpp"
#include "bettors.hpp"

#include <algorithm>
#include <new>
#include <vector>

using namespace bbe_abi;

struct bbe_bettors {
    uint32_t n = 0;
    uint32_t per_kind[4] = {0, 0, 0, 0};
    uint8_t* kind = nullptr;  // device, grouped by kind
    float* param = nullptr;
    uint32_t* id = nullptr;
};

static void destroy(bbe_bettors* b) {
    if (!b) return;
    (void)hipFree(b->kind);
    (void)hipFree(b->param);
    (void)hipFree(b->id);
    delete b;
}

BBE_API int bbe_race_trace(const bbe_race* race, const bbe_state* state, uint64_t seed,
                           uint32_t request, uint32_t sim, uint32_t max_rows, float* trace,
                           uint32_t* n_rows, void* stream) {
    if (!race) return fail(BBE_EINVAL, "race is NULL");
    if (!trace || !n_rows) return fail(BBE_EINVAL, "NULL output");
    if (max_rows < 1 || max_rows > BBE_TICK_LIMIT + 1u)
        return fail(BBE_EINVAL, "max_rows must be in 1..BBE_TICK_LIMIT+1");
    bbe::TraceArgs a;
    std::memset(&a, 0, sizeof a);
    a.rc = race->rc;
    a.pace = race->pace;
    int rc = check_state(race, state, a.d0, a.s0, a.id0, &a.t0);
    if (rc != BBE_OK) return rc;
    a.request = request;
    a.sim = sim;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.max_rows = max_rows;
    a.trace = trace;
    a.rows_out = n_rows;
    hipError_t e = BBE_HIP(bbe::launch_race_trace(a, static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching race_trace_kernel");
    return ok();
}

BBE_API int bbe_bettors_create(const uint8_t* kind, const float* param, int n_bettors,
                               bbe_bettors** out) {
    if (!out) return fail(BBE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!kind || !param) return fail(BBE_EINVAL, "NULL argument");
    if (n_bettors < 1) return fail(BBE_EINVAL, "n_bettors must be >= 1");
    for (int b = 0; b < n_bettors; ++b) {
        const float p = param[b];
        switch (kind[b]) {
            case BBE_BETTOR_ZI:
            case BBE_BETTOR_LW:
                break;
            case BBE_BETTOR_UD:
                if (!std::isfinite(p) || !(p >= 0.0f))
                    return fail(BBE_EINVAL, "bettor %d: UD distance must be finite and >= 0", b);
                break;
            case BBE_BETTOR_LINEX:
                if (!(p >= 1.0f && p <= (float)BBE_TICK_LIMIT) || p != std::floor(p))
                    return fail(BBE_EINVAL,
                                "bettor %d: LinEx window must be an integer in 1..BBE_TICK_LIMIT",
                                b);
                break;
            default:
                return fail(BBE_EINVAL, "bettor %d: unknown kind %d", b, (int)kind[b]);
        }
    }
    // group by kind, keeping the caller's order within a kind
    std::vector<uint32_t> order((size_t)n_bettors);
    for (int b = 0; b < n_bettors; ++b) order[(size_t)b] = (uint32_t)b;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return kind[x] < kind[y]; });
    std::vector<uint8_t> k((size_t)n_bettors);
    std::vector<float> p((size_t)n_bettors);
    for (size_t j = 0; j < order.size(); ++j) {
        k[j] = kind[order[j]];
        // ZI and LW ignore their parameter; store 0 so no stray value is read
        p[j] = (k[j] == BBE_BETTOR_UD || k[j] == BBE_BETTOR_LINEX) ? param[order[j]] : 0.0f;
    }
    bbe_bettors* b = new (std::nothrow) bbe_bettors();
    if (!b) return fail(BBE_ENOMEM, "out of host memory");
    b->n = (uint32_t)n_bettors;
    for (int i = 0; i < n_bettors; ++i) b->per_kind[kind[i]] += 1;
    const size_t nb = (size_t)n_bettors;
    if (dev_alloc(&b->kind, nb) != hipSuccess ||
        dev_alloc(&b->param, nb * sizeof(float)) != hipSuccess ||
        dev_alloc(&b->id, nb * sizeof(uint32_t)) != hipSuccess) {
        destroy(b);
        return fail(BBE_ENOMEM, "device allocation of %d bettors failed", n_bettors);
    }
    hipError_t e = BBE_HIP(hipMemcpy(b->kind, k.data(), nb, hipMemcpyHostToDevice));
    if (e == hipSuccess) e = hipMemcpy(b->param, p.data(), nb * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->id, order.data(), nb * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        destroy(b);
        return hip_fail(e, "copying the bettors");
    }
    *out = b;
    return ok();
}

BBE_API void bbe_bettors_free(bbe_bettors* b) { destroy(b); }

BBE_API int bbe_bettors_count(const bbe_bettors* b, uint32_t* per_kind) {
    if (!b || !per_kind) return fail(BBE_EINVAL, "NULL argument");
    for (int i = 0; i < 4; ++i) per_kind[i] = b->per_kind[i];
    return ok();
}

BBE_API int bbe_bettor_views(const bbe_bettors* b, const float* trace, uint32_t n_rows, int n,
                             float track_len, uint32_t t0, uint32_t first_row, uint32_t n_eval,
                             uint64_t seed, uint8_t* views, uint32_t* counts, void* stream) {
    if (!b || !trace) return fail(BBE_EINVAL, "NULL argument");
    if (!views && !counts) return fail(BBE_EINVAL, "views and counts are both NULL");
    if (n < 1 || n > BBE_MAX_COMPETITORS)
        return fail(BBE_EINVAL, "n must be in 1..%d", BBE_MAX_COMPETITORS);
    if (!std::isfinite(track_len) || !(track_len > 0.0f))
        return fail(BBE_EINVAL, "track_len must be finite and > 0");
    if (n_rows < 1) return fail(BBE_EINVAL, "the trace needs at least one row");
    if ((uint64_t)first_row + n_eval > n_rows)
        return fail(BBE_EINVAL, "rows first_row .. first_row + n_eval - 1 exceed the trace");
    bbe::ViewArgs a;
    std::memset(&a, 0, sizeof a);
    a.trace = trace;
    a.n = n;
    a.L = track_len;
    a.t0 = t0;
    a.first_row = first_row;
    a.n_eval = n_eval;
    a.kind = b->kind;
    a.param = b->param;
    a.id = b->id;
    a.n_bettors = b->n;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.views = views;
    a.counts = counts;
    hipError_t e = BBE_HIP(bbe::launch_bettor_views(a, static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching bettor_views_kernel");
    return ok();
}

BBE_API int bbe_rp_views(const uint64_t* wins, int n_bettors, int n, int row_stride,
                         uint8_t* views, uint32_t* counts, void* stream) {
    if (!views && !counts) return fail(BBE_EINVAL, "views and counts are both NULL");
    if (n < 1 || n > BBE_MAX_COMPETITORS)
        return fail(BBE_EINVAL, "n must be in 1..%d", BBE_MAX_COMPETITORS);
    if (row_stride < n) return fail(BBE_EINVAL, "row_stride must be >= n");
    if (n_bettors < 0) return fail(BBE_EINVAL, "n_bettors must be >= 0");
    if (n_bettors > 0 && !wins) return fail(BBE_EINVAL, "wins is NULL");
    hipError_t e = BBE_HIP(bbe::launch_rp_views(reinterpret_cast<const unsigned long long*>(wins),
                                        (uint32_t)n_bettors, n, row_stride, views, counts,
                                        static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching rp_views_kernel");
    return ok();
}
