// abi_internal.hpp -- pieces of the C ABI implementation shared by its
// translation units: the race handle, error reporting, state validation.
#pragma once

#include "../../include/bbe.h"
#include "kernels.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#define BBE_API extern "C" __attribute__((visibility("default")))

struct bbe_race {
    int n;
    float L;
    bbe_competitor comp[BBE_MAX_COMPETITORS];
    bbe::RaceConst rc;
    bbe::RacePace pace;  // all zero unless bbe_race_set_pace
};

namespace bbe_abi {

extern thread_local std::string g_err;

inline int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

inline int ok() {
    g_err.clear();
    return BBE_OK;
}

// Host-side fault injection, for the tests of the error paths.  The
// environment variable BBE_FAULT_INJECT, read once per process, names the
// calls to fail: "alloc:K1,K2,..." fails the K-th device allocation made
// through dev_alloc (counted from 1 over the process) as an out-of-memory
// error, and "device:K1,..." replaces the K-th HIP call made through BBE_HIP
// by a hipErrorLaunchFailure result without making it; the two may be
// given together, separated by a space.  Unset, nothing is counted and
// nothing fails.
enum FaultKind { kFaultAlloc = 0, kFaultDevice = 1 };
bool fault(FaultKind kind);

inline hipError_t dev_alloc(void** p, size_t bytes) {
    if (fault(kFaultAlloc)) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

template <class T>
inline hipError_t dev_alloc(T** p, size_t bytes) {
    return dev_alloc(reinterpret_cast<void**>(p), bytes);
}

#define BBE_HIP(call) \
    (::bbe_abi::fault(::bbe_abi::kFaultDevice) ? hipErrorLaunchFailure : (call))

inline int hip_fail(hipError_t e, const char* what) {
    return fail(BBE_EDEVICE, "%s: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
}

inline int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

// Validates one competitor and fills its derived constants.
inline int setup_competitor(const bbe_competitor& c, float L, int idx, bbe::RaceConst& rc) {
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
    // the kernels use espan * 2^-16, exact for 0 and for spans >= 2^-110
    if (espan != 0.0f && !(espan >= 0x1p-110f))
        return fail(BBE_EINVAL, "competitor %d: pref*(hi-lo) must be 0 or at least 2^-110",
                    idx);
    rc.elo[idx] = elo;
    rc.espan16[idx] = espan * 0x1p-16f;
    rc.alpha[idx] = alpha;
    rc.beta[idx] = beta;
    rc.theta[idx] = c.theta;
    double slowest = (double)elo * (1.0 - std::fabs((double)c.rho));
    if (!(slowest > 0.0) || (double)L / slowest > (double)BBE_EXPECTED_TICK_BOUND)
        return fail(BBE_EINVAL,
                    "competitor %d: slowest free step %.3g needs more than %d ticks to cover "
                    "the track",
                    idx, slowest, BBE_EXPECTED_TICK_BOUND);
    return BBE_OK;
}

// Puts a state (competitor order) into slot order: positions ascending,
// equal positions by competitor index (a stable insertion sort).
inline void to_slot_order(int n, const float* d, const float* s, float* d_out, float* s_out,
                   uint8_t* id_out) {
    int idx[BBE_MAX_COMPETITORS];
    for (int c = 0; c < n; ++c) {
        int k = c;
        while (k > 0 && d[idx[k - 1]] > d[c]) {
            idx[k] = idx[k - 1];
            --k;
        }
        idx[k] = c;
    }
    for (int k = 0; k < n; ++k) {
        d_out[k] = d[idx[k]];
        s_out[k] = s[idx[k]];
        id_out[k] = (uint8_t)idx[k];
    }
}

// Validates a state and writes it in slot order (state == NULL: start of
// race, every competitor at 0, ordered by index).
inline int check_state(int n, float L, const bbe_state* st, float* d0, float* s0, uint8_t* id0,
                       uint32_t* t0) {
    float d[BBE_MAX_COMPETITORS], s[BBE_MAX_COMPETITORS];
    if (!st) {
        for (int c = 0; c < n; ++c) d[c] = s[c] = 0.0f;
        *t0 = 0;
        to_slot_order(n, d, s, d0, s0, id0);
        return BBE_OK;
    }
    if (st->tick > 0xFFFFFFFFu - BBE_TICK_LIMIT)
        return fail(BBE_EINVAL, "state tick %u too large", st->tick);
    if (!st->pos || !st->prev_step) return fail(BBE_EINVAL, "state needs pos and prev_step");
    for (int c = 0; c < n; ++c) {
        float p = st->pos[c], q = st->prev_step[c];
        if (!std::isfinite(p) || p < 0.0f || !(p < L))
            return fail(BBE_EINVAL, "state: pos[%d] must be finite and in [0, L)", c);
        if (!std::isfinite(q) || !(q > 0.0f))
            return fail(BBE_EINVAL, "state: prev_step[%d] must be finite and > 0", c);
        d[c] = p + 0.0f;  // -0 becomes +0
        s[c] = q;
    }
    *t0 = st->tick;
    to_slot_order(n, d, s, d0, s0, id0);
    return BBE_OK;
}

inline int check_state(const bbe_race* r, const bbe_state* st, float* d0, float* s0, uint8_t* id0,
                       uint32_t* t0) {
    return check_state(r->n, r->L, st, d0, s0, id0, t0);
}

}  // namespace bbe_abi
