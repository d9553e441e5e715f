// race_sim.hpp -- one simulated race per lane (paper Section 3, Eq. 1).
//
// A lane holds the positions d[] and previous steps s[] of its simulation
// in registers (N is a compile-time competitor count, so every competitor
// index is static).  Finished competitors are parked at +inf, which removes
// them from the "competitor ahead" search; their update is masked.
//
// One tick (absolute tick t -> t+1), all from the start-of-tick state:
//   1. draws: Philox4x32-10(key = seed, ctr = (t, sim, request, b)) for
//      blocks b = 0 .. ceil(N/4)-1; competitor c takes word c&3 of block
//      c>>2 and u = (w >> 8) * 2^-24;
//   2. competitor ahead: over all pairs, the smallest positive gap
//      fl(d_i - d_c) and the previous step of that competitor, the lowest
//      index winning equal gaps (pairs are visited in ascending index order
//      and only a strictly smaller key replaces the current one);
//   3. Eq. 1: R = alpha + beta*d; free: S = R*(elo + espan*u); blocked
//      (gap <= theta): S = R*min(s_c, s_ahead);
//   4. synchronous update d += S, s = S for running competitors; a
//      competitor whose new position reaches L crosses the line;
//   5. this tick's finishers are ranked after the earlier ones, among
//      themselves by the fraction fl((L - d_old)/S), then by index.
#pragma once

#include "race_common.hpp"

namespace bbe {

template <int N>
struct LaneState {
    float d[N];
    float s[N];
    uint32_t t;
    int nfin;
    int winner;
};

template <int N>
__device__ __forceinline__ void lane_reset(LaneState<N>& st, const float* __restrict__ d0,
                                           const float* __restrict__ s0, uint32_t t0) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
        st.d[c] = d0[c];
        st.s[c] = s0[c];
    }
    st.t = t0;
    st.nfin = 0;
    st.winner = -1;
}

// Advance one tick.  Returns the number of competitors that stepped.
// `order_row` (may be null) receives the finishers of this tick at their
// ranks.
template <int N>
__device__ __forceinline__ int lane_tick(LaneState<N>& st, const RaceConst& rc, uint32_t sim,
                                         uint32_t request, uint32_t k0, uint32_t k1,
                                         uint8_t* __restrict__ order_row) {
    // 1. draws
    float u[N];
#pragma unroll
    for (int b = 0; b < (N + 3) / 4; ++b) {
        U4 w = philox4x32_10(st.t, sim, request, (uint32_t)b, k0, k1);
        if (4 * b + 0 < N) u[4 * b + 0] = unit24(w.x);
        if (4 * b + 1 < N) u[4 * b + 1] = unit24(w.y);
        if (4 * b + 2 < N) u[4 * b + 2] = unit24(w.z);
        if (4 * b + 3 < N) u[4 * b + 3] = unit24(w.w);
    }

    // 2. competitor ahead
    uint32_t best[N];
    float s_ahead[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
        best[c] = 0xFFFFFFFFu;
        s_ahead[c] = 0.0f;
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
#pragma unroll
        for (int b = a + 1; b < N; ++b) {
            uint32_t g = __float_as_uint(st.d[b] - st.d[a]);
            uint32_t ka = gap_key_fwd(g);
            uint32_t kb = gap_key_rev(g);
            if (ka < best[a]) {
                best[a] = ka;
                s_ahead[a] = st.s[b];
            }
            if (kb < best[b]) {
                best[b] = kb;
                s_ahead[b] = st.s[a];
            }
        }
    }

    // 3. Eq. 1
    float S[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
        float R = rc.alpha[c] + rc.beta[c] * st.d[c];
        float x = rc.elo[c] + rc.espan[c] * u[c];
        float s_free = R * x;
        float s_blocked = R * fminf(st.s[c], s_ahead[c]);
        S[c] = (best[c] < rc.theta_bits[c]) ? s_blocked : s_free;
    }

    // 4. synchronous update; crossers keep their start-of-tick position
    //    until they are ranked
    const float L = rc.L;
    uint32_t cross = 0;
    int nrun = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        bool run = st.d[c] < L;
        float dn = st.d[c] + S[c];
        bool cr = run && (dn >= L);
        cross |= (uint32_t)cr << c;
        st.d[c] = (run && !cr) ? dn : st.d[c];
        st.s[c] = run ? S[c] : st.s[c];
        nrun += run ? 1 : 0;
    }
    st.t += 1;

    // 5. rank this tick's finishers
    if (cross) {
        if (cross & (cross - 1u)) {
            float fr[N];
#pragma unroll
            for (int c = 0; c < N; ++c)
                if ((cross >> c) & 1u) fr[c] = (L - st.d[c]) / st.s[c];
#pragma unroll
            for (int c = 0; c < N; ++c) {
                if (!((cross >> c) & 1u)) continue;
                int r = st.nfin;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    if (i == c || !((cross >> i) & 1u)) continue;
                    if (fr[i] < fr[c] || (fr[i] == fr[c] && i < c)) ++r;
                }
                if (r == 0) st.winner = c;
                if (order_row) order_row[r] = (uint8_t)c;
            }
        } else {
            int c = __builtin_ctz(cross);
            if (st.nfin == 0) st.winner = c;
            if (order_row) order_row[st.nfin] = (uint8_t)c;
        }
        st.nfin += __builtin_popcount(cross);
#pragma unroll
        for (int c = 0; c < N; ++c)
            if ((cross >> c) & 1u) st.d[c] = __builtin_inff();
    }
    return nrun;
}

}  // namespace bbe
