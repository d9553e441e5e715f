// race_sim.hpp -- one simulated race per lane, 64 lanes in lockstep
// (paper Section 3, Eq. 1).
//
// Layout.  A lane keeps its competitors in N register "slots" sorted by
// position (ascending; finished competitors are parked at +inf at the
// top).  Slot k holds the position d[k], the previous step s[k] and the
// index id[k] of the competitor that occupies it, which locates its draw
// and its parameter record in LDS.  Slots are kept in
// (position, competitor index) order, so the competitor ahead of slot k is
// the first slot above it with a larger position -- slot k+1 unless
// positions are equal -- and the query of Eq. 1 costs O(1) per competitor
// instead of a scan over all pairs.
//
// One tick (all 64 lanes at the same absolute tick t):
//   1. draws in competitor order: Philox4x32-10(key = seed,
//      ctr = (t, sim, request, b)) for blocks b = 0 .. ceil(N/4)-1;
//      competitor c takes word c&3 of block c>>2, u = (w >> 8) * 2^-24; the
//      draws go to the lane's column of an LDS table and each slot reads
//      the draw of its own competitor;
//   2. competitor ahead: the running competitor with the smallest position
//      greater than d_c (lowest index among equal positions); gap =
//      fl(d_ahead - d_c), +inf if nobody is ahead;
//   3. Eq. 1: R = alpha + beta*d; free: S = R*(elo + espan*u); blocked
//      (gap <= theta): S = R*min(s_c, s_ahead);
//   4. synchronous update d += S, s = S of the running competitors; a
//      competitor whose new position reaches L crosses the line;
//   5. this tick's finishers are ranked after the earlier ones, among
//      themselves by the fraction fl((L - d_old)/S), then by index, and are
//      parked at +inf;
//   6. bubble passes restore the slot order.
#pragma once

#include "race_common.hpp"

namespace bbe {

template <int N>
struct Slots {
    float d[N];
    float s[N];
    uint32_t id[N];
};

__device__ __forceinline__ float lds_f32(const char* smem, uint32_t off) {
    return *reinterpret_cast<const float*>(smem + off);
}

__device__ __forceinline__ void lds_st_f32(char* smem, uint32_t off, float v) {
    *reinterpret_cast<float*>(smem + off) = v;
}

// Writes the parameter records of a race into a wave's record block:
// record c = (elo, espan, alpha, beta, theta, -, -, -) at pbase + 32*c.
template <int N>
__device__ __forceinline__ void write_params(char* smem, uint32_t pbase, const RaceConst& rc,
                                            int lane) {
    if (lane < N) {
        float4* rec = reinterpret_cast<float4*>(smem + pbase + lane * 32);
        rec[0] = make_float4(rc.elo[lane], rc.espan[lane], rc.alpha[lane], rc.beta[lane]);
        rec[1] = make_float4(rc.theta[lane], 0.0f, 0.0f, 0.0f);
    }
}

// Loads an initial state already in slot order (positions ascending, equal
// positions by competitor index).
template <int N>
__device__ __forceinline__ void slots_reset(Slots<N>& sl, const float* __restrict__ d0,
                                            const float* __restrict__ s0,
                                            const uint8_t* __restrict__ id0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        sl.d[k] = d0[k];
        sl.s[k] = s0[k];
        sl.id[k] = id0[k];
    }
}

// Steps 1-4 for one lane.  `ucol` is the byte offset of this lane's column
// of the draw table (competitor c's draw at ucol + 256*c), `pbase` that of
// the wave's parameter records.  Returns the bit mask of slots that crossed
// the line (their d[] still holds the start-of-tick position).
template <int N>
__device__ __forceinline__ uint32_t slots_tick(Slots<N>& sl, char* smem, uint32_t ucol,
                                               uint32_t pbase, float L, uint32_t t,
                                               uint32_t sim, uint32_t request, uint32_t k0,
                                               uint32_t k1) {
    // 1. draws, competitor order, into this lane's column
#pragma unroll
    for (int b = 0; b < (N + 3) / 4; ++b) {
        U4 w = philox4x32_10(t, sim, request, (uint32_t)b, k0, k1);
        if (4 * b + 0 < N) lds_st_f32(smem, ucol + (4 * b + 0) * 256, unit24(w.x));
        if (4 * b + 1 < N) lds_st_f32(smem, ucol + (4 * b + 1) * 256, unit24(w.y));
        if (4 * b + 2 < N) lds_st_f32(smem, ucol + (4 * b + 2) * 256, unit24(w.z));
        if (4 * b + 3 < N) lds_st_f32(smem, ucol + (4 * b + 3) * 256, unit24(w.w));
    }

    // 2.-4. Slots from the top down.  Slots are in (position, index) order,
    //    so the competitor ahead of slot k is the first slot above it with a
    //    larger position: slot k+1, or -- where positions are equal -- the
    //    one found for slot k+1, carried down in (nd, ns).  The start-of-tick
    //    position and step of slot k+1 are kept in (d_up, s_up) because the
    //    update overwrites the slot (synchronous update).  Each slot's draw
    //    and parameter record are read from LDS kPf slots ahead of use.
    constexpr int kPf = 4;
    float pu[N], pth[N];
    float4 pp[N];
#pragma unroll
    for (int k = N - 1; k >= 0 && k >= N - kPf; --k) {
        const uint32_t id = sl.id[k];
        pu[k] = lds_f32(smem, ucol + (id << 8));
        pp[k] = *reinterpret_cast<const float4*>(smem + pbase + (id << 5));
        pth[k] = lds_f32(smem, pbase + (id << 5) + 16);
    }
    float nd = __builtin_inff(), ns = 0.0f;
    float d_up = __builtin_inff(), s_up = 0.0f;
    uint32_t cross = 0;
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        if (k - kPf >= 0) {
            const uint32_t id = sl.id[k - kPf];
            pu[k - kPf] = lds_f32(smem, ucol + (id << 8));
            pp[k - kPf] = *reinterpret_cast<const float4*>(smem + pbase + (id << 5));
            pth[k - kPf] = lds_f32(smem, pbase + (id << 5) + 16);
        }
        const float d = sl.d[k];
        const float s = sl.s[k];
        const bool gt = d_up > d;
        nd = gt ? d_up : nd;
        ns = gt ? s_up : ns;
        // Eq. 1
        const float4 p = pp[k];
        float R = p.z + p.w * d;
        float x = p.x + p.y * pu[k];
        float s_free = R * x;
        // min of two positive steps (ns = 0 only when nobody is ahead)
        float s_min = __uint_as_float(min(__float_as_uint(s), __float_as_uint(ns)));
        float s_blocked = R * s_min;
        float gap = nd - d;  // +inf when nobody is ahead
        float S = (gap <= pth[k]) ? s_blocked : s_free;
        // synchronous update
        bool run = d < L;
        float dn = d + S;
        bool cr = run && (dn >= L);
        cross |= cr ? (1u << k) : 0u;
        sl.d[k] = (run && !cr) ? dn : d;
        sl.s[k] = run ? S : s;
        d_up = d;
        s_up = s;
    }
    return cross;
}

// Step 5: rank this tick's finishers (slot mask `cross`) after the `nfin`
// earlier ones, record them, park them at +inf.  Returns the number ranked.
template <int N>
__device__ __forceinline__ int slots_finish(Slots<N>& sl, uint32_t cross, float L, int nfin,
                                            int& winner, uint8_t* __restrict__ row) {
    float fr[N];
    const bool multi = (cross & (cross - 1u)) != 0u;
    if (multi) {
#pragma unroll
        for (int k = 0; k < N; ++k)
            if ((cross >> k) & 1u) fr[k] = (L - sl.d[k]) / sl.s[k];
    }
    int ranked = 0;
    uint32_t rem = cross;
    while (rem) {
        int bk = -1;
        float bf = 0.0f;
        uint32_t bid = 32u;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            if (!((rem >> k) & 1u)) continue;
            uint32_t idk = sl.id[k];
            float f = multi ? fr[k] : 0.0f;
            bool better = (bk < 0) || (f < bf) || (f == bf && idk < bid);
            bk = better ? k : bk;
            bf = better ? f : bf;
            bid = better ? idk : bid;
        }
        int r = nfin + ranked;
        if (r == 0) winner = (int)bid;
        if (row) row[r] = (uint8_t)bid;
        ++ranked;
        rem &= ~(1u << bk);
    }
#pragma unroll
    for (int k = 0; k < N; ++k)
        if ((cross >> k) & 1u) sl.d[k] = __builtin_inff();
    return ranked;
}

// Order key of a slot: position first (non-negative floats and +inf order
// like their bit patterns), then the competitor index.
__device__ __forceinline__ uint64_t slot_key(float d, uint32_t id) {
    return ((uint64_t)__float_as_uint(d) << 32) | id;
}

// Step 6: one bubble pass restoring (position, index) order.  Each
// compare-exchange is branch-free (unsigned min/max of the position bit
// patterns, selects of the rest) and is skipped when no lane of the wave
// needs it.  Returns true (wave-uniform) if any lane swapped.  Lanes whose
// simulation has ended are sorted too; their slots are no longer read.
template <int N>
__device__ __forceinline__ bool slots_bubble(Slots<N>& sl) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        bool sw = slot_key(sl.d[k], sl.id[k]) > slot_key(sl.d[k + 1], sl.id[k + 1]);
        if (__builtin_amdgcn_ballot_w64(sw)) {
            uint32_t a = __float_as_uint(sl.d[k]), b = __float_as_uint(sl.d[k + 1]);
            float s0 = sw ? sl.s[k + 1] : sl.s[k];
            float s1 = sw ? sl.s[k] : sl.s[k + 1];
            uint32_t i0 = sw ? sl.id[k + 1] : sl.id[k];
            uint32_t i1 = sw ? sl.id[k] : sl.id[k + 1];
            sl.d[k] = __uint_as_float(a < b ? a : b);
            sl.d[k + 1] = __uint_as_float(a < b ? b : a);
            sl.s[k] = s0;
            sl.s[k + 1] = s1;
            sl.id[k] = i0;
            sl.id[k + 1] = i1;
            any = true;
        }
    }
    return any;
}

// Step 6 in full: passes until no lane of the wave swaps (the usual tick
// needs one pass that swaps and one that confirms).
template <int N>
__device__ __forceinline__ void slots_restore(Slots<N>& sl) {
    while (slots_bubble<N>(sl)) {
    }
}


// One generation: up to 64 simulations of one race from one state, one per
// lane, in lockstep from tick t0.  `live` marks the lanes that hold a
// simulation (index `sim`); `row` (or null) receives its finish order.
// Winners go to the LDS histogram `hist`; competitor-steps add to `steps`.
template <int N>
__device__ __forceinline__ void run_generation(char* smem, uint32_t ucol, uint32_t pbase,
                                               float L, const float* __restrict__ d0,
                                               const float* __restrict__ s0,
                                               const uint8_t* __restrict__ id0, uint32_t t0,
                                               bool live, uint32_t sim, uint32_t request,
                                               uint32_t k0, uint32_t k1, int stop_after,
                                               uint8_t* __restrict__ row, uint32_t* hist,
                                               unsigned long long& steps) {
    Slots<N> sl;
    slots_reset<N>(sl, d0, s0, id0);
    uint32_t t = t0;
    int nfin = 0, winner = -1;
    while (__builtin_amdgcn_ballot_w64(live)) {
        if (live) {
            uint32_t cross = slots_tick<N>(sl, smem, ucol, pbase, L, t, sim, request, k0, k1);
            if (cross) {
                int k = slots_finish<N>(sl, cross, L, nfin, winner, row);
                nfin += k;
                steps += (unsigned long long)k * (t + 1 - t0);
            }
            if (nfin >= stop_after || t + 1 - t0 >= kTickLimit) {
                if (winner >= 0) atomicAdd(&hist[winner], 1u);
                if (row)
                    for (int r = nfin; r < N; ++r) row[r] = 0xFF;
                steps += (unsigned long long)(N - nfin) * (t + 1 - t0);
                live = false;
            }
        }
        t += 1;
        slots_restore<N>(sl);
    }
}

}  // namespace bbe
