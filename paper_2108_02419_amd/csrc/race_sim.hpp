// race_sim.hpp -- one simulated race per lane, 64 lanes in lockstep
// (paper Section 3, Eq. 1).
//
// Layout.  A lane keeps its competitors in N register "slots" sorted by
// position (ascending; finished competitors are parked at the top with a
// NaN position).  Slot k holds the position d[k], the LDS byte offset
// rec[k] of its competitor's parameter record (pbase + 32 * competitor
// index; it also locates the competitor's draw) and the previous step s[k].
// Slots are ordered by the 64-bit key (bits(d) << 32) | rec: non-negative
// floats, +inf and the parking NaN order like their bit patterns, and rec
// grows with the competitor index, so this is (position, index) order.  The
// competitor ahead of slot k is then the first slot above it with a larger
// position -- slot k+1 unless positions are equal -- and the query of Eq. 1
// costs O(1) per competitor instead of a scan over all pairs.
//
// One tick (all 64 lanes at the same absolute tick t):
//   1. draws in competitor order: Philox4x32-10(key = seed,
//      ctr = (t, sim, request, b)) for blocks b = 0 .. ceil(N/8)-1;
//      competitor c takes word (c>>1)&3 of block c>>3, its high half for
//      even c and its low half for odd c, as the integer k (u = k * 2^-16);
//      the draws go to the lane's column of an LDS table and each slot
//      reads the draw of its own competitor;
//   2. competitor ahead: the running competitor with the smallest position
//      greater than d_c (lowest index among equal positions); gap =
//      fl(d_ahead - d_c), +inf if nobody is ahead;
//   3. Eq. 1: R = alpha + beta*d (+ gamma*min(t, tau) in the paced
//      variants); free: S = R*(elo + espan*u); blocked (gap <= theta):
//      S = R*min(s_c, s_ahead);
//   4. synchronous update d += S, s = S of the running competitors; a
//      competitor whose new position reaches L crosses the line;
//   5. this tick's finishers are ranked after the earlier ones, among
//      themselves by the fraction fl((L - d_old)/S), then by index, and are
//      parked (position NaN: every comparison with it is false, so a parked
//      slot never crosses again and is never "ahead" of anyone);
//   6. compare-exchange passes, alternately upward and downward, restore the
//      slot order.
#pragma once

#include "race_common.hpp"

#include <type_traits>

namespace bbe {

template <int N>
struct Slots {
    float d[N];
    uint32_t rec[N];
    float s[N];
};

// Order key of a slot.
__device__ __forceinline__ uint64_t slot_key(float d, uint32_t rec) {
    return ((uint64_t)__float_as_uint(d) << 32) | rec;
}

__device__ __forceinline__ float lds_f32(const char* smem, uint32_t off) {
    return *reinterpret_cast<const float*>(smem + off);
}

__device__ __forceinline__ void lds_st_f32(char* smem, uint32_t off, float v) {
    *reinterpret_cast<float*>(smem + off) = v;
}

// The parking position of finished competitors (a quiet NaN whose bit
// pattern exceeds that of +inf).
__device__ __forceinline__ float parked() {
    return __uint_as_float(0x7FC00000u);
}

// How slots_tick adds the time term gamma*min(t, tau) of R:
//   kPaceOff    no time term (gamma = 0 everywhere);
//   kPaceInline every slot reads its competitor's gamma and tau and forms the
//               term itself (lanes may be at different ticks);
//   kPaceTable  all lanes of the wave are at the same tick: lane c forms
//               competitor c's term once per tick into its record, and every
//               slot adds it.  The term is the same rounded product either
//               way, so the three modes agree bit for bit.
enum Pace : int { kPaceOff = 0, kPaceInline = 1, kPaceTable = 2 };

// Writes the parameter records of a race into a record block: record c =
// (elo, espan16, alpha, beta, theta, gamma | term, tau, gamma) at
// pbase + 32*c; the time-term fields are written (by the same lane,
// afterwards) by write_pace.  Offset 20 holds gamma for kPaceInline and
// the current tick's term for kPaceTable.
template <int N>
__device__ __forceinline__ void write_params(char* smem, uint32_t pbase, const RaceConst& rc,
                                            int lane) {
    if (lane < N) {
        float4* rec = reinterpret_cast<float4*>(smem + pbase + lane * 32);
        rec[0] = make_float4(rc.elo[lane], rc.espan16[lane], rc.alpha[lane], rc.beta[lane]);
        rec[1] = make_float4(rc.theta[lane], 0.0f, 0.0f, 0.0f);
    }
}

template <int N>
__device__ __forceinline__ void write_pace(char* smem, uint32_t pbase, const RacePace& pc,
                                          int lane) {
    if (lane < N) {
        float* rec = reinterpret_cast<float*>(smem + pbase + lane * 32);
        rec[5] = pc.gamma[lane];
        rec[6] = pc.tau[lane];
        rec[7] = pc.gamma[lane];
    }
}

// Loads an initial state already in slot order (positions ascending, equal
// positions by competitor index); `pbase` locates the parameter records.
template <int N>
__device__ __forceinline__ void slots_reset(Slots<N>& sl, const float* __restrict__ d0,
                                            const float* __restrict__ s0,
                                            const uint8_t* __restrict__ id0, uint32_t pbase) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        sl.d[k] = d0[k];
        sl.rec[k] = pbase + 32u * id0[k];
        sl.s[k] = s0[k];
    }
}

// Steps 1-4 for one lane.  `ucol` is the byte offset of this lane's column
// of the draw table (competitor c's draw at ucol + 256*c), `pbase` that of
// the parameter records.  Returns the bit mask of slots that crossed the
// line (their position still holds the start-of-tick value; their s holds
// the step S that took them over).  kPace selects how the time term of R
// is added (with gamma = 0 it adds +0, so every mode agrees on unpaced
// races).  Only the A lowest slots are stepped: the caller guarantees that
// slots A .. N-1 are parked in every lane (a parked slot's step changes
// nothing: it stays parked and is never ahead of anyone).
template <int N, Pace kPace = kPaceOff, int A = N>
__device__ __forceinline__ uint32_t slots_tick(Slots<N>& sl, char* smem, uint32_t ucol,
                                               uint32_t pbase, float L, uint32_t t,
                                               uint32_t sim, uint32_t request, uint32_t k0,
                                               uint32_t k1) {
    const float tf = (float)t;
    if constexpr (kPace == kPaceTable) {
        // this tick's term of competitor c, formed by lane c (t is the same
        // in every lane) into its record for the wave's slots to add
        const uint32_t lane = __lane_id();
        if (lane < (uint32_t)N) {
            const uint32_t r = pbase + 32u * lane;
            const float2 tg = *reinterpret_cast<const float2*>(smem + r + 24u);  // (tau, gamma)
            lds_st_f32(smem, r + 20u, tg.y * fminf(tf, tg.x));
        }
        // the wave's LDS operations complete in order; keep the compiler
        // from moving the slots' reads above this store
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // 1. draws, competitor order, into this lane's column
#pragma unroll
    for (int b = 0; b < (N + 7) / 8; ++b) {
        const U4 w = philox4x32_10(t, sim, request, (uint32_t)b, k0, k1);
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 8 * b + 2 * j;
            if (c < N) lds_st_f32(smem, ucol + c * 256, draw_hi(words[j]));
            if (c + 1 < N) lds_st_f32(smem, ucol + (c + 1) * 256, draw_lo(words[j]));
        }
    }

    // 2.-4. Slots from the top down.  Slots are in (position, index) order,
    //    so the competitor ahead of slot k is the first slot above it with a
    //    larger position: slot k+1, or -- where positions are equal -- the
    //    one found for slot k+1, carried down in (nd, ns).  The start-of-tick
    //    position and step of slot k+1 are kept in (d_up, s_up) because the
    //    update overwrites the slot (synchronous update).  The draw of
    //    competitor c sits at ucol + 256*c = ubias + 8*rec; each slot's draw
    //    and parameter record are read from LDS kPf slots ahead of use.
    const uint32_t ubias = ucol - 8u * pbase;
    constexpr int kPf = 4;
    float pu[N], pth[N], pga[N], pta[N];
    float4 pp[N];
#pragma unroll
    for (int k = A - 1; k >= 0 && k >= A - kPf; --k) {
        const uint32_t rec = sl.rec[k];
        pu[k] = lds_f32(smem, ubias + (rec << 3));
        pp[k] = *reinterpret_cast<const float4*>(smem + rec);
        if constexpr (kPace == kPaceInline) {
            const float4 q = *reinterpret_cast<const float4*>(smem + rec + 16);
            pth[k] = q.x;
            pga[k] = q.y;
            pta[k] = q.z;
        } else if constexpr (kPace == kPaceTable) {
            const float2 q = *reinterpret_cast<const float2*>(smem + rec + 16);
            pth[k] = q.x;
            pga[k] = q.y;  // the term itself
        } else {
            pth[k] = lds_f32(smem, rec + 16);
        }
    }
    float nd = __builtin_inff(), ns = 0.0f;
    float d_up = __builtin_inff(), s_up = 0.0f;
    uint32_t cross = 0;
#pragma unroll
    for (int k = A - 1; k >= 0; --k) {
        if (k - kPf >= 0) {
            const uint32_t rec = sl.rec[k - kPf];
            pu[k - kPf] = lds_f32(smem, ubias + (rec << 3));
            pp[k - kPf] = *reinterpret_cast<const float4*>(smem + rec);
            if constexpr (kPace == kPaceInline) {
                const float4 q = *reinterpret_cast<const float4*>(smem + rec + 16);
                pth[k - kPf] = q.x;
                pga[k - kPf] = q.y;
                pta[k - kPf] = q.z;
            } else if constexpr (kPace == kPaceTable) {
                const float2 q = *reinterpret_cast<const float2*>(smem + rec + 16);
                pth[k - kPf] = q.x;
                pga[k - kPf] = q.y;
            } else {
                pth[k - kPf] = lds_f32(smem, rec + 16);
            }
        }
        const float d = sl.d[k];
        const float s = sl.s[k];
        const bool gt = d_up > d;  // false next to a parked (NaN) slot
        nd = gt ? d_up : nd;
        ns = gt ? s_up : ns;
        // Eq. 1
        const float4 p = pp[k];
        float R = p.z + p.w * d;
        if constexpr (kPace == kPaceInline) R = R + pga[k] * fminf(tf, pta[k]);
        if constexpr (kPace == kPaceTable) R = R + pga[k];
        float x = p.x + p.y * pu[k];
        // min of two positive steps (ns = 0 only when nobody is ahead)
        float s_min = __uint_as_float(min(__float_as_uint(s), __float_as_uint(ns)));
        float gap = nd - d;  // +inf when nobody is ahead
        // R*s_min when blocked, R*x when free (one product of the selected
        // factor rounds exactly as the product taken in that branch)
        float S = R * ((gap <= pth[k]) ? s_min : x);
        // synchronous update; a parked slot computes NaN and stays parked
        float dn = d + S;
        bool cr = dn >= L;
        cross = cross + cross + (cr ? 1u : 0u);  // slot k lands on bit k
        sl.d[k] = cr ? d : dn;
        sl.s[k] = S;
        d_up = d;
        s_up = s;
    }
    return cross;
}

// Step 5: ranks this tick's finishers (slot mask `cross`) after the `nfin`
// earlier ones, records them, and parks every crossing slot (position NaN);
// returns the number ranked.  `rank` is false in lanes whose simulation has
// already ended: their finishers are parked but not recorded.  In one pass
// over the crossing slots, each finisher is compacted -- entry j (the j-th
// set bit of `cross`) holds its competitor index in the lane's column of a
// byte table, at icol + 64*j, and, when there are several, its crossing
// fraction in the lane's (already consumed) column of the draw table, at
// ucol + 256*j -- and its slot is parked.  The entries are then picked in
// (fraction, index) order by a selection over those c entries, so the work
// grows with c^2 for the few finishers of a tick rather than with c*N.
template <int N, int A = N>
__device__ __forceinline__ int slots_rank_park(Slots<N>& sl, uint32_t cross, bool rank, float L,
                                               char* smem, uint32_t ucol, uint32_t icol,
                                               uint32_t pbase, int nfin, int& winner,
                                               uint8_t* __restrict__ row) {
    const int c = __builtin_popcount(cross);
#pragma unroll
    for (int k = 0; k < A; ++k)
        if ((cross >> k) & 1u) {
            if (rank) {
                const uint32_t j = __builtin_popcount(cross & ((1u << k) - 1u));
                smem[icol + 64u * j] = (char)((sl.rec[k] - pbase) >> 5);
                // a lone finisher needs no fraction
                if (c > 1) lds_st_f32(smem, ucol + 256u * j, (L - sl.d[k]) / sl.s[k]);
            }
            sl.d[k] = parked();
        }
    if (!rank) return 0;
    uint32_t used = 0u;
    for (int r = 0; r < c; ++r) {
        int bj = -1;
        float bf = 0.0f;
        uint32_t bid = 0u;
        for (int j = 0; j < c; ++j) {
            const float f = lds_f32(smem, ucol + 256u * j);
            const uint32_t id = (uint8_t)smem[icol + 64u * j];
            const bool better =
                !((used >> j) & 1u) && ((bj < 0) || (f < bf) || (f == bf && id < bid));
            bj = better ? j : bj;
            bf = better ? f : bf;
            bid = better ? id : bid;
        }
        used |= 1u << bj;  // c - r > 0 entries are unused, so bj >= 0
        const int rr = nfin + r;
        if (rr == 0) winner = (int)bid;
        if (row) row[rr] = (uint8_t)bid;
    }
    return c;
}

// Step 5 (ranking): ranks this tick's finishers (slot mask `cross`) after
// the `nfin` earlier ones and records them; returns the number ranked.  A
// lone finisher needs no fraction.  Several are compacted first -- entry j
// (the j-th set bit of `cross`) holds the finisher's fraction in the lane's
// (already consumed) column of the draw table, at ucol + 256*j, and its
// competitor index in the lane's column of a byte table, at icol + 64*j --
// and then picked in (fraction, index) order by a selection over those c
// entries, so the work grows with c^2 for the few finishers of a tick
// rather than with c*N.
template <int N>
__device__ __forceinline__ int slots_rank(const Slots<N>& sl, uint32_t cross, float L,
                                          char* smem, uint32_t ucol, uint32_t icol,
                                          uint32_t pbase, int nfin, int& winner,
                                          uint8_t* __restrict__ row) {
    if ((cross & (cross - 1u)) == 0u) {
        uint32_t rec = 0u;
#pragma unroll
        for (int k = 0; k < N; ++k) rec = ((cross >> k) & 1u) ? sl.rec[k] : rec;
        const uint32_t id = (rec - pbase) >> 5;
        if (nfin == 0) winner = (int)id;
        if (row) row[nfin] = (uint8_t)id;
        return 1;
    }
#pragma unroll
    for (int k = 0; k < N; ++k)
        if ((cross >> k) & 1u) {
            const uint32_t j = __builtin_popcount(cross & ((1u << k) - 1u));
            lds_st_f32(smem, ucol + 256u * j, (L - sl.d[k]) / sl.s[k]);
            smem[icol + 64u * j] = (char)((sl.rec[k] - pbase) >> 5);
        }
    const int c = __builtin_popcount(cross);
    uint32_t used = 0u;
    for (int r = 0; r < c; ++r) {
        int bj = -1;
        float bf = 0.0f;
        uint32_t bid = 0u;
        for (int j = 0; j < c; ++j) {
            const float f = lds_f32(smem, ucol + 256u * j);
            const uint32_t id = (uint8_t)smem[icol + 64u * j];
            const bool better =
                !((used >> j) & 1u) && ((bj < 0) || (f < bf) || (f == bf && id < bid));
            bj = better ? j : bj;
            bf = better ? f : bf;
            bid = better ? id : bid;
        }
        used |= 1u << bj;  // c - r > 0 entries are unused, so bj >= 0
        const int rr = nfin + r;
        if (rr == 0) winner = (int)bid;
        if (row) row[rr] = (uint8_t)bid;
    }
    return c;
}

// Step 5 (parking): the slots of mask `cross` get the parking position.
template <int N>
__device__ __forceinline__ void slots_park(Slots<N>& sl, uint32_t cross) {
#pragma unroll
    for (int k = 0; k < N; ++k)
        if ((cross >> k) & 1u) sl.d[k] = parked();
}

// Step 6: compare-exchange of slots k and k+1: three v_swap_b32 under the
// execution mask of the lanes that need the exchange, skipped when none
// does (the first pass of a tick exchanges most pairs in some lane, later
// passes few).
__device__ __forceinline__ void vswap(float& a, float& b) {
    asm volatile("v_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void vswap(uint32_t& a, uint32_t& b) {
    asm volatile("v_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}

template <int N>
__device__ __forceinline__ void slots_cx(Slots<N>& sl, int k) {
    if (slot_key(sl.d[k], sl.rec[k]) > slot_key(sl.d[k + 1], sl.rec[k + 1])) {
        vswap(sl.d[k], sl.d[k + 1]);
        vswap(sl.rec[k], sl.rec[k + 1]);
        vswap(sl.s[k], sl.s[k + 1]);
    }
}

// One upward pass (k = 0 .. N-2; carries a slot up any distance).  Returns
// true if the result may still be out of order: each slot is final once the
// pass has left it, so the pass checks every finished neighbour pair.
template <int N, int A = N>
__device__ __forceinline__ bool slots_pass_up(Slots<N>& sl) {
    bool bad = false;
#pragma unroll
    for (int k = 0; k < A - 1; ++k) {
        slots_cx<N>(sl, k);
        if (k >= 1)
            bad |= slot_key(sl.d[k - 1], sl.rec[k - 1]) > slot_key(sl.d[k], sl.rec[k]);
    }
    return bad;
}

// One upward pass that also re-exchanges the pair below after each step
// (k = 0 .. A-2: pairs k, then k-1), so a slot passed by two others moves
// down two places in one pass.  A tick's overtakes then need one such pass
// in most ticks where plain up/down passes need two: by a CPU replay of
// the 20-competitor workload, 1.24 passes and 22 order checks per tick
// instead of 2.22 and 40, for the same number of compare-exchanges.
// Checks every pair once the pass has left it.
template <int N, int A = N>
__device__ __forceinline__ bool slots_pass_up2(Slots<N>& sl) {
    bool bad = false;
#pragma unroll
    for (int k = 0; k < A - 1; ++k) {
        slots_cx<N>(sl, k);
        if (k >= 1) slots_cx<N>(sl, k - 1);
        if (k >= 2)
            bad |= slot_key(sl.d[k - 2], sl.rec[k - 2]) > slot_key(sl.d[k - 1], sl.rec[k - 1]);
    }
    if constexpr (A >= 3)
        bad |= slot_key(sl.d[A - 3], sl.rec[A - 3]) > slot_key(sl.d[A - 2], sl.rec[A - 2]);
    if constexpr (A >= 2)
        bad |= slot_key(sl.d[A - 2], sl.rec[A - 2]) > slot_key(sl.d[A - 1], sl.rec[A - 1]);
    return bad;
}

// One downward pass (k = N-2 .. 0; carries a slot down any distance).
template <int N, int A = N>
__device__ __forceinline__ bool slots_pass_down(Slots<N>& sl) {
    bool bad = false;
#pragma unroll
    for (int k = A - 2; k >= 0; --k) {
        slots_cx<N>(sl, k);
        if (k + 2 <= A - 1)
            bad |= slot_key(sl.d[k + 1], sl.rec[k + 1]) > slot_key(sl.d[k + 2], sl.rec[k + 2]);
    }
    return bad;
}

// Step 6 in full: alternate passes until every active lane of the wave is
// in order (a tick's overtakes need one pass in most lanes, two where a
// slot moves down by more than two places).  Sorting the A lowest slots
// suffices when slots A .. N-1 are parked in every lane: the order among
// parked slots is never used.
template <int N, int A = N>
__device__ __forceinline__ void slots_restore(Slots<N>& sl) {
    for (;;) {
        if (!__builtin_amdgcn_ballot_w64(slots_pass_up2<N, A>(sl))) break;
        if (!__builtin_amdgcn_ballot_w64(slots_pass_down<N, A>(sl))) break;
    }
}

// Runs f(std::integral_constant<int, A>) for A = N, N - kStep, ... (A >=
// kStep) one after the other for as long as f returns true.
template <int A, int kStep, class F>
__device__ __forceinline__ void run_phases(F& f) {
    if (f(std::integral_constant<int, A>{})) {
        if constexpr (A - kStep >= kStep) run_phases<A - kStep, kStep>(f);
    }
}

// One generation: up to 64 simulations of one race from one state, one per
// lane, in lockstep from tick t0.  `live` marks the lanes that hold a
// simulation (index `sim`); `row` (or null) receives its finish order.
// Lanes whose simulation has ended keep stepping with the others (their
// results are no longer recorded), so the tick needs no divergent branch.
// Winners go to the LDS histogram `hist`; competitor-steps add to `steps`.
// kRankPark selects slots_rank_park (one pass that ranks and parks) over
// slots_rank followed by slots_park; the two give the same results, and
// each kernel takes the one its register allocation does better with.
// kSkipStep > 0 stops stepping and sorting the top slots once they are
// parked in every lane, kSkipStep slots at a time (a copy of the tick per
// active count): late in a generation most lanes have parked most of their
// competitors.
template <int N, Pace kPace = kPaceOff, bool kRankPark = true, int kSkipStep = 0>
__device__ __forceinline__ void run_generation(char* smem, uint32_t ucol, uint32_t icol,
                                               uint32_t pbase,
                                               float L, const float* __restrict__ d0,
                                               const float* __restrict__ s0,
                                               const uint8_t* __restrict__ id0, uint32_t t0,
                                               bool live, uint32_t sim, uint32_t request,
                                               uint32_t k0, uint32_t k1, int stop_after,
                                               uint8_t* __restrict__ row, uint32_t* hist,
                                               unsigned long long& steps) {
    Slots<N> sl;
    slots_reset<N>(sl, d0, s0, id0, pbase);
    uint32_t t = t0;
    int nfin = 0, winner = -1;
    // One phase steps the A lowest slots (slots A .. N-1 are parked in every
    // lane) until the generation ends (returns false) or the next kSkipStep
    // slots down are parked in every lane too (returns true).
    auto phase = [&](auto act) -> bool {
        constexpr int A = decltype(act)::value;
        while (__builtin_amdgcn_ballot_w64(live)) {
            // the Philox products that depend on the simulation index only
            // are recomputed each tick rather than held (or spilled) across
            // the phases' loops
            uint32_t sim_t = sim;
            __asm__ volatile("" : "+v"(sim_t));
            const uint32_t cross =
                slots_tick<N, kPace, A>(sl, smem, ucol, pbase, L, t, sim_t, request, k0, k1);
            const bool any = __builtin_amdgcn_ballot_w64(cross != 0u) != 0;
            if (any) {
                if constexpr (kRankPark) {
                    const bool rank = live && cross;
                    const int k = slots_rank_park<N, A>(sl, cross, rank, L, smem, ucol, icol,
                                                        pbase, nfin, winner, row);
                    if (rank) {
                        nfin += k;
                        steps += (unsigned long long)k * (t + 1 - t0);
                    }
                } else {
                    if (live && cross) {
                        const int k = slots_rank<N>(sl, cross, L, smem, ucol, icol, pbase, nfin,
                                                    winner, row);
                        nfin += k;
                        steps += (unsigned long long)k * (t + 1 - t0);
                    }
                    slots_park<N>(sl, cross);
                }
            }
            if (live && (nfin >= stop_after || t + 1 - t0 >= kTickLimit)) {
                if (winner >= 0) atomicAdd(&hist[winner], 1u);
                if (row)
                    for (int r = nfin; r < N; ++r) row[r] = 0xFF;
                steps += (unsigned long long)(N - nfin) * (t + 1 - t0);
                live = false;
            }
            t += 1;
            slots_restore<N, A>(sl);
            if constexpr (kSkipStep > 0 && A - kSkipStep >= kSkipStep) {
                // sorted again, so a lane's parked slots are its top ones:
                // the next kSkipStep slots down are parked everywhere iff the
                // lowest of them is
                if (any && !__builtin_amdgcn_ballot_w64(__float_as_uint(sl.d[A - kSkipStep]) !=
                                                        __float_as_uint(parked())))
                    return true;
            }
        }
        return false;
    };
    if constexpr (kSkipStep > 0) {
        run_phases<N, kSkipStep>(phase);
    } else {
        // the same tick over all N slots, written out as a plain loop (the
        // batch kernel's register allocation is tuned on this form)
        while (__builtin_amdgcn_ballot_w64(live)) {
            const uint32_t cross =
                slots_tick<N, kPace>(sl, smem, ucol, pbase, L, t, sim, request, k0, k1);
            if (__builtin_amdgcn_ballot_w64(cross != 0u)) {
                if constexpr (kRankPark) {
                    const bool rank = live && cross;
                    const int k = slots_rank_park<N>(sl, cross, rank, L, smem, ucol, icol,
                                                     pbase, nfin, winner, row);
                    if (rank) {
                        nfin += k;
                        steps += (unsigned long long)k * (t + 1 - t0);
                    }
                } else {
                    if (live && cross) {
                        const int k = slots_rank<N>(sl, cross, L, smem, ucol, icol, pbase, nfin,
                                                    winner, row);
                        nfin += k;
                        steps += (unsigned long long)k * (t + 1 - t0);
                    }
                    slots_park<N>(sl, cross);
                }
            }
            if (live && (nfin >= stop_after || t + 1 - t0 >= kTickLimit)) {
                if (winner >= 0) atomicAdd(&hist[winner], 1u);
                if (row)
                    for (int r = nfin; r < N; ++r) row[r] = 0xFF;
                steps += (unsigned long long)(N - nfin) * (t + 1 - t0);
                live = false;
            }
            t += 1;
            slots_restore<N>(sl);
        }
    }
}

// Writes a lane's state in competitor order (prefix runs).
template <int N>
__device__ __forceinline__ void slots_store(const Slots<N>& sl, uint32_t pbase,
                                            float* __restrict__ pos_out,
                                            float* __restrict__ prev_out) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const uint32_t c = (sl.rec[k] - pbase) >> 5;
        pos_out[c] = sl.d[k];
        prev_out[c] = sl.s[k];
    }
}

}  // namespace bbe
