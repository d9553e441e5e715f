// bettors.hpp -- argument blocks and launchers of the in-play side: the
// trace of the race the bettors watch and the views of the cheap bettor
// rules (paper Section 5).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "race_common.hpp"

namespace bbe {

// Positions of one simulation, row 0 = the start state, row r after r
// ticks, until the tick before the first crossing or max_rows rows.
struct TraceArgs {
    RaceConst rc;
    float d0[kMaxN];  // start state in slot order, as in SimArgs
    float s0[kMaxN];
    uint8_t id0[kMaxN];
    uint32_t t0;
    uint32_t request;
    uint32_t sim;
    uint32_t k0, k1;
    uint32_t max_rows;
    float* trace;       // [max_rows][n]
    uint32_t* rows_out;  // [1]
    RacePace pace;
};

// Bettor kinds, as numbered in the C ABI.
enum : uint8_t { kZI = 0, kLW = 1, kUD = 2, kLinEx = 3 };

// Views of a bettor population at trace rows first_row .. first_row +
// n_eval - 1.  The population is stored grouped by kind (stable), so that
// the waves of a launch run one rule each: slot j holds bettor id[j].
struct ViewArgs {
    const float* trace;  // [n_rows][n]
    int n;
    float L;
    uint32_t t0;         // tick of trace row 0
    uint32_t first_row;
    uint32_t n_eval;
    const uint8_t* kind;   // [n_bettors], grouped by kind
    const float* param;    // [n_bettors], same order
    const uint32_t* id;    // [n_bettors], caller's bettor index of each slot
    uint32_t n_bettors;
    uint32_t k0, k1;       // ZI draws: Philox key
    uint8_t* views;        // [n_eval][n_bettors] by caller index, or null
    uint32_t* counts;      // [n_eval][n], or null; cleared by the launcher
};

constexpr int kViewBlock = 256;
constexpr int kViewRowsPerBlock = 8;
// rows of history staged in LDS for LinEx windows (longer windows read the
// trace in global memory)
constexpr int kViewWindow = 120;

hipError_t launch_race_trace(const TraceArgs& a, hipStream_t s);
hipError_t launch_bettor_views(const ViewArgs& a, hipStream_t s);
// RP(d) views from win counts [n_bettors][stride]; counts [n] cleared first.
hipError_t launch_rp_views(const unsigned long long* wins, uint32_t n_bettors, int n, int stride,
                           uint8_t* views, uint32_t* counts, hipStream_t s);

}  // namespace bbe
