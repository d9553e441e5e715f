// kernels.hpp -- kernel argument blocks and launchers shared by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "race_common.hpp"

namespace bbe {

// Monte-Carlo over simulations sim_begin .. sim_begin + n_sims - 1 of one
// race from one state.  Passed by value (kernel arguments).
struct SimArgs {
    RaceConst rc;
    float d0[kMaxN];
    float s0[kMaxN];
    uint32_t t0;
    uint32_t sim_begin;
    uint32_t n_sims;
    uint32_t request;
    uint32_t k0, k1;  // Philox key = seed
    int stop_after;
    uint8_t* orders;            // [n_sims][n] or null
    unsigned long long* wins;   // [n], zeroed before launch, or null
    unsigned long long* steps;  // [1], zeroed before launch, or null
};

struct PrefixArgs {
    RaceConst rc;
    float d0[kMaxN];
    float s0[kMaxN];
    uint32_t t0;
    uint32_t request;
    uint32_t sim;
    uint32_t k0, k1;
    float target;
    uint32_t* tick_out;
    float* pos_out;
    float* prev_out;
};

int mc_block_size();
int mc_blocks_per_cu(int n);
hipError_t launch_race_mc(const SimArgs& a, int grid, hipStream_t s);
hipError_t launch_race_prefix(const PrefixArgs& a, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_win_probs(const unsigned long long* wins, int n_rows, int n, int stride,
                            double* probs, hipStream_t s);

}  // namespace bbe
