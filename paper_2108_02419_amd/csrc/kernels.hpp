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
    // initial state in slot order: positions ascending, equal positions by
    // competitor index; id0[k] is the competitor in slot k
    float d0[kMaxN];
    float s0[kMaxN];
    uint8_t id0[kMaxN];
    uint32_t t0;
    uint32_t sim_begin;
    uint32_t n_sims;
    uint32_t request;
    uint32_t k0, k1;  // Philox key = seed
    int stop_after;
    uint8_t* orders;            // [n_sims][n] or null
    unsigned long long* wins;   // [n], zeroed before launch, or null
    unsigned long long* steps;  // [1], zeroed before launch, or null
    RacePace pace;
};

struct PrefixArgs {
    RaceConst rc;
    float d0[kMaxN];  // slot order, as in SimArgs
    float s0[kMaxN];
    uint8_t id0[kMaxN];
    uint32_t t0;
    uint32_t request;
    uint32_t sim;
    uint32_t k0, k1;
    float target;
    uint32_t max_ticks;  // stop after this many ticks at the latest
    uint32_t* tick_out;
    float* pos_out;
    float* prev_out;
    RacePace pace;
};

int mc_block_size();
int mc_blocks_per_cu(int n, bool paced);
// the paced variants (race_kernels_paced.hip), used by the two above
int mc_blocks_per_cu_paced(int n);
hipError_t launch_race_mc_paced(const SimArgs& a, int grid, hipStream_t s);
hipError_t launch_race_mc(const SimArgs& a, int grid, hipStream_t s);
hipError_t launch_race_prefix(const PrefixArgs& a, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
// Finish-order tallies over an orders matrix [n_sims][n] (see order_kernels.hip);
// both clear their counts first.
hipError_t launch_rank_counts(const uint8_t* orders, uint32_t n_sims, int n,
                              unsigned long long* counts, hipStream_t s);
hipError_t launch_order_pmf(const uint8_t* orders, uint32_t n_sims, int n, int n_fact,
                            unsigned long long* counts, hipStream_t s);
hipError_t launch_win_probs(const unsigned long long* wins, int n_rows, int n, int stride,
                            double* probs, hipStream_t s);

}  // namespace bbe

namespace bbe {

// One request of a batch: a race, an initial state in slot order and a
// range of simulations of stream (seed, request).  Read by whole waves
// (uniform loads).
struct alignas(16) ReqDesc {
    RaceConst rc;
    float d0[kMaxN];
    float s0[kMaxN];
    uint8_t id0[kMaxN];
    uint32_t t0;
    uint32_t request;
    uint32_t sim_begin;
    uint32_t n_sims;
    int stop_after;
    // in-play state generation only: simulation index and leader target
    uint32_t prefix_sim;
    float target;
    RacePace pace;
};

// A work item of the persistent kernel: simulations [first, first + count)
// of request `req` (count <= 64 * generations per chunk).
struct Chunk {
    uint32_t req;
    uint32_t first;
    uint32_t count;
    uint32_t n;
};

// One launch serves the work items chunks[0 .. n_chunks) of every
// competitor count (chunk.n selects the template instance).
struct BatchArgs {
    const ReqDesc* reqs;
    const Chunk* chunks;
    uint32_t n_chunks;
    uint32_t* queue;            // the launch's work-queue head, zeroed before launch
    unsigned long long* wins;   // [n_reqs][kMaxN], zeroed before launch
    unsigned long long* steps;  // [1] or null, zeroed before launch
    uint32_t k0, k1;
};

// paced: the items include a race with a time term of R (some gamma != 0)
hipError_t launch_batch_mc(const BatchArgs& a, int waves_per_block, int grid, bool paced,
                           hipStream_t s);
int batch_blocks_per_cu(int waves_per_block, bool paced);
// the paced variant (batch_kernels_paced.hip), used by the two above
hipError_t launch_batch_mc_paced(const BatchArgs& a, int waves_per_block, int grid,
                                 hipStream_t s);
int batch_blocks_per_cu_paced(int waves_per_block);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int n, hipStream_t s);
hipError_t launch_batch_probs(const unsigned long long* wins, const ReqDesc* reqs, int n_reqs,
                              double* probs, hipStream_t s);
hipError_t launch_prefix_batch(const ReqDesc* reqs, int n_reqs, uint32_t k0, uint32_t k1,
                               uint32_t* tick_out, float* pos_out, float* prev_out,
                               hipStream_t s);

}  // namespace bbe
