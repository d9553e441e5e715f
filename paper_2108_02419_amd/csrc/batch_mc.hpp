// batch_mc.hpp -- the persistent batch kernel template (see
// batch_kernels.hip).  Its plain variant is instantiated in
// batch_kernels.hip and its paced variant (time term of R) in
// batch_kernels_paced.hip, each in a translation unit of its own so that
// neither affects the other's code generation.
#pragma once

#include "kernels.hpp"
#include "race_sim.hpp"

#include <utility>

namespace bbe {

// Per-wave LDS: draw table [kMaxN][64] floats, parameter records, win
// histogram, the request's start state in slot order (positions, previous
// steps, competitor ids) so that it does not occupy registers, and the
// byte table the ranking of several same-tick finishers uses.
constexpr uint32_t kWaveU = kMaxN * 256;
constexpr uint32_t kWavePar = kMaxN * 32;
constexpr uint32_t kWaveHist = 128;
constexpr uint32_t kWaveInit = kMaxN * 12;
constexpr uint32_t kWaveIds = kMaxN * 64;  // finisher ids of a tick, u8[N][64]
constexpr uint32_t kWaveBytes = kWaveU + kWavePar + kWaveHist + kWaveInit + kWaveIds;

__device__ __forceinline__ unsigned long long wave_sum_u64b(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Parked slots stop being stepped 2 at a time once every lane has parked
// them, from N = 6 on.  From N = 18 on, the copies of the tick fit in the
// registers only with ranking and parking in one pass (slots_rank_park).
// The paced variant skips 4 at a time for N = 12 .. 17 only: it spills
// from N = 18 on either way.
template <int N, bool kPaced>
constexpr int batch_skip_step() {
    if constexpr (kPaced) return (N >= 12 && N <= 17) ? 4 : 0;
    return N >= 6 ? 2 : 0;
}

template <int N, bool kPaced>
constexpr bool batch_rank_park() {
    return !kPaced && N >= 18;
}

template <int N, bool kPaced>
__device__ __forceinline__ void run_chunk(const ReqDesc& rq, const Chunk& ch, char* smem,
                                          uint32_t wbase, int lane, uint32_t k0, uint32_t k1,
                                          unsigned long long* wins_row,
                                          unsigned long long& steps) {
    const uint32_t ucol = wbase + lane * 4;
    const uint32_t icol = wbase + kWaveU + kWavePar + kWaveHist + kWaveInit + lane;
    const uint32_t pbase = wbase + kWaveU;
    uint32_t* hist = reinterpret_cast<uint32_t*>(smem + wbase + kWaveU + kWavePar);
    float* d0 = reinterpret_cast<float*>(smem + wbase + kWaveU + kWavePar + kWaveHist);
    float* s0 = d0 + kMaxN;
    uint8_t* id0 = reinterpret_cast<uint8_t*>(s0 + kMaxN);
    write_params<N>(smem, pbase, rq.rc, lane);
    if constexpr (kPaced) write_pace<N>(smem, pbase, rq.pace, lane);
    if (lane < N) {
        hist[lane] = 0u;
        d0[lane] = rq.d0[lane];
        s0[lane] = rq.s0[lane];
        id0[lane] = rq.id0[lane];
    }
    for (uint32_t g = 0; g < ch.count; g += 64) {
        const bool live = g + lane < ch.count;
        const uint32_t sim = rq.sim_begin + ch.first + g + lane;
        // re-read the start state from LDS each generation rather than
        // keeping 3N registers live across the loop
        __asm__ volatile("" ::: "memory");
        run_generation<N, kPaced ? kPaceTable : kPaceOff, batch_rank_park<N, kPaced>(),
                       batch_skip_step<N, kPaced>()>(
            smem, ucol, icol, pbase, rq.rc.L, d0, s0, id0, rq.t0, live, sim, rq.request, k0, k1,
            rq.stop_after, nullptr, hist, steps);
    }
    if (lane < N) {
        uint32_t w = hist[lane];
        if (w) atomicAdd(&wins_row[lane], (unsigned long long)w);
    }
}

// Runs a work item with the template instance of its competitor count (a
// wave-uniform switch on n).
template <bool kPaced, int... I>
__device__ __forceinline__ void run_chunk_any(int n, const ReqDesc& rq, const Chunk& ch,
                                              char* smem, uint32_t wbase, int lane, uint32_t k0,
                                              uint32_t k1, unsigned long long* wins_row,
                                              unsigned long long& steps,
                                              std::integer_sequence<int, I...>) {
    (void)((n == I + 1 ? (run_chunk<I + 1, kPaced>(rq, ch, smem, wbase, lane, k0, k1, wins_row,
                                                    steps),
                          true)
                       : false) ||
           ...);
}

// The persistent kernel: one launch serves the work items of every
// competitor count (one launch for the plain races, one for the paced);
// waves take items from one global queue, ordered longest first across the
// whole batch, so that the shortest items end the launch.  Up to 4 waves per
// workgroup (blockDim.x = 64 * waves); the register budget aims at 4 waves
// per SIMD (the largest instance fits in 128 VGPRs without spilling).
template <bool kPaced>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
    batch_mc_kernel(const BatchArgs a) {
    extern __shared__ __attribute__((aligned(16))) char smem[];  // waves * kWaveBytes
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const uint32_t wbase = wave * kWaveBytes;
    unsigned long long steps = 0ull;
    for (;;) {
        uint32_t ci = 0;
        if (lane == 0) ci = atomicAdd(a.queue, 1u);
        ci = __builtin_amdgcn_readfirstlane(ci);
        if (ci >= a.n_chunks) break;
        const Chunk ch = a.chunks[ci];
        const int n = (int)__builtin_amdgcn_readfirstlane(ch.n);
        run_chunk_any<kPaced>(n, a.reqs[ch.req], ch, smem, wbase, lane, a.k0, a.k1,
                              a.wins + (size_t)ch.req * kMaxN, steps,
                              std::make_integer_sequence<int, kMaxN>{});
    }
    steps = wave_sum_u64b(steps);
    if (a.steps && lane == 0 && steps) atomicAdd(a.steps, steps);
}

}  // namespace bbe
