// race_mc.hpp -- the Monte-Carlo kernel template (see race_kernels.hip).
// Its plain variant is instantiated in race_kernels.hip and its paced
// variant (time term of R) in race_kernels_paced.hip, each in a translation
// unit of its own so that neither affects the other's code generation.
#pragma once

#include "kernels.hpp"
#include "race_sim.hpp"

namespace bbe {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;

// Parameter records: one table for the workgroup, or one per wave in the
// paced variant (each wave writes its own tick's time terms into them).
template <int N, bool kPaced = false>
struct BlockLds {
    static constexpr uint32_t kU = 0;                                      // [wave] u tables
    static constexpr uint32_t kPar = ((kWaves * N * 256 + 1023) / 1024) * 1024;  // records
    static constexpr uint32_t kParBytes = kPaced ? ((kWaves * N * 32 + 1023) / 1024) * 1024 : 1024;
    static constexpr uint32_t kWins = kPar + kParBytes;                   // u32[N]
    static constexpr uint32_t kSteps = kWins + 128;                        // u64
    static constexpr uint32_t kInit = kSteps + 16;  // start state: d0, s0 (f32[N]), id0 (u8[N])
    static constexpr uint32_t kIds = kInit + kMaxN * 12;  // [wave] finisher ids, u8[N][64]
    // [wave] finish orders of the wave's current generation, u8[64][N]
    static constexpr uint32_t kOrd = kIds + kWaves * N * 64;
    static constexpr uint32_t kBytes = kOrd + kWaves * 64 * N;
};

// Copies `bytes` bytes of a wave's LDS order table to global memory with
// coalesced 4-byte stores (byte stores for an unaligned destination and
// for the tail).
__device__ __forceinline__ void flush_orders(const char* tab, uint8_t* __restrict__ dst,
                                             uint32_t bytes, int lane) {
    uint32_t done = 0;
    if ((reinterpret_cast<uintptr_t>(dst) & 3u) == 0) {
        const uint32_t words = bytes >> 2;
        for (uint32_t w = lane; w < words; w += 64)
            reinterpret_cast<uint32_t*>(dst)[w] = reinterpret_cast<const uint32_t*>(tab)[w];
        done = words << 2;
    }
    for (uint32_t i = done + lane; i < bytes; i += 64) dst[i] = (uint8_t)tab[i];
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Waves per SIMD the register allocation aims for (4: the body fits in 128
// VGPRs without spilling).
template <int N, bool kPaced = false>
constexpr int mc_waves_per_eu() {
    return 4;
}

// Parked slots stop being stepped 2 at a time once every lane has parked
// them (from N = 6 on; smaller races gain too little for the extra copies
// of the tick).
template <int N>
constexpr int mc_skip_step() {
    return N >= 6 ? 2 : 0;
}

template <int N, bool kPaced>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(mc_waves_per_eu<N, kPaced>()))) race_mc_kernel(const SimArgs a) {
    using Lay = BlockLds<N, kPaced>;
    __shared__ __attribute__((aligned(1024))) char smem[Lay::kBytes];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const uint32_t ucol = Lay::kU + wave * (N * 256) + lane * 4;
    const uint32_t icol = Lay::kIds + wave * (N * 64) + lane;
    // plain: one record table for the workgroup (every wave simulates the
    // same race), at a compile-time offset; paced: one table per wave
    const uint32_t pbase =
        kPaced ? Lay::kPar + (uint32_t)__builtin_amdgcn_readfirstlane(wave) * (N * 32u)
               : Lay::kPar;
    uint32_t* s_wins = reinterpret_cast<uint32_t*>(smem + Lay::kWins);
    unsigned long long* s_steps = reinterpret_cast<unsigned long long*>(smem + Lay::kSteps);

    float* s_d0 = reinterpret_cast<float*>(smem + Lay::kInit);
    float* s_s0 = s_d0 + kMaxN;
    uint8_t* s_id0 = reinterpret_cast<uint8_t*>(s_s0 + kMaxN);
    if constexpr (kPaced) {
        write_params<N>(smem, pbase, a.rc, lane);
        write_pace<N>(smem, pbase, a.pace, lane);
    } else {
        write_params<N>(smem, pbase, a.rc, (int)threadIdx.x);
    }
    if (threadIdx.x < N) {
        s_wins[threadIdx.x] = 0u;
        s_d0[threadIdx.x] = a.d0[threadIdx.x];
        s_s0[threadIdx.x] = a.s0[threadIdx.x];
        s_id0[threadIdx.x] = a.id0[threadIdx.x];
    }
    if (threadIdx.x == 0) *s_steps = 0ull;
    __syncthreads();

    const float L = a.rc.L;
    const uint64_t wave_stride = (uint64_t)gridDim.x * kWaves * 64;
    unsigned long long steps = 0ull;

    // finish orders go to the wave's LDS table during a generation and to
    // HBM in one coalesced flush at its end
    char* otab = smem + Lay::kOrd + wave * (64 * N);
    for (uint64_t base = ((uint64_t)blockIdx.x * kWaves + wave) * 64; base < a.n_sims;
         base += wave_stride) {
        const uint64_t j = base + lane;
        const bool live = j < a.n_sims;
        uint8_t* row = (a.orders && live) ? reinterpret_cast<uint8_t*>(otab + lane * N) : nullptr;
        // re-read the start state from LDS each generation rather than
        // keeping it live (in registers) across the loop
        __asm__ volatile("" ::: "memory");
        run_generation<N, kPaced ? kPaceTable : kPaceOff, true, mc_skip_step<N>()>(
            smem, ucol, icol, pbase, L, s_d0, s_s0, s_id0, a.t0, live, a.sim_begin + (uint32_t)j,
            a.request, a.k0, a.k1, a.stop_after, row, s_wins, steps);
        if (a.orders) {
            // the wave's LDS operations complete in order; keep the compiler
            // from moving the table's reads above the lanes' writes (and the
            // next generation's writes above these reads)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const uint64_t rows = a.n_sims - base < 64 ? a.n_sims - base : 64;
            flush_orders(otab, a.orders + base * N, (uint32_t)(rows * N), lane);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }

    steps = wave_sum_u64(steps);
    if (lane == 0) atomicAdd(s_steps, steps);
    __syncthreads();
    if (a.wins && threadIdx.x < N) {
        uint32_t w = s_wins[threadIdx.x];
        if (w) atomicAdd(&a.wins[threadIdx.x], (unsigned long long)w);
    }
    if (a.steps && threadIdx.x == 0) atomicAdd(a.steps, *s_steps);
}

}  // namespace bbe
