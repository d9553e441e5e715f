// race_kernels.hip -- gfx950 kernels of the race Monte-Carlo (paper Section 3,
// Eq. 1; Section 6: repeated seeded runs estimate the finish-order PMF).
//
// race_mc_kernel<N>: each wave runs "generations" of 64 simulations, one
// per lane, all lanes at the same tick (the draws' counter tick is then
// wave-uniform); a generation ends when all its lanes have finished, and the
// wave moves on to the next 64 simulation indices of its grid stride.  Wins
// are counted in an LDS histogram (one LDS atomic per finished simulation)
// and flushed with one 64-bit global atomic per competitor per workgroup;
// competitor-steps are summed per simulation from the finishing ticks and
// reduced per wave and per workgroup the same way.
#include "kernels.hpp"
#include "race_sim.hpp"

#include <utility>

namespace bbe {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;

template <int N>
struct BlockLds {
    static constexpr uint32_t kU = 0;                                      // [wave] u tables
    static constexpr uint32_t kPar = ((kWaves * N * 256 + 1023) / 1024) * 1024;  // records
    static constexpr uint32_t kWins = kPar + 1024;                        // u32[N]
    static constexpr uint32_t kSteps = kWins + 128;                        // u64
    static constexpr uint32_t kInit = kSteps + 16;  // start state: d0, s0 (f32[N]), id0 (u8[N])
    static constexpr uint32_t kBytes = kInit + kMaxN * 12;
};

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Waves per SIMD the register allocation aims for: 4 where the body fits in
// 128 VGPRs without spilling, else 3.
template <int N>
constexpr int mc_waves_per_eu() {
    return 4;
}

template <int N>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(mc_waves_per_eu<N>()))) race_mc_kernel(const SimArgs a) {
    using Lay = BlockLds<N>;
    __shared__ __attribute__((aligned(1024))) char smem[Lay::kBytes];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const uint32_t ucol = Lay::kU + wave * (N * 256) + lane * 4;
    // one record table for the workgroup (every wave simulates the same
    // race), at a compile-time offset
    const uint32_t pbase = Lay::kPar;
    uint32_t* s_wins = reinterpret_cast<uint32_t*>(smem + Lay::kWins);
    unsigned long long* s_steps = reinterpret_cast<unsigned long long*>(smem + Lay::kSteps);

    float* s_d0 = reinterpret_cast<float*>(smem + Lay::kInit);
    float* s_s0 = s_d0 + kMaxN;
    uint8_t* s_id0 = reinterpret_cast<uint8_t*>(s_s0 + kMaxN);
    write_params<N>(smem, pbase, a.rc, (int)threadIdx.x);
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

    for (uint64_t base = ((uint64_t)blockIdx.x * kWaves + wave) * 64; base < a.n_sims;
         base += wave_stride) {
        const uint64_t j = base + lane;
        const bool live = j < a.n_sims;
        uint8_t* row = (a.orders && live) ? a.orders + j * N : nullptr;
        // re-read the start state from LDS each generation rather than
        // keeping it live (in registers) across the loop
        __asm__ volatile("" ::: "memory");
        run_generation<N>(smem, ucol, pbase, L, s_d0, s_s0, s_id0, a.t0, live,
                          a.sim_begin + (uint32_t)j, a.request, a.k0, a.k1, a.stop_after, row,
                          s_wins, steps);
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

// One lane advances one simulation until the leader reaches the target.
template <int N>
__global__ void __launch_bounds__(64) race_prefix_kernel(const PrefixArgs a) {
    constexpr uint32_t kPar = ((N * 256 + 1023) / 1024) * 1024;
    __shared__ __attribute__((aligned(1024))) char smem[kPar + 1024];
    const int lane = threadIdx.x;
    const uint32_t ucol = lane * 4;
    write_params<N>(smem, kPar, a.rc, lane);
    __syncthreads();
    if (lane != 0) return;
    Slots<N> sl;
    slots_reset<N>(sl, a.d0, a.s0, a.id0, kPar);
    uint32_t t = a.t0;
    bool ok = true;
    for (;;) {
        if (sl.d[N - 1] >= a.target) break;  // slots ascending: the leader is last
        if (t - a.t0 >= a.max_ticks) break;
        if (t - a.t0 >= kTickLimit) {
            ok = false;
            break;
        }
        uint32_t cross =
            slots_tick<N>(sl, smem, ucol, kPar, a.rc.L, t, a.sim, a.request, a.k0, a.k1);
        t += 1;
        if (cross) {
            ok = false;
            break;
        }
        slots_restore<N>(sl);
    }
    *a.tick_out = ok ? t : 0xFFFFFFFFu;
    slots_store<N>(sl, kPar, a.pos_out, a.prev_out);
}

__global__ void zero_u64_kernel(unsigned long long* __restrict__ p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void win_probs_kernel(const unsigned long long* __restrict__ wins, int n_rows, int n,
                                 int stride, double* __restrict__ probs) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int r = i / n, c = i - r * n;
    if (r >= n_rows) return;
    const unsigned long long* row = wins + (size_t)r * stride;
    unsigned long long tot = 0;
    for (int k = 0; k < n; ++k) tot += row[k];
    probs[(size_t)r * stride + c] = tot ? (double)row[c] / (double)tot : 1.0 / (double)n;
}

// ---------------------------------------------------------------- launchers

template <int N>
static hipError_t launch_mc_n(const SimArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(race_mc_kernel<N>, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int N>
static int occupancy_n() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, race_mc_kernel<N>, kBlock, 0) !=
        hipSuccess)
        nb = 1;
    return nb > 0 ? nb : 1;
}

template <int N>
static hipError_t launch_prefix_n(const PrefixArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(race_prefix_kernel<N>, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int... I>
static hipError_t dispatch_mc(int n, const SimArgs& a, int grid, hipStream_t s,
                              std::integer_sequence<int, I...>) {
    using Fn = hipError_t (*)(const SimArgs&, int, hipStream_t);
    static constexpr Fn table[] = {launch_mc_n<I + 1>...};
    return table[n - 1](a, grid, s);
}

template <int... I>
static int dispatch_occ(int n, std::integer_sequence<int, I...>) {
    using Fn = int (*)();
    static constexpr Fn table[] = {occupancy_n<I + 1>...};
    return table[n - 1]();
}

template <int... I>
static hipError_t dispatch_prefix(int n, const PrefixArgs& a, hipStream_t s,
                                  std::integer_sequence<int, I...>) {
    using Fn = hipError_t (*)(const PrefixArgs&, hipStream_t);
    static constexpr Fn table[] = {launch_prefix_n<I + 1>...};
    return table[n - 1](a, s);
}

using Seq = std::make_integer_sequence<int, kMaxN>;

int mc_block_size() { return kBlock; }

int mc_blocks_per_cu(int n) {
    static int cache[kMaxN + 1] = {0};
    if (!cache[n]) cache[n] = dispatch_occ(n, Seq{});
    return cache[n];
}

hipError_t launch_race_mc(const SimArgs& a, int grid, hipStream_t s) {
    return dispatch_mc(a.rc.n, a, grid, s, Seq{});
}

hipError_t launch_race_prefix(const PrefixArgs& a, hipStream_t s) {
    return dispatch_prefix(a.rc.n, a, s, Seq{});
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_win_probs(const unsigned long long* wins, int n_rows, int n, int stride,
                            double* probs, hipStream_t s) {
    long total = (long)n_rows * n;
    hipLaunchKernelGGL(win_probs_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       wins, n_rows, n, stride, probs);
    return hipGetLastError();
}

}  // namespace bbe
