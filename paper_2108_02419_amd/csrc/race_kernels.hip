// race_kernels.hip -- gfx950 kernels of the race Monte-Carlo (paper Section 3,
// Eq. 1; Section 6: repeated seeded runs estimate the finish-order PMF).
//
// race_mc_kernel<N>: one simulation per lane.  When a lane's simulation ends
// it takes the next simulation index (lane id + k * grid size), so lanes
// stay busy although simulations end at different ticks.  Wins are counted
// in an LDS histogram (one LDS atomic per finished simulation) and flushed
// with one 64-bit global atomic per competitor per workgroup; competitor-
// steps are reduced per wave and per workgroup the same way.
#include "kernels.hpp"
#include "race_sim.hpp"

#include <utility>

namespace bbe {

constexpr int kBlock = 256;

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int N>
__global__ void __launch_bounds__(kBlock) race_mc_kernel(const SimArgs a) {
    __shared__ uint32_t s_wins[N];
    __shared__ unsigned long long s_steps;
    if (threadIdx.x < N) s_wins[threadIdx.x] = 0u;
    if (threadIdx.x == 0) s_steps = 0ull;
    __syncthreads();

    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long steps = 0ull;

    LaneState<N> st;
    lane_reset<N>(st, a.d0, a.s0, a.t0);
    bool active = j < a.n_sims;
    while (active) {
        uint8_t* row = a.orders ? a.orders + j * N : nullptr;
        steps += (unsigned)lane_tick<N>(st, a.rc, a.sim_begin + (uint32_t)j, a.request, a.k0, a.k1,
                                        row);
        if (st.nfin >= a.stop_after || st.t - a.t0 >= kTickLimit) {
            if (st.winner >= 0) atomicAdd(&s_wins[st.winner], 1u);
            if (row)
                for (int r = st.nfin; r < N; ++r) row[r] = 0xFF;
            j += stride;
            active = j < a.n_sims;
            lane_reset<N>(st, a.d0, a.s0, a.t0);
        }
    }

    steps = wave_sum_u64(steps);
    if ((threadIdx.x & 63) == 0) atomicAdd(&s_steps, steps);
    __syncthreads();
    if (a.wins && threadIdx.x < N) {
        uint32_t w = s_wins[threadIdx.x];
        if (w) atomicAdd(&a.wins[threadIdx.x], (unsigned long long)w);
    }
    if (a.steps && threadIdx.x == 0) atomicAdd(a.steps, s_steps);
}

// One lane advances one simulation until the leader reaches the target.
template <int N>
__global__ void __launch_bounds__(64) race_prefix_kernel(const PrefixArgs a) {
    if (threadIdx.x != 0) return;
    LaneState<N> st;
    lane_reset<N>(st, a.d0, a.s0, a.t0);
    bool ok = true;
    for (;;) {
        float lead = st.d[0];
#pragma unroll
        for (int c = 1; c < N; ++c) lead = fmaxf(lead, st.d[c]);
        if (lead >= a.target) break;
        if (st.t - a.t0 >= kTickLimit) {
            ok = false;
            break;
        }
        lane_tick<N>(st, a.rc, a.sim, a.request, a.k0, a.k1, nullptr);
        if (st.nfin > 0) {
            ok = false;
            break;
        }
    }
    *a.tick_out = ok ? st.t : 0xFFFFFFFFu;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        a.pos_out[c] = st.d[c];
        a.prev_out[c] = st.s[c];
    }
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
