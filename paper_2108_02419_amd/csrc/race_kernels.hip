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
// reduced per wave and per workgroup the same way.  kPaced selects the
// variant that evaluates the time term of R (races with some gamma != 0).
#include "kernels.hpp"
#include "race_mc.hpp"
#include "race_sim.hpp"

#include <utility>

namespace bbe {

// One lane advances one simulation until the leader reaches the target.
template <int N>
__global__ void __launch_bounds__(64) race_prefix_kernel(const PrefixArgs a) {
    constexpr uint32_t kPar = ((N * 256 + 1023) / 1024) * 1024;
    __shared__ __attribute__((aligned(1024))) char smem[kPar + 1024];
    const int lane = threadIdx.x;
    const uint32_t ucol = lane * 4;
    write_params<N>(smem, kPar, a.rc, lane);
    write_pace<N>(smem, kPar, a.pace, lane);
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
            slots_tick<N, kPaceInline>(sl, smem, ucol, kPar, a.rc.L, t, a.sim, a.request, a.k0, a.k1);
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
    // 64-bit index: n_rows * n may exceed 2^31
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t r = i / (size_t)n;
    const int c = (int)(i - r * (size_t)n);
    if (r >= (size_t)n_rows) return;
    const unsigned long long* row = wins + r * (size_t)stride;
    unsigned long long tot = 0;
    for (int k = 0; k < n; ++k) tot += row[k];
    probs[r * (size_t)stride + c] = tot ? (double)row[c] / (double)tot : 1.0 / (double)n;
}

// ---------------------------------------------------------------- launchers

template <int N>
static hipError_t launch_mc_n(const SimArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((race_mc_kernel<N, false>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int N>
static int occupancy_n() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, race_mc_kernel<N, false>, kBlock, 0) !=
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

int mc_blocks_per_cu(int n, bool paced) {
    if (paced) return mc_blocks_per_cu_paced(n);
    static int cache[kMaxN + 1] = {};
    if (!cache[n]) cache[n] = dispatch_occ(n, Seq{});
    return cache[n];
}

hipError_t launch_race_mc(const SimArgs& a, int grid, hipStream_t s) {
    if (a.pace.paced) return launch_race_mc_paced(a, grid, s);
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
