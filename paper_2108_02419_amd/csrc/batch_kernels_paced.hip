// batch_kernels_paced.hip -- the persistent batch kernel's paced variant,
// for groups holding a race whose responsiveness carries the time term
// gamma*min(t, tau) (paper Section 3, R_c(t, d)).  A translation unit of its
// own, so that the plain variant's code generation stays as it is.
#include "batch_mc.hpp"
#include "kernels.hpp"

#include <utility>

namespace bbe {

template <int N>
static hipError_t launch_batch_paced_n(const BatchArgs& a, int waves_per_block, int grid,
                                       hipStream_t s) {
    hipLaunchKernelGGL((batch_mc_kernel<N, true>), dim3(grid), dim3(64 * waves_per_block),
                       waves_per_block * kWaveBytes, s, a);
    return hipGetLastError();
}

template <int N>
static int batch_occupancy_paced_n(int waves_per_block) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_mc_kernel<N, true>,
                                                     64 * waves_per_block,
                                                     waves_per_block * kWaveBytes) != hipSuccess)
        nb = 1;
    return nb > 0 ? nb : 1;
}

template <int... I>
static hipError_t dispatch_batch_paced(int n, const BatchArgs& a, int w, int grid, hipStream_t s,
                                       std::integer_sequence<int, I...>) {
    using Fn = hipError_t (*)(const BatchArgs&, int, int, hipStream_t);
    static constexpr Fn table[] = {launch_batch_paced_n<I + 1>...};
    return table[n - 1](a, w, grid, s);
}

template <int... I>
static int dispatch_batch_occ_paced(int n, int w, std::integer_sequence<int, I...>) {
    using Fn = int (*)(int);
    static constexpr Fn table[] = {batch_occupancy_paced_n<I + 1>...};
    return table[n - 1](w);
}

hipError_t launch_batch_mc_paced(const BatchArgs& a, int n, int waves_per_block, int grid,
                                 hipStream_t s) {
    return dispatch_batch_paced(n, a, waves_per_block, grid, s,
                                std::make_integer_sequence<int, kMaxN>{});
}

int batch_blocks_per_cu_paced(int n, int waves_per_block) {
    static int cache[kMaxN + 1][5] = {};
    int& c = cache[n][waves_per_block];
    if (!c)
        c = dispatch_batch_occ_paced(n, waves_per_block, std::make_integer_sequence<int, kMaxN>{});
    return c;
}

}  // namespace bbe
