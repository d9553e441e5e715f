// race_kernels_paced.hip -- the Monte-Carlo kernel's paced variant: the
// responsiveness carries the time term gamma*min(t, tau) (paper Section 3,
// R_c(t, d)).  A translation unit of its own, so that the plain variant's
// code generation in race_kernels.hip stays as it is.
#include "kernels.hpp"
#include "race_mc.hpp"

#include <utility>

namespace bbe {

template <int N>
static hipError_t launch_paced_n(const SimArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((race_mc_kernel<N, true>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int N>
static int occupancy_paced_n() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, race_mc_kernel<N, true>, kBlock, 0) !=
        hipSuccess)
        nb = 1;
    return nb > 0 ? nb : 1;
}

template <int... I>
static hipError_t dispatch_paced(int n, const SimArgs& a, int grid, hipStream_t s,
                                 std::integer_sequence<int, I...>) {
    using Fn = hipError_t (*)(const SimArgs&, int, hipStream_t);
    static constexpr Fn table[] = {launch_paced_n<I + 1>...};
    return table[n - 1](a, grid, s);
}

template <int... I>
static int dispatch_occ_paced(int n, std::integer_sequence<int, I...>) {
    using Fn = int (*)();
    static constexpr Fn table[] = {occupancy_paced_n<I + 1>...};
    return table[n - 1]();
}

int mc_blocks_per_cu_paced(int n) {
    static int cache[kMaxN + 1] = {};
    if (!cache[n]) cache[n] = dispatch_occ_paced(n, std::make_integer_sequence<int, kMaxN>{});
    return cache[n];
}

hipError_t launch_race_mc_paced(const SimArgs& a, int grid, hipStream_t s) {
    return dispatch_paced(a.rc.n, a, grid, s, std::make_integer_sequence<int, kMaxN>{});
}

}  // namespace bbe
