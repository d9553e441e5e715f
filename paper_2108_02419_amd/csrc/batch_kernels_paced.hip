// batch_kernels_paced.hip -- the persistent batch kernel's paced variant,
// for the work items of races whose responsiveness carries the time term
// gamma*min(t, tau) (paper Section 3, R_c(t, d)).  A translation unit of its
// own, so that the plain variant's code generation stays as it is.
#include "batch_mc.hpp"
#include "kernels.hpp"

#include <utility>

namespace bbe {

hipError_t launch_batch_mc_paced(const BatchArgs& a, int waves_per_block, int grid,
                                 hipStream_t s) {
    hipLaunchKernelGGL((batch_mc_kernel<true>), dim3(grid), dim3(64 * waves_per_block),
                       waves_per_block * kWaveBytes, s, a);
    return hipGetLastError();
}

int batch_blocks_per_cu_paced(int waves_per_block) {
    static int cache[5] = {};
    int& c = cache[waves_per_block];
    if (!c) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_mc_kernel<true>,
                                                         64 * waves_per_block,
                                                         waves_per_block * kWaveBytes) !=
                hipSuccess ||
            nb < 1)
            nb = 1;
        c = nb;
    }
    return c;
}

}  // namespace bbe
