// order_kernels.hip -- tallies over finish orders (paper Section 6: the
// finish orders of repeated seeded runs estimate a probability mass function
// over the n! possible orders; Section 3: a bettor's view of a race is a set
// of such frequentist estimates).
//
// rank_counts_kernel: counts[c][r] += 1 for every simulation in which
// competitor c finished at rank r (finish-position / place probabilities).
// order_pmf_kernel (n <= 7): counts[lexicographic rank of the order] += 1
// for every simulation whose order is complete.
// Both privatise the tally in LDS (u32 per workgroup) and flush it with one
// 64-bit atomic per non-zero bin; rows are read one simulation per thread.
#include "kernels.hpp"

namespace bbe {

constexpr int kOrdBlock = 256;

__global__ void __launch_bounds__(kOrdBlock)
    rank_counts_kernel(const uint8_t* __restrict__ orders, uint32_t n_sims, int n,
                       unsigned long long* __restrict__ counts) {
    __shared__ uint32_t hist[kMaxN * kMaxN];
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_sims; s += stride) {
        const uint8_t* row = orders + s * (uint64_t)n;
        for (int r = 0; r < n; ++r) {
            const int c = row[r];
            if (c < n) atomicAdd(&hist[c * n + r], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n * n; i += blockDim.x)
        if (hist[i]) atomicAdd(&counts[i], (unsigned long long)hist[i]);
}

// Lexicographic rank of a complete order (its Lehmer code read in the
// factorial number system); -1 if some rank is unfilled (0xFF) or holds an
// index >= n.
__device__ __forceinline__ int lex_rank(const uint8_t* row, int n) {
    int rank = 0;
    for (int i = 0; i < n; ++i) {
        const int v = row[i];
        if (v >= n) return -1;
        int smaller = 0;
        for (int j = i + 1; j < n; ++j) smaller += (row[j] < v) ? 1 : 0;
        rank = rank * (n - i) + smaller;
    }
    return rank;
}

__global__ void __launch_bounds__(kOrdBlock)
    order_pmf_kernel(const uint8_t* __restrict__ orders, uint32_t n_sims, int n, int n_fact,
                     unsigned long long* __restrict__ counts) {
    extern __shared__ uint32_t bins[];  // [n!]
    for (int i = threadIdx.x; i < n_fact; i += blockDim.x) bins[i] = 0u;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_sims; s += stride) {
        const int k = lex_rank(orders + s * (uint64_t)n, n);
        if (k >= 0) atomicAdd(&bins[k], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_fact; i += blockDim.x)
        if (bins[i]) atomicAdd(&counts[i], (unsigned long long)bins[i]);
}

static int order_grid(uint32_t n_sims) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint64_t want = ((uint64_t)n_sims + kOrdBlock - 1) / kOrdBlock;
    const uint64_t cap = (uint64_t)cus * 8;
    return (int)(want < 1 ? 1 : (want < cap ? want : cap));
}

hipError_t launch_rank_counts(const uint8_t* orders, uint32_t n_sims, int n,
                              unsigned long long* counts, hipStream_t s) {
    hipError_t e = launch_zero_u64(counts, n * n, s);
    if (e != hipSuccess || n_sims == 0) return e;
    hipLaunchKernelGGL(rank_counts_kernel, dim3(order_grid(n_sims)), dim3(kOrdBlock), 0, s,
                       orders, n_sims, n, counts);
    return hipGetLastError();
}

hipError_t launch_order_pmf(const uint8_t* orders, uint32_t n_sims, int n, int n_fact,
                            unsigned long long* counts, hipStream_t s) {
    hipError_t e = launch_zero_u64(counts, n_fact, s);
    if (e != hipSuccess || n_sims == 0) return e;
    hipLaunchKernelGGL(order_pmf_kernel, dim3(order_grid(n_sims)), dim3(kOrdBlock),
                       n_fact * sizeof(uint32_t), s, orders, n_sims, n, n_fact, counts);
    return hipGetLastError();
}

}  // namespace bbe
