// batch_kernels.hip -- uneven batches of Monte-Carlo requests in one
// persistent launch (the paper's dry-run workload: many bettors each asking
// for their own simulations of the race in play, Sections 3 and 6).
//
// batch_mc_kernel: one persistent launch for the whole batch (a second one
// for races with a time term of R, the paced variant), grid sized to the
// resident capacity of the GPU; every wave repeatedly takes the next work
// item from a global atomic counter (one atomic per item, issued by lane
// 0), runs that item's simulations one generation of 64 at a time with the
// template instance of its competitor count and the request's parameters in
// its LDS records, and flushes the item's wins with one 64-bit atomic per
// competitor.  Items are ordered by expected work, largest first, so the
// smallest work ends the queue.
#include "batch_mc.hpp"
#include "kernels.hpp"
#include "race_sim.hpp"

#include <utility>

namespace bbe {

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// probs[r][c] = wins[r][c] / sum_c wins[r][c] for c < n_r (1/n_r if the row
// is empty), 0 for the padding columns.
__global__ void batch_probs_kernel(const unsigned long long* __restrict__ wins,
                                   const ReqDesc* __restrict__ reqs, int n_reqs,
                                   double* __restrict__ probs) {
    // 64-bit index: n_reqs * 20 may exceed 2^31
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t r = i / kMaxN;
    const int c = (int)(i - r * kMaxN);
    if (r >= (size_t)n_reqs) return;
    const int n = reqs[r].rc.n;
    const unsigned long long* row = wins + r * kMaxN;
    unsigned long long tot = 0;
    for (int k = 0; k < n; ++k) tot += row[k];
    double p = 0.0;
    if (c < n) p = tot ? (double)row[c] / (double)tot : 1.0 / (double)n;
    probs[r * kMaxN + c] = p;
}

// In-play states for a batch: lane i advances simulation prefix_sim of
// request i until its leader reaches the target.  Each lane has its own
// race, so each lane has its own parameter records.
constexpr uint32_t kPfxWaveU = kMaxN * 256;
constexpr uint32_t kPfxLanePar = kMaxN * 32;

template <int N>
__device__ void run_prefix_lane(const ReqDesc& rq, char* smem, uint32_t ucol, uint32_t pbase,
                                int lane, uint32_t k0, uint32_t k1, uint32_t* tick_out,
                                float* pos_out, float* prev_out) {
    for (int c = 0; c < N; ++c) {
        float4* rec = reinterpret_cast<float4*>(smem + pbase + c * 32);
        rec[0] = make_float4(rq.rc.elo[c], rq.rc.espan16[c], rq.rc.alpha[c], rq.rc.beta[c]);
        rec[1] = make_float4(rq.rc.theta[c], rq.pace.gamma[c], rq.pace.tau[c], 0.0f);
    }
    Slots<N> sl;
    slots_reset<N>(sl, rq.d0, rq.s0, rq.id0, pbase);
    uint32_t t = rq.t0;
    bool ok = true;
    for (;;) {
        if (sl.d[N - 1] >= rq.target) break;
        if (t - rq.t0 >= kTickLimit) {
            ok = false;
            break;
        }
        uint32_t cross =
            slots_tick<N, kPaceInline>(sl, smem, ucol, pbase, rq.rc.L, t, rq.prefix_sim, rq.request, k0,
                                k1);
        t += 1;
        if (cross) {
            ok = false;
            break;
        }
        slots_restore<N>(sl);
    }
    *tick_out = ok ? t : 0xFFFFFFFFu;
    for (int c = 0; c < kMaxN; ++c) {
        pos_out[c] = 0.0f;
        prev_out[c] = 0.0f;
    }
    slots_store<N>(sl, pbase, pos_out, prev_out);
}

__global__ void __launch_bounds__(64) prefix_batch_kernel(const ReqDesc* __restrict__ reqs,
                                                          int n_reqs, uint32_t k0, uint32_t k1,
                                                          uint32_t* tick_out, float* pos_out,
                                                          float* prev_out) {
    __shared__ __attribute__((aligned(16))) char smem[kPfxWaveU + 64 * kPfxLanePar];
    const int lane = threadIdx.x;
    const int i = blockIdx.x * 64 + lane;
    if (i >= n_reqs) return;
    const ReqDesc& rq = reqs[i];
    const uint32_t ucol = lane * 4;
    const uint32_t pbase = kPfxWaveU + lane * kPfxLanePar;
    float* po = pos_out + (size_t)i * kMaxN;
    float* pv = prev_out + (size_t)i * kMaxN;
    switch (rq.rc.n) {
#define BBE_CASE(n) \
    case n:         \
        run_prefix_lane<n>(rq, smem, ucol, pbase, lane, k0, k1, tick_out + i, po, pv); \
        break;
        BBE_CASE(1) BBE_CASE(2) BBE_CASE(3) BBE_CASE(4) BBE_CASE(5)
        BBE_CASE(6) BBE_CASE(7) BBE_CASE(8) BBE_CASE(9) BBE_CASE(10)
        BBE_CASE(11) BBE_CASE(12) BBE_CASE(13) BBE_CASE(14) BBE_CASE(15)
        BBE_CASE(16) BBE_CASE(17) BBE_CASE(18) BBE_CASE(19) BBE_CASE(20)
#undef BBE_CASE
        default:
            tick_out[i] = 0xFFFFFFFFu;
            break;
    }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_batch_mc(const BatchArgs& a, int waves_per_block, int grid, bool paced,
                           hipStream_t s) {
    if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
        return hipErrorInvalidValue;
    if (paced) return launch_batch_mc_paced(a, waves_per_block, grid, s);
    hipLaunchKernelGGL((batch_mc_kernel<false>), dim3(grid), dim3(64 * waves_per_block),
                       waves_per_block * kWaveBytes, s, a);
    return hipGetLastError();
}

int batch_blocks_per_cu(int waves_per_block, bool paced) {
    if (waves_per_block < 1 || waves_per_block > 4) return 1;
    if (paced) return batch_blocks_per_cu_paced(waves_per_block);
    static int cache[5] = {};
    int& c = cache[waves_per_block];
    if (!c) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_mc_kernel<false>,
                                                         64 * waves_per_block,
                                                         waves_per_block * kWaveBytes) !=
                hipSuccess ||
            nb < 1)
            nb = 1;
        c = nb;
    }
    return c;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_batch_probs(const unsigned long long* wins, const ReqDesc* reqs, int n_reqs,
                              double* probs, hipStream_t s) {
    long total = (long)n_reqs * kMaxN;
    hipLaunchKernelGGL(batch_probs_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       wins, reqs, n_reqs, probs);
    return hipGetLastError();
}

hipError_t launch_prefix_batch(const ReqDesc* reqs, int n_reqs, uint32_t k0, uint32_t k1,
                               uint32_t* tick_out, float* pos_out, float* prev_out,
                               hipStream_t s) {
    if (n_reqs <= 0) return hipSuccess;
    hipLaunchKernelGGL(prefix_batch_kernel, dim3((n_reqs + 63) / 64), dim3(64), 0, s, reqs, n_reqs,
                       k0, k1, tick_out, pos_out, prev_out);
    return hipGetLastError();
}

}  // namespace bbe
