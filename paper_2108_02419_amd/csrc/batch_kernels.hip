// batch_kernels.hip -- uneven batches of Monte-Carlo requests in one
// persistent launch (the paper's dry-run workload: many bettors each asking
// for their own simulations of the race in play, Sections 3 and 6).
//
// batch_mc_kernel<N>: one persistent launch per competitor count present in
// the batch (each with the register budget of its own N), grid sized to the
// resident capacity of the GPU; every wave repeatedly takes the next work
// item of its group from a global atomic counter (one atomic per item,
// issued by lane 0), runs that item's simulations one generation of 64 at a
// time with the request's parameters in its LDS records, and flushes the
// item's wins with one 64-bit atomic per competitor.  Within a group, items
// are ordered by expected length, longest first, so the shortest work ends
// the queue.
#include "kernels.hpp"
#include "race_sim.hpp"

#include <utility>

namespace bbe {

// Per-wave LDS: draw table [kMaxN][64] floats, parameter records, win
// histogram, and the request's start state in slot order (positions,
// previous steps, competitor ids) so that it does not occupy registers.
constexpr uint32_t kWaveU = kMaxN * 256;
constexpr uint32_t kWavePar = kMaxN * 32;
constexpr uint32_t kWaveHist = 128;
constexpr uint32_t kWaveInit = kMaxN * 12;
constexpr uint32_t kWaveBytes = kWaveU + kWavePar + kWaveHist + kWaveInit;

__device__ __forceinline__ unsigned long long wave_sum_u64b(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int N>
__device__ __forceinline__ void run_chunk(const ReqDesc& rq, const Chunk& ch, char* smem,
                                          uint32_t wbase, int lane, uint32_t k0, uint32_t k1,
                                          unsigned long long* wins_row,
                                          unsigned long long& steps) {
    const uint32_t ucol = wbase + lane * 4;
    const uint32_t pbase = wbase + kWaveU;
    uint32_t* hist = reinterpret_cast<uint32_t*>(smem + wbase + kWaveU + kWavePar);
    float* d0 = reinterpret_cast<float*>(smem + wbase + kWaveU + kWavePar + kWaveHist);
    float* s0 = d0 + kMaxN;
    uint8_t* id0 = reinterpret_cast<uint8_t*>(s0 + kMaxN);
    write_params<N>(smem, pbase, rq.rc, lane);
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
        run_generation<N>(smem, ucol, pbase, rq.rc.L, d0, s0, id0, rq.t0, live, sim,
                          rq.request, k0, k1, rq.stop_after, nullptr, hist, steps);
    }
    if (lane < N) {
        uint32_t w = hist[lane];
        if (w) atomicAdd(&wins_row[lane], (unsigned long long)w);
    }
}

// Waves per SIMD the register allocation aims for: 4 where the body fits in
// 128 VGPRs without spilling, else 3.
template <int N>
constexpr int batch_waves_per_eu() {
    return 4;
}

// Persistent kernel for the work items of one competitor count; up to 4
// waves per workgroup (blockDim.x = 64 * waves).
template <int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(batch_waves_per_eu<N>())))
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
        run_chunk<N>(a.reqs[ch.req], ch, smem, wbase, lane, a.k0, a.k1,
                     a.wins + (size_t)ch.req * kMaxN, steps);
    }
    steps = wave_sum_u64b(steps);
    if (a.steps && lane == 0 && steps) atomicAdd(a.steps, steps);
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// probs[r][c] = wins[r][c] / sum_c wins[r][c] for c < n_r (1/n_r if the row
// is empty), 0 for the padding columns.
__global__ void batch_probs_kernel(const unsigned long long* __restrict__ wins,
                                   const ReqDesc* __restrict__ reqs, int n_reqs,
                                   double* __restrict__ probs) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int r = i / kMaxN, c = i - r * kMaxN;
    if (r >= n_reqs) return;
    const int n = reqs[r].rc.n;
    const unsigned long long* row = wins + (size_t)r * kMaxN;
    unsigned long long tot = 0;
    for (int k = 0; k < n; ++k) tot += row[k];
    double p = 0.0;
    if (c < n) p = tot ? (double)row[c] / (double)tot : 1.0 / (double)n;
    probs[(size_t)r * kMaxN + c] = p;
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
        rec[1] = make_float4(rq.rc.theta[c], 0.0f, 0.0f, 0.0f);
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
            slots_tick<N>(sl, smem, ucol, pbase, rq.rc.L, t, rq.prefix_sim, rq.request, k0, k1);
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

template <int N>
static hipError_t launch_batch_n(const BatchArgs& a, int waves_per_block, int grid,
                                 hipStream_t s) {
    hipLaunchKernelGGL(batch_mc_kernel<N>, dim3(grid), dim3(64 * waves_per_block),
                       waves_per_block * kWaveBytes, s, a);
    return hipGetLastError();
}

template <int N>
static int batch_occupancy_n(int waves_per_block) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_mc_kernel<N>,
                                                     64 * waves_per_block,
                                                     waves_per_block * kWaveBytes) != hipSuccess)
        nb = 1;
    return nb > 0 ? nb : 1;
}

template <int... I>
static hipError_t dispatch_batch(int n, const BatchArgs& a, int w, int grid, hipStream_t s,
                                 std::integer_sequence<int, I...>) {
    using Fn = hipError_t (*)(const BatchArgs&, int, int, hipStream_t);
    static constexpr Fn table[] = {launch_batch_n<I + 1>...};
    return table[n - 1](a, w, grid, s);
}

template <int... I>
static int dispatch_batch_occ(int n, int w, std::integer_sequence<int, I...>) {
    using Fn = int (*)(int);
    static constexpr Fn table[] = {batch_occupancy_n<I + 1>...};
    return table[n - 1](w);
}

hipError_t launch_batch_mc(const BatchArgs& a, int n, int waves_per_block, int grid,
                           hipStream_t s) {
    if (n < 1 || n > kMaxN || (waves_per_block != 1 && waves_per_block != 2 &&
                               waves_per_block != 4))
        return hipErrorInvalidValue;
    return dispatch_batch(n, a, waves_per_block, grid, s,
                          std::make_integer_sequence<int, kMaxN>{});
}

int batch_blocks_per_cu(int n, int waves_per_block) {
    static int cache[kMaxN + 1][5] = {};
    if (n < 1 || n > kMaxN || waves_per_block < 1 || waves_per_block > 4) return 1;
    int& c = cache[n][waves_per_block];
    if (!c) c = dispatch_batch_occ(n, waves_per_block, std::make_integer_sequence<int, kMaxN>{});
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
