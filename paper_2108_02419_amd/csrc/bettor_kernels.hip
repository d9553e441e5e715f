// bettor_kernels.hip -- the in-play side of the model on gfx950: the trace
// of the race that bettors watch (paper Section 3: the race state is the
// vector of positions, advanced tick by tick by Eq. 1) and the views of the
// cheap bettor rules of Section 5 (LinEx, LW, UD, ZI) over that trace.
//
// race_trace_kernel<N>: one lane advances one simulation with the same
// slot code as the Monte-Carlo kernels and writes the positions after every
// tick, stopping before the first tick in which a competitor reaches the
// line (the winner market closes then).
//
// bettor_views_kernel: one thread per bettor, a block of 256 bettors over
// chunks of kViewRowsPerBlock trace rows.  The bettors are stored grouped by
// kind, so nearly every wave runs a single rule.  Per chunk the block stages
// the chunk's rows in LDS -- with up to kViewWindow rows of history before
// them where the block holds LinEx bettors -- one thread per row finds its
// leader and runner-up, and every thread forms its views:
//   LW     the leader (ties to the lowest index);
//   UD     the runner-up while fl(x_P1 - x_P2) < D, else the leader;
//   LinEx  over a window w = min(N, r) ticks, the competitor with the least
//          remaining distance fl(L - x) per displacement fl(x - x_back),
//          among those that moved; the two ratios are compared exactly by
//          cross-multiplying in double precision (products of two floats
//          are exact there); with w = 0 or nobody moving, the leader;
//   ZI     a uniform competitor, floor(w * n / 2^32) for the first word w
//          of the Philox block with counter (t, bettor, ~0, ~0).
// Views are tallied per row in an LDS histogram and flushed with one
// global atomic per competitor and row per block.
#include "bettors.hpp"
#include "race_sim.hpp"

#include <utility>

namespace bbe {

template <int N>
__device__ __forceinline__ void slots_store_pos(const Slots<N>& sl, uint32_t pbase,
                                                float* __restrict__ row) {
#pragma unroll
    for (int k = 0; k < N; ++k) row[(sl.rec[k] - pbase) >> 5] = sl.d[k];
}

template <int N>
__global__ void __launch_bounds__(64) race_trace_kernel(const TraceArgs a) {
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
    slots_store_pos<N>(sl, kPar, a.trace);
    uint32_t rows = 1;
    uint32_t t = a.t0;
    // at most max_rows - 1 <= 2^20 ticks
    while (rows < a.max_rows) {
        const uint32_t cross =
            slots_tick<N, kPaceInline>(sl, smem, ucol, kPar, a.rc.L, t, a.sim, a.request, a.k0, a.k1);
        if (cross) break;
        t += 1;
        slots_restore<N>(sl);
        slots_store_pos<N>(sl, kPar, a.trace + (size_t)rows * N);
        ++rows;
    }
    *a.rows_out = rows;
}

// Leader and runner-up of one row (ties to the lowest index) and the
// distance between them; p2 = p1 and gap = 0 when n = 1.
__device__ __forceinline__ void row_leaders(const float* __restrict__ x, int n, int& p1, int& p2,
                                            float& gap) {
    float xr[kMaxN];
#pragma unroll
    for (int c = 0; c < kMaxN; ++c) xr[c] = c < n ? x[c] : 0.0f;
    p1 = 0;
    float b1 = xr[0];
#pragma unroll
    for (int c = 1; c < kMaxN; ++c)
        if (c < n && xr[c] > b1) {
            b1 = xr[c];
            p1 = c;
        }
    p2 = -1;
    float b2 = 0.0f;
#pragma unroll
    for (int c = 0; c < kMaxN; ++c)
        if (c < n && c != p1 && (p2 < 0 || xr[c] > b2)) {
            b2 = xr[c];
            p2 = c;
        }
    gap = p2 < 0 ? 0.0f : b1 - b2;
    if (p2 < 0) p2 = p1;
}

// LinEx pick over rows x (now) and back (w ticks earlier): least
// fl(L - x_c) / fl(x_c - back_c) among positive displacements, compared
// exactly; -1 if nobody moved.
__device__ __forceinline__ int linex_scan(const float* __restrict__ x,
                                          const float* __restrict__ back, int n, float L) {
    float xr[kMaxN], br[kMaxN];
#pragma unroll
    for (int c = 0; c < kMaxN; ++c) {
        xr[c] = c < n ? x[c] : 0.0f;
        br[c] = c < n ? back[c] : 0.0f;
    }
    int best = -1;
    float bre = 0.0f, bdi = 1.0f;
#pragma unroll
    for (int c = 0; c < kMaxN; ++c) {
        const float disp = xr[c] - br[c];
        const float rem = L - xr[c];
        const bool better = c < n && disp > 0.0f &&
                            (best < 0 || (double)rem * (double)bdi < (double)bre * (double)disp);
        best = better ? c : best;
        bre = better ? rem : bre;
        bdi = better ? disp : bdi;
    }
    return best;
}

__global__ void __launch_bounds__(kViewBlock) bettor_views_kernel(const ViewArgs a) {
    constexpr int R = kViewRowsPerBlock;
    __shared__ float s_rows[(kViewWindow + R) * kMaxN];
    __shared__ uint32_t s_cnt[R * kMaxN];
    __shared__ int s_p1[R], s_p2[R];
    __shared__ float s_gap[R];
    const int n = a.n;
    const uint32_t j = blockIdx.x * kViewBlock + threadIdx.x;
    const bool have = j < a.n_bettors;
    const uint8_t kind = have ? a.kind[j] : (uint8_t)kLW;
    const float param = have ? a.param[j] : 0.0f;
    const uint32_t id = have ? a.id[j] : 0u;
    // bettors are grouped by kind with LinEx last: the block holds LinEx
    // bettors iff its last one is
    const uint32_t last = min(blockIdx.x * kViewBlock + kViewBlock, a.n_bettors) - 1;
    const bool block_linex = a.kind[last] == kLinEx;

    for (uint32_t i0 = blockIdx.y * R; i0 < a.n_eval; i0 += gridDim.y * R) {
        const int nr = (int)min((uint32_t)R, a.n_eval - i0);
        const uint32_t r0 = a.first_row + i0;
        // rows lo .. r0 + nr - 1 in LDS: the chunk, and for LinEx blocks up
        // to kViewWindow rows of history before it
        const uint32_t lo = block_linex ? (r0 > (uint32_t)kViewWindow ? r0 - kViewWindow : 0u) : r0;
        const int nstage = (int)(r0 - lo + nr) * n;
        const float* __restrict__ src = a.trace + (size_t)lo * n;
        for (int k = threadIdx.x; k < nstage; k += kViewBlock) s_rows[k] = src[k];
        if ((int)threadIdx.x < nr * n) s_cnt[threadIdx.x] = 0u;
        __syncthreads();
        if ((int)threadIdx.x < nr) {
            int p1, p2;
            float gap;
            row_leaders(s_rows + (size_t)(r0 - lo + threadIdx.x) * n, n, p1, p2, gap);
            s_p1[threadIdx.x] = p1;
            s_p2[threadIdx.x] = p2;
            s_gap[threadIdx.x] = gap;
        }
        __syncthreads();

        for (int ii = 0; ii < nr; ++ii) {
            const uint32_t r = r0 + ii;
            int v = s_p1[ii];
            if (kind == kZI) {
                const U4 w = philox4x32_10(a.t0 + r, id, 0xFFFFFFFFu, 0xFFFFFFFFu, a.k0, a.k1);
                v = (int)(((uint64_t)w.x * (uint32_t)n) >> 32);
            } else if (kind == kUD) {
                if (n > 1 && s_gap[ii] < param) v = s_p2[ii];
            } else if (kind == kLinEx) {
                const uint32_t w = min((uint32_t)param, r);
                if (w > 0) {
                    const float* x = s_rows + (size_t)(r - lo) * n;
                    const uint32_t rb = r - w;
                    const int best = rb >= lo
                                         ? linex_scan(x, s_rows + (size_t)(rb - lo) * n, n, a.L)
                                         : linex_scan(x, a.trace + (size_t)rb * n, n, a.L);
                    if (best >= 0) v = best;
                }
            }
            if (have) {
                if (a.views) a.views[(size_t)(i0 + ii) * a.n_bettors + id] = (uint8_t)v;
                atomicAdd(&s_cnt[ii * n + v], 1u);
            }
        }
        __syncthreads();
        if (a.counts && (int)threadIdx.x < nr * n && s_cnt[threadIdx.x])
            atomicAdd(&a.counts[(size_t)i0 * n + threadIdx.x], s_cnt[threadIdx.x]);
    }
}

// RP(d) views: the competitor with the most dry-run wins (lowest index on
// ties), one thread per bettor row of the win-count matrix.
__global__ void __launch_bounds__(kViewBlock)
    rp_views_kernel(const unsigned long long* __restrict__ wins, uint32_t n_bettors, int n,
                    int stride, uint8_t* __restrict__ views, uint32_t* __restrict__ counts) {
    __shared__ uint32_t s_cnt[kMaxN];
    if ((int)threadIdx.x < n) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t b = blockIdx.x * kViewBlock + threadIdx.x;
    if (b < n_bettors) {
        const unsigned long long* __restrict__ row = wins + (size_t)b * stride;
        int best = 0;
        unsigned long long bw = row[0];
        for (int c = 1; c < n; ++c) {
            const unsigned long long w = row[c];
            if (w > bw) {
                bw = w;
                best = c;
            }
        }
        if (views) views[b] = (uint8_t)best;
        atomicAdd(&s_cnt[best], 1u);
    }
    __syncthreads();
    if (counts && (int)threadIdx.x < n && s_cnt[threadIdx.x])
        atomicAdd(&counts[threadIdx.x], s_cnt[threadIdx.x]);
}

__global__ void zero_u32_kernel(uint32_t* __restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------- launchers

template <int N>
static hipError_t launch_trace_n(const TraceArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(race_trace_kernel<N>, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int... I>
static hipError_t dispatch_trace(int n, const TraceArgs& a, hipStream_t s,
                                 std::integer_sequence<int, I...>) {
    using Fn = hipError_t (*)(const TraceArgs&, hipStream_t);
    static constexpr Fn table[] = {launch_trace_n<I + 1>...};
    return table[n - 1](a, s);
}

hipError_t launch_race_trace(const TraceArgs& a, hipStream_t s) {
    return dispatch_trace(a.rc.n, a, s, std::make_integer_sequence<int, kMaxN>{});
}

hipError_t launch_bettor_views(const ViewArgs& a, hipStream_t s) {
    if (a.n_eval == 0 || a.n_bettors == 0) return hipSuccess;
    if (a.counts) {
        const size_t total = (size_t)a.n_eval * a.n;
        hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                           s, a.counts, total);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const unsigned gx = (a.n_bettors + kViewBlock - 1) / kViewBlock;
    const unsigned gy_need = (a.n_eval + kViewRowsPerBlock - 1) / kViewRowsPerBlock;
    const unsigned gy = gy_need < 65535u ? gy_need : 65535u;
    hipLaunchKernelGGL(bettor_views_kernel, dim3(gx, gy), dim3(kViewBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rp_views(const unsigned long long* wins, uint32_t n_bettors, int n, int stride,
                           uint8_t* views, uint32_t* counts, hipStream_t s) {
    if (counts) {
        hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(256), 0, s, counts, (size_t)n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_bettors == 0) return hipSuccess;
    hipLaunchKernelGGL(rp_views_kernel, dim3((n_bettors + kViewBlock - 1) / kViewBlock),
                       dim3(kViewBlock), 0, s, wins, n_bettors, n, stride, views, counts);
    return hipGetLastError();
}

}  // namespace bbe
