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
// up to kViewRowsPerBlock trace rows.  The bettors are stored grouped by
// kind, so nearly every wave runs a single rule.  Per row the block stages
// the positions in LDS, one thread finds the leader and the runner-up, and
// every thread forms its view:
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
// global atomic per competitor per block.
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
            slots_tick<N>(sl, smem, ucol, kPar, a.rc.L, t, a.sim, a.request, a.k0, a.k1);
        if (cross) break;
        t += 1;
        slots_restore<N>(sl);
        slots_store_pos<N>(sl, kPar, a.trace + (size_t)rows * N);
        ++rows;
    }
    *a.rows_out = rows;
}

__global__ void __launch_bounds__(kViewBlock) bettor_views_kernel(const ViewArgs a) {
    __shared__ float s_x[kMaxN];
    __shared__ uint32_t s_cnt[kMaxN];
    __shared__ int s_p1, s_p2;
    __shared__ float s_gap;
    const int n = a.n;
    const uint32_t j = blockIdx.x * kViewBlock + threadIdx.x;
    const bool have = j < a.n_bettors;
    const uint8_t kind = have ? a.kind[j] : (uint8_t)kLW;
    const float param = have ? a.param[j] : 0.0f;
    const uint32_t id = have ? a.id[j] : 0u;

    for (uint32_t i0 = blockIdx.y * kViewRowsPerBlock; i0 < a.n_eval;
         i0 += gridDim.y * kViewRowsPerBlock) {
        const uint32_t i1 = min(i0 + (uint32_t)kViewRowsPerBlock, a.n_eval);
        for (uint32_t i = i0; i < i1; ++i) {
            const uint32_t r = a.first_row + i;
            if ((int)threadIdx.x < n) {
                s_x[threadIdx.x] = a.trace[(size_t)r * n + threadIdx.x];
                s_cnt[threadIdx.x] = 0u;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int p1 = 0;
                for (int c = 1; c < n; ++c)
                    if (s_x[c] > s_x[p1]) p1 = c;
                int p2 = -1;
                for (int c = 0; c < n; ++c)
                    if (c != p1 && (p2 < 0 || s_x[c] > s_x[p2])) p2 = c;
                s_p1 = p1;
                s_p2 = p2 < 0 ? p1 : p2;
                s_gap = p2 < 0 ? 0.0f : s_x[p1] - s_x[p2];
            }
            __syncthreads();

            int v = s_p1;
            if (kind == kZI) {
                const U4 w = philox4x32_10(a.t0 + r, id, 0xFFFFFFFFu, 0xFFFFFFFFu, a.k0, a.k1);
                v = (int)(((uint64_t)w.x * (uint32_t)n) >> 32);
            } else if (kind == kUD) {
                if (n > 1 && s_gap < param) v = s_p2;
            } else if (kind == kLinEx) {
                const uint32_t w = min((uint32_t)param, r);
                if (w > 0) {
                    const float* __restrict__ back = a.trace + (size_t)(r - w) * n;
                    int best = -1;
                    float br = 0.0f, bd = 1.0f;
                    for (int c = 0; c < n; ++c) {
                        const float xc = s_x[c];
                        const float disp = xc - back[c];
                        if (disp > 0.0f) {
                            const float rem = a.L - xc;
                            if (best < 0 || (double)rem * (double)bd < (double)br * (double)disp) {
                                best = c;
                                br = rem;
                                bd = disp;
                            }
                        }
                    }
                    if (best >= 0) v = best;
                }
            }
            if (have) {
                if (a.views) a.views[(size_t)i * a.n_bettors + id] = (uint8_t)v;
                atomicAdd(&s_cnt[v], 1u);
            }
            __syncthreads();
            if (a.counts && (int)threadIdx.x < n && s_cnt[threadIdx.x])
                atomicAdd(&a.counts[(size_t)i * n + threadIdx.x], s_cnt[threadIdx.x]);
        }
    }
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

}  // namespace bbe
