// mlp_kernels.hip -- the surrogate network on gfx950 matrix cores: a
// 160 -> 256 -> 256 -> 256 -> 20 perceptron (ReLU, masked softmax) mapping an
// encoded in-play race state to win probabilities, trained on Monte-Carlo
// win frequencies (the frequentist estimates of paper Section 3) with a
// soft cross-entropy and Adam.
//
// Products use v_mfma_f32_16x16x32_bf16: bfloat16 operands, float32
// accumulation.  Operand fragments (one 16x32 block of A, one 32x16 block of
// B per instruction): lane l holds row / column (l % 16) and the 8
// consecutive reduction indices 8*(l/16) .. 8*(l/16)+7; the 16x16 float
// result: lane l holds column (l % 16) of rows 4*(l/16) .. 4*(l/16)+3.
//
// Rounding points (round to nearest even): features, weights used in
// products, hidden activations after ReLU, dz and the back-propagated
// gradients; biases, logits, probabilities, loss and weight gradients are
// float32.
#include "mlp.hpp"

namespace bbe {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float floatx4;

__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 16 rows x 32 reduction indices from a row-major LDS tile (stride S).
__device__ __forceinline__ bf16x8 frag_lds(const uint16_t* t, int S, int row0, int k0, int lane) {
    return *reinterpret_cast<const bf16x8*>(t + (row0 + (lane & 15)) * S + k0 + 8 * (lane >> 4));
}
// 16 rows (of a [N][K] row-major global matrix) x 32 reduction indices.
__device__ __forceinline__ bf16x8 frag_glb(const uint16_t* __restrict__ W, int K, int n0, int k0,
                                          int lane) {
    return *reinterpret_cast<const bf16x8*>(W + (size_t)(n0 + (lane & 15)) * K + k0 +
                                            8 * (lane >> 4));
}

// acc[rb][cb] = in[16*RB x K] (LDS) * W[n_base .. n_base + 16*NCB, 0 .. K)^T.
// The k blocks are accumulated in the same order for every row, so a row's
// result does not depend on how many rows its workgroup holds.
template <int RB, int K, int NCB>
__device__ __forceinline__ void tile_gemm(const uint16_t* in, int S, const uint16_t* __restrict__ W,
                                          int n_base, floatx4 (&acc)[RB][NCB], int lane) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a[RB], b[NCB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) a[rb] = frag_lds(in, S, rb * 16, k0, lane);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) b[cb] = frag_glb(W, K, n_base + cb * 16, k0, lane);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = mfma(a[rb], b[cb], acc[rb][cb]);
    }
}

// Rows per workgroup of the forward and backward-data kernels: 16 * RB,
// RB = 1, 2 or 4, chosen per launch so that small batches still spread
// over the chip.
constexpr int kS = kHid + 8;         // LDS row stride of hidden tiles (bank spread)
constexpr int kSin = kIn + 8;        // LDS row stride of the feature tile
constexpr int kSout = kOutP + 8;     // LDS row stride of the dz tile

// Copies rows [row0, row0 + R) of a [B][K] bf16 matrix into an LDS tile
// (stride S), zero rows past B.  16-byte pieces.
template <int R, int K>
__device__ __forceinline__ void load_tile(uint16_t* t, int S, const uint16_t* __restrict__ g,
                                          int row0, int B) {
    constexpr int P = K / 8;
    for (int i = threadIdx.x; i < R * P; i += blockDim.x) {
        int r = i / P, c = (i - r * P) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (row0 + r < B) v = *reinterpret_cast<const uint4*>(g + (size_t)(row0 + r) * K + c);
        *reinterpret_cast<uint4*>(t + r * S + c) = v;
    }
}

// Hidden layer epilogue: bias, ReLU, bfloat16 into LDS (and global).
template <int RB, int NCB>
__device__ __forceinline__ void hidden_out(const floatx4 (&acc)[RB][NCB], int n_base,
                                           const float* __restrict__ bias, uint16_t* out, int S,
                                           uint16_t* __restrict__ g, int row0, int B, int lane) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int n = n_base + cb * 16 + (lane & 15);
            const float bn = bias[n];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = rb * 16 + 4 * (lane >> 4) + i;
                uint16_t h = to_bf16(fmaxf(acc[rb][cb][i] + bn, 0.0f));
                out[r * S + n] = h;
                if (g && row0 + r < B) g[(size_t)(row0 + r) * kHid + n] = h;
            }
        }
}

// Forward pass of 16 * RB rows; optional softmax cross-entropy epilogue.
template <int RB>
__global__ void __launch_bounds__(256) mlp_fwd_kernel(const MlpFwdArgs a) {
    constexpr int R = 16 * RB;
    __shared__ __attribute__((aligned(16))) uint16_t bufA[R * kS];
    __shared__ __attribute__((aligned(16))) uint16_t bufB[R * kS];
    __shared__ float logit[R][kOutP + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = blockIdx.x * R;

    load_tile<R, kIn>(bufA, kSin, a.x, row0, a.B);
    __syncthreads();
    {
        floatx4 acc[RB][4];
        tile_gemm<RB, kIn, 4>(bufA, kSin, a.w1, wave * 64, acc, lane);
        hidden_out<RB, 4>(acc, wave * 64, a.b1, bufB, kS, a.h1, row0, a.B, lane);
    }
    __syncthreads();
    {
        floatx4 acc[RB][4];
        tile_gemm<RB, kHid, 4>(bufB, kS, a.w2, wave * 64, acc, lane);
        hidden_out<RB, 4>(acc, wave * 64, a.b2, bufA, kS, a.h2, row0, a.B, lane);
    }
    __syncthreads();
    {
        floatx4 acc[RB][4];
        tile_gemm<RB, kHid, 4>(bufA, kS, a.w3, wave * 64, acc, lane);
        hidden_out<RB, 4>(acc, wave * 64, a.b3, bufB, kS, a.h3, row0, a.B, lane);
    }
    __syncthreads();
    if (wave < 2) {  // 32 padded outputs: two column blocks, one per wave
        floatx4 acc[RB][1];
        tile_gemm<RB, kHid, 1>(bufB, kS, a.w4, wave * 16, acc, lane);
        const int n = wave * 16 + (lane & 15);
        const float bn = n < kOut ? a.b4[n] : 0.0f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) logit[rb * 16 + 4 * (lane >> 4) + i][n] = acc[rb][0][i] + bn;
    }
    __syncthreads();

    // Masked softmax over the slots that hold a competitor, one row a thread.
    const int r = threadIdx.x;
    if (r < R && row0 + r < a.B) {
        const size_t row = (size_t)(row0 + r);
        const int nv = min(max(a.n_valid[row], 1), kOut);  // 1..20 slots hold competitors
        float mx = -__builtin_inff();
        for (int c = 0; c < nv; ++c) mx = fmaxf(mx, logit[r][c]);
        float e[kOut], sum = 0.0f;
        for (int c = 0; c < kOut; ++c) {
            e[c] = c < nv ? expf(logit[r][c] - mx) : 0.0f;
            sum += e[c];
        }
        const float inv = 1.0f / sum;
        float ent = 0.0f, ce = 0.0f;
        for (int c = 0; c < kOut; ++c) {
            float q = e[c] * inv;
            if (a.probs) a.probs[row * kOut + c] = q;
            if (a.logits) a.logits[row * kOutP + c] = c < nv ? logit[r][c] : -__builtin_inff();
            if (c < nv) {
                float lq = (logit[r][c] - mx) - logf(sum);
                if (q > 0.0f) ent -= q * lq;
                if (a.target) {
                    float p = a.target[row * kOut + c];
                    ce -= p * lq;
                    a.dz[row * kOutP + c] = to_bf16((q - p) * a.inv_batch);
                }
            } else if (a.target) {
                a.dz[row * kOutP + c] = 0;
            }
        }
        if (a.target)
            for (int c = kOut; c < kOutP; ++c) a.dz[row * kOutP + c] = 0;
        if (a.entropy) a.entropy[row] = ent;
        if (a.loss) atomicAdd(a.loss, ce * a.inv_batch);
    }
}

// Backward-data epilogue: gradient times ReLU mask of the forward
// activation, bfloat16 into LDS (if given) and global.
template <int RB>
__device__ __forceinline__ void grad_out(const floatx4 (&acc)[RB][4], int n_base,
                                         const uint16_t* __restrict__ h, uint16_t* out, int S,
                                         uint16_t* __restrict__ g, int row0, int B, int lane) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int n = n_base + cb * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = rb * 16 + 4 * (lane >> 4) + i;
                uint16_t v = 0;
                if (row0 + r < B && h[(size_t)(row0 + r) * kHid + n] != 0)
                    v = to_bf16(acc[rb][cb][i]);
                if (out) out[r * S + n] = v;
                if (row0 + r < B) g[(size_t)(row0 + r) * kHid + n] = v;
            }
        }
}

// Gradients with respect to the three hidden layers' pre-activations, for
// 16 * RB rows.
template <int RB>
__global__ void __launch_bounds__(256) mlp_bwd_data_kernel(const MlpBwdArgs a) {
    constexpr int R = 16 * RB;
    __shared__ __attribute__((aligned(16))) uint16_t bufA[R * kS];
    __shared__ __attribute__((aligned(16))) uint16_t bufB[R * kS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = blockIdx.x * R;
    load_tile<R, kOutP>(bufA, kSout, a.dz4, row0, a.B);
    __syncthreads();
    {
        floatx4 acc[RB][4];
        tile_gemm<RB, kOutP, 4>(bufA, kSout, a.w4t, wave * 64, acc, lane);
        grad_out<RB>(acc, wave * 64, a.h3, bufB, kS, a.dz3, row0, a.B, lane);
    }
    __syncthreads();
    {
        floatx4 acc[RB][4];
        tile_gemm<RB, kHid, 4>(bufB, kS, a.w3t, wave * 64, acc, lane);
        grad_out<RB>(acc, wave * 64, a.h2, bufA, kS, a.dz2, row0, a.B, lane);
    }
    __syncthreads();
    {
        floatx4 acc[RB][4];
        tile_gemm<RB, kHid, 4>(bufA, kS, a.w2t, wave * 64, acc, lane);
        grad_out<RB>(acc, wave * 64, a.h1, nullptr, kS, a.dz1, row0, a.B, lane);
    }
}

// Weight gradients dW[n][k] = sum over the batch rows of dz[r][n] * h[r][k],
// and bias gradients db[n] = sum over the rows of dz[r][n].
// One workgroup: a 64 (n) x 64 (k) tile of one layer over one chunk of
// kWgRows rows (blockIdx.y); it stores its tile once -- into the gradient
// itself when the batch is one chunk, else into that chunk's partial
// vector, which mlp_wreduce_kernel sums in chunk order.  The tile at k0 = 0
// also sums its 64 dz columns over the chunk (each wave a quarter of the
// rows in order, the quarters added in wave order) for the bias gradient.
// No atomics, so the gradient (and training) is the same bit for bit from
// run to run.  Both operands are staged transposed in LDS so that fragments
// are contiguous.
constexpr int kWgS = kWgRows + 8;

__global__ void __launch_bounds__(256) mlp_wgrad_kernel(const MlpWgradArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t tz[64 * kWgS];  // [n][r]
    __shared__ __attribute__((aligned(16))) uint16_t th[64 * kWgS];  // [k][r]
    const WgradTile t = a.tiles[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r0 = blockIdx.y * kWgRows;
    const LayerGrad& L = a.layers[t.layer];
    // stage: element (r, n) of dz -> tz[n][r]; (r, k) of h -> th[k][r]
    for (int i = threadIdx.x; i < kWgRows * 64; i += blockDim.x) {
        int r = i >> 6, c = i & 63;
        int row = r0 + r;
        uint16_t z = 0, h = 0;
        if (row < a.B) {
            if (t.n0 + c < L.n_rows) z = L.dz[(size_t)row * L.dz_stride + t.n0 + c];
            if (t.k0 + c < L.K) h = L.h[(size_t)row * L.K + t.k0 + c];
        }
        tz[c * kWgS + r] = z;
        th[c * kWgS + r] = h;
    }
    __syncthreads();
    // wave w: n rows [16w, 16w+16) of the tile, all 64 k columns
    floatx4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < kWgRows; k0 += 32) {
        bf16x8 fa = frag_lds(tz, kWgS, wave * 16, k0, lane);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma(fa, frag_lds(th, kWgS, cb * 16, k0, lane), acc[cb]);
    }
    float* out = gridDim.y == 1 ? L.gw : a.part + (size_t)blockIdx.y * kNParams + L.woff;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int k = t.k0 + cb * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int n = t.n0 + wave * 16 + 4 * (lane >> 4) + i;
            if (n < L.n_rows && k < L.K) out[(size_t)n * L.K + k] = acc[cb][i];
        }
    }
    if (t.k0 == 0) {  // uniform per workgroup
        __shared__ float bpart[4][64];
        constexpr int kQ = kWgRows / 4;
        float sum = 0.0f;
        const uint16_t* col = tz + lane * kWgS + wave * kQ;
        for (int r = 0; r < kQ; ++r) sum += from_bf16(col[r]);
        bpart[wave][lane] = sum;
        __syncthreads();
        const int n = t.n0 + lane;
        if (wave == 0 && n < L.n_rows) {
            const float b = ((bpart[0][lane] + bpart[1][lane]) + bpart[2][lane]) + bpart[3][lane];
            if (gridDim.y == 1)
                L.gb[n] = b;
            else
                a.part[(size_t)blockIdx.y * kNParams + L.woff + L.n_rows * L.K + n] = b;
        }
    }
}

// Sum of the per-chunk partial gradients (weights and biases), chunk 0
// first: one thread per parameter of the four layers (each layer's weights
// then its bias, as packed).
__global__ void __launch_bounds__(256) mlp_wreduce_kernel(const MlpWgradArgs a, int n_chunks) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const LayerGrad& L = a.layers[l];
        const int nw = L.n_rows * L.K;
        if (i < nw + L.n_rows) {
            const float* p = a.part + L.woff + i;
            float s = p[0];
            for (int c = 1; c < n_chunks; ++c) s += p[(size_t)c * kNParams];
            if (i < nw)
                L.gw[i] = s;
            else
                L.gb[i - nw] = s;
            return;
        }
        i -= nw + L.n_rows;
    }
}

// Adam on the float32 master parameters (optional) and refresh of the
// bfloat16 copies used by the products: w[n][k] and, for layers 2-4, the
// transposed copy wt[k][n].
__global__ void mlp_adam_kernel(const MlpAdamArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    float w = a.params[i];
    if (a.grad) {
        const float g = a.grad[i];
        const float m = a.beta1 * a.m[i] + (1.0f - a.beta1) * g;
        const float v = a.beta2 * a.v[i] + (1.0f - a.beta2) * (g * g);
        a.m[i] = m;
        a.v[i] = v;
        const float mh = m * a.inv_bc1;
        const float vh = v * a.inv_bc2;
        w = w - a.lr * mh / (sqrtf(vh) + a.eps);
        a.params[i] = w;
    }
    const uint16_t h = to_bf16(w);
    // locate i in the packed layout
    if (i < kOffB1) {
        a.w1[i] = h;
    } else if (i >= kOffW2 && i < kOffB2) {
        int j = i - kOffW2, n = j / kHid, k = j - n * kHid;
        a.w2[j] = h;
        a.w2t[k * kHid + n] = h;
    } else if (i >= kOffW3 && i < kOffB3) {
        int j = i - kOffW3, n = j / kHid, k = j - n * kHid;
        a.w3[j] = h;
        a.w3t[k * kHid + n] = h;
    } else if (i >= kOffW4 && i < kOffB4) {
        int j = i - kOffW4, n = j / kHid, k = j - n * kHid;
        a.w4[j] = h;
        a.w4t[k * kOutP + n] = h;
    }
}

// State encoding: one state per half-wave (32 lanes), lane c of the half
// for competitor c.  Slots hold competitors by expected remaining ticks
// T = (L-d) / ((lo+hi)*0.5 * (1 + rho*d/L)) (R_c taken at the midpoint of
// the remaining distance), smallest first, equal T by lower index: a
// competitor's slot is the number of competitors before it in that order.
// Early in a race that orders the field by strength, late in it by
// position.  Positions enter only relative to other competitors or to the
// line (bfloat16 keeps about 2.5 significant digits: an absolute position
// would lose the gaps that decide a race).  8 float32 features per slot,
// rounded to bfloat16: remaining distance (L-d)/L, gap to the leader /
// (75 dt), gap to the competitor directly ahead on the track (position
// order, equal positions by lower index) / (7.5 dt) capped at 4 (4 for the
// leader), previous step / (7.5 dt), mean free step (lo+hi)/(15 dt),
// (hi-lo)/(hi+lo), rho/0.2, and (T - T_min)/10; zero padding.  Each lane
// writes its slot's 8 features as one 16-byte store, so a state's 320-byte
// row is written by 20 adjacent stores.
__global__ void __launch_bounds__(256) encode_kernel(const EncodeArgs a) {
    const int lane = threadIdx.x & 63;
    const int half = lane & 32;                // first lane of this state's half-wave
    const int c = lane & 31;                   // competitor of this lane
    const long b = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 5;  // state
    const bool in = b < a.B;
    const int n = in ? min(max(a.n[b], 0), kMaxN) : 0;
    const bool act = c < n;
    const float L = a.track_len;
    float d = 0.0f, s = 0.0f, lo = 0.0f, hi = 0.0f, rho = 0.0f;
    if (act) {
        d = a.pos[b * kMaxN + c];
        s = a.prev[b * kMaxN + c];
        const float* cp = a.comp + (b * kMaxN + c) * 5;
        lo = cp[0];
        hi = cp[1];
        rho = cp[3];
    }
    const float rmid = 1.0f + rho * (d / L);
    const float T = act ? (L - d) / (((lo + hi) * 0.5f) * rmid) : __builtin_inff();
    // slot = competitors before this one in (T, index) order; the position
    // of the competitor directly ahead on the track; the leader's position;
    // the smallest expected remaining time
    int slot = 0;
    bool has_ahead = false;
    float d_above = __builtin_inff(), d_lead = -__builtin_inff(), tmin = __builtin_inff();
    // every lane runs all kMaxN steps (the two halves may hold different n)
    for (int i = 0; i < kMaxN; ++i) {
        const float di = __shfl(d, half + i, 64);
        const float Ti = __shfl(T, half + i, 64);
        const bool valid = i < n;
        slot += (valid && (Ti < T || (Ti == T && i < c))) ? 1 : 0;
        // directly ahead: the lowest of those ahead in (position, index) order
        const bool ahead = valid && (di > d || (di == d && i < c));
        has_ahead = has_ahead || ahead;
        d_above = ahead ? fminf(d_above, di) : d_above;
        d_lead = valid ? fmaxf(d_lead, di) : d_lead;
        tmin = valid ? fminf(tmin, Ti) : tmin;
    }
    if (!in || c >= kMaxN) return;
    uint16_t* x = a.x + b * kIn;
    if (act) {
        const float gap = has_ahead ? fminf((d_above - d) / a.c75, 4.0f) : 4.0f;
        const float f[8] = {(L - d) / L,     (d_lead - d) / a.c750, gap,
                            s / a.c75,       (lo + hi) / a.c15,     (hi - lo) / (hi + lo),
                            rho / 0.2f,      (T - tmin) / 10.0f};
        uint4 v;
        v.x = (uint32_t)to_bf16(f[0]) | ((uint32_t)to_bf16(f[1]) << 16);
        v.y = (uint32_t)to_bf16(f[2]) | ((uint32_t)to_bf16(f[3]) << 16);
        v.z = (uint32_t)to_bf16(f[4]) | ((uint32_t)to_bf16(f[5]) << 16);
        v.w = (uint32_t)to_bf16(f[6]) | ((uint32_t)to_bf16(f[7]) << 16);
        *reinterpret_cast<uint4*>(x + slot * 8) = v;
        if (a.slot) a.slot[b * kMaxN + slot] = c;
        if (a.target) a.target[b * kMaxN + slot] = (float)a.probs_in[b * kMaxN + c];
    } else {
        // lanes n .. 19 clear the padding slots n .. 19
        *reinterpret_cast<uint4*>(x + c * 8) = make_uint4(0u, 0u, 0u, 0u);
        if (a.slot) a.slot[b * kMaxN + c] = -1;
        if (a.target) a.target[b * kMaxN + c] = 0.0f;
    }
}

__global__ void fill_f32_kernel(float* __restrict__ p, float v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- launchers

// Row blocks per workgroup for a batch: the most (up to 4) that still give
// at least 256 workgroups, else 1.
static int row_blocks(int B) {
    if ((B + 63) / 64 >= 256) return 4;
    if ((B + 31) / 32 >= 256) return 2;
    return 1;
}
hipError_t launch_mlp_fwd(const MlpFwdArgs& a, hipStream_t s) {
    switch (row_blocks(a.B)) {
        case 4: hipLaunchKernelGGL(mlp_fwd_kernel<4>, dim3((a.B + 63) / 64), dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(mlp_fwd_kernel<2>, dim3((a.B + 31) / 32), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(mlp_fwd_kernel<1>, dim3((a.B + 15) / 16), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}
hipError_t launch_mlp_bwd_data(const MlpBwdArgs& a, hipStream_t s) {
    switch (row_blocks(a.B)) {
        case 4: hipLaunchKernelGGL(mlp_bwd_data_kernel<4>, dim3((a.B + 63) / 64), dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(mlp_bwd_data_kernel<2>, dim3((a.B + 31) / 32), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(mlp_bwd_data_kernel<1>, dim3((a.B + 15) / 16), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}
hipError_t launch_mlp_wgrad(const MlpWgradArgs& a, int n_tiles, hipStream_t s) {
    const int n_chunks = (a.B + kWgRows - 1) / kWgRows;
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(n_tiles, n_chunks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n_chunks > 1) {
        hipLaunchKernelGGL(mlp_wreduce_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, s, a,
                           n_chunks);
        e = hipGetLastError();
    }
    return e;
}
hipError_t launch_mlp_adam(const MlpAdamArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_encode(const EncodeArgs& a, hipStream_t s) {
    // 8 states per 256-thread workgroup
    hipLaunchKernelGGL(encode_kernel, dim3((unsigned)(((long)a.B + 7) / 8)), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, float v, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace bbe
