// race_common.hpp -- device-side building blocks of the race model on gfx950.
//
// Race model: paper Section 3 and Eq. 1 (Cliff, Hawkins, Keen & Lau-Soto,
// EMSS 2021).  Every arithmetic step is single precision, one rounding per
// operation (the library is built with -ffp-contract=off), in the operation
// order that the C ABI documents, so that a simulation is a deterministic
// function of (race, state, seed, request, sim index).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bbe {

constexpr int kMaxN = 20;
constexpr uint32_t kTickLimit = 1u << 20;

// Per-race constants, each rounded once to float32 on the host:
//   elo = fl(P*lo), espan = fl(P*fl(hi - lo))   free step = elo + espan*u
//   alpha = fl(1 - rho), beta = fl(fl(2*rho)/L) R_c(d) = alpha + beta*d
//   theta                                        blocked iff gap <= theta
// The kernels take the draw as the integer k (a 16-bit half of a Philox
// word, u = k * 2^-16) and the span pre-scaled, espan16 = espan * 2^-16: a
// power-of-two scaling, exact whenever espan is 0 or at least 2^-110 (the
// host rejects other spans), so fl(espan16 * k) = fl(espan * u) bit for bit.
struct RaceConst {
    float L;
    int n;
    float elo[kMaxN];
    float espan16[kMaxN];
    float alpha[kMaxN];
    float beta[kMaxN];
    float theta[kMaxN];
};

// Time term of R (R += fl(gamma * min(t, tau)) on the absolute tick t);
// `paced` is set when some gamma != 0 and selects the kernels that evaluate
// it.  Kept apart from RaceConst, at the end of the argument blocks, so the
// plain kernels see the same argument layout as without it.
struct RacePace {
    float gamma[kMaxN];
    float tau[kMaxN];
    int paced;
};

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Each round forms the
// 64-bit products of the two even counter words with the round multipliers
// (one v_mad_u64_u32 each); the high halves are xored with the odd words
// and the round key (one three-input v_bitop3_b32 each once all three
// operands vary per lane), the low halves
// become the new odd words, and the key advances by the Weyl increments.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // truth table of a ^ b ^ c
}

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        // In the race kernels the counter words t, request and block are
        // wave-uniform and only `sim` varies per lane, so the first rounds
        // mix at most one lane-varying word into each xor: plain xors let
        // the compiler keep the uniform parts on the scalar unit there.
        uint32_t n0, n2;
        if (r < 3) {
            n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        } else {
            n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
            n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        }
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// The two draws of a Philox word as integers in [0, 2^16), exact in
// float32: the high half (even competitor) and the low half (odd
// competitor); the uniform of the model is u = k * 2^-16.
__device__ __forceinline__ float draw_hi(uint32_t w) {
    return (float)(w >> 16);
}
__device__ __forceinline__ float draw_lo(uint32_t w) {
    return (float)(w & 0xFFFFu);
}

}  // namespace bbe
