// mlp.hpp -- sizes, packed parameter layout and kernel arguments of the
// surrogate network.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "race_common.hpp"

namespace bbe {

constexpr int kIn = 160;    // 20 slots x 8 features
constexpr int kHid = 256;
constexpr int kOut = 20;
constexpr int kOutP = 32;   // output rows padded to two 16-wide blocks

// Packed float32 parameters: W1 [256][160], b1, W2 [256][256], b2,
// W3 [256][256], b3, W4 [20][256], b4.
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHid * kIn;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kHid;
constexpr int kOffW4 = kOffB3 + kHid;
constexpr int kOffB4 = kOffW4 + kOut * kHid;
constexpr int kNParams = kOffB4 + kOut;
static_assert(kNParams == 177940, "parameter count");

struct MlpFwdArgs {
    const uint16_t* x;        // [B][160] bf16
    const int32_t* n_valid;   // [B]
    int B;
    const uint16_t *w1, *w2, *w3, *w4;  // bf16 [256][160], [256][256] x2, [32][256]
    const float *b1, *b2, *b3, *b4;
    uint16_t *h1, *h2, *h3;   // [B][256] bf16 or null
    float* probs;             // [B][20] or null
    float* entropy;           // [B] or null
    float* logits;            // [B][32] or null
    const float* target;      // [B][20] or null (training)
    uint16_t* dz;             // [B][32] bf16 (training)
    float* loss;              // [1] (training, accumulated)
    float inv_batch;
};

struct MlpBwdArgs {
    int B;
    const uint16_t* dz4;  // [B][32]
    const uint16_t *w4t, *w3t, *w2t;  // [256][32], [256][256], [256][256]
    const uint16_t *h1, *h2, *h3;
    uint16_t *dz3, *dz2, *dz1;  // [B][256]
};

struct LayerGrad {
    const uint16_t* dz;  // [B][dz_stride]
    int dz_stride;
    const uint16_t* h;   // [B][K] input of the layer
    int K;
    int n_rows;          // outputs of the layer
    float* gw;           // [n_rows][K]
    float* gb;           // [n_rows]
    int woff;            // offset of gw in the packed parameter vector
};

// Rows of the batch per weight-gradient work item.
constexpr int kWgRows = 256;

struct WgradTile {
    int layer, n0, k0, pad;
};

struct MlpWgradArgs {
    int B;
    LayerGrad layers[4];
    const WgradTile* tiles;
    // partial weight gradients, one packed parameter vector per chunk of
    // kWgRows rows (needed when B > kWgRows); summed in chunk order
    float* part;
};

struct MlpAdamArgs {
    float* params;
    float *m, *v;
    const float* grad;  // null: refresh the bf16 copies only
    float lr, beta1, beta2, eps, inv_bc1, inv_bc2;
    uint16_t *w1, *w2, *w3, *w4, *w2t, *w3t, *w4t;
};

struct EncodeArgs {
    const float* comp;   // [B][20][5]
    const int32_t* n;    // [B]
    const float* pos;    // [B][20]
    const float* prev;   // [B][20]
    int B;
    float track_len, c75, c15, c750;  // 7.5 dt, 15 dt, 75 dt
    uint16_t* x;         // [B][160]
    int32_t* slot;       // [B][20] or null
    const double* probs_in;  // [B][20] competitor order, or null
    float* target;           // [B][20] slot order (with probs_in)
};

hipError_t launch_mlp_fwd(const MlpFwdArgs& a, hipStream_t s);
hipError_t launch_mlp_bwd_data(const MlpBwdArgs& a, hipStream_t s);
hipError_t launch_mlp_wgrad(const MlpWgradArgs& a, int n_tiles, hipStream_t s);
hipError_t launch_mlp_adam(const MlpAdamArgs& a, hipStream_t s);
hipError_t launch_encode(const EncodeArgs& a, hipStream_t s);
hipError_t launch_fill_f32(float* p, float v, int n, hipStream_t s);

}  // namespace bbe
